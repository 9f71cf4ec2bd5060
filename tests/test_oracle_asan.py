"""The oracle under AddressSanitizer, LeakSanitizer and UndefinedBehaviorSanitizer (host only).

tests/asan_oracle_driver.c drives every oracle path on small melts; this test builds it with gcc
and the sanitizers into a temporary directory and runs it.  Any invalid access, leak or undefined
operation ends the run with a non-zero status and a report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_is_clean_under_address_leak_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_oracle")
    build = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "oracle"),
             os.path.join(HERE, "asan_oracle_driver.c"), os.path.join(ROOT, "oracle", "ecmc_oracle.c"), "-lm", "-o", exe]
    subprocess.run(build, check=True, capture_output=True, text=True, timeout=120)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "every path ran" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
