"""Build the gfx950 library ``libecmc.so`` in-tree with hipcc.

Flags: -O3, IEEE binary64 without contraction (-ffp-contract=off: the event
arithmetic must be reproducible bit for bit), packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libecmc.so")
# (source, extra macros, object tag): the phase and sweep kernels are built a second time for
# harmonic springs, the sweep kernel a third time for the push-off
SOURCES = [(os.path.join(CSRC, f), d, t) for f, d, t in (
    ("ecmc_kernels.hip", (), ""), ("ecmc_phase.hip", (), ""), ("ecmc_phase.hip", ("ECMC_SPRING_TU=1",), ".spring"),
    ("ecmc_sweep.hip", (), ""), ("ecmc_sweep.hip", ("ECMC_SPRING_TU=1",), ".spring"),
    ("ecmc_sweep.hip", ("ECMC_PUSH_TU=1",), ".push"), ("ecmc_api.cpp", (), ""))]
HEADERS = [os.path.join(CSRC, f) for f in ("ecmc_device.h", "ecmc_internal.h")]
ARCH = os.environ.get("ECMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libecmc.so)")


def build(verbose: bool = False, out: str = LIB, defines: tuple = ()) -> str:
    """Compile the library to ``out``; ``defines`` are extra -D macros (tuning knobs).

    Each source is compiled to an object of its own, all at once, then linked."""
    from concurrent.futures import ThreadPoolExecutor
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-ffp-contract=off", "-fno-fast-math",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include")] + [f"-D{d}" for d in defines]
    objs = [out + "." + os.path.basename(src) + tag + ".o" for src, _, tag in SOURCES]

    def compile_one(src_obj):
        (src, extra, _), obj = src_obj
        cmd = [hipcc()] + flags + [f"-D{d}" for d in extra] + ["-c", "-o", obj, "-x", "hip", src]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd).returncode

    try:
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            codes = list(ex.map(compile_one, zip(SOURCES, objs)))
        if any(codes):
            raise subprocess.CalledProcessError(max(codes), "hipcc -c")
        tmp = out + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
