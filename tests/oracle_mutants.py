"""Mutation check of the oracle pins (run by hand: ``python tests/oracle_mutants.py``).

Each entry plants one plausible mistake in a copy of the oracle source, builds it into
a temporary library, and runs ``tests/test_oracle_pins.py`` against it through the
``ECMC_ORACLE_LIB`` override.  A pin suite worth trusting fails on every mutant except
the ones marked equivalent (they change no observable result).
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC_PATH = os.path.join(ROOT, "oracle", "ecmc_oracle.c")

MUTANTS = {
    "hs_plus": ("double v = dpar - sqrt(s->sig2 - dperp2);", "double v = dpar + sqrt(s->sig2 - dperp2);"),
    "tether_minus": ("double v = dpar + sqrt(t);", "double v = dpar - sqrt(t);"),
    "perp_drop": ("*dperp2 = pb + pc;", "*dperp2 = pb;"),
    "wrap_sign": ("if (w[a] > 0) d[a] = d[a] + s->L;", "if (w[a] > 0) d[a] = d[a] - s->L;"),
    "dpar_sign": ("*dpar = sgn > 0 ? d[axis] : -d[axis];", "*dpar = d[axis];"),
    "no_tether": ("consider(&best, tether_candidate(s, dpar, dperp2), q, 1, dpar);\n    }\n    return best;",
                  "}\n    return best;"),
    "delta_sign": ("s->sum_delta += b.dpar - b.x;", "s->sum_delta += b.dpar + b.x;"),
    "no_reflect": ("sgn = -sgn;\n            }\n            continue;", "p = b.j;\n            }\n            continue;"),
    "wall_pass": ("if (cell_in_domain(s, dm, cn)) {", "if (1) {"),
    "cell_skip": ("for (int dx = -1; dx <= 1; ++dx) {\n                const int raw",
                  "for (int dx = -1; dx <= 0; ++dx) {\n                const int raw"),
    "rg_index": ("if (rg2) rg2[q] = g / (double)N;", "if (rg2) rg2[q] = g / (double)(N - 1);"),
    "pivot_rng": ("const int32_t p = mot[below(u[0], (uint32_t)m)];",
                  "const int32_t p = mot[below(u[0], (uint32_t)(m > 1 ? m - 1 : m))];"),
    "period_half": ("const double r = fmod(*xmax, W + W);", "const double r = fmod(*xmax, W);"),
    "swap_skip_j": ("        if (u >= 0 && dist2(s, rp, u == p ? rj : &s->r[3 * u]) > s->b2) return 0;\n", ""),
    "swap_image_sign": ("        s->img[3 * p + a] += sh;", "        s->img[3 * p + a] -= sh;"),
    # equivalent mutants: no observable difference is expected
    # (W = 0 means every event between the two reflections had zero length, so the zero-length
    # cycle search ends the same EC a few steps later with the same positions)
    "period_no_cycle (equivalent)": ("if (!(W > 0.0)) {", "if (W < 0.0) {"),
    "tie_kind (equivalent)": ("(j == b->j && kind < b->kind)", "(j == b->j && kind > b->kind)"),
    "face_add (rounding only)": ("*ra = sgn > 0 ? s->bnd[c + 1] : s->bnd[c];", "*ra = sgn > 0 ? *ra + xc : *ra - xc;"),
}


def main(names):
    src = open(SRC_PATH).read()
    header = os.path.join(ROOT, "oracle", "ecmc_oracle.h")
    bad = 0
    for name in names or list(MUTANTS):
        a, b = MUTANTS[name]
        assert src.count(a) == 1, name
        d = tempfile.mkdtemp()
        with open(os.path.join(d, "m.c"), "w") as f:
            f.write(src.replace(a, b).replace('#include "ecmc_oracle.h"', f'#include "{header}"'))
        lib = os.path.join(d, "lib.so")
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-o", lib,
                        os.path.join(d, "m.c"), "-lm"], check=True)
        env = dict(os.environ, ECMC_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                            os.path.join(HERE, "test_oracle_pins.py")], env=env, capture_output=True, text=True,
                           cwd=ROOT)
        caught = r.returncode != 0
        if not caught and "(" not in name:
            bad += 1
        tail = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
        print(f"{name:28s} {'CAUGHT' if caught else 'missed'}  {tail}", flush=True)
    return bad


if __name__ == "__main__":
    sys.exit(1 if main(sys.argv[1:]) else 0)
