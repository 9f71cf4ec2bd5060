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
    "no_tether": ("consider(&best, orc_bond_x(s, dpar, dperp2, g ? g[t] : -1.0), q, 1, dpar);\n    }\n    return best;",
                  "}\n    return best;"),
    "delta_sign": ("ORC_C_TETHER_LIFT]++;\n                s->sum_delta += b.dpar - b.x;",
                   "ORC_C_TETHER_LIFT]++;\n                s->sum_delta += b.dpar + b.x;"),
    "no_reflect": ("sgn = -sgn;\n            }\n            continue;", "p = b.j;\n            }\n            continue;"),
    "wall_pass": ("if (cell_in_domain(s, dm, cn)) {", "if (1) {"),
    "cell_skip": ("for (int dx = -1; dx <= 1; ++dx) {\n                const int raw",
                  "for (int dx = -1; dx <= 0; ++dx) {\n                const int raw"),
    "rg_index": ("if (rg2) rg2[q] = g / (double)N;", "if (rg2) rg2[q] = g / (double)(N - 1);"),
    "pivot_rng": ("const int32_t p = starts[below(u[0], (uint32_t)ms)];\n                            const uint32_t",
                  "const int32_t p = starts[below(u[0], (uint32_t)(ms > 1 ? ms - 1 : ms))];\n"
                  "                            const uint32_t"),
    "period_half": ("const double r = fmod(*xmax, W + W);", "const double r = fmod(*xmax, W);"),
    "swap_skip_j": ("        if (u >= 0 && dist2(s, rp, u == p ? rj : &s->r[3 * u]) > s->b2) return 0;\n", ""),
    "swap_image_sign": ("        s->img[3 * p + a] += sh;", "        s->img[3 * p + a] -= sh;"),
    "spring_b0_present": ("sqrt(dpar > 0.0 ? dperp2 : dpar * dpar + dperp2)", "sqrt(dpar * dpar + dperp2)"),
    "spring_energy_sign": ("sqrt(e * e + g)", "sqrt(fabs(e * e - g))"),
    "spring_no_cap": ("    if (be2 > s->b2) be2 = s->b2;\n", ""),
    "spring_half_energy": ("g[t] = -orc_ln(u) * s->two_over_k;", "g[t] = -orc_ln(u) * s->two_over_k * 0.5;"),
    "spring_stale_draw": ("const uint32_t ctr[4] = {step, dm->ec, dm->domain, dm->sweep};",
                          "const uint32_t ctr[4] = {0u, dm->ec, dm->domain, dm->sweep};"),
    "ln_series_short": ("for (int n = 10; n >= 0; --n)", "for (int n = 8; n >= 0; --n)"),
    "ln_reduction": ("if (f < 0.70710678118654752440) {", "if (f < 0.5) {"),
    "pair_drop_z": ("const double r = sqrt((q0 + q1) + q2);", "const double r = sqrt(q0 + q1);"),
    "pair_twice": ("for (int64_t j = i + 1; j < s->nb; ++j) {\n            double d[3];",
                   "for (int64_t j = 0; j < s->nb; ++j) {\n            if (j == i) continue;\n            double d[3];"),
    "pair_no_image": ("for (int a = 0; a < 3; ++a) d[a] = mi(s, s->r[3 * j + a] - s->r[3 * i + a]);\n            const double q0",
                      "for (int a = 0; a < 3; ++a) d[a] = s->r[3 * j + a] - s->r[3 * i + a];\n            const double q0"),
    "r2n_lag_shift": ("sum[t2 - t] += (q0 + q1) + q2;", "sum[t2 - t - 1] += (q0 + q1) + q2;"),
    "r2n_no_image": ("for (int k = 0; k < 3; ++k) R[k] += mi(s, s->r[3 * i1 + k] - s->r[3 * i0 + k]);",
                     "for (int k = 0; k < 3; ++k) R[k] += s->r[3 * i1 + k] - s->r[3 * i0 + k];"),
    "r2n_drop_z": ("sum[t2 - t] += (q0 + q1) + q2;", "sum[t2 - t] += q0 + q1;"),
    "e2e_squared": ("floor(sqrt(r2[q]) / rmax * (double)nbins)", "floor(r2[q] / rmax * (double)nbins)"),
    "push_no_ignore": ("    if (s->push && dpar * dpar + dperp2 < s->ov2) return 0; /* push-off: an overlapping pair */\n", ""),
    "push_start_all": ("if (!s->push || overlaps_any(s, list[i])) out[k++] = list[i];", "out[k++] = list[i];"),
    "push_margin": ("s->ov2 = s->sig2 * (1.0 - 1e-9);", "s->ov2 = s->sig2 * (1.0 + 1e-9);"),
    # the periodic reduction: applied from the first reflection on (it then ends every EC at its
    # first reflection), or the switch to the plain loop ignored
    "period_first_reflection": ("ORC_C_WALL]++;\n            if (!s->spring && !s->no_skip && reflected && periodic(",
                                "ORC_C_WALL]++;\n            if (!s->spring && !s->no_skip && periodic("),
    "plain_loop_ignored": ("s->no_skip = on ? 0 : 1;", "s->no_skip = 0;"),
    # the zero-length cycle search never finds the repeated state
    "cycle_never_detected": ("if (p == saved_p && sgn == saved_sgn && c == saved_c) {", "if (0) {"),
    # tile-joint with 1-cell tiles accepted (no bead could leave its cell)
    "joint_accepts_single_cells": ("(tiling == 2 && (D < 2 ||", "(tiling == 2 && (D < 1 ||"),
    "joint_moves": ("        if (((c[a] - dm->off[a]) % s->n + s->n) % s->n % dm->P >= dm->D) return 0;\n", ""),
    # equivalent mutants: no observable difference is expected
    # (W = 0 means every event between the two reflections had zero length, so the zero-length
    # cycle search ends the same EC a few steps later with the same positions)
    "period_no_cycle (equivalent)": ("if (!(W > 0.0)) {", "if (W < 0.0) {"),
    "tie_kind (equivalent)": ("(j == b->j && kind < b->kind)", "(j == b->j && kind > b->kind)"),
    # (the two energies of a step are independent uniforms: which bond takes which changes
    # trajectories, which the GPU parity tests see, but no distribution)
    "spring_slot_swap (equivalent)": ("consider(&best, orc_bond_x(s, dpar, dperp2, g ? g[t] : -1.0), q, 1, dpar);",
                                      "consider(&best, orc_bond_x(s, dpar, dperp2, g ? g[1 - t] : -1.0), q, 1, dpar);"),
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
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
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
