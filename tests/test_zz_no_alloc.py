"""The allocation-free R^2(n) entry point (partial sums in the library's static per-device array)
against the workspace entry point, through the C ABI, and against the oracle.

Both entry points run the same kernels with the same number of blocks, so the sums are taken in
the same order and the results must be identical; the oracle's are within the rounding bound of
the R^2(n) sums (Sec. II.B).  Two calls in a row share the one array: the second, on a smaller
input, must not see what the first left there.
"""
import numpy as np
import pytest

import oracle
from paper_1502_06447_amd import ecmc, inputs

pytestmark = pytest.mark.gpu


def _tol(pairs):
    return 1e-11 + pairs.max() * 2.0 ** -53


def test_noalloc_internal_distances_match_the_workspace_call():
    big = inputs.lattice_chains(16384, 64, 0.45, seed=3)    # 1,048,576 beads: all 2^20 partial-sum slots
    small = inputs.lattice_chains(500, 32, 0.45, seed=2)    # 500 blocks x 41 lags
    gb = ecmc.Melt.from_melt(big, ecmc.Options())
    opts = dict(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16)
    gs = ecmc.Melt.from_melt(small, ecmc.Options(**opts))
    os_ = oracle.Oracle.from_melt(small, n_cells=16)
    for s in range(2):
        gs.sweep(16000, 20.0, 610 + s)
        os_.sweep(16000, 20.0, 610 + s, tiling=ecmc.TILING_CHECKER, D=2)
    gs.synchronize()
    assert np.array_equal(gs.positions(), os_.positions())

    # first call: the benchmark-sized melt fills the whole array
    print("noalloc: 16384 x 64, n_max 63", flush=True)
    r2n, cn = gb.internal_distances_noalloc(63)
    r2w, cw = gb.internal_distances(63)
    assert np.array_equal(cn, cw) and cn[63] == 16384
    assert np.array_equal(r2n, r2w)
    ro, co = oracle.Oracle.from_melt(big, n_cells=gb.n_cells).internal_distances(63)
    assert np.array_equal(cn, co)
    assert np.allclose(r2n, ro, rtol=_tol(cn), atol=0), np.abs(r2n[1:] / ro[1:] - 1).max()

    # second call: a smaller input on the array the first call left full
    print("noalloc: 500 x 32, n_max 40", flush=True)
    r2n2, cn2 = gs.internal_distances_noalloc(40)
    r2w2, cw2 = gs.internal_distances(40)
    assert np.array_equal(cn2, cw2) and np.array_equal(r2n2, r2w2)
    ro2, co2 = os_.internal_distances(40)
    assert np.array_equal(cn2, co2)
    assert np.allclose(r2n2, ro2, rtol=_tol(cn2), atol=0)
    assert np.all(r2n2[32:] == 0.0) and r2n2[0] == 0.0

    # the large input again, after the small one: the same result as the first time
    r2n3, _ = gb.internal_distances_noalloc(63)
    assert np.array_equal(r2n3, r2n)


def test_noalloc_internal_distances_refuse_what_the_workspace_call_refuses():
    small = inputs.saw_chains(16, 16, 0.30, seed=1)
    g = ecmc.Melt.from_melt(small, ecmc.Options(tiling=ecmc.TILING_WHOLE))
    for n_max in (-1, 2048):
        with pytest.raises(ecmc.EcmcError):
            g.internal_distances_noalloc(n_max)
    r2, cnt = g.internal_distances_noalloc(0)
    assert r2[0] == 0.0 and cnt[0] == 256
