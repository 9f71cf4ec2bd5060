"""GPU tests of the boundary's stream and failure handling, through the C ABI.

- The larger staging tiers of a by-phases sweep run on a second stream only when the caller
  gives one; the result is the same either way (the tiers take disjoint domains of a colour).
- A dependency wait of the one-launch sweep that runs out of time leaves its domain as it was:
  the guard is forced from the host with a wait limit of one microsecond, every kernel still
  ends normally, the call reports ECMC_E_DEVICE, and the state stays valid (no overlap, no
  stretched bond, every bead listed in its own cell).
"""
import numpy as np
import pytest

from paper_1502_06447_amd import ecmc, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def melt_c2():
    return inputs.lattice_chains(500, 32, 0.45, seed=2)


def test_side_stream_gives_the_same_sweeps(melt_c2):
    import torch
    # D = 3 frames hold about 340 beads: a 256-bead first tier leaves many domains to the next
    opts = ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=3, n_cells=18, schedule=ecmc.SCHED_PHASES,
                        stage_tier=256)
    side = torch.cuda.Stream()
    runs = []
    for s in (None, side):
        g = ecmc.Melt.from_melt(melt_c2, opts, side_stream=s)
        for k in range(2):
            g.sweep(16000, 20.0, 300 + k)
        g.synchronize()
        runs.append((g.positions(), g.cells(), g.images(), g.counters()))
        g.close()
    (p0, c0, i0, n0), (p1, c1, i1, n1) = runs
    assert np.array_equal(p0, p1) and np.array_equal(c0, c1) and np.array_equal(i0, i1)
    assert n0 == n1 and n0["ec"] >= 32000


def test_a_wait_that_runs_out_leaves_a_valid_state(melt_c2):
    g = ecmc.Melt.from_melt(melt_c2, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16,
                                                  wait_limit_us=1))
    g.sweep(16000, 20.0, 404)
    with pytest.raises(ecmc.EcmcError) as e:
        g.synchronize()
    assert e.value.code == ecmc.E_DEVICE and "ran out of time" in str(e.value)
    assert g.counters()["error_flags"] & (1 << 5)
    g.clear_error()
    assert g.counters()["error_flags"] == 0
    # colour-0 domains never wait; every domain that gave up did nothing
    c = g.counters()
    assert 0 < c["ec"] < 16000
    assert g.check_state(1e-12) == {"overlaps": 0, "stretched": 0, "misplaced": 0}
    pos = g.positions()
    assert np.all(np.isfinite(pos)) and np.all((pos >= 0.0) & (pos <= melt_c2.L))
