"""GPU tests of the boundary's stream and failure handling, through the C ABI.

- The larger staging tiers of a by-phases sweep run on a second stream only when the caller
  gives one; the result is the same either way (the tiers take disjoint domains of a colour).
- A dependency wait of the one-launch sweep that runs out of time leaves its domain as it was:
  the guard is forced from the host with a wait limit of one microsecond, every kernel still
  ends normally, the call reports ECMC_E_DEVICE, and the state stays valid (no overlap, no
  stretched bond, every bead listed in its own cell).
- The running device sums of the observables agree with the per-sweep observables, for a single
  melt and for a batch.
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
    # sum_delta is a floating-point sum over domains in completion order: equal to rounding
    assert {k: v for k, v in n0.items() if k != "sum_delta"} == {k: v for k, v in n1.items() if k != "sum_delta"}
    assert abs(n0["sum_delta"] - n1["sum_delta"]) <= 1e-12 * abs(n0["sum_delta"]) and n0["ec"] >= 32000


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


def test_pair_correlation_of_the_dense_melt(melt_c2):
    """g(r) from the GPU pair counts, normalised by the library: zero inside the hard core
    (no two beads closer than sigma), a contact peak above 1 just outside it (Sec. II: dense
    hard spheres at eta = 0.45), and the same numbers as the library call on the counts."""
    g = ecmc.Melt.from_melt(melt_c2, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16))
    for k in range(3):
        g.sweep(16000, 20.0, 500 + k)
    r_max = 0.95 * g.h
    gr = g.pair_correlation(40, r_max)
    h = g.pair_histogram(40, r_max)
    assert np.array_equal(gr, ecmc.pair_correlation(h, r_max, melt_c2.n_beads, melt_c2.L ** 3))
    edges = np.linspace(0.0, r_max, 41)
    assert np.all(gr[edges[1:] <= 1.0] == 0.0)
    assert gr[np.searchsorted(edges, 1.0)] > 1.5


def test_observables_accumulate_matches_the_per_sweep_observables(melt_c2):
    """The running device sums of the observables (averages over sweeps, Sec. IV.A) against the
    per-sweep results of ecmc_observables: <R^2> and <R_g^2> to rounding (the sums are atomic adds
    in any order), the bond-length histogram exactly.  A reset clears them; another bin count
    without a reset is refused."""
    g = ecmc.Melt.from_melt(melt_c2, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16))
    g.observables_accumulate(nbins=24)  # cleared by the reset below
    g.observables_reset()
    r2s, rg2s, hist = [], [], np.zeros(24, dtype=np.int64)
    for k in range(3):
        g.sweep(16000, 20.0, 600 + k)
        g.observables_accumulate(nbins=24)
        o = g.observables(nbins=24)
        r2s.append(o["r2"].mean())
        rg2s.append(o["rg2"].mean())
        hist += o["hist"]
    m = g.observables_mean()
    assert m["samples"] == 3
    assert abs(m["r2"] - np.mean(r2s)) <= 1e-12 * np.mean(r2s)
    assert abs(m["rg2"] - np.mean(rg2s)) <= 1e-12 * np.mean(rg2s)
    assert np.array_equal(m["hist"], hist) and hist.sum() == 3 * 500 * 31
    with pytest.raises(ecmc.EcmcError) as e:
        g.observables_accumulate(nbins=10)
    assert e.value.code == ecmc.E_ARG
    g.observables_reset()
    assert g.observables_mean()["samples"] == 0
    g.observables_accumulate(nbins=10)
    m = g.observables_mean()
    assert m["samples"] == 1 and m["hist"].sum() == 500 * 31
    o = g.observables(nbins=10)
    assert np.array_equal(m["hist"], o["hist"]) and abs(m["r2"] - o["r2"].mean()) <= 1e-12 * o["r2"].mean()


def test_observables_accumulate_over_a_batch_of_melts():
    """The running sums over a batch: every polymer of every melt counts once per sample, so the
    means equal those of the per-sweep observables over all polymers of the batch."""
    melts = inputs.batch_melts(4, 11, n_choices=(16, 32, 64), beads_range=(1000, 3000))
    g = ecmc.Melt.from_batch(melts, ecmc.Options())
    r2s, rg2s, hist = [], [], np.zeros(16, dtype=np.int64)
    for k in range(2):
        g.sweep(g.n_beads, 20.0, 700 + k)
        g.observables_accumulate(nbins=16)
        o = g.observables(nbins=16)
        assert o["n_poly"] == sum(m.n_poly for m in melts)
        r2s.append(o["r2"].mean())
        rg2s.append(o["rg2"].mean())
        hist += o["hist"]
    m = g.observables_mean()
    assert m["samples"] == 2 and np.array_equal(m["hist"], hist)
    assert abs(m["r2"] - np.mean(r2s)) <= 1e-12 * np.mean(r2s)
    assert abs(m["rg2"] - np.mean(rg2s)) <= 1e-12 * np.mean(rg2s)
