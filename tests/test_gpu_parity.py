"""GPU parity: the gfx950 event-chain kernels against the CPU oracle, through the C ABI.

FP64 path: on the same start, seed and schedule the GPU must reproduce the oracle's
event sequence (kind, pivot, struck bead, per domain and EC) bit for bit and its
positions to 1e-9 sigma (they are expected to agree exactly).
"""
import numpy as np
import pytest

import oracle
from paper_1502_06447_amd import ecmc, inputs

pytestmark = pytest.mark.gpu

KEY = ("sweep", "domain", "ec", "step")


class _Pair:
    """The same melt on the GPU and in the oracle, swept with identical arguments."""

    def __init__(self, melt, tiling, D=2, n_cells=0, log=2_000_000, **kw):
        opts = ecmc.Options(tiling=tiling, domain_cells=D, n_cells=n_cells, event_log_capacity=log, **kw)
        self.g = ecmc.Melt.from_melt(melt, opts)
        self.o = oracle.Oracle.from_melt(melt, n_cells=n_cells)
        self.o.set_swap(kw.get("swap_moves", False))
        self.o.set_spring(kw.get("spring_k", 0.0))
        if log:
            self.o.enable_log(log)
        self.tiling, self.D = tiling, D
        assert self.g.n_cells == self.o.n_cells and self.g.h == self.o.h

    def sweep(self, n_ec, ell, seed, colour_mask=0xFF):
        self.g.sweep(n_ec, ell, seed, colour_mask=colour_mask)
        self.o.sweep(n_ec, ell, seed, tiling=self.tiling, D=self.D, colour_mask=colour_mask)


def _pair(melt, tiling, D=2, n_cells=0, log=2_000_000, **kw):
    p = _Pair(melt, tiling, D=D, n_cells=n_cells, log=log, **kw)
    return p, p.g, p.o


def _sorted(log):
    return log[np.lexsort((log["step"], log["ec"], log["domain"], log["sweep"]))]


def _compare(g, o, tol=1e-9):
    g.synchronize()
    lg = _sorted(g.event_log())
    lo = _sorted(o.event_log())
    m = min(len(lg), len(lo))
    if len(lg) != len(lo) or not np.array_equal(lg, lo):
        diff = np.flatnonzero(lg[:m] != lo[:m])
        bad = diff[0] if len(diff) else m
        raise AssertionError(f"logs differ (gpu {len(lg)}, oracle {len(lo)} records); first divergent record "
                             f"{bad}: gpu {lg[bad] if bad < len(lg) else None} oracle "
                             f"{lo[bad] if bad < len(lo) else None}")
    dp = np.abs(g.positions() - o.positions()).max()
    assert dp <= tol, dp
    assert np.array_equal(g.cells(), o.cells())
    assert np.array_equal(g.images(), o.images())
    cg = g.counters()
    co, dsum = o.counters()
    for k, idx in (("hs_lift", oracle.C_HS_LIFT), ("tether_lift", oracle.C_TETHER_LIFT),
                   ("hs_reflect", oracle.C_HS_REFLECT), ("tether_reflect", oracle.C_TETHER_REFLECT),
                   ("wall", oracle.C_WALL), ("cross", oracle.C_CROSS), ("ec", oracle.C_EC),
                   ("steps", oracle.C_STEPS), ("periodic", oracle.C_PERIOD), ("cycle", oracle.C_CYCLE),
                   ("swap", oracle.C_SWAP)):
        assert cg[k] == co[idx], k
    assert cg["sum_delta"] == pytest.approx(dsum, rel=1e-9, abs=1e-9)  # FP64 atomic sum over domains
    return len(lg), dp


@pytest.mark.parametrize("exact", [False, True])
def test_whole_box_c1_event_sequence_bit_exact(melt_c1, exact):
    """16 x 16 melt, eta = 0.30, whole box (n = 5): 3 sweeps of 2,000 ECs with ell = 10 sigma,
    with the single-precision screen and with the plain FP64 search."""
    p, g, o = _pair(melt_c1, ecmc.TILING_WHOLE, precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED)
    for s in range(3):
        p.sweep(2000, 10.0, 11 + s)
    n, dp = _compare(g, o)
    assert n > 100_000
    print(f"{n} events, max |dr| {dp}")


@pytest.mark.parametrize("exact,sched", [(False, ecmc.SCHED_SWEEP), (True, ecmc.SCHED_SWEEP),
                                         (False, ecmc.SCHED_PHASES)])
def test_checkerboard_c1_event_sequence_bit_exact(melt_c1, exact, sched):
    """Checkerboard decomposition on the 16 x 16 melt (n = 4, D = 2: one domain per colour):
    walls, immotile reflections, every domain frame wrapping the periodic box; one launch per
    sweep (each domain waits for its neighbours of earlier colours) and one per phase."""
    p, g, o = _pair(melt_c1, ecmc.TILING_CHECKER, D=2, n_cells=4, precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED,
                    schedule=sched)
    for s in range(4):
        p.sweep(256, 10.0, 70 + s)
    n, _ = _compare(g, o)
    assert n > 10_000


@pytest.mark.parametrize("tiling,exact", [(ecmc.TILING_WHOLE, False), (ecmc.TILING_CHECKER, False),
                                          (ecmc.TILING_CHECKER, True)])
def test_swap_moves_c1_event_sequence_bit_exact(melt_c1, tiling, exact):
    """Swap moves (Sec. II.C) on the 16 x 16 melt: every proposal, acceptance, exchange of
    positions and image correction as in the oracle, whole box and checkerboard."""
    p, g, o = _pair(melt_c1, tiling, D=2, n_cells=0 if tiling == ecmc.TILING_WHOLE else 4, swap_moves=True,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED)
    for s in range(4):
        p.sweep(256, 10.0, 170 + s)
    n, _ = _compare(g, o)
    assert n > 10_000 and g.counters()["swap"] > 100


@pytest.fixture(scope="module")
def melt_c2():
    return inputs.lattice_chains(500, 32, 0.45, seed=2)


@pytest.mark.parametrize("D,n_cells,exact,sched", [(2, 16, False, ecmc.SCHED_SWEEP), (2, 16, False, ecmc.SCHED_PHASES),
                                                   (3, 18, False, ecmc.SCHED_SWEEP), (3, 18, True, ecmc.SCHED_SWEEP),
                                                   (3, 18, False, ecmc.SCHED_PHASES)])
def test_c2_dense_melt_bit_exact(melt_c2, D, n_cells, exact, sched):
    """500 x 32 melt at eta = 0.45 (n = 16, D = 2: 64 domains per colour; n = 18, D = 3: 27),
    2 sweeps of 16,000 ECs with ell = 20 sigma, by both schedules."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=D, n_cells=n_cells, log=40_000_000,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED, schedule=sched)
    for s in range(2):
        p.sweep(16000, 20.0, 5 + s)
    n, _ = _compare(g, o)
    assert n > 250_000


@pytest.mark.parametrize("exact,tier", [(True, 448), (False, 448), (True, 384)])
def test_c2_dense_melt_wide_staging_tiers_bit_exact(melt_c2, exact, tier):
    """The 500 x 32 melt (n = 18, D = 3, frames of about 340 beads) staged in the 448-bead tier (7
    beads per lane) and the 384-bead tier (6 per lane; the frames above it run from workspace
    slots), 2 sweeps of 16,000 ECs: every event as in the oracle."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=3, n_cells=18, log=40_000_000,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED, stage_tier=tier)
    for s in range(2):
        p.sweep(16000, 20.0, 15 + s)
    n, _ = _compare(g, o)
    assert n > 250_000


def _clustered(melt, grow):
    """The chains of `melt` that do not cross its periodic boundary, unchanged, in a box `grow`
    times wider: a dense region next to an empty one, so that domain frames hold very
    different bead counts (the densest far above what the mean density asks for)."""
    L, n_per = melt.L, melt.n_per
    ch = melt.positions.reshape(melt.n_poly, n_per, 3)
    keep = np.all(np.abs(np.diff(ch, axis=1)) < 0.5 * L, axis=(1, 2))
    m = int(keep.sum())
    i = np.arange(m * n_per, dtype=np.int32).reshape(m, n_per)
    bonds = np.stack([i[:, :-1].ravel(), i[:, 1:].ravel()], axis=1).astype(np.int32)
    return inputs.Melt(L=L * grow, positions=ch[keep].reshape(-1, 3).copy(), bonds=bonds, sigma=melt.sigma,
                       b_max=melt.b_max, n_poly=m, n_per=n_per)


@pytest.mark.parametrize("sched", [ecmc.SCHED_SWEEP, ecmc.SCHED_PHASES])
def test_clustered_melt_large_frames_bit_exact(melt_c2, sched):
    """The 500 x 32 melt (eta = 0.45) in a box 1.35 times wider (n = 24, D = 2): the staging
    area is sized for the mean density, so the dense domains (about 180 beads in a frame)
    overflow it and run from workspace slots (one launch per sweep) or from the larger
    staging tiers (by phases); event sequence and state as in the oracle."""
    m = _clustered(melt_c2, 1.35)
    frame = 64 * m.n_beads / 24 ** 3
    p, g, o = _pair(m, ecmc.TILING_CHECKER, D=2, n_cells=24, log=40_000_000, schedule=sched)
    # the densest 4^3-cell frames hold more than twice the mean
    cells = np.floor(m.positions / g.h).astype(int) % 24
    dense = np.zeros((24, 24, 24), int)
    np.add.at(dense, (cells[:, 0], cells[:, 1], cells[:, 2]), 1)
    win = sum(np.roll(dense, (-a, -b, -c), axis=(0, 1, 2)) for a in range(4) for b in range(4) for c in range(4))
    assert win.max() > 2 * frame > 100
    for s in range(2):
        p.sweep(m.n_beads, 20.0, 41 + s)
    n, _ = _compare(g, o)
    assert n > 100_000


def test_swap_moves_c2_dense_melt_bit_exact(melt_c2):
    """Swap moves in the 500 x 32 melt at eta = 0.45 (n = 18, D = 3), 2 sweeps."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=3, n_cells=18, log=40_000_000, swap_moves=True)
    for s in range(2):
        p.sweep(16000, 20.0, 25 + s)
    n, _ = _compare(g, o)
    assert n > 250_000 and g.counters()["swap"] > 100


def test_observables_match_oracle(melt_c2):
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=3, log=0)
    p.sweep(16000, 20.0, 3)
    og = g.observables(nbins=32)
    oo = o.observables(nbins=32)
    assert og["n_poly"] == oo["n_poly"] == 500
    np.testing.assert_allclose(og["r2"], oo["r2"], rtol=1e-12)
    np.testing.assert_allclose(og["rg2"], oo["rg2"], rtol=1e-12)
    np.testing.assert_allclose(og["mid"], oo["mid"], rtol=0, atol=1e-9)
    assert np.array_equal(og["hist"], oo["hist"])


def test_shape_analysis_matches_oracle(melt_c2):
    """Gyration tensors, eigenvalues and unwrapped centres of mass per polymer (appendix shape
    analysis; the centre of mass of g2) against the oracle, after 2 sweeps of the 500 x 32 melt;
    the ensemble descriptors of Table II from both."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=3, n_cells=18, log=0)
    for s in range(2):
        p.sweep(16000, 20.0, 31 + s)
    sg, so = g.shape(), o.shape()
    assert sg["n_poly"] == so["n_poly"] == 500
    tr = so["gyr"][:, :3].sum(axis=1)[:, None]
    assert np.all(np.abs(sg["gyr"] - so["gyr"]) <= 1e-10 * tr)
    assert np.all(np.abs(sg["eig"] - so["eig"]) <= 1e-9 * tr)
    np.testing.assert_allclose(sg["com"], so["com"], rtol=0, atol=1e-9)
    dg, do = ecmc.shape_descriptors(sg["eig"]), oracle.shape_descriptors(so["eig"])
    for k in do:
        assert abs(dg[k] - do[k]) < 1e-9, k


def test_edge_cases_zero_length_and_empty(melt_c1):
    """ell = 0 (every EC ends at once), n_chains = 0 (nothing runs, the sweep counter still
    advances), and a dilute box where most domains are empty."""
    p, g, o = _pair(melt_c1, ecmc.TILING_CHECKER, D=2, n_cells=4)
    p.sweep(300, 0.0, 1)
    p.sweep(0, 10.0, 2)
    assert g.sweep_counter == o.sweep_counter == 2
    n, _ = _compare(g, o)
    assert n == 304                      # K = ceil(300 / 8) = 38 ECs in each of the 8 domains
    dil = inputs.hs_fluid(40, 0.02, seed=4)
    p, g, o = _pair(dil, ecmc.TILING_CHECKER, D=3, n_cells=6)
    for s in range(3):
        p.sweep(500, 5.0, 9 + s)
    _compare(g, o)


def test_error_paths_from_host():
    """A staging area smaller than a domain's beads and an EC iteration cap of 1 are
    reported as errors at the next synchronising call; the kernels still exit normally."""
    m = inputs.lattice_chains(64, 64, 0.45, seed=7)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, stage_capacity=64))
    g.sweep(4096, 20.0, 1)
    with pytest.raises(ecmc.EcmcError) as e:
        g.synchronize()
    assert e.value.code == ecmc.E_CELL_OVERFLOW
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, event_cap=1))
    g.sweep(4096, 20.0, 1)
    with pytest.raises(ecmc.EcmcError) as e:
        g.synchronize()
    assert e.value.code == ecmc.E_STUCK


def test_checkpoint_restore_continues_bit_exact(melt_c1):
    a = ecmc.Melt.from_melt(melt_c1, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=4))
    b = ecmc.Melt.from_melt(melt_c1, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=4))
    a.sweep(256, 10.0, 1)
    a.sweep(256, 10.0, 2)
    b.sweep(256, 10.0, 1)
    state = (b.positions(), b.cells(), b.images(), b.sweep_counter)
    c = ecmc.Melt.from_melt(melt_c1, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=4))
    c.set_state(*state)
    c.sweep(256, 10.0, 2)
    assert np.array_equal(a.positions(), c.positions())
    assert np.array_equal(a.images(), c.images())


def _brute_check(p, c, bonds, L, h, n, tol=1e-10):
    """Overlaps, stretched bonds and misplaced beads of a state by brute force (numpy)."""
    d = p[None, :, :] - p[:, None, :]
    d -= L * np.round(d / L)
    q = np.einsum("ijk,ijk->ij", d, d)
    iu = np.triu_indices(len(p), 1)
    overlaps = int(np.count_nonzero(q[iu] < 1.0 * (1 - tol)))
    b = p[bonds[:, 1]] - p[bonds[:, 0]]
    b -= L * np.round(b / L)
    stretched = int(np.count_nonzero(np.einsum("ij,ij->i", b, b) > 1.4 ** 2 * (1 + tol)))
    hi = np.where(c + 1 < n, (c + 1) * h, L)
    misplaced = int(np.count_nonzero(np.any((p < c * h) | (p > hi), axis=1)))
    return {"overlaps": overlaps, "stretched": stretched, "misplaced": misplaced}


def test_state_check_counts_planted_faults(melt_c1):
    """The device state check on the 16 x 16 melt: nothing after three sweeps.  Then faults are
    planted from the host through set_state, which accepts a coordinate up to 1e-12 past its cell:
    a chain end moved along its bond to 3 sigma from its partner, and a bead put 4e-13 past its
    cell's upper face.  The counts equal a brute-force count of the planted state."""
    g = ecmc.Melt.from_melt(melt_c1, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=4))
    for s in range(3):
        g.sweep(256, 10.0, 60 + s)
    g.synchronize()
    assert g.check_state() == {"overlaps": 0, "stretched": 0, "misplaced": 0}
    pos, cells, img = g.positions(), g.cells(), g.images()
    L, h, n = melt_c1.L, g.h, g.n_cells
    assert _brute_check(pos, cells, melt_c1.bonds, L, h, n) == {"overlaps": 0, "stretched": 0, "misplaced": 0}
    p, c = pos.copy(), cells.copy()
    d = pos[0] - pos[1]
    d -= L * np.round(d / L)
    p[0] = np.mod(pos[1] + 3.0 * d / np.linalg.norm(d), L)
    c[0] = np.minimum(np.floor(p[0] / h).astype(np.int32), n - 1)
    k = next(i for i in range(8, len(p)) if c[i, 0] < n - 1)
    p[k, 0] = (c[k, 0] + 1) * h + 4e-13
    g.set_state(p, c, img, g.sweep_counter)
    got = g.check_state()
    want = _brute_check(p, c, melt_c1.bonds, L, h, n)
    assert got == want and got["stretched"] >= 1 and got["misplaced"] == 1, (got, want)
    with pytest.raises(ecmc.EcmcError):
        g.check_state(tol=0.1)


def test_checkpoint_file_resume_gives_identical_event_logs(melt_c2, tmp_path):
    """Checkpoint and resume through a file on the 500 x 32 melt: four sweeps in one run against two
    sweeps, a checkpoint file, a new context restored from it and two more sweeps.  The last two
    sweeps' event logs, the final state and the counters of those sweeps are identical."""
    opts = dict(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16, event_log_capacity=4_000_000)
    a = ecmc.Melt.from_melt(melt_c2, ecmc.Options(**opts))
    for s in range(2):
        a.sweep(16000, 20.0, 30 + s)
    path = str(tmp_path / "ckpt.npz")
    a.save_checkpoint(path)
    a.clear_event_log()
    a.reset_counters()
    for s in range(2, 4):
        a.sweep(16000, 20.0, 30 + s)
    a.synchronize()
    b = ecmc.Melt.from_melt(melt_c2, ecmc.Options(**opts))
    b.load_checkpoint(path)
    for s in range(2, 4):
        b.sweep(16000, 20.0, 30 + s)
    b.synchronize()
    la, lb = _sorted(a.event_log()), _sorted(b.event_log())
    assert len(la) > 100_000 and np.array_equal(la, lb)
    assert np.array_equal(a.positions(), b.positions()) and np.array_equal(a.images(), b.images())
    ca, cb = a.counters(), b.counters()
    assert all(ca[k] == cb[k] for k in ("hs_lift", "tether_lift", "hs_reflect", "wall", "cross", "ec", "steps"))


# ------------------------------------------------------------------ full-size sample
@pytest.fixture(scope="module")
def melt_c3():
    return inputs.lattice_chains(16384, 64, 0.45, seed=3)


def _sampled_domains(m, swap, precision=ecmc.PREC_MIXED, seed=77):
    """One colour phase of a 1,048,576-bead melt (n = 76, D = 2) on the GPU; the oracle replays 32
    sampled domains of that phase, whose beads must end identical (positions, cells, images)."""
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, swap_moves=swap,
                                            precision=precision))
    assert g.n_cells == 76
    n_ec = m.n_beads
    g.sweep(n_ec, 20.0, seed, colour_mask=0x01)
    g.synchronize()
    o = oracle.Oracle.from_melt(m)
    o.set_swap(swap)
    cells0 = o.cells()
    rng = np.random.default_rng(0)
    nd = 38
    colour0 = [d for d in range(nd ** 3) if (d % nd) % 2 == 0 and (d // nd % nd) % 2 == 0 and (d // nd ** 2) % 2 == 0]
    pick = np.sort(rng.choice(colour0, 32, replace=False))
    o.sweep_subset(n_ec, 20.0, seed, 2, 0x01, pick)
    # the beads of the sampled domains: offsets of sweep 0 from the Philox draw (0, 0, 0, 1)
    from tests.test_oracle_pins import _philox_py
    u = _philox_py([0, 0, 0, 1], [seed, 0])
    off = np.array([(u[a] * 2) >> 32 for a in range(3)])
    dom = ((cells0 - off) % 76) // 2
    did = dom[:, 0] + nd * (dom[:, 1] + nd * dom[:, 2])
    mine = np.flatnonzero(np.isin(did, pick))
    op = o.positions()
    assert np.count_nonzero(np.any(op[mine] != m.positions[mine], axis=1)) > 100
    gp = g.positions()
    assert np.array_equal(gp[mine], op[mine])
    assert np.array_equal(g.cells()[mine], o.cells()[mine])
    assert np.array_equal(g.images()[mine], o.images()[mine])
    c, _ = o.counters()
    assert c[oracle.C_EC] == 20 * len(np.unique(did[np.isin(did, pick)]))
    return g


@pytest.mark.parametrize("swap", [False, True])
def test_c3_full_size_sampled_domains(melt_c3, swap):
    """1,048,576 beads (16,384 x 64, eta = 0.45, n = 76, D = 2) in the launch configuration
    the benchmark times: one colour phase on the GPU; the oracle replays 32 sampled domains
    of that phase (domains of one phase never interact), and the beads of those domains
    must end with identical positions, cells and image counters; without and with swaps."""
    g = _sampled_domains(melt_c3, swap)
    assert (g.counters()["swap"] > 0) == swap   # over the whole phase (rarely accepted from a lattice start)


@pytest.fixture(scope="module")
def melt_c5():
    return inputs.lattice_chains(2048, 512, 0.45, seed=5)


@pytest.mark.parametrize("swap,precision", [(False, ecmc.PREC_MIXED), (True, ecmc.PREC_MIXED), (True, ecmc.PREC_FP64)])
def test_c5_long_chains_full_size_sampled_domains(melt_c5, swap, precision):
    """The long-chain melt (2,048 chains of 512 beads, 1,048,576 beads, eta = 0.45) as the
    benchmark's --workload c5 runs it, without and with swaps, in the mixed and the plain FP64
    search: one colour phase on the GPU, 32 sampled domains replayed by the oracle, identical."""
    g = _sampled_domains(melt_c5, swap, precision, seed=78)
    assert g.counters()["error_flags"] == 0


def test_c5_middle_bead_msd(melt_c5):
    """g1 and g2 of the long chains: the GPU's start snapshot (middle bead 256 and centre of mass of
    every chain, unwrapped) equals the oracle's; over four sweeps the device series gives g1, g2
    equal to the numpy definition on the same series, with g1 growing."""
    import torch
    g = ecmc.Melt.from_melt(melt_c5, ecmc.Options(swap_moves=True))
    snaps = torch.empty((5, 2048, 6), dtype=torch.float64, device="cuda")
    g.snapshot(out=snaps[0])
    g.synchronize()
    ref = oracle.Oracle.from_melt(melt_c5).snapshot()
    assert np.allclose(snaps[0].cpu().numpy(), ref, rtol=0, atol=1e-9 * melt_c5.L)
    for s in range(4):
        g.sweep(melt_c5.n_beads, 20.0, 820 + s)
        g.snapshot(out=snaps[s + 1])
    g.synchronize()
    got = snaps.cpu().numpy()
    g1, g2 = g.msd(snaps)
    r1, r2 = oracle.msd_series(got)
    assert np.allclose(g1, r1, rtol=1e-12, atol=0) and np.allclose(g2, r2, rtol=1e-12, atol=0)
    assert 0.0 < g1[1] < g1[2] < g1[4]


@pytest.mark.parametrize("precision", [ecmc.PREC_MIXED, ecmc.PREC_FP64])
def test_c3_subsample_r2_and_drift_against_the_oracle(precision):
    """A 4,096-bead subsample of the large-melt workload (64 chains of 64 at eta = 0.45, ell = 20,
    D = 2), ten full sweeps in each precision against the oracle's: no position drift at all and
    the same <R^2> and <R_g^2> to the summation order."""
    m = inputs.lattice_chains(64, 64, 0.45, seed=12)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, precision=precision))
    o = oracle.Oracle.from_melt(m, n_cells=g.n_cells)
    for s in range(10):
        g.sweep(m.n_beads, 20.0, 40 + s)
        o.sweep(m.n_beads, 20.0, 40 + s, tiling=1, D=2)
    g.synchronize()
    assert np.array_equal(g.positions(), o.positions()) and np.array_equal(g.images(), o.images())
    og, oo = g.observables(nbins=8), o.observables(nbins=8)
    assert og["r2"].mean() == pytest.approx(oo["r2"].mean(), rel=1e-12)
    assert og["rg2"].mean() == pytest.approx(oo["rg2"].mean(), rel=1e-12)
    assert g.counters()["ec"] == o.counters()[0][oracle.C_EC] >= 10 * m.n_beads
    assert g.counters()["error_flags"] == 0


def test_c3_schedules_agree_at_full_size(melt_c3):
    """At 1,048,576 beads (6,859 domains per colour, a few hundred of them above the LDS
    staging area) two sweeps in one launch each and two sweeps by colour phases end in the
    same state bit for bit: positions, cells, images and every counter."""
    m = melt_c3
    runs = []
    for sched in (ecmc.SCHED_SWEEP, ecmc.SCHED_PHASES):
        g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, schedule=sched))
        for s in range(2):
            g.sweep(m.n_beads, 20.0, 300 + s)
        g.synchronize()
        runs.append((g.positions(), g.cells(), g.images(), g.counters()))
        g.close()
    (p0, c0, i0, k0), (p1, c1, i1, k1) = runs
    assert np.array_equal(p0, p1) and np.array_equal(c0, c1) and np.array_equal(i0, i1)
    for k in k0:
        if k == "sum_delta":
            assert k0[k] == pytest.approx(k1[k], rel=1e-9)
        else:
            assert k0[k] == k1[k], k
    assert k0["ec"] > 2_000_000 and k0["error_flags"] == 0


def test_c3_invariants_after_full_sweeps(melt_c3):
    """Properties that hold at any size: after full sweeps of the 1M-bead melt no pair of
    beads overlaps and no tether is stretched (checked on the host with a cell grid)."""
    m = melt_c3
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2))
    for s in range(2):
        g.sweep(m.n_beads, 20.0, 500 + s)
    g.synchronize()
    assert g.check_state() == {"overlaps": 0, "stretched": 0, "misplaced": 0}
    pos = g.positions()
    L = m.L
    # shape analysis of all 16,384 chains against the oracle put into the same state
    o = oracle.Oracle.from_melt(m)
    o.set_state(pos, g.cells(), g.images(), g.sweep_counter)
    sg, so = g.shape(), o.shape()
    tr = so["gyr"][:, :3].sum(axis=1)[:, None]
    assert np.all(np.abs(sg["gyr"] - so["gyr"]) <= 1e-10 * tr) and np.all(np.abs(sg["eig"] - so["eig"]) <= 1e-9 * tr)
    np.testing.assert_allclose(sg["com"], so["com"], rtol=0, atol=1e-8)
    d = pos[m.bonds[:, 1]] - pos[m.bonds[:, 0]]
    d -= L * np.round(d / L)
    assert np.einsum("ij,ij->i", d, d).max() <= 1.4 ** 2 * (1 + 1e-10)
    cells = g.cells()
    h = g.h
    assert np.all(pos >= cells * h - 1e-12) and np.all(pos <= np.minimum((cells + 1) * h, L) + 1e-12)
    n = g.n_cells
    flat = cells[:, 0] + n * (cells[:, 1] + n * cells[:, 2])
    order = np.argsort(flat, kind="stable")
    start = np.searchsorted(flat[order], np.arange(n ** 3 + 1))
    min_d2 = np.inf
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = (((cells[:, 0] + dx) % n) + n * (((cells[:, 1] + dy) % n) + n * ((cells[:, 2] + dz) % n)))
                cnt = start[nb + 1] - start[nb]
                for t in range(int(cnt.max())):
                    has = cnt > t
                    j = order[start[nb[has]] + t]
                    i = np.flatnonzero(has)
                    keep = j != i
                    dd = pos[j[keep]] - pos[i[keep]]
                    dd -= L * np.round(dd / L)
                    if dd.size:
                        min_d2 = min(min_d2, float(np.einsum("ij,ij->i", dd, dd).min()))
    assert min_d2 >= 1.0 - 1e-10


# ------------------------------------------------------------------ statistics on the GPU
@pytest.mark.parametrize("tiling,D,L", [(ecmc.TILING_WHOLE, 1, 8.0), (ecmc.TILING_CHECKER, 2, 6.0)])
def test_gpu_dimer_bond_length_distribution(tiling, D, L):
    """Isolated tethered dimer: p(r) = 3 r^2 / (b^3 - sigma^3) on [sigma, b].  Successive
    samples are correlated (lag-1 autocorrelation near 0.3), so the KS test takes every
    fifth one."""
    from scipy import stats
    m = inputs.dimer(L, seed=21)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=tiling, domain_cells=D))
    r = np.empty(6000)
    for k in range(len(r)):
        g.sweep(3, 7.3, 4000 + k)
        p = g.positions()
        d = p[1] - p[0]
        d -= L * np.round(d / L)
        r[k] = np.linalg.norm(d)
    cdf = lambda x: np.clip((x ** 3 - 1.0) / (1.4 ** 3 - 1.0), 0, 1)
    assert stats.kstest(r[::5], cdf).pvalue > 1e-3


# ---------------------------------------------------------------- batches of independent melts
@pytest.fixture(scope="module")
def small_batch():
    """Four melts of the batched workload's kinds (N from 16 to 64, 1,000 to 3,000 beads,
    eta from 0.35 to 0.45), each in its own box."""
    return inputs.batch_melts(4, 11, n_choices=(16, 32, 64), beads_range=(1000, 3000))


def _split_log(log, info):
    sel = (log["domain"] >= info["first_domain"]) & (log["domain"] < info["first_domain"] + info["n_domains"])
    part = log[sel].copy()
    part["domain"] -= info["first_domain"]
    for k in ("pivot", "target"):
        ok = part[k] >= 0
        part[k][ok] -= info["first_bead"]
    return part


@pytest.mark.parametrize("exact", [False, True])
def test_batch_every_melt_matches_the_oracle(small_batch, exact):
    """A batch sweeps all its melts in one launch; melt m draws from random stream m.  Replayed
    alone in the oracle (stream m, the batch's ECs per domain), every melt must give the same
    event sequence, positions, cells and images; the counters add up over the melts."""
    melts = small_batch
    g = ecmc.Melt.from_batch(melts, ecmc.Options(event_log_capacity=20_000_000,
                                                 precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED))
    assert g.n_melts == len(melts)
    infos = [g.melt_info(m) for m in range(len(melts))]
    total_domains = sum(i["n_domains"] for i in infos)
    n_ec = g.n_beads
    K = -(-n_ec // total_domains)
    for s in range(2):
        g.sweep(n_ec, 20.0, 61 + s)
    g.synchronize()
    log = g.event_log()
    pos, cells, img = g.positions(), g.cells(), g.images()
    tot = np.zeros(oracle.NCNT, dtype=np.uint64)
    for m, (melt, info) in enumerate(zip(melts, infos)):
        o = oracle.Oracle.from_melt(melt, n_cells=info["n_cells"])
        o.set_stream(m)
        o.enable_log(10_000_000)
        for s in range(2):
            o.sweep(K * info["n_domains"], 20.0, 61 + s, tiling=1, D=info["domain_cells"])
        lg = _sorted(_split_log(log, info))
        lo = _sorted(o.event_log())
        assert len(lg) == len(lo) and np.array_equal(lg, lo), f"melt {m}: logs differ ({len(lg)} vs {len(lo)})"
        b0, nb = info["first_bead"], info["n_beads"]
        assert np.array_equal(pos[b0:b0 + nb], o.positions()), m
        assert np.array_equal(cells[b0:b0 + nb], o.cells()), m
        assert np.array_equal(img[b0:b0 + nb], o.images()), m
        tot += np.asarray(o.counters()[0], dtype=np.uint64)
    cg = g.counters()
    assert cg["hs_lift"] == tot[oracle.C_HS_LIFT] and cg["ec"] == tot[oracle.C_EC] and cg["steps"] == tot[oracle.C_STEPS]
    assert len(log) > 100_000


def test_batch_of_one_is_the_single_melt(melt_c2):
    """A batch holding one melt sweeps exactly as the single-melt context."""
    a = ecmc.Melt.from_melt(melt_c2, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=16))
    b = ecmc.Melt.from_batch([melt_c2], ecmc.Options(), n_cells=[16], domain_cells=[2])
    for s in range(3):
        a.sweep(16000, 20.0, 91 + s)
        b.sweep(16000, 20.0, 91 + s)
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.images(), b.images())
    assert a.sweep_counter == b.sweep_counter == 3


def test_graph_of_sweeps_replays_like_eager_sweeps(small_batch):
    """Three sweeps captured into a HIP graph on the context's stream, replayed twice with
    eager work and synchronisation in between: after each replay the state equals three more
    eager sweeps of a twin context (the sweep counter and stamps advance on the device)."""
    import torch
    s = torch.cuda.Stream()
    g = ecmc.Melt.from_batch(small_batch, ecmc.Options(), stream=s)
    e = ecmc.Melt.from_batch(small_batch, ecmc.Options())
    n_ec = g.n_beads
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        for _ in range(3):
            g.sweep(n_ec, 20.0, 5)
    for rep in range(2):
        graph.replay()
        for _ in range(3):
            e.sweep(n_ec, 20.0, 5)
        torch.cuda.synchronize()
        assert g.sweep_counter == e.sweep_counter == 3 * (rep + 1)
        assert np.array_equal(g.positions(), e.positions()), rep
        assert np.array_equal(g.cells(), e.cells()), rep
        ce, cg = e.counters(), g.counters()
        assert all(ce[k] == cg[k] for k in ("hs_lift", "hs_reflect", "ec", "steps", "cross", "wall")), rep


def test_autotuner_returns_a_configuration_that_runs(small_batch, tmp_path):
    """The autotuner times its candidates on a scratch workspace and returns per-melt cells and
    domain edges and a staging tier that a batch context accepts and sweeps with.  Through a
    cache file, a second call returns the stored choice without timing anything."""
    melts = small_batch
    nb = sum(m.n_beads for m in melts)
    opts = ecmc.Options()
    cache = str(tmp_path / "tune.json")
    nc, dc, res = ecmc.ecmc_tune_batch(melts, 1.0, 1.4, ecmc._native_options(opts), nb, 20.0, trial_sweeps=1,
                                       cache=cache)
    assert res["candidates"] >= 1 and res["ecs_per_s"] > 0 and res["stage_tier"] in (64, 128, 192, 256, 384, 512)
    assert res["cached"] is False
    nc2, dc2, res2 = ecmc.ecmc_tune_batch(melts, 1.0, 1.4, ecmc._native_options(opts), nb, 20.0, trial_sweeps=1,
                                          cache=cache)
    assert res2["cached"] is True and (nc2, dc2) == (nc, dc)
    assert {k: v for k, v in res2.items() if k != "cached"} == {k: v for k, v in res.items() if k != "cached"}
    for m, n, D in zip(melts, nc, dc):
        assert n >= 4 and D >= 2 and n % D == 0 and (n // D) % 2 == 0 and m.L / n > 1.4
    opts.stage_tier = res["stage_tier"]
    g = ecmc.Melt.from_batch(melts, opts, n_cells=nc, domain_cells=dc)
    g.sweep(nb, 20.0, 3)
    g.synchronize()
    assert g.counters()["ec"] > 0


# ------------------------------------------------------------------ harmonic springs (Eq. (2))
@pytest.fixture(scope="module")
def melt_c1_spring():
    """The 16 x 16 parity melt with room for stretched bonds: springs capped at 1.8 sigma."""
    return inputs.saw_chains(16, 16, 0.30, seed=1, b_max=1.8)


@pytest.mark.parametrize("tiling,exact,sched", [(ecmc.TILING_WHOLE, False, ecmc.SCHED_SWEEP),
                                                (ecmc.TILING_WHOLE, True, ecmc.SCHED_SWEEP),
                                                (ecmc.TILING_CHECKER, False, ecmc.SCHED_SWEEP),
                                                (ecmc.TILING_CHECKER, True, ecmc.SCHED_SWEEP),
                                                (ecmc.TILING_CHECKER, False, ecmc.SCHED_PHASES)])
def test_springs_c1_event_sequence_bit_exact(melt_c1_spring, tiling, exact, sched):
    """Spring bonds (k sigma^2 = 30, capped at 1.8 sigma) on the 16 x 16 melt: the energy draw
    of every step and bond, every spring lift and spring reflection as in the oracle, whole
    box (n = 4) and checkerboard (n = 4, D = 2), both precisions and both schedules."""
    whole = tiling == ecmc.TILING_WHOLE
    p, g, o = _pair(melt_c1_spring, tiling, D=2, n_cells=4, spring_k=30.0, schedule=sched,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED)
    for s in range(3):
        p.sweep(2000 if whole else 256, 10.0, 400 + s)
    n, _ = _compare(g, o)
    c = g.counters()
    assert n > 10_000 and c["tether_lift"] > 100 and c["periodic"] == 0
    if not whole:
        assert c["tether_reflect"] > 0 and c["wall"] > 0


@pytest.fixture(scope="module")
def melt_c2_spring():
    return inputs.lattice_chains(500, 32, 0.45, seed=2, b_max=1.6)


@pytest.mark.parametrize("exact,sched", [(False, ecmc.SCHED_SWEEP), (True, ecmc.SCHED_SWEEP),
                                         (False, ecmc.SCHED_PHASES)])
def test_springs_c2_dense_melt_bit_exact(melt_c2_spring, exact, sched):
    """500 x 32 spring melt at eta = 0.45 (k sigma^2 = 30, cap 1.6 sigma, n = 16, D = 2: 64
    domains per colour), 2 sweeps of 16,000 ECs with ell = 20 sigma."""
    p, g, o = _pair(melt_c2_spring, ecmc.TILING_CHECKER, D=2, n_cells=16, log=40_000_000, spring_k=30.0,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED, schedule=sched)
    for s in range(2):
        p.sweep(16000, 20.0, 500 + s)
    n, _ = _compare(g, o)
    assert n > 250_000


@pytest.mark.parametrize("exact", [True, False])
def test_springs_c2_in_the_448_bead_tier_bit_exact(melt_c2_spring, exact):
    """The 500 x 32 spring melt (n = 16, D = 2, frames of about 250 beads) staged in the 448-bead tier
    (7 beads per lane, the motile beads as mask words), 2 sweeps of 16,000 ECs: every event as in
    the oracle."""
    p, g, o = _pair(melt_c2_spring, ecmc.TILING_CHECKER, D=2, n_cells=16, log=40_000_000, spring_k=30.0,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED, stage_tier=448)
    for s in range(2):
        p.sweep(16000, 20.0, 540 + s)
    n, _ = _compare(g, o)
    assert n > 250_000


@pytest.mark.parametrize("sched", [ecmc.SCHED_SWEEP, ecmc.SCHED_PHASES])
def test_springs_clustered_large_frames_bit_exact(melt_c2_spring, sched):
    """Springs in the clustered 500 x 32 melt (box 1.35 times wider, n = 20, D = 2, cap 1.6 sigma):
    the staging area is sized for the mean density, so the dense frames (more than twice the mean)
    run from workspace slots (one launch per sweep) or from the larger staging tiers (by phases),
    where the search evaluates every staged bead in full; every event as in the oracle."""
    m = _clustered(melt_c2_spring, 1.35)
    frame = 64 * m.n_beads / 20 ** 3
    p, g, o = _pair(m, ecmc.TILING_CHECKER, D=2, n_cells=20, log=40_000_000, spring_k=30.0,
                    precision=ecmc.PREC_FP64, schedule=sched)
    cells = np.floor(m.positions / g.h).astype(int) % 20
    dense = np.zeros((20, 20, 20), int)
    np.add.at(dense, (cells[:, 0], cells[:, 1], cells[:, 2]), 1)
    win = sum(np.roll(dense, (-a, -b, -c), axis=(0, 1, 2)) for a in range(4) for b in range(4) for c in range(4))
    assert win.max() > 2 * frame > 100
    for s in range(2):
        p.sweep(m.n_beads, 20.0, 61 + s)
    n, _ = _compare(g, o)
    assert n > 100_000


def test_springs_tile_joint_c2_dense_melt_bit_exact(melt_c2_spring):
    """The 500 x 32 spring melt (cap 1.6 sigma) on 2^3-cell tiles at pitch 3 (n = 15: 125 tiles in
    one phase, the joints immotile): 2 sweeps of 16,000 ECs with ell = 20 sigma, every event as in
    the oracle."""
    p, g, o = _pair(melt_c2_spring, ecmc.TILING_JOINT, D=2, n_cells=15, log=40_000_000, spring_k=30.0)
    for s in range(2):
        p.sweep(16000, 20.0, 520 + s)
    n, _ = _compare(g, o)
    c = g.counters()
    assert n > 250_000 and c["tether_lift"] > 50 and c["periodic"] == 0 and c["wall"] > 0


@pytest.fixture(scope="module")
def melt_c3_spring():
    return inputs.lattice_chains(16384, 64, 0.45, seed=3, b_max=1.8)


def test_springs_tile_joint_c3_full_size_clean_and_precision_exact(melt_c3_spring):
    """The 1,048,576-bead spring melt (cap 1.8 sigma) at full size on 2^3-cell tiles at pitch 3
    (57^3 cells): one sweep in each precision ends in identical states with identical counters,
    and the device state check finds no overlap, stretched bond or misplaced bead."""
    runs = []
    for prec in (ecmc.PREC_MIXED, ecmc.PREC_FP64):
        g = ecmc.Melt.from_melt(melt_c3_spring, ecmc.Options(tiling=ecmc.TILING_JOINT, domain_cells=2, n_cells=57,
                                                             spring_k=30.0, precision=prec))
        g.sweep(melt_c3_spring.n_beads, 20.0, 88)
        g.synchronize()
        assert g.check_state() == {"overlaps": 0, "stretched": 0, "misplaced": 0}
        runs.append((g.positions(), g.images(), g.counters()))
        g.close()
    (p0, i0, c0), (p1, i1, c1) = runs
    assert np.array_equal(p0, p1) and np.array_equal(i0, i1)
    assert all(c0[k] == c1[k] for k in ("hs_lift", "tether_lift", "hs_reflect", "tether_reflect", "wall", "ec", "steps"))
    assert c0["ec"] >= melt_c3_spring.n_beads and c0["tether_lift"] > 0 and c0["error_flags"] == 0


def test_springs_c3_full_size_sampled_domains(melt_c3_spring):
    """1,048,576 beads bonded by springs (k sigma^2 = 30, cap 1.8 sigma: n = 56, D = 2) in
    the launch configuration the benchmark times for springs (one launch per sweep): after
    one full sweep the oracle replays 24 sampled domains of colour 0 from the start, and the
    beads of those domains must end with identical positions, cells and images (colour 0
    runs first, so its domains see only the start)."""
    m = melt_c3_spring
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=56, spring_k=30.0))
    n = g.n_cells
    assert n == 56
    nd = n // 2
    o = oracle.Oracle.from_melt(m, n_cells=56)
    o.set_spring(30.0)
    assert o.n_cells == n
    cells0 = o.cells()
    n_ec = m.n_beads
    g.sweep(n_ec, 20.0, 91)
    g.synchronize()
    rng = np.random.default_rng(1)
    colour0 = [d for d in range(nd ** 3) if (d % nd) % 2 == 0 and (d // nd % nd) % 2 == 0 and (d // nd ** 2) % 2 == 0]
    pick = np.sort(rng.choice(colour0, 24, replace=False))
    o.sweep_subset(n_ec, 20.0, 91, 2, 0x01, pick)
    from tests.test_oracle_pins import _philox_py
    u = _philox_py([0, 0, 0, 1], [91, 0])
    off = np.array([(u[a] * 2) >> 32 for a in range(3)])
    dom = ((cells0 - off) % n) // 2
    did = dom[:, 0] + nd * (dom[:, 1] + nd * dom[:, 2])
    mine = np.flatnonzero(np.isin(did, pick))
    # a domain moves only the beads it holds when it starts, and they stay inside it, so the
    # later colours of the sweep leave the beads of colour-0 domains as colour 0 left them
    op = o.positions()
    assert np.count_nonzero(np.any(op[mine] != m.positions[mine], axis=1)) > 100
    assert np.array_equal(g.positions()[mine], op[mine])
    assert np.array_equal(g.cells()[mine], o.cells()[mine])
    assert np.array_equal(g.images()[mine], o.images()[mine])
    c = g.counters()
    assert c["error_flags"] == 0 and c["tether_lift"] > 0 and c["periodic"] == 0


def test_springs_refused_with_swaps_and_bad_constants(melt_c1_spring):
    """Host-side validation: a spring constant outside [1e-6, 1e12] or combined with swap
    moves is refused before anything runs."""
    for kw in ({"spring_k": -1.0}, {"spring_k": 1e-9}, {"spring_k": float("nan")},
               {"spring_k": 30.0, "swap_moves": True}):
        with pytest.raises(ecmc.EcmcError):
            ecmc.Melt.from_melt(melt_c1_spring, ecmc.Options(tiling=ecmc.TILING_WHOLE, **kw))


# ------------------------------------------------------------------ analysis: g1, g2, W(R), g(r)
def test_snapshots_and_msd_match_the_oracle(melt_c2):
    """A run of 6 sweeps on the 500 x 32 melt with a snapshot after each (middle bead and centre
    of mass, unwrapped): the GPU snapshots equal the oracle's (same trajectory, the sums of the
    unwrapping to rounding), and g1, g2 of the GPU series agree with the oracle's numpy
    definition on the same series to 1e-12."""
    import torch
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=2, n_cells=16, log=0)
    snaps = torch.empty((7, g.n_poly, 6), dtype=torch.float64, device="cuda")
    host = []
    g.snapshot(out=snaps[0])
    host.append(o.snapshot())
    for s in range(6):
        p.sweep(16000, 20.0, 900 + s)
        g.snapshot(out=snaps[s + 1])
        host.append(o.snapshot())
    g.synchronize()
    ref = np.stack(host)
    got = snaps.cpu().numpy()
    assert np.allclose(got, ref, rtol=0, atol=1e-9 * melt_c2.L), np.abs(got - ref).max()
    g1, g2 = g.msd(snaps)
    r1, r2 = oracle.msd_series(got)
    assert np.allclose(g1, r1, rtol=1e-12, atol=0) and np.allclose(g2, r2, rtol=1e-12, atol=0)
    assert g1[0] == 0.0 and g1[-1] > g1[1] > 0.0


def test_end_to_end_and_pair_histograms_match_the_oracle(melt_c2):
    """W(R) and the pair counts behind g(r) after two sweeps of the 500 x 32 melt, against the
    oracle in the same state: the pair counts bit for bit (the same distances in the same
    arithmetic); W(R) bit for bit except for polymers whose |R| lies within 1e-9 of a bin edge
    (the GPU sums the bond vectors in another order)."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=2, n_cells=16, log=0)
    for s in range(2):
        p.sweep(16000, 20.0, 950 + s)
    g.synchronize()
    hp = g.pair_histogram(64, g.h)
    assert np.array_equal(hp, o.pair_histogram(64, g.h))
    assert hp[: int(64 / g.h)].sum() == 0 and hp.sum() > 5 * melt_c2.n_beads
    rmax, nb = 40.0, 80
    hw = g.end_to_end_histogram(nb, rmax)
    ho = o.end_to_end_histogram(nb, rmax)
    R = np.sqrt(o.observables(nbins=1)["r2"])
    edge = np.abs(R / rmax * nb - np.round(R / rmax * nb)) < 1e-9 * nb
    assert np.abs(hw - ho).sum() <= 2 * np.count_nonzero(edge)
    assert hw.sum() == 500
    with pytest.raises(ecmc.EcmcError):
        g.pair_histogram(10, 1.01 * g.h)


# Internal distances R^2(n): the GPU sums squares of differences of prefix sums of the bond
# vectors, blockwise; the oracle walks every pair bond by bond.  Both are FP64 and round
# differently.  With unit roundoff u = 2^-53, chains of N beads with bonds below 1.4 and
# |R| >= sigma = 1 for n >= 1, a prefix sum is off by at most N^2 * 1.4 u, which puts a relative
# error below 2 * 2 N^2 * 1.4 u on a squared length (N = 64: 2.5e-12); the sum of m positive
# terms adds at most m u on either side (m = 16,000 at the 500 x 32 melt: 1.8e-12).  The
# tests use 1e-11 below 20,000 pairs per lag, and m u + 1e-11 above.
def _r2n_tol(pairs):
    return 1e-11 + pairs.max() * 2.0 ** -53


def test_internal_distances_match_the_oracle(melt_c2):
    """R^2(n) for n = 0..40 (past the 32-bead chains) after three sweeps of the 500 x 32 melt,
    against the oracle in the same state: identical pair counts, means to the rounding bound,
    zeros beyond the chains, and the same result on a second call (a fixed summation order)."""
    p, g, o = _pair(melt_c2, ecmc.TILING_CHECKER, D=2, n_cells=16, log=0)
    for s in range(3):
        p.sweep(16000, 20.0, 970 + s)
    g.synchronize()
    r2, cnt = g.internal_distances(40)
    r2o, cnto = o.internal_distances(40)
    assert np.array_equal(cnt, cnto) and np.array_equal(cnt[:32], 500 * (32 - np.arange(32)))
    assert np.allclose(r2, r2o, rtol=_r2n_tol(cnt), atol=0), np.abs(r2 / np.where(r2o > 0, r2o, 1) - 1).max()
    assert r2[0] == 0.0 and np.all(r2[32:] == 0.0) and 1.0 <= r2[1] <= 1.4 ** 2  # n = 1: bonds in [sigma, b_max]
    r2b, _ = g.internal_distances(40)
    assert np.array_equal(r2, r2b)
    assert g.internal_distances(0)[0][0] == 0.0
    with pytest.raises(ecmc.EcmcError):
        g.internal_distances(2048)


def test_internal_distances_of_a_batch_match_the_oracle(small_batch):
    """A batch of four melts with chains of 16 to 64 beads, each in its own box: the GPU's
    R^2(n) over the whole batch equals the pair-weighted mean of the oracle's per-melt results."""
    g = ecmc.Melt.from_batch(small_batch, ecmc.Options())
    g.sweep(g.n_beads, 20.0, 990)
    g.synchronize()
    r2, cnt = g.internal_distances(70)
    pos = g.positions()
    tot, ctot, b0 = np.zeros(71), np.zeros(71, dtype=np.int64), 0
    for m, melt in enumerate(small_batch):
        info = g.melt_info(m)
        nb = info["n_beads"]
        o = oracle.Oracle.from_melt(melt, n_cells=info["n_cells"])
        o.set_stream(m)
        o.sweep(-(-g.n_beads // sum(g.melt_info(k)["n_domains"] for k in range(g.n_melts))) * info["n_domains"],
                20.0, 990, tiling=1, D=info["domain_cells"])
        assert np.array_equal(pos[b0:b0 + nb], o.positions()), m
        r, c = o.internal_distances(70)
        tot += r * c
        ctot += c
        b0 += nb
    assert np.array_equal(cnt, ctot)
    want = np.divide(tot, ctot, out=np.zeros_like(tot), where=ctot > 0)
    assert np.allclose(r2, want, rtol=_r2n_tol(cnt), atol=0)
    assert np.all(r2[64:] == 0.0)


def test_internal_distances_c3_full_size(melt_c3):
    """The 1,048,576-bead benchmark melt (16,384 chains of 64) in its start state, chains wrapped
    through the box: R^2(n) for every n against the oracle on the whole melt."""
    g = ecmc.Melt.from_melt(melt_c3, ecmc.Options())
    r2, cnt = g.internal_distances(63)
    o = oracle.Oracle.from_melt(melt_c3, n_cells=g.n_cells)
    r2o, cnto = o.internal_distances(63)
    assert np.array_equal(cnt, cnto) and cnt[63] == 16384
    assert np.allclose(r2, r2o, rtol=_r2n_tol(cnt), atol=0), np.abs(r2[1:] / r2o[1:] - 1).max()


# ------------------------------------------------------------------ push-off (Sec. II.B)
def _pushoff_pair(melt, n, log=4_000_000):
    g = ecmc.Melt.from_melt(melt, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=n, cell_capacity=32,
                                               overlapping_start=True, event_log_capacity=log))
    o = oracle.Oracle(melt.L, melt.sigma, melt.b_max, melt.positions, melt.bonds, n_cells=n, overlapping=True)
    o.enable_log(log)
    return g, o


def _phantom_cells(melt):
    n = int(melt.L // melt.b_max)
    while melt.L / n <= melt.b_max or n % 2 or (n // 2) % 2:
        n -= 1
    return n


def test_pushoff_sweeps_bit_exact():
    """Push-off sweeps (overlapping pairs are no events, ECs start at overlapping beads) on 200
    phantom chains of 16 beads at eta = 0.30 (n = 12, D = 2): at working diameters 0.5, 0.8 and
    1, two sweeps each with ECs of length 2 sigma; every event, the positions, cells, images,
    counters and the overlap counts as in the oracle."""
    m = inputs.phantom_chains(200, 16, 0.30, seed=6)
    n = _phantom_cells(m)
    g, o = _pushoff_pair(m, n)
    seed = 0
    for d in (0.5, 0.8, 1.0):
        o.set_pushoff(d)
        assert g.count_overlaps(d) == o.count_overlaps(d)
        for _ in range(2):
            g.pushoff_sweep(m.n_beads, 2.0, 300 + seed, d)
            o.sweep(m.n_beads, 2.0, 300 + seed, tiling=1, D=2)
            seed += 1
        assert g.count_overlaps(d) == o.count_overlaps(d)
    n_ev, _ = _compare(g, o)
    assert n_ev > 1000


def test_pushoff_loop_reaches_a_valid_start():
    """The native slow push-off (ten working diameters up to sigma, sweeps until no overlap is
    left at each) on 150 phantom chains of 32 beads at eta = 0.35 (c = 1.9; the oracle, run the
    same way, needs 585 sweeps at the last diameter): no overlap is left, the state is a valid
    start (the oracle's plain create accepts it: no pair closer than sigma, no bond longer than
    b_max), and plain sweeps run on it."""
    m = inputs.phantom_chains(150, 32, 0.35, seed=9)
    n = _phantom_cells(m)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=n, cell_capacity=32,
                                            overlapping_start=True))
    assert g.count_overlaps(1.0) > 300
    sweeps, left = g.pushoff(0.1, 10, ell=2.0, seed=5, max_sweeps=5000)
    print(f"push-off: {sweeps} sweeps, {left} overlaps left")
    assert left == 0 and g.count_overlaps(1.0) == 0
    oracle.Oracle(m.L, 1.0, m.b_max, g.positions(), m.bonds, n_cells=n)
    g.sweep(m.n_beads, 20.0, 11)
    g.synchronize()


def test_pushoff_reaches_a_valid_start_at_the_benchmark_density():
    """The slow push-off of Sec. II.B at eta = 0.45 (100 phantom chains of 32 beads, c = 1.9):
    20 working diameters from 0.145 sigma to sigma, ECs of 2 sigma, sweeps at each until no
    overlap is left.  It ends with no overlap, the device state check is clean, the oracle's
    plain create accepts the state as a start, and the internal distances R^2(n)/n stay close to
    the phantom walk's law at short range (the push-off only nudges the chains apart)."""
    m = inputs.phantom_chains(100, 32, 0.45, seed=9)
    n = _phantom_cells(m)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_CHECKER, domain_cells=2, n_cells=n, cell_capacity=32,
                                            overlapping_start=True))
    assert g.count_overlaps(1.0) > 1000
    sweeps, left = g.pushoff(0.145, 20, ell=2.0, seed=1, max_sweeps=20000)
    print(f"push-off at eta 0.45: {sweeps} sweeps, {left} overlaps left")
    assert left == 0 and g.count_overlaps(1.0) == 0
    assert g.check_state(1e-12) == {"overlaps": 0, "stretched": 0, "misplaced": 0}
    oracle.Oracle(m.L, 1.0, m.b_max, g.positions(), m.bonds, n_cells=n)
    r2, cnt = g.internal_distances(8)
    assert cnt[1] == 100 * 31 and 1.0 <= r2[1] <= 1.4 ** 2


def test_c4_full_batch_sampled_melts_match_the_oracle():
    """The 256-melt batch of the benchmark (8.4M beads, N from 16 to 256, eta 0.35-0.45) at full
    size in its launch configuration (one dependency-ordered launch per sweep for all melts, the
    256-bead staging tier the autotuner picks, larger frames in workspace slots): after two
    sweeps, five sampled melts (the smallest, the largest, the one with the largest cells and two
    at random) replayed alone in the oracle (stream m, the batch's ECs per domain) end with the
    same positions, cells and images bit for bit."""
    melts = inputs.batch_melts(256, 3)
    g = ecmc.Melt.from_batch(melts, ecmc.Options(stage_tier=256))
    infos = [g.melt_info(m) for m in range(g.n_melts)]
    total_domains = sum(i["n_domains"] for i in infos)
    n_ec = g.n_beads
    K = -(-n_ec // total_domains)
    for s in range(2):
        g.sweep(n_ec, 20.0, 1000 + s)
    g.synchronize()
    assert g.counters()["error_flags"] == 0
    pos, cells, img = g.positions(), g.cells(), g.images()
    sizes = [i["n_beads"] for i in infos]
    edge = [i["cell_size"] for i in infos]
    rng = np.random.default_rng(2)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argmax(edge))}
                  | set(int(x) for x in rng.choice(len(melts), 2, replace=False)))
    for m in pick:
        info, melt = infos[m], melts[m]
        o = oracle.Oracle.from_melt(melt, n_cells=info["n_cells"])
        o.set_stream(m)
        for s in range(2):
            o.sweep(K * info["n_domains"], 20.0, 1000 + s, tiling=1, D=info["domain_cells"])
        b0, nb = info["first_bead"], info["n_beads"]
        assert np.array_equal(pos[b0:b0 + nb], o.positions()), m
        assert np.array_equal(cells[b0:b0 + nb], o.cells()), m
        assert np.array_equal(img[b0:b0 + nb], o.images()), m


# ------------------------------------------------------------------ tile-joint partition (Sec. II.A)
@pytest.mark.parametrize("exact", [False, True])
def test_tile_joint_c3_subsample_event_sequence_bit_exact(exact):
    """The tile-joint partition on a 64 x 64 melt at eta = 0.45 (n = 12: 2^3-cell tiles at pitch 3,
    64 tiles in one phase; joints immotile): 3 sweeps of 4,096 ECs, every event as in the oracle,
    both precisions."""
    m = inputs.lattice_chains(64, 64, 0.45, seed=7)
    p, g, o = _pair(m, ecmc.TILING_JOINT, D=2, n_cells=12, log=20_000_000,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED)
    for s in range(3):
        p.sweep(4096, 20.0, 600 + s)
    n, _ = _compare(g, o)
    assert n > 50_000 and g.counters()["wall"] > 0


@pytest.mark.parametrize("D,n_cells", [(2, 18), (3, 16)])
def test_tile_joint_c2_dense_melt_bit_exact(melt_c2, D, n_cells):
    """Tile-joint on the 500 x 32 melt at eta = 0.45 (n = 18: pitch 3 with 2^3-cell tiles, 216
    tiles; n = 16: pitch 4 with 3^3-cell tiles, 64 tiles), 2 sweeps of 16,000 ECs with ell = 20 sigma."""
    p, g, o = _pair(melt_c2, ecmc.TILING_JOINT, D=D, n_cells=n_cells, log=40_000_000)
    for s in range(2):
        p.sweep(16000, 20.0, 700 + s)
    n, _ = _compare(g, o)
    assert n > 100_000


# ------------------------------------------------------------------ zero-length cycles
@pytest.mark.parametrize("exact", [False, True])
def test_zero_length_cycle_event_sequence_bit_exact(exact):
    """Three beads (sigma = 5, b_max = 6, every distance exact) where a move along x, or a move of
    the tethered pair along y or z, is a run of zero-length events that comes round for ever (A
    touches B, B's tether to C is taut, C touches A; the tether alone stops B and C across it).
    Whole-box sweeps of 6 ECs: the GPU ends the same ECs with CYCLE at the same step as the
    oracle, in both precisions, and what moves freely moves the same."""
    c = np.array([16.0, 16.0, 16.0])
    pos = np.array([c - [3.0, 4.0, 0.0], c, c - [6.0, 0.0, 0.0]])
    m = inputs.Melt(L=32.0, positions=pos, bonds=np.array([[1, 2]], dtype=np.int32), sigma=5.0, b_max=6.0)
    p, g, o = _pair(m, ecmc.TILING_WHOLE, n_cells=4, log=10_000,
                    precision=ecmc.PREC_FP64 if exact else ecmc.PREC_MIXED)
    for s in range(4):
        p.sweep(6, 7.5, 40 + s)
    n, _ = _compare(g, o)
    assert g.counters()["cycle"] >= 2


# ------------------------------------------------------------------ statistics on the GPU
@pytest.mark.parametrize("eta,n_beads", [(0.10, 500), (0.20, 500)])
def test_gpu_pressure_from_lifts_matches_carnahan_starling(eta, n_beads):
    """Unbonded spheres in whole-box mode on the GPU: beta P / rho = 1 + <sum of lift separations
    along v> / ell (the event-chain pressure estimator) against Carnahan-Starling, within 2 %
    (500 spheres, 400 sweeps of 500 ECs with ell = 4 sigma after 20 melting sweeps)."""
    cs = (1 + eta + eta ** 2 - eta ** 3) / (1 - eta) ** 3
    m = inputs.hs_fluid(n_beads, eta, seed=3)
    g = ecmc.Melt.from_melt(m, ecmc.Options(tiling=ecmc.TILING_WHOLE))
    ell = 4.0
    for s in range(20):
        g.sweep(n_beads, ell, 50 + s)
    g.synchronize()
    c0 = g.counters()
    for s in range(400):
        g.sweep(n_beads, ell, 500 + s)
    g.synchronize()
    c1 = g.counters()
    n_ec = c1["ec"] - c0["ec"]
    Z = 1 + (c1["sum_delta"] - c0["sum_delta"]) / (n_ec * ell)
    assert abs(Z - cs) / cs < 0.02, (Z, cs)
