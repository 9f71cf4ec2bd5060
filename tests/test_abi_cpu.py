"""CPU-only checks of the C ABI: the library loads, exports every declared symbol,
and the host-side validation answers without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1502_06447_amd import ecmc, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ecmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ecmc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = ecmc.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ecmc.EXPORTS)


def test_status_strings_and_defaults():
    L = ecmc.lib()
    for code in range(-8, 1):
        assert L.ecmc_status_str(code)
    o = ecmc.ecmc_default_options()
    assert o.precision == ecmc.PREC_FP64 and o.tiling == ecmc.TILING_CHECKER and o.domain_cells == 2


def test_workspace_size_and_geometry_errors():
    o = ecmc.ecmc_default_options()
    n = ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    assert n > 1 << 20 * 0 and n > 50 * (1 << 20)
    o.domain_cells = 3  # 76 cells per axis is not divisible by 3
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    assert e.value.code == ecmc.E_BOX
    o.domain_cells = 1  # the partition would never move (offset always 0): not ergodic
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    assert e.value.code == ecmc.E_BOX
    o.tiling = ecmc.TILING_JOINT  # 1-cell tiles: a wall at every face, no bead ever leaves its cell
    for n_cells in (0, 58, 76):
        o.n_cells = n_cells
        with pytest.raises(ecmc.EcmcError) as e:
            ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
        assert e.value.code == ecmc.E_BOX
    o.domain_cells, o.n_cells = 2, 75  # 2^3-cell tiles at pitch 3
    assert ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o) > 0
    o = ecmc.ecmc_default_options()
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(5.0, 1.0, 1.4, 10, o)          # n = 3 < 4
    assert e.value.code == ecmc.E_BOX
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(20.0, 1.0, 0.9, 10, o)         # l_max < sigma
    assert e.value.code == ecmc.E_ARG
    o.precision = 7                                              # neither FP64 nor MIXED
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(20.0, 1.0, 1.4, 10, o)
    assert e.value.code == ecmc.E_ARG
    o = ecmc.ecmc_default_options()
    o.schedule = 2                                               # neither SWEEP nor PHASES
    with pytest.raises(ecmc.EcmcError) as e:
        ecmc.ecmc_workspace_size(20.0, 1.0, 1.4, 10, o)
    assert e.value.code == ecmc.E_ARG


def test_sweep_schedule_reserves_staging_slots():
    """The one-launch sweep stages the rare domains above the LDS capacity in workspace slots
    (512 of them at the 1,048,576-bead melt, each for a full frame of 4^3 cells x 16 beads,
    40 bytes a bead); by phases, or with a fixed staging capacity, there are none."""
    o = ecmc.ecmc_default_options()
    sweep = ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    o.schedule = ecmc.SCHED_PHASES
    phases = ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    assert sweep - phases >= 512 * 1024 * 40 and sweep - phases < 512 * 1024 * 40 + 4 * 76 ** 3
    o.schedule = ecmc.SCHED_SWEEP
    o.stage_capacity = 192
    fixed = ecmc.ecmc_workspace_size(106.8551, 1.0, 1.4, 1 << 20, o)
    assert fixed - phases < 4096


def _init_status(pos, bonds, L=10.0, tiling=ecmc.TILING_WHOLE, workspace=True):
    """ecmc_init with a placeholder workspace address: the host validation runs before
    anything is copied to the device, so invalid inputs are refused without a GPU."""
    o = ecmc.ecmc_default_options()
    o.tiling = tiling
    if workspace:
        o.workspace = 1 << 20
        o.workspace_bytes = 1 << 40
    h = ctypes.c_void_p()
    p = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
    return ecmc.lib().ecmc_init(ctypes.byref(h), L, 1.0, 1.4, p.shape[0], p.ctypes.data, b.shape[0],
                                b.ctypes.data if b.size else None, ctypes.byref(o))


def test_host_validation_without_gpu():
    two = np.array([[1.0, 1.0, 1.0], [1.5, 1.0, 1.0]])
    assert _init_status(two, np.zeros((0, 2))) == ecmc.E_OVERLAP
    far = np.array([[1.0, 1.0, 1.0], [2.5, 1.0, 1.0]])
    assert _init_status(far, [[0, 1]]) == ecmc.E_TETHER
    tri = np.array([[1.0, 1.0, 1.0], [2.2, 1.0, 1.0], [3.4, 1.0, 1.0]])
    assert _init_status(tri, [[0, 1], [1, 2], [2, 0]]) == ecmc.E_ARG          # ring
    assert _init_status(tri, [[0, 1], [0, 1]]) == ecmc.E_ARG                  # duplicate
    assert _init_status(np.array([[np.nan, 1.0, 1.0]]), np.zeros((0, 2))) == ecmc.E_ARG
    assert _init_status(tri, [[0, 1]], workspace=False) == ecmc.E_WORKSPACE
    assert _init_status(tri, [[0, 1]], L=5.0) == ecmc.E_BOX


def test_generators_shapes(melt_c1):
    m = melt_c1
    assert m.positions.shape == (256, 3) and m.bonds.shape == (240, 2)
    assert abs(m.eta - 0.30) < 1e-12
    big = inputs.lattice_chains(64, 64, 0.45, seed=2)
    assert big.n_beads == 4096 and abs(big.eta - 0.45) < 1e-12
    d = big.positions[big.bonds[:, 1]] - big.positions[big.bonds[:, 0]]
    d -= big.L * np.round(d / big.L)
    r = np.linalg.norm(d, axis=1)
    assert r.min() >= 1.0 and r.max() <= 1.4


def test_product_shape_descriptors_agree_with_oracle():
    """The binding's ensemble shape descriptors (host post-processing of the GPU's per-polymer
    eigenvalues) against the oracle's own implementation, on random eigenvalue sets."""
    import oracle
    rng = np.random.default_rng(3)
    lam = np.sort(rng.gamma(2.0, 1.0, size=(4000, 3)), axis=1)[:, ::-1]
    a, b = ecmc.shape_descriptors(lam), oracle.shape_descriptors(lam)
    for k in b:
        assert abs(a[k] - b[k]) < 1e-12, k


def test_tuner_cache_key_and_file(tmp_path):
    """The tuner cache: the key is stable for equal inputs and changes with a melt's box, its bead
    count, ell, an option that changes what runs, the GPU and the library; a stored result comes
    back as written, other keys survive a second store, and a damaged file reads as a miss."""
    melts = inputs.batch_melts(3, 11, n_choices=(16, 32), beads_range=(1000, 3000))
    opt = ecmc.ecmc_default_options()
    args = (melts, 1.0, 1.4, opt, 2000, 20.0, 2, "gpu-a", "lib-1")
    k0 = ecmc.tune_key(*args)
    assert k0 == ecmc.tune_key(*args) and len(k0) == 64
    other = list(melts)
    other[1] = inputs.batch_melts(3, 12, n_choices=(16, 32), beads_range=(1000, 3000))[1]
    changed = [ecmc.tune_key(other, *args[1:]),
               ecmc.tune_key(melts, 1.0, 1.4, opt, 2001, 20.0, 2, "gpu-a", "lib-1"),
               ecmc.tune_key(melts, 1.0, 1.4, opt, 2000, 10.0, 2, "gpu-a", "lib-1"),
               ecmc.tune_key(melts, 1.0, 1.4, opt, 2000, 20.0, 2, "gpu-b", "lib-1"),
               ecmc.tune_key(melts, 1.0, 1.4, opt, 2000, 20.0, 2, "gpu-a", "lib-2")]
    opt2 = ecmc.ecmc_default_options()
    opt2.swap_moves = 1
    changed.append(ecmc.tune_key(melts, 1.0, 1.4, opt2, 2000, 20.0, 2, "gpu-a", "lib-1"))
    # the tuner times both searches, so the precision option does not change the key
    opt3 = ecmc.ecmc_default_options()
    opt3.precision = ecmc.PREC_MIXED
    assert ecmc.tune_key(melts, 1.0, 1.4, opt3, 2000, 20.0, 2, "gpu-a", "lib-1") == k0
    assert len(set(changed + [k0])) == len(changed) + 1
    path = str(tmp_path / "tune.json")
    assert ecmc.tune_cache_get(path, k0) is None
    res = {"stage_tier": 256, "policy": 0, "ms_per_sweep": 1.5, "ecs_per_s": 2e8, "candidates": 3, "cached": False}
    ecmc.tune_cache_put(path, k0, [12, 14, 16], [2, 2, 2], res)
    ecmc.tune_cache_put(path, changed[0], [8, 8, 8], [2, 2, 2], dict(res, stage_tier=128))
    nc, dc, got = ecmc.tune_cache_get(path, k0)
    assert nc == [12, 14, 16] and dc == [2, 2, 2] and got == {k: v for k, v in res.items() if k != "cached"}
    assert ecmc.tune_cache_get(path, changed[0])[2]["stage_tier"] == 128
    with open(path, "w") as f:
        f.write("{not json")
    assert ecmc.tune_cache_get(path, k0) is None


def test_bench_partition_defaults():
    """bench.py's workload geometry: tethers and springs both default to the 2^3-cell checkerboard;
    an explicit --tiling or --domain-cells wins; the tile-joint grid is divisible by the pitch with
    cells wider than the bond cap; no default partition has domains or tiles of a single cell."""
    import argparse
    import bench
    ns = lambda **kw: argparse.Namespace(**{"workload": "c3", "tiling": None, "domain_cells": 0, "springs": 0.0, **kw})
    assert (bench.workload_of(ns())["tiling"], bench.workload_of(ns())["D"]) == (1, 2)
    w = bench.workload_of(ns(springs=30.0))
    assert (w["tiling"], w["D"]) == (1, 2)
    w = bench.workload_of(ns(springs=30.0, tiling="joint"))
    assert (w["tiling"], w["D"]) == (2, 2)
    w = bench.workload_of(ns(springs=30.0, tiling="joint", domain_cells=3))
    assert (w["tiling"], w["D"]) == (2, 3)
    L = 106.85512104226243
    n = bench.grid_cells(L, 1.8, bench.workload_of(ns(springs=30.0)))
    assert n == 56 and n % 4 == 0 and L / n > 1.8
    n = bench.grid_cells(L, 1.8, bench.workload_of(ns(springs=30.0, tiling="joint")))
    assert n == 57 and n % 3 == 0 and L / n > 1.8


def test_pair_correlation_pools_the_melts_of_a_batch():
    """g(r) of two melts from their summed pair counts: each bin over the summed ideal-gas
    counts N_m (N_m - 1) / 2 * 4 pi (r_hi^3 - r_lo^3) / (3 V_m); one melt alone reduces to it."""
    import numpy as np
    hist = np.array([0, 3, 40, 125, 260], dtype=np.int64)
    r_max, nb, vol = 1.5, np.array([500, 2000]), np.array([1000.0, 8000.0])
    g = ecmc.pair_correlation(hist, r_max, nb, vol)
    edges = np.linspace(0.0, r_max, 6)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    ideal = sum(n * (n - 1) / 2.0 / v for n, v in zip(nb, vol)) * shell
    assert np.allclose(g, hist / ideal, rtol=1e-14, atol=0)
    assert np.allclose(ecmc.pair_correlation(hist, r_max, 500, 1000.0), hist / (500 * 499 / 2 / 1000.0 * shell),
                       rtol=1e-14, atol=0)
    with pytest.raises(ecmc.EcmcError):
        ecmc.pair_correlation(hist, -1.0, 500, 1000.0)


def test_shape_descriptors_take_any_eigenvalue_order():
    import numpy as np
    rng = np.random.default_rng(4)
    lam = rng.uniform(0.1, 3.0, (50, 3))
    a = ecmc.shape_descriptors(np.sort(lam, axis=1)[:, ::-1])
    b = ecmc.shape_descriptors(rng.permuted(lam, axis=1))
    assert all(abs(a[k] - b[k]) < 1e-13 * max(1.0, abs(a[k])) for k in a)
    with pytest.raises(ecmc.EcmcError):
        ecmc.shape_descriptors(np.zeros((2, 3)))


def test_bench_profiled_values_follow_the_kernel_source_hash(tmp_path):
    """bench.py takes measured HBM traffic and LDS figures from a committed counter summary only while
    the kernel sources still hash to the value recorded there (null otherwise, or without a summary)."""
    import bench
    good = tmp_path / "good.md"
    good.write_text(f"text\n- `kernel_source_sha256`: `{bench.kernel_source_hash()}`\n"
                    "- `hbm_bytes_per_launch_fp64`: `1.5e+09`\n- `lds_bank_conflict_ratio_fp64`: `6.0e-03`\n")
    assert bench.profiled_value("hbm_bytes_per_launch_fp64", str(good)) == 1.5e9
    assert bench.profiled_value("lds_bank_conflict_ratio_fp64", str(good)) == 6.0e-3
    assert bench.profiled_value("hbm_bytes_per_launch_mixed", str(good)) is None
    stale = tmp_path / "stale.md"
    stale.write_text("- `kernel_source_sha256`: `0`\n- `hbm_bytes_per_launch_fp64`: `1.5e+09`\n")
    assert bench.profiled_value("hbm_bytes_per_launch_fp64", str(stale)) is None
    assert bench.profiled_value("hbm_bytes_per_launch_fp64", str(tmp_path / "absent.md")) is None
    h = bench.host_cpu()
    assert isinstance(h["logical_cpus"], int) and h["logical_cpus"] >= 1
