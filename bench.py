"""Throughput of the event-chain hot path on one MI355X.

Workload (default): a melt of M = 16,384 chains x N = 64 tethered hard spheres
(1,048,576 beads), packing fraction 0.45, sigma = 1, tether l_max = 1.4 sigma,
periodic cube L = 106.855 sigma with 76 cells per axis, checkerboard domains of
2^3 cells (6,859 active domains per colour phase).  One step = one sweep: a new
partition, the 8 colour phases, N_beads event chains of length ell = 20 sigma in
all, then the observables (R^2, R_g^2, bond histogram, middle-bead positions).
Synthetic start: a jittered lattice walk (seeded), melted by the warm-up sweeps.

Metric: collision events/s (hard-sphere and tether lifts plus reflections off
immotile beads; cell crossings and wall reflections excluded), with bead-sweeps/s
(ECs started per second) alongside.  The roofline figure prices every collision
event at the algorithmic bytes of a cell-list search over the 18-cell forward
neighbourhood (1,384 B at this density, FP64) against 8 TB/s of HBM; the kernel
stages each domain once per sweep and runs its chains from LDS and registers, so its
measured HBM traffic is far below.  The plain FP64 search is the default; the screened
(mixed) search, which gives the same results, is timed after it in the same run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c5|c4] [--precision fp64|mixed]
       [--swap] [--springs K [--spring-cap B]]

--springs K bonds the same chains by harmonic springs (k/2)(b - sigma)^2 of constant K (Eq. (2);
the paper's melts use K = 30), capped at B sigma (default 1.8, which cuts off a Boltzmann weight
of 3e-5 of a free bond); the cells then have edge > B.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per collision event (FP64): 18 cells x rho h^3 candidates x (24 B
# position + 4 B id) + 18 x 4 B cell counts + 3 x 28 B (pivot and its two partners)
# + 24 B write-back
def bytes_per_event(beads_per_cell: float) -> float:
    return 18 * beads_per_cell * 28 + 18 * 4 + 3 * 28 + 24


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "ecmc_sweep_c3_1M_hbm_traffic.md")
BATCH_COUNTERS = os.path.join(ROOT, "profiles", "ecmc_sweep_c4_256melts_counters.md")
# the sources the profiled sweep kernel is built from: its translation unit and the headers it includes
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1502_06447_amd", "csrc", f)
                  for f in ("ecmc_device.h", "ecmc_internal.h", "ecmc_sweep.hip")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def profiled_value(key: str, summary: str = TRAFFIC_SUMMARY):
    """A value of a committed counter summary (rocprofv3 runs of the sweep kernel; by default the
    C3 one), or None when there is none or the kernel sources have changed since the counters were
    taken."""
    if not os.path.exists(summary):
        return None
    fields = {}
    for line in open(summary):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].strip().split(": ", 1)
            fields[k.strip("`")] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash() or key not in fields:
        return None
    return float(fields[key])


def measured_traffic(precision: str):
    """HBM bytes per sweep launch of the given search (fp64 or mixed): FETCH_SIZE + WRITE_SIZE."""
    return profiled_value(f"hbm_bytes_per_launch_{precision}")


WORKLOADS = {
    "c3": dict(M=16384, N=64, eta=0.45, ell=20.0, D=2, label="16384 chains x 64 beads (1,048,576), eta=0.45"),
    "c2": dict(M=500, N=32, eta=0.45, ell=20.0, D=3, label="500 chains x 32 beads (16,000), eta=0.45"),
    "c5": dict(M=2048, N=512, eta=0.45, ell=20.0, D=2, label="2048 chains x 512 beads (1,048,576), eta=0.45"),
    # the batched form: independent melts, N uniform in {16, ..., 256}, 2k-64k beads each,
    # eta uniform in [0.35, 0.45]; one tuned launch per sweep, sweeps replayed from a HIP graph
    "c4": dict(melts=256, ell=20.0, label="256 independent melts, N in {16,32,64,128,256}, 2,048-65,536 beads "
                                         "each, eta in [0.35, 0.45]"),
}


def checker_cells(L: float, b_max: float, D: int) -> int:
    """The largest cell grid with edge > b_max that a checkerboard of D^3-cell domains tiles
    (n a multiple of D with n / D even)."""
    n = int(L // b_max)
    while n > 0 and (L / n <= b_max or n % D or (n // D) % 2):
        n -= 1
    return n


def grid_cells(L: float, b_max: float, w) -> int:
    """Cells per axis for the workload's partition: the checkerboard grid, or for tile-joint
    (tiles of D^3 cells at pitch D + 1) the largest n with edge > b_max that the pitch divides."""
    if w.get("tiling", 1) == 2:
        P = w["D"] + 1
        n = int(L // b_max)
        while n > 0 and (L / n <= b_max or n % P or n // P < 2):
            n -= 1
        return n
    return checker_cells(L, b_max, w["D"])


def host_cpu() -> dict:
    """The host the CPU baseline ran on: CPU model, logical CPUs, and those this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(w, seconds: float = 12.0, seed: int = 5, swap: bool = False, spring_k: float = 0.0,
                 b_max: float = 1.4) -> dict:
    """The CPU oracle (serial, one core) on a bounded sample of the same workload: an
    independent 64 x 64 melt at the same packing fraction, ell, domain size and bonds."""
    import oracle
    from paper_1502_06447_amd import inputs

    m = inputs.lattice_chains(64, 64, w["eta"], seed=seed, b_max=b_max)
    n = grid_cells(m.L, b_max, w)
    o = oracle.Oracle.from_melt(m, n_cells=n)
    o.set_swap(swap)
    o.set_spring(spring_k)
    for s in range(2):  # melt the lattice like the GPU warm-up does
        o.sweep(m.n_beads, w["ell"], 100 + s, tiling=w.get("tiling", 1), D=w["D"])
    c0, _ = o.counters()
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        o.sweep(m.n_beads, w["ell"], 200 + k, tiling=w.get("tiling", 1), D=w["D"])
        k += 1
    dt = time.perf_counter() - t0
    c1, _ = o.counters()
    ev = int(sum(c1[i] - c0[i] for i in (oracle.C_HS_LIFT, oracle.C_TETHER_LIFT, oracle.C_HS_REFLECT,
                                          oracle.C_TETHER_REFLECT, oracle.C_SWAP)))
    return {"value": ev / dt, "unit": "collision events/s", "cores": 1, "kind": "oracle",
            "sample": f"64 x 64 beads (4,096), eta={w['eta']}, ell={w['ell']}, "
                      + ("tile-joint " if w.get("tiling", 1) == 2 else "") + f"D={w['D']}, {n}^3 cells"
                      + (f", springs k={spring_k} capped at {b_max}" if spring_k else "") + f": {k} sweeps "
                      f"after 2 warm-up sweeps, {dt:.1f} s, single thread",
            "ec_per_s": float(c1[oracle.C_EC] - c0[oracle.C_EC]) / dt, "host": host_cpu()}


def _oracle_worker(args):
    """One independent oracle instance (its own 64 x 64 melt and seeds) for `seconds` of work:
    (collision events, ECs, seconds)."""
    w, seconds, seed, spring_k, b_max = args
    import oracle
    from paper_1502_06447_amd import inputs
    m = inputs.lattice_chains(64, 64, w["eta"], seed=seed, b_max=b_max)
    o = oracle.Oracle.from_melt(m, n_cells=grid_cells(m.L, b_max, w))
    o.set_spring(spring_k)
    for s in range(2):
        o.sweep(m.n_beads, w["ell"], 100 + s, tiling=w.get("tiling", 1), D=w["D"])
    c0, _ = o.counters()
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        o.sweep(m.n_beads, w["ell"], 200 + k, tiling=w.get("tiling", 1), D=w["D"])
        k += 1
    dt = time.perf_counter() - t0
    c1, _ = o.counters()
    ev = int(sum(c1[i] - c0[i] for i in (oracle.C_HS_LIFT, oracle.C_TETHER_LIFT, oracle.C_HS_REFLECT,
                                          oracle.C_TETHER_REFLECT, oracle.C_SWAP)))
    return ev, int(c1[oracle.C_EC] - c0[oracle.C_EC]), dt


def cpu_baseline_all_cores(w, seconds: float = 1.5, spring_k: float = 0.0, b_max: float = 1.4) -> dict:
    """The oracle on every host core at once (up to 16): P independent instances, each on its own
    64 x 64 melt (independent by construction, as the domains of one colour or the melts of a
    batch are), for `seconds` each.  Forked before the GPU is touched."""
    import multiprocessing as mp
    P = max(1, min(os.cpu_count() or 1, 16))
    with mp.get_context("fork").Pool(P) as pool:
        res = pool.map(_oracle_worker, [(w, seconds, 50 + i, spring_k, b_max) for i in range(P)])
    wall = max(r[2] for r in res)
    return {"value": sum(r[0] for r in res) / wall, "unit": "collision events/s", "cores": P, "kind": "oracle",
            "sample": f"{P} independent 64 x 64 melts (4,096 beads each), one per core, {seconds} s each after "
                      "2 warm-up sweeps",
            "ec_per_s": sum(r[1] for r in res) / wall}


def copy_bandwidth(gib: int = 2, reps: int = 5) -> float:
    """HBM bandwidth of a plain device-to-device copy on this GPU, GB/s (read + written bytes
    over the best of a few HIP-event-timed copies)."""
    import torch
    n = gib << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n / best / 1e9


def precision_check(melt, w, sweeps: int, swap: bool = False, spring_k: float = 0.0) -> dict:
    """Both precisions from the same start through the same sweeps (untimed): the screened
    kernel must reproduce the plain FP64 kernel bit for bit.  Reported: the largest position
    difference, the shift of <R^2>, whether every event count agrees, and the event sequences
    compared record by record (sorted by sweep, domain, EC and step): the index of the first
    record where they differ (null: identical).  Springs run about 300 events per EC, whose
    logs (~10 GB at this size) are not taken."""
    import numpy as np
    from paper_1502_06447_amd import ecmc
    # about 9 records per tether EC (collision events, wall reflections, the periodic skip, the end)
    log_cap = 0 if spring_k > 0 else int(16 * melt.n_beads * sweeps)
    res = {}
    for name, prec in (("mixed", ecmc.PREC_MIXED), ("fp64", ecmc.PREC_FP64)):
        g = ecmc.Melt.from_melt(melt, ecmc.Options(tiling=w.get("tiling", 1), domain_cells=w["D"], precision=prec,
                                                   swap_moves=swap, spring_k=spring_k,
                                                   n_cells=grid_cells(melt.L, melt.b_max, w),
                                                   event_log_capacity=log_cap))
        for i in range(sweeps):
            g.sweep(melt.n_beads, w["ell"], 7000 + i)
        g.synchronize()
        log = None
        if log_cap:
            log = g.event_log()
            log = log[np.lexsort((log["step"], log["ec"], log["domain"], log["sweep"]))]
        res[name] = (g.positions(), g.observables(nbins=32)["r2"].mean(), g.counters(), log)
        g.close()
    (pm, r2m, cm, lm), (pf, r2f, cf, lf) = res["mixed"], res["fp64"]
    out = {"sweeps": sweeps, "beads": int(melt.n_beads), "positions_identical": bool(np.array_equal(pm, pf)),
           "max_position_drift": float(np.abs(pm - pf).max()), "r2_mixed": float(r2m), "r2_fp64": float(r2f),
           "r2_shift": float(r2m - r2f),
           # event counts exactly; the sum of lift overlaps to rounding (atomic adds in any order)
           "event_counts_identical": all(cm[k] == cf[k] for k in cm if k not in ("error_flags", "sum_delta")),
           "sum_delta_rel_diff": float(abs(cm["sum_delta"] - cf["sum_delta"]) / max(abs(cf["sum_delta"]), 1e-300))}
    if log_cap:
        m = min(len(lm), len(lf))
        diff = np.flatnonzero(lm[:m] != lf[:m])
        first = int(diff[0]) if len(diff) else (m if len(lm) != len(lf) else None)
        out["event_records"] = int(len(lf))
        out["first_divergent_event"] = first
        if first is not None and first < m:
            out["first_divergent_key"] = {k: int(lf[first][k]) for k in ("sweep", "domain", "ec", "step")}
    return out


def batch_precision_check(melts, opts, nc, dc, ell: float, sweeps: int) -> dict:
    """Both precisions from the same start through the same sweeps of the whole batch."""
    import numpy as np
    from paper_1502_06447_amd import ecmc
    nb = sum(m.n_beads for m in melts)
    res = {}
    for name, prec in (("mixed", ecmc.PREC_MIXED), ("fp64", ecmc.PREC_FP64)):
        o = ecmc.Options(**{**opts.__dict__, "precision": prec})
        g = ecmc.Melt.from_batch(melts, o, n_cells=nc, domain_cells=dc)
        for i in range(sweeps):
            g.sweep(nb, ell, 7000 + i)
        g.synchronize()
        res[name] = (g.positions(), g.counters())
        g.close()
    (pm, cm), (pf, cf) = res["mixed"], res["fp64"]
    return {"sweeps": sweeps, "beads": int(nb), "positions_identical": bool(np.array_equal(pm, pf)),
            "max_position_drift": float(np.abs(pm - pf).max()),
            "event_counts_identical": all(cm[k] == cf[k] for k in cm if k not in ("error_flags", "sum_delta"))}


def batch_cpu_baseline(melt, ell: float, D: int, n_cells: int, seconds: float) -> dict:
    """The CPU oracle (serial, one core) on one melt of the batch, same schedule rules."""
    import oracle
    o = oracle.Oracle.from_melt(melt, n_cells=n_cells)
    o.sweep(melt.n_beads, ell, 100, tiling=1, D=D)
    c0, _ = o.counters()
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        o.sweep(melt.n_beads, ell, 200 + k, tiling=1, D=D)
        k += 1
    dt = time.perf_counter() - t0
    c1, _ = o.counters()
    ev = int(sum(c1[i] - c0[i] for i in (oracle.C_HS_LIFT, oracle.C_TETHER_LIFT, oracle.C_HS_REFLECT,
                                          oracle.C_TETHER_REFLECT, oracle.C_SWAP)))
    return {"value": ev / dt, "unit": "collision events/s", "cores": 1, "kind": "oracle",
            "sample": f"melt 0 of the batch ({melt.n_beads} beads, N={melt.n_per}, eta={melt.eta:.3f}), "
                      f"{n_cells}^3 cells, D={D}: {k} sweeps after 1 warm-up sweep, {dt:.1f} s, single thread",
            "ec_per_s": float(c1[oracle.C_EC] - c0[oracle.C_EC]) / dt, "host": host_cpu()}


def copy_probe(mib: int) -> None:
    """One device-to-device copy of mib MiB (a plain copy kernel of known size, the scale for
    hardware byte counters); nothing for mib = 0."""
    if mib <= 0:
        return
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    print(f"# copy probe: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)


def main_batch(args):
    """The batched workload: tuned geometry and staging, K sweeps captured into one HIP graph
    (the sweep loop), replayed once in the timed region after W eager warm-up sweeps."""
    import numpy as np
    import torch
    from paper_1502_06447_amd import ecmc, inputs

    w = WORKLOADS["c4"]
    torch.cuda.set_device(0)
    copy_probe(args.copy_probe)
    melts = inputs.batch_melts(w["melts"], args.seed)
    nb = sum(m.n_beads for m in melts)
    ell = w["ell"]
    prec = ecmc.PREC_MIXED if args.precision == "mixed" else ecmc.PREC_FP64
    opts = ecmc.Options(precision=prec, swap_moves=args.swap)
    tune = None
    nc = dc = None
    if not args.no_tune:
        t0 = time.perf_counter()
        nc, dc, tune = ecmc.ecmc_tune_batch(melts, 1.0, 1.4, ecmc._native_options(opts), nb, ell, trial_sweeps=2,
                                            cache=args.tune_cache)
        tune["seconds"] = time.perf_counter() - t0
        opts.stage_tier = tune["stage_tier"]
        opts.precision = tune["precision"]
        print(f"# tuned: stage tier {tune['stage_tier']}, policy {tune['policy']}, precision {tune['precision']}, "
              f"{tune['candidates']} candidates, {tune['seconds']:.1f} s{' (cached)' if tune['cached'] else ''}",
              file=sys.stderr, flush=True)
    prec_name = "fp64" if opts.precision == ecmc.PREC_FP64 else "mixed"
    stream = torch.cuda.Stream()
    g = ecmc.Melt.from_batch(melts, opts, n_cells=nc, domain_cells=dc, stream=stream)
    infos = [g.melt_info(m) for m in range(g.n_melts)]
    cells = sum(i["n_cells"] ** 3 for i in infos)
    print(f"# c4: {len(melts)} melts, {nb} beads, {cells} cells, staging {g.stage_capacity}", file=sys.stderr,
          flush=True)
    for i in range(args.warmup):
        g.sweep(nb, ell, 1000 + i)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    g.synchronize()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        for i in range(args.steps):
            g.sweep(nb, ell, 1000 + args.warmup + i)
    torch.cuda.synchronize()
    c0 = g.counters()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c1 = g.counters()
    g.synchronize()
    kernel_s = e0.elapsed_time(e1) / 1e3
    d = {k: c1[k] - c0[k] for k in c1 if k not in ("error_flags",)}
    events = d["hs_lift"] + d["tether_lift"] + d["hs_reflect"] + d["tether_reflect"] + d["swap"]
    ecs = d["ec"]
    value = events / dt
    # algorithmic bytes per event at the bead-weighted mean occupancy of a cell
    occ = sum(i["n_beads"] * (i["n_beads"] / i["n_cells"] ** 3) for i in infos) / nb
    B = bytes_per_event(occ)
    achieved = events * B / kernel_s / 1e9 if kernel_s > 0 else 0.0
    # the committed counters are of the configuration the tuner picks for this batch (the first
    # geometry policy, 256-bead tier, plain FP64 search); another choice has none
    profiled = (bool(tune) and tune["policy"] == 0 and opts.stage_tier == 256 and opts.precision == ecmc.PREC_FP64
                and not args.swap)
    traffic = profiled_value("hbm_bytes_per_launch_fp64", BATCH_COUNTERS) if profiled else None
    out = {
        "metric": "collision events/s",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"c4: {w['label']}, ell={ell} sigma, checkerboard (tuned per melt), FP64 results "
                        f"({prec_name} event search{', tuned' if tune else ''}), sweep loop replayed from one HIP graph",
            "melts": len(melts), "beads": nb, "cells": cells, "precision": prec_name,
            "swap_moves": bool(args.swap), "stage_capacity": g.stage_capacity, "parallelism": "single GPU",
            "domain_cells_used": sorted(set(i["domain_cells"] for i in infos)),
        },
        "tune": tune,
        "bead_sweeps_per_s": ecs / dt,
        "events_per_ec": events / max(ecs, 1),
        "counters": {k: int(v) if isinstance(v, int) else v for k, v in d.items()},
        "kernel_ms_per_step": kernel_s * 1e3 / args.steps,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_event": B,
            "lds_bank_conflict_ratio": (profiled_value("lds_bank_conflict_ratio_fp64", BATCH_COUNTERS)
                                        if profiled else None),
            "note": "algorithmic bytes (18-cell forward cell-list scan per collision event, bead-weighted mean "
                    "cell occupancy) over the HIP-event time of the graph replay; traffic: measured HBM bytes "
                    "per sweep launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated by a copy)",
        },
    }
    if traffic is not None:
        out["roofline"]["traffic_bytes_per_event"] = traffic / (events / args.steps)
        out["roofline"]["traffic_GBps"] = traffic * args.steps / kernel_s / 1e9 if kernel_s > 0 else None
    if not args.no_precision_check:
        out["precision_check"] = batch_precision_check(melts, opts, nc, dc, ell, sweeps=2)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(melts[0], ell, infos[0]["domain_cells"], infos[0]["n_cells"],
                                                 seconds=args.cpu_seconds)
        out["cpu_baseline"]["vs_gpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def msd_run(g, nb: int, w, sweeps: int, seed0: int) -> dict:
    """Untimed: continue the run for `sweeps` sweeps with a snapshot of every chain's middle bead and
    centre of mass after each (Sec. IV.A), then g1 and g2 over all time origins on the GPU; reported at
    lags 1, 2, 4, ... sweeps with the collision events the run took."""
    import torch
    snaps = torch.empty((sweeps + 1, g.n_poly, 6), dtype=torch.float64, device="cuda")
    c0 = g.counters()
    g.snapshot(out=snaps[0])
    t0 = time.perf_counter()
    for s in range(sweeps):
        g.sweep(nb, w["ell"], seed0 + s)
        g.snapshot(out=snaps[s + 1])
        if (s + 1) % 100 == 0:
            g.synchronize()
            print(f"# msd run: {s + 1}/{sweeps} sweeps", file=sys.stderr, flush=True)
    g1, g2 = g.msd(snaps)
    dt = time.perf_counter() - t0
    c1 = g.counters()
    ev = sum(c1[k] - c0[k] for k in ("hs_lift", "tether_lift", "hs_reflect", "tether_reflect", "swap"))
    lags = [1 << k for k in range(sweeps.bit_length()) if (1 << k) <= sweeps]
    return {"sweeps": sweeps, "collision_events": int(ev), "seconds": dt, "lags_sweeps": lags,
            "g1": [float(g1[d]) for d in lags], "g2": [float(g2[d]) for d in lags],
            "note": "middle bead (g1) and middle bead relative to the centre of mass (g2), sigma^2, averaged "
                    "over chains and time origins; from the start state, not an equilibrated melt"}


def workload_of(args) -> dict:
    """The workload's parameters with the partition chosen on the command line.  Without one,
    tethers and springs both run on the checkerboard of 2^3-cell domains (every partition on
    offer has domains of at least 2 cells per edge: smaller ones would keep each bead in its
    cell for good)."""
    tiling = args.tiling or "checker"
    w = dict(WORKLOADS[args.workload], tiling=2 if tiling == "joint" else 1)
    if args.domain_cells > 0:
        w["D"] = args.domain_cells
    return w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=("mixed", "fp64"),
                    help="fp64 (default, the faster on every workload measured): every staged bead evaluated in "
                         "FP64 at every event (the plain kernel); mixed: single-precision screen + FP64 evaluation "
                         "of the beads it cannot rule out; identical results.  The other one is timed after the "
                         "main run.  c4: the autotuner's choice unless --no-tune")
    ap.add_argument("--swap", action="store_true", help="swap moves at hard-sphere contacts (Sec. II.C)")
    ap.add_argument("--springs", type=float, default=0.0, metavar="K",
                    help="bonds as harmonic springs of constant K (Eq. (2), k_B T / sigma^2); 0 = tethers")
    ap.add_argument("--tiling", default=None, choices=("checker", "joint"),
                    help="checker: D^3-cell domains in 8 colour phases (the default); joint: the "
                         "tile-joint partition (D^3-cell tiles at pitch D + 1 with immotile joints, one phase; "
                         "D >= 2)")
    ap.add_argument("--domain-cells", type=int, default=0, metavar="D",
                    help="domain (checkerboard) or tile (tile-joint) edge in cells; 0 = the workload's (2)")
    ap.add_argument("--spring-cap", type=float, default=1.8, metavar="B",
                    help="with --springs: bond length cap in sigma (cells get an edge > B)")
    ap.add_argument("--no-precision-check", action="store_true",
                    help="skip the untimed comparison of the two precisions after the timed steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--msd-sweeps", type=int, default=0, metavar="S",
                    help="after the timed steps (untimed): S more sweeps with a snapshot after each, and g1, g2 "
                         "(Sec. IV.A) at lags 1, 2, 4, ... sweeps in the JSON line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="c4: skip the autotuner (automatic geometry and staging)")
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="c4: reuse a tuning result stored in this file for the same batch, GPU and library")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device once (a plain copy kernel of known size, "
                         "the scale for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); a multi-GPU run is not part of this build",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        if args.springs:
            print("--springs is not offered for the batched workload", file=sys.stderr)
            sys.exit(2)
        return main_batch(args)
    b_max = args.spring_cap if args.springs else 1.4
    all_cores = None
    if not args.no_cpu_baseline:
        # the all-cores oracle leg runs first, in forked workers, before this process touches the GPU
        all_cores = cpu_baseline_all_cores(workload_of(args), spring_k=args.springs, b_max=b_max)

    import numpy as np
    import torch
    from paper_1502_06447_amd import ecmc, inputs

    w = workload_of(args)
    torch.cuda.set_device(0)
    copy_probe(args.copy_probe)
    melt = inputs.lattice_chains(w["M"], w["N"], w["eta"], seed=args.seed, b_max=b_max)
    n_cells = grid_cells(melt.L, b_max, w)
    nb = melt.n_beads

    def timed_run(precision: str):
        """W untimed and K timed sweeps of a fresh context, each followed by the observables, which
        are added to running device sums (no host round trip between sweeps); their means over the
        K timed sweeps are read after the timed region."""
        prec = ecmc.PREC_MIXED if precision == "mixed" else ecmc.PREC_FP64
        g = ecmc.Melt.from_melt(melt, ecmc.Options(tiling=w.get("tiling", 1), domain_cells=w["D"], time_kernels=True,
                                                   precision=prec, swap_moves=args.swap, spring_k=args.springs,
                                                   n_cells=n_cells))

        def step(i):
            g.sweep(nb, w["ell"], 1000 + i)
            g.observables_accumulate(nbins=32)

        for i in range(args.warmup):
            step(i)
            print(f"# {precision} warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
        g.synchronize()
        g.kernel_time()
        g.observables_reset()
        c0 = g.counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(args.warmup + i)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.synchronize()
        c1 = g.counters()
        kms, launches = g.kernel_time()
        d = {k: c1[k] - c0[k] for k in c1 if k not in ("error_flags",)}
        events = d["hs_lift"] + d["tether_lift"] + d["hs_reflect"] + d["tether_reflect"] + d["swap"]
        print(f"# {precision}: {args.steps} timed sweeps in {dt:.4f} s", file=sys.stderr, flush=True)
        return g, dt, d, events, kms, launches

    g, dt, d, events, kms, launches = timed_run(args.precision)
    obs = g.observables_mean()
    n = g.n_cells
    beads_per_cell = nb / n ** 3
    print(f"# {args.workload}: {nb} beads, L={melt.L:.4f}, n={n}, h={g.h:.4f}, staging {g.stage_capacity}",
          file=sys.stderr, flush=True)
    ecs = d["ec"]
    value = events / dt
    B = bytes_per_event(beads_per_cell)
    kernel_s = kms / 1e3  # HIP events around each sweep launch (or colour phase, by phases)
    achieved = events * B / kernel_s / 1e9 if kernel_s > 0 else 0.0
    plain_c3 = args.workload == "c3" and not args.swap and not args.springs and w["tiling"] == 1
    traffic = measured_traffic(args.precision) if plain_c3 else None
    out = {
        "metric": "collision events/s",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {w['label']}, ell={w['ell']} sigma, "
                        + (f"checkerboard D={w['D']}, " if w["tiling"] == 1 else
                           f"tile-joint {w['D']}^3-cell tiles at pitch {w['D'] + 1}, ")
                        + f"{n}^3 cells, FP64 results ({args.precision} event search)"
                        + (", swap moves" if args.swap else "")
                        + (f", harmonic springs k={args.springs} capped at {b_max} sigma" if args.springs else ""),
            "precision": args.precision, "swap_moves": bool(args.swap),
            "tiling": "checkerboard" if w["tiling"] == 1 else "tile-joint",
            "bonds": (f"spring k={args.springs}, cap {b_max} sigma" if args.springs else "tether 1.4 sigma"),
            "beads": nb, "chains": w["M"], "beads_per_chain": w["N"], "eta": w["eta"], "ell": w["ell"],
            "domain_cells": w["D"], "cells_per_axis": n, "parallelism": "single GPU",
        },
        "bead_sweeps_per_s": ecs / dt,
        "events_per_ec": events / max(ecs, 1),
        "counters": {k: int(v) if isinstance(v, int) else v for k, v in d.items()},
        "observables": {"r2_mean": obs["r2"], "rg2_mean": obs["rg2"], "samples": obs["samples"],
                        "note": "<R^2>, <R_g^2> per chain over the timed sweeps, sampled after each on the "
                                "device"},
        "kernel_ms_per_step": kms / args.steps,
        "timed_launches": launches,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": events * B / max(launches, 1),
            "bytes_per_event": B,
            "note": "achieved: algorithmic bytes (18-cell forward cell-list scan per collision event) over the "
                    "HIP-event time of the sweep launches ("
                    + ("one dependency-ordered kernel per sweep" if w.get("tiling", 1) == 1 else
                       "the tile-joint phase: its staging tiers on two streams, one phase per sweep")
                    + "); traffic: measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated "
                      "by a copy)",
        },
    }
    # the other precision timed in the same way, from the same start and seeds: its results are
    # the same FP64 trajectory, so the two rates compare like for like
    other = "fp64" if args.precision == "mixed" else "mixed"
    g_o, dt_o, d_o, events_o, kms_o, launches_o = timed_run(other)
    del g_o
    ach_o = events_o * B / (kms_o / 1e3) / 1e9 if kms_o > 0 else 0.0
    out[other] = {
        "value": events_o / dt_o, "unit": "events/s", "ms_per_step": dt_o / args.steps * 1e3,
        "bead_sweeps_per_s": d_o["ec"] / dt_o, "kernel_ms_per_step": kms_o / args.steps,
        "roofline_achieved_GBps": ach_o, "frac": ach_o / HBM_PEAK_GBS,
        "same_trajectory": bool(events_o == events and d_o["ec"] == ecs),
        "traffic": measured_traffic(other) if plain_c3 else None,
        "lds_bank_conflict_ratio": profiled_value(f"lds_bank_conflict_ratio_{other}") if plain_c3 else None,
    }
    # LDS bank-conflict cycles over LDS-active cycles of the sweep kernel (SQ counters)
    out["roofline"]["lds_bank_conflict_ratio"] = (profiled_value(f"lds_bank_conflict_ratio_{args.precision}")
                                                  if plain_c3 else None)
    if traffic is not None:
        # the measured HBM bytes of a launch per collision event, and as a rate over the launch time
        out["roofline"]["traffic_bytes_per_event"] = traffic / (events / max(launches, 1))
        out["roofline"]["traffic_GBps"] = traffic * launches / kernel_s / 1e9 if kernel_s > 0 else None
    out["roofline"]["measured_copy_GBps"] = copy_bandwidth()
    if args.msd_sweeps > 0:
        out["msd"] = msd_run(g, nb, w, args.msd_sweeps, 1000 + args.warmup + args.steps)
    if not args.no_precision_check:
        out["precision_check"] = precision_check(melt, w, sweeps=2, swap=args.swap, spring_k=args.springs)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, seconds=args.cpu_seconds, swap=args.swap, spring_k=args.springs,
                                           b_max=b_max)
        out["cpu_baseline"]["vs_gpu"] = value / out["cpu_baseline"]["value"]
        out["cpu_baseline"]["all_cores"] = all_cores
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
