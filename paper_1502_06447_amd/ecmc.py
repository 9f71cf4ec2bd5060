"""Python binding of the C ABI in ``include/ecmc.h`` (ctypes; argument marshalling only).

Every step of the event-chain path runs in the gfx950 kernels of ``libecmc.so``.
PyTorch only supplies the device workspace (a uint8 tensor) and the stream.  If
the library is missing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; ECMC_LIB names another build of the same sources (a tuning variant)
LIB_PATH = os.environ.get("ECMC_LIB") or os.path.join(_HERE, "libecmc.so")

OK, E_ARG, E_OVERLAP, E_TETHER, E_BOX, E_CELL_OVERFLOW, E_STUCK, E_DEVICE, E_WORKSPACE = 0, -1, -2, -3, -4, -5, -6, -7, -8
PREC_FP64, PREC_MIXED = 0, 1
TILING_WHOLE, TILING_CHECKER, TILING_JOINT = 0, 1, 2
SCHED_SWEEP, SCHED_PHASES = 0, 1
EV_HS_LIFT, EV_TETHER_LIFT, EV_HS_REFLECT, EV_TETHER_REFLECT, EV_WALL, EV_END, EV_PERIOD, EV_CYCLE, EV_SWAP = range(9)

EVENT_DTYPE = np.dtype([
    ("sweep", "<u4"), ("domain", "<u4"), ("ec", "<u4"), ("step", "<u4"),
    ("pivot", "<i4"), ("target", "<i4"), ("kind", "<u4"), ("colour", "<u4"),
])


class ecmc_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("tiling", ctypes.c_int32),
        ("n_cells", ctypes.c_int32),
        ("domain_cells", ctypes.c_int32),
        ("cell_capacity", ctypes.c_int32),
        ("stage_capacity", ctypes.c_int32),
        ("event_cap", ctypes.c_int64),
        ("event_log_capacity", ctypes.c_int64),
        ("time_kernels", ctypes.c_int32),
        ("swap_moves", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("stage_tier", ctypes.c_int32),
        ("overlapping_start", ctypes.c_int32),
        ("spring_k", ctypes.c_double),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("side_stream", ctypes.c_void_p),
        ("wait_limit_us", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ecmc_melt_desc(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double),
        ("n_beads", ctypes.c_int64),
        ("positions", ctypes.c_void_p),
        ("n_bonds", ctypes.c_int64),
        ("bonds", ctypes.c_void_p),
        ("n_cells", ctypes.c_int32),
        ("domain_cells", ctypes.c_int32),
    ]


class ecmc_melt_info(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double), ("cell_size", ctypes.c_double),
        ("first_bead", ctypes.c_int64), ("n_beads", ctypes.c_int64),
        ("first_polymer", ctypes.c_int64), ("n_polymers", ctypes.c_int64),
        ("first_domain", ctypes.c_int64), ("n_domains", ctypes.c_int64),
        ("n_cells", ctypes.c_int32), ("domain_cells", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ecmc_tune_result(ctypes.Structure):
    _fields_ = [("stage_tier", ctypes.c_int32), ("policy", ctypes.c_int32), ("ms_per_sweep", ctypes.c_double),
                ("ecs_per_s", ctypes.c_double), ("candidates", ctypes.c_int32), ("precision", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ecmc_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("hs_lift", "tether_lift", "hs_reflect", "tether_reflect", "wall", "cross", "ec", "steps",
                 "periodic", "cycle", "swap")] + [
        ("sum_delta", ctypes.c_double), ("error_flags", ctypes.c_uint32), ("pad", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class EcmcError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: {msg} (status {code})")
        self.code = code


_lib = None

EXPORTS = (
    "ecmc_default_options", "ecmc_workspace_size", "ecmc_init", "ecmc_sweep", "ecmc_sweep_colours",
    "ecmc_synchronize", "ecmc_observables", "ecmc_shape", "ecmc_get_positions", "ecmc_get_cells", "ecmc_get_images",
    "ecmc_get_counters", "ecmc_reset_counters", "ecmc_get_event_log", "ecmc_clear_event_log",
    "ecmc_set_state", "ecmc_kernel_time", "ecmc_sweep_counter", "ecmc_n_cells", "ecmc_cell_size",
    "ecmc_stage_capacity", "ecmc_destroy", "ecmc_status_str", "ecmc_last_error",
    "ecmc_workspace_size_batch", "ecmc_init_batch", "ecmc_n_melts", "ecmc_get_melt_info",
    "ecmc_tune_workspace_size", "ecmc_tune_batch", "ecmc_snapshot", "ecmc_msd", "ecmc_end_to_end_histogram",
    "ecmc_pair_histogram", "ecmc_pushoff_sweep", "ecmc_count_overlaps", "ecmc_pushoff", "ecmc_internal_distances",
    "ecmc_check_state", "ecmc_screen_constants", "ecmc_internal_distances_noalloc", "ecmc_clear_error",
    "ecmc_shape_descriptors", "ecmc_pair_correlation", "ecmc_observables_accumulate", "ecmc_observables_mean",
    "ecmc_observables_reset",
)


def lib():
    """Load libecmc.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (no CPU fallback exists)")
    # torch's HIP runtime is loaded first: the library's shares the process with it, and the
    # other order leaves the library without a device
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    i32, i64, u32, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    st = ctypes.c_int
    opt_p = P(ecmc_options)
    sig = {
        "ecmc_default_options": (None, [opt_p]),
        "ecmc_workspace_size": (st, [dbl, dbl, dbl, i64, opt_p, P(ctypes.c_size_t)]),
        "ecmc_screen_constants": (st, [dbl, dbl, dbl, i64, opt_p, vp, vp]),
        "ecmc_init": (st, [P(vp), dbl, dbl, dbl, i64, vp, i64, vp, opt_p]),
        "ecmc_sweep": (st, [vp, i64, dbl, u64]),
        "ecmc_sweep_colours": (st, [vp, i64, dbl, u64, u32]),
        "ecmc_synchronize": (st, [vp]),
        "ecmc_observables": (st, [vp, i32, vp, vp, vp, vp, P(i64)]),
        "ecmc_observables_accumulate": (st, [vp, i32]),
        "ecmc_observables_mean": (st, [vp, P(dbl), P(dbl), vp, P(i64)]),
        "ecmc_observables_reset": (st, [vp]),
        "ecmc_shape": (st, [vp, vp, vp, vp, P(i64)]),
        "ecmc_snapshot": (st, [vp, vp]),
        "ecmc_msd": (st, [vp, vp, i64, vp]),
        "ecmc_end_to_end_histogram": (st, [vp, i32, dbl, vp]),
        "ecmc_pair_histogram": (st, [vp, i32, dbl, vp]),
        "ecmc_internal_distances": (st, [vp, i32, vp, vp]),
        "ecmc_internal_distances_noalloc": (st, [vp, i32, vp, vp]),
        "ecmc_check_state": (st, [vp, dbl, P(i64), P(i64), P(i64)]),
        "ecmc_pushoff_sweep": (st, [vp, i64, dbl, u64, dbl]),
        "ecmc_count_overlaps": (st, [vp, dbl, P(i64)]),
        "ecmc_pushoff": (st, [vp, dbl, i32, dbl, u64, i64, P(i64), P(i64)]),
        "ecmc_get_positions": (st, [vp, vp]),
        "ecmc_get_cells": (st, [vp, vp]),
        "ecmc_get_images": (st, [vp, vp]),
        "ecmc_get_counters": (st, [vp, P(ecmc_counters)]),
        "ecmc_reset_counters": (st, [vp]),
        "ecmc_clear_error": (st, [vp]),
        "ecmc_shape_descriptors": (st, [vp, i64, vp]),
        "ecmc_pair_correlation": (st, [vp, i32, dbl, i32, vp, vp, vp]),
        "ecmc_get_event_log": (st, [vp, vp, i64, P(i64)]),
        "ecmc_clear_event_log": (st, [vp]),
        "ecmc_set_state": (st, [vp, vp, vp, vp, u32]),
        "ecmc_kernel_time": (st, [vp, P(dbl), P(i64)]),
        "ecmc_sweep_counter": (u32, [vp]),
        "ecmc_n_cells": (i32, [vp]),
        "ecmc_cell_size": (dbl, [vp]),
        "ecmc_stage_capacity": (i32, [vp]),
        "ecmc_workspace_size_batch": (st, [i32, P(ecmc_melt_desc), dbl, dbl, opt_p, P(ctypes.c_size_t)]),
        "ecmc_init_batch": (st, [P(vp), i32, P(ecmc_melt_desc), dbl, dbl, opt_p]),
        "ecmc_n_melts": (i32, [vp]),
        "ecmc_get_melt_info": (st, [vp, i32, P(ecmc_melt_info)]),
        "ecmc_tune_workspace_size": (st, [i32, P(ecmc_melt_desc), dbl, dbl, opt_p, P(ctypes.c_size_t)]),
        "ecmc_tune_batch": (st, [i32, P(ecmc_melt_desc), dbl, dbl, opt_p, i64, dbl, i32, P(i32), P(i32),
                                 P(ecmc_tune_result)]),
        "ecmc_destroy": (None, [vp]),
        "ecmc_status_str": (ctypes.c_char_p, [st]),
        "ecmc_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int, what: str, ctx=None):
    if code != OK:
        msg = lib().ecmc_last_error(ctx).decode()
        raise EcmcError(code, what, msg or lib().ecmc_status_str(code).decode())


# ---------------------------------------------------------------- thin wrappers (same names)
def ecmc_default_options() -> ecmc_options:
    o = ecmc_options()
    lib().ecmc_default_options(ctypes.byref(o))
    return o


def ecmc_workspace_size(box: float, sigma: float, l_max: float, n_beads: int, opt: ecmc_options) -> int:
    n = ctypes.c_size_t()
    _check(lib().ecmc_workspace_size(box, sigma, l_max, n_beads, ctypes.byref(opt), ctypes.byref(n)),
           "ecmc_workspace_size")
    return n.value


def ecmc_screen_constants(box: float, sigma: float, l_max: float, n_beads: int, opt: ecmc_options) -> dict:
    """The single-precision screen's constants for this geometry (host only): p_sure, in_lo, in_hi,
    err (float32 values) and the cell edge h, frame edge X and box L."""
    out = np.zeros(4, dtype=np.float32)
    geo = np.zeros(3, dtype=np.float64)
    _check(lib().ecmc_screen_constants(box, sigma, l_max, n_beads, ctypes.byref(opt), out.ctypes.data,
                                       geo.ctypes.data), "ecmc_screen_constants")
    return {"p_sure": out[0], "in_lo": out[1], "in_hi": out[2], "err": out[3], "h": float(geo[0]),
            "X": float(geo[1]), "L": float(geo[2])}


def ecmc_init(box, sigma, l_max, positions, bonds, opt: ecmc_options):
    pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
    bnd = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
    h = ctypes.c_void_p()
    _check(lib().ecmc_init(ctypes.byref(h), box, sigma, l_max, pos.shape[0], pos.ctypes.data, bnd.shape[0],
                           bnd.ctypes.data if bnd.size else None, ctypes.byref(opt)), "ecmc_init")
    return h


def _melt_descs(melts, n_cells=None, domain_cells=None):
    """ecmc_melt_desc array for inputs.Melt-like objects; the returned arrays must outlive the call."""
    keep = []
    descs = (ecmc_melt_desc * len(melts))()
    for i, m in enumerate(melts):
        pos = np.ascontiguousarray(m.positions, dtype=np.float64).reshape(-1, 3)
        bnd = np.ascontiguousarray(m.bonds, dtype=np.int32).reshape(-1, 2)
        keep += [pos, bnd]
        descs[i].box = float(m.L)
        descs[i].n_beads = pos.shape[0]
        descs[i].positions = pos.ctypes.data
        descs[i].n_bonds = bnd.shape[0]
        descs[i].bonds = bnd.ctypes.data if bnd.size else None
        descs[i].n_cells = int(n_cells[i]) if n_cells is not None else 0
        descs[i].domain_cells = int(domain_cells[i]) if domain_cells is not None else 0
    return descs, keep


def ecmc_workspace_size_batch(melts, sigma: float, l_max: float, opt: ecmc_options, n_cells=None,
                              domain_cells=None) -> int:
    descs, keep = _melt_descs(melts, n_cells, domain_cells)
    n = ctypes.c_size_t()
    _check(lib().ecmc_workspace_size_batch(len(melts), descs, sigma, l_max, ctypes.byref(opt), ctypes.byref(n)),
           "ecmc_workspace_size_batch")
    return n.value


def ecmc_init_batch(melts, sigma: float, l_max: float, opt: ecmc_options, n_cells=None, domain_cells=None):
    descs, keep = _melt_descs(melts, n_cells, domain_cells)
    h = ctypes.c_void_p()
    _check(lib().ecmc_init_batch(ctypes.byref(h), len(melts), descs, sigma, l_max, ctypes.byref(opt)),
           "ecmc_init_batch")
    return h


# Options that change what a sweep runs, and so the tuner's choice (the workspace, the stream and
# the staging tier the tuner itself picks are left out).
# (the precision is not among them: the tuner times both searches whatever the option says)
_TUNE_OPTION_FIELDS = ("tiling", "n_cells", "domain_cells", "cell_capacity", "stage_capacity",
                       "event_cap", "event_log_capacity", "swap_moves", "schedule", "overlapping_start", "spring_k")


def tune_key(melts, sigma: float, l_max: float, opt: ecmc_options, n_chains: int, ell: float, trial_sweeps: int,
             device_name: str, library_digest: str) -> str:
    """Key of a tuning result (SHA-256 hex): the geometry of every melt (box edge, beads, bonds),
    sigma and l_max, the options that change what runs, the ECs per sweep, ell and the trial
    length, the GPU's name and a digest of the library that was timed."""
    items = {
        "melts": [[float(m.L).hex(), int(m.n_beads), int(len(m.bonds))] for m in melts],
        "sigma": float(sigma).hex(), "l_max": float(l_max).hex(),
        "options": {k: (getattr(opt, k).hex() if isinstance(getattr(opt, k), float) else int(getattr(opt, k)))
                    for k in _TUNE_OPTION_FIELDS},
        "n_chains": int(n_chains), "ell": float(ell).hex(), "trial_sweeps": int(trial_sweeps),
        "device": str(device_name), "library": str(library_digest),
    }
    return hashlib.sha256(json.dumps(items, sort_keys=True).encode()).hexdigest()


def tune_cache_get(path: str, key: str):
    """The cached (n_cells, domain_cells, result) under key in the JSON file at path, or None."""
    try:
        with open(path) as f:
            entry = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not entry:
        return None
    return list(entry["n_cells"]), list(entry["domain_cells"]), dict(entry["result"])


def tune_cache_put(path: str, key: str, n_cells, domain_cells, result: dict) -> None:
    """Store a tuning result under key in the JSON file at path (other keys kept; the file is
    replaced in one rename, so a reader never sees half of it)."""
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        table = {}
    table[key] = {"n_cells": [int(x) for x in n_cells], "domain_cells": [int(x) for x in domain_cells],
                  "result": {k: v for k, v in result.items() if k != "cached"}}
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _library_digest() -> str:
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        for block in iter(lambda: f.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()


def ecmc_tune_batch(melts, sigma: float, l_max: float, opt: ecmc_options, n_chains: int, ell: float,
                    trial_sweeps: int = 2, device: str = "cuda", cache: str | None = None):
    """Run the library's autotuner on a scratch workspace (a torch tensor freed on return).
    Returns (n_cells, domain_cells, result): per-melt geometry and the chosen staging tier.
    With cache (a JSON file path) a result stored for the same key (see tune_key) is returned
    without timing anything, and a new one is stored; result["cached"] says which."""
    import torch
    key = None
    if cache:
        key = tune_key(melts, sigma, l_max, opt, n_chains, ell, trial_sweeps, torch.cuda.get_device_name(device),
                       _library_digest())
        hit = tune_cache_get(cache, key)
        if hit is not None:
            hit[2]["cached"] = True
            return hit
    descs, keep = _melt_descs(melts)
    n = ctypes.c_size_t()
    _check(lib().ecmc_tune_workspace_size(len(melts), descs, sigma, l_max, ctypes.byref(opt), ctypes.byref(n)),
           "ecmc_tune_workspace_size")
    scratch = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
    o = ecmc_options.from_buffer_copy(opt)
    o.workspace = (scratch.data_ptr() + 255) & ~255
    o.workspace_bytes = n.value
    nc = (ctypes.c_int32 * len(melts))()
    dc = (ctypes.c_int32 * len(melts))()
    res = ecmc_tune_result()
    _check(lib().ecmc_tune_batch(len(melts), descs, sigma, l_max, ctypes.byref(o), int(n_chains), float(ell),
                                 int(trial_sweeps), nc, dc, ctypes.byref(res)), "ecmc_tune_batch")
    torch.cuda.synchronize()
    del scratch
    result = res.as_dict()
    if cache:
        tune_cache_put(cache, key, list(nc), list(dc), result)
    result["cached"] = False
    return list(nc), list(dc), result


def ecmc_sweep(ctx, n_chains: int, ell: float, seed: int):
    _check(lib().ecmc_sweep(ctx, int(n_chains), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF), "ecmc_sweep", ctx)


def ecmc_sweep_colours(ctx, n_chains: int, ell: float, seed: int, colour_mask: int):
    _check(lib().ecmc_sweep_colours(ctx, int(n_chains), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                    int(colour_mask)), "ecmc_sweep_colours", ctx)


def ecmc_synchronize(ctx):
    _check(lib().ecmc_synchronize(ctx), "ecmc_synchronize", ctx)


def ecmc_destroy(ctx):
    lib().ecmc_destroy(ctx)


# ---------------------------------------------------------------- convenience object
@dataclass
class Options:
    tiling: int = TILING_CHECKER
    domain_cells: int = 2
    n_cells: int = 0
    cell_capacity: int = 0
    stage_capacity: int = 0
    event_cap: int = 0
    event_log_capacity: int = 0
    time_kernels: bool = False
    precision: int = PREC_FP64
    swap_moves: bool = False
    schedule: int = SCHED_SWEEP
    stage_tier: int = 0
    spring_k: float = 0.0  # > 0: harmonic springs of this constant, capped at l_max
    overlapping_start: bool = False  # accept overlaps in the start (the push-off's phantom chains)
    wait_limit_us: int = 0  # guard on a dependency wait of the one-launch sweep (0 = 30 s)


def _native_options(o: "Options") -> ecmc_options:
    opt = ecmc_default_options()
    opt.precision = o.precision
    opt.tiling = o.tiling
    opt.domain_cells = o.domain_cells
    opt.n_cells = o.n_cells
    opt.cell_capacity = o.cell_capacity
    opt.stage_capacity = o.stage_capacity
    opt.event_cap = o.event_cap
    opt.event_log_capacity = o.event_log_capacity
    opt.time_kernels = 1 if o.time_kernels else 0
    opt.swap_moves = 1 if o.swap_moves else 0
    opt.schedule = o.schedule
    opt.stage_tier = o.stage_tier
    opt.spring_k = float(o.spring_k)
    opt.overlapping_start = 1 if o.overlapping_start else 0
    opt.wait_limit_us = int(o.wait_limit_us)
    return opt


class Melt:
    """A melt (or a batch of independent melts) resident on the GPU: the context plus its
    torch-owned workspace."""

    def __init__(self, L: float, sigma: float, b_max: float, positions, bonds, options: Options | None = None,
                 device: str = "cuda", stream=None, side_stream=None):
        opt = _native_options(options or Options())
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        self._attach(opt, ecmc_workspace_size(L, sigma, b_max, pos.shape[0], opt), device, stream, options, side_stream)
        self.L, self.sigma, self.b_max = float(L), float(sigma), float(b_max)
        self.n_beads = pos.shape[0]
        self.ctx = ecmc_init(L, sigma, b_max, pos, bonds, opt)
        # linear chains (the library rejects anything else): one polymer per bead minus bonds
        self.n_poly = self.n_beads - int(np.asarray(bonds).reshape(-1, 2).shape[0])

    def _attach(self, opt, nbytes, device, stream, options, side_stream=None):
        import torch
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        opt.workspace = (base + 255) & ~255
        opt.workspace_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        opt.stream = self.stream.cuda_stream
        self.side_stream = side_stream
        opt.side_stream = side_stream.cuda_stream if side_stream is not None else None
        self.opt = opt
        self.log_capacity = int((options or Options()).event_log_capacity)

    @classmethod
    def from_batch(cls, melts, options: Options | None = None, n_cells=None, domain_cells=None, device: str = "cuda",
                   stream=None):
        """Independent melts (inputs.Melt-like: L, positions, bonds, sigma, b_max) in one context:
        they sweep together in one launch per sweep.  Per-bead and per-polymer results are the
        melts' own, concatenated in melt order (see melt_info)."""
        o = options or Options()
        opt = _native_options(o)
        sigma, b_max = float(melts[0].sigma), float(melts[0].b_max)
        if any(float(m.sigma) != sigma or float(m.b_max) != b_max for m in melts):
            raise ValueError("the melts of a batch share sigma and b_max")
        self = cls.__new__(cls)
        self._attach(opt, ecmc_workspace_size_batch(melts, sigma, b_max, opt, n_cells, domain_cells), device, stream, o)
        self.L, self.sigma, self.b_max = None, sigma, b_max
        self.n_beads = sum(int(np.asarray(m.positions).reshape(-1, 3).shape[0]) for m in melts)
        self.ctx = ecmc_init_batch(melts, sigma, b_max, opt, n_cells, domain_cells)
        self.n_poly = sum(self.melt_info(i)["n_polymers"] for i in range(len(melts)))
        return self

    @property
    def n_melts(self) -> int:
        return lib().ecmc_n_melts(self.ctx)

    def melt_info(self, m: int) -> dict:
        info = ecmc_melt_info()
        _check(lib().ecmc_get_melt_info(self.ctx, int(m), ctypes.byref(info)), "ecmc_get_melt_info", self.ctx)
        return info.as_dict()

    @classmethod
    def from_melt(cls, melt, options: Options | None = None, **kw):
        return cls(melt.L, melt.sigma, melt.b_max, melt.positions, melt.bonds, options, **kw)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            ecmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- path
    def sweep(self, n_chains: int, ell: float, seed: int, colour_mask: int = 0xFF):
        if colour_mask == 0xFF:
            ecmc_sweep(self.ctx, n_chains, ell, seed)
        else:
            ecmc_sweep_colours(self.ctx, n_chains, ell, seed, colour_mask)

    def synchronize(self):
        ecmc_synchronize(self.ctx)

    # -- state
    @property
    def n_cells(self) -> int:
        return lib().ecmc_n_cells(self.ctx)

    @property
    def h(self) -> float:
        return lib().ecmc_cell_size(self.ctx)

    @property
    def stage_capacity(self) -> int:
        return lib().ecmc_stage_capacity(self.ctx)

    @property
    def sweep_counter(self) -> int:
        return lib().ecmc_sweep_counter(self.ctx)

    def positions(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3))
        _check(lib().ecmc_get_positions(self.ctx, out.ctypes.data), "ecmc_get_positions", self.ctx)
        return out

    def cells(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3), dtype=np.int32)
        _check(lib().ecmc_get_cells(self.ctx, out.ctypes.data), "ecmc_get_cells", self.ctx)
        return out

    def images(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3), dtype=np.int32)
        _check(lib().ecmc_get_images(self.ctx, out.ctypes.data), "ecmc_get_images", self.ctx)
        return out

    def counters(self) -> dict:
        c = ecmc_counters()
        _check(lib().ecmc_get_counters(self.ctx, ctypes.byref(c)), "ecmc_get_counters", self.ctx)
        return c.as_dict()

    def reset_counters(self):
        _check(lib().ecmc_reset_counters(self.ctx), "ecmc_reset_counters", self.ctx)

    def clear_error(self):
        """Clear the device error word after handling the error it caused."""
        _check(lib().ecmc_clear_error(self.ctx), "ecmc_clear_error", self.ctx)

    def event_log(self) -> np.ndarray:
        n = ctypes.c_int64()
        _check(lib().ecmc_get_event_log(self.ctx, None, 0, ctypes.byref(n)), "ecmc_get_event_log", self.ctx)
        if n.value > self.log_capacity:
            raise EcmcError(E_ARG, "event_log", f"log overflow: {n.value} records > capacity {self.log_capacity}")
        out = np.zeros(n.value, dtype=EVENT_DTYPE)
        _check(lib().ecmc_get_event_log(self.ctx, out.ctypes.data, n.value, ctypes.byref(n)), "ecmc_get_event_log",
               self.ctx)
        return out

    def clear_event_log(self):
        _check(lib().ecmc_clear_event_log(self.ctx), "ecmc_clear_event_log", self.ctx)

    def set_state(self, pos, cells, img, sweep_counter: int):
        p = np.ascontiguousarray(pos, dtype=np.float64)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        i = np.ascontiguousarray(img, dtype=np.int32)
        _check(lib().ecmc_set_state(self.ctx, p.ctypes.data, c.ctypes.data, i.ctypes.data, int(sweep_counter)),
               "ecmc_set_state", self.ctx)

    def save_checkpoint(self, path: str) -> None:
        """Write the state a run resumes from (positions, cells, image counters, sweep counter) to an
        .npz file.  The random numbers are counter-based on (seed, sweep counter, domain, EC), so a
        context restored from it continues bit for bit as the original would."""
        np.savez(path, positions=self.positions(), cells=self.cells(), images=self.images(),
                 sweep_counter=np.array([self.sweep_counter], dtype=np.uint32), n_beads=np.array([self.n_beads]))

    def load_checkpoint(self, path: str) -> None:
        """Restore a state written by save_checkpoint into this context (same melt geometry)."""
        with np.load(path, allow_pickle=False) as f:
            if int(f["n_beads"][0]) != self.n_beads:
                raise ValueError(f"checkpoint holds {int(f['n_beads'][0])} beads, this melt {self.n_beads}")
            self.set_state(f["positions"], f["cells"], f["images"], int(f["sweep_counter"][0]))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().ecmc_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)), "ecmc_kernel_time", self.ctx)
        return ms.value, n.value

    def observables(self, nbins: int = 20) -> dict:
        n_poly = ctypes.c_int64()
        M = self.n_poly
        r2 = np.zeros(M)
        rg2 = np.zeros(M)
        hist = np.zeros(nbins, dtype=np.int64)
        mid = np.zeros((M, 3))
        _check(lib().ecmc_observables(self.ctx, nbins, r2.ctypes.data, rg2.ctypes.data, hist.ctypes.data,
                                      mid.ctypes.data, ctypes.byref(n_poly)), "ecmc_observables", self.ctx)
        assert n_poly.value == M
        return {"r2": r2, "rg2": rg2, "hist": hist, "mid": mid, "n_poly": M}

    def observables_accumulate(self, nbins: int = 20):
        """Add this state's observables (sums over polymers of R^2 and R_g^2, the bond-length
        histogram) to running device sums; asynchronous, no host round trip."""
        _check(lib().ecmc_observables_accumulate(self.ctx, int(nbins)), "ecmc_observables_accumulate", self.ctx)
        self._acc_nbins = int(nbins)

    def observables_mean(self) -> dict:
        """<R^2>, <R_g^2> per polymer and sample, the summed bond-length histogram and the sample
        count of the running sums (synchronises)."""
        r2, rg2, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        hist = np.zeros(max(getattr(self, "_acc_nbins", 0), 1), dtype=np.int64)
        _check(lib().ecmc_observables_mean(self.ctx, ctypes.byref(r2), ctypes.byref(rg2), hist.ctypes.data,
                                           ctypes.byref(n)), "ecmc_observables_mean", self.ctx)
        return {"r2": r2.value, "rg2": rg2.value, "hist": hist[:getattr(self, "_acc_nbins", 0)], "samples": n.value}

    def observables_reset(self):
        _check(lib().ecmc_observables_reset(self.ctx), "ecmc_observables_reset", self.ctx)
        self._acc_nbins = 0

    def pushoff_sweep(self, n_chains: int, ell: float, seed: int, diameter: float):
        """One push-off sweep (Sec. II.B) at working diameter d: overlapping pairs are no events,
        ECs start at overlapping beads."""
        _check(lib().ecmc_pushoff_sweep(self.ctx, int(n_chains), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                        float(diameter)), "ecmc_pushoff_sweep", self.ctx)

    def count_overlaps(self, diameter: float) -> int:
        """Pairs closer than d (squared distance below d^2 (1 - 1e-9))."""
        n = ctypes.c_int64()
        _check(lib().ecmc_count_overlaps(self.ctx, float(diameter), ctypes.byref(n)), "ecmc_count_overlaps", self.ctx)
        return n.value

    def pushoff(self, d_start: float, stages: int, ell: float = 2.0, seed: int = 1, max_sweeps: int = 10000):
        """The slow push-off: working diameters from d_start up to sigma in `stages` steps, push-off
        sweeps at each until no overlap is left.  Returns (sweeps run, overlaps left)."""
        done, left = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ecmc_pushoff(self.ctx, float(d_start), int(stages), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                  int(max_sweeps), ctypes.byref(done), ctypes.byref(left)), "ecmc_pushoff", self.ctx)
        return done.value, left.value

    def snapshot(self, out=None):
        """Middle bead and centre of mass of every polymer, image-unwrapped, as a device tensor
        [M, 6] (queued on the melt's stream, no synchronisation): one time point for g1 and g2."""
        import torch
        if out is None:
            out = torch.empty((self.n_poly, 6), dtype=torch.float64, device=self.workspace.device)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() != 6 * self.n_poly:
            raise ValueError("snapshot buffer must be a contiguous float64 tensor of n_poly x 6")
        _check(lib().ecmc_snapshot(self.ctx, out.data_ptr()), "ecmc_snapshot", self.ctx)
        return out

    def msd(self, snaps) -> tuple:
        """g1 and g2 (Sec. IV.A) for lags 0..T-1 from a device tensor of snapshots [T, M, 6],
        averaged over polymers and time origins, computed on the GPU; numpy arrays."""
        import torch
        if snaps.dtype != torch.float64 or not snaps.is_contiguous() or snaps.dim() != 3 \
                or snaps.shape[1] != self.n_poly or snaps.shape[2] != 6:
            raise ValueError("snapshots must be a contiguous float64 tensor [T, n_poly, 6]")
        T = snaps.shape[0]
        out = torch.empty(2 * T, dtype=torch.float64, device=snaps.device)
        _check(lib().ecmc_msd(self.ctx, snaps.data_ptr(), T, out.data_ptr()), "ecmc_msd", self.ctx)
        self.synchronize()
        o = out.cpu().numpy()
        return o[:T].copy(), o[T:].copy()

    def end_to_end_histogram(self, nbins: int, r_max: float) -> np.ndarray:
        """W(R): polymers per bin of |R| (width r_max / nbins; |R| >= r_max in the last bin)."""
        h = np.zeros(int(nbins), dtype=np.int64)
        _check(lib().ecmc_end_to_end_histogram(self.ctx, int(nbins), float(r_max), h.ctypes.data),
               "ecmc_end_to_end_histogram", self.ctx)
        return h

    def check_state(self, tol: float = 1e-10) -> dict:
        """Invariants of the current state counted on the GPU: overlapping pairs (closer than
        sigma (1 - tol)), stretched bonds (longer than l_max (1 + tol)) and misplaced beads."""
        ov, st, mp = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ecmc_check_state(self.ctx, float(tol), ctypes.byref(ov), ctypes.byref(st), ctypes.byref(mp)),
               "ecmc_check_state", self.ctx)
        return {"overlaps": ov.value, "stretched": st.value, "misplaced": mp.value}

    def internal_distances(self, n_max: int) -> tuple[np.ndarray, np.ndarray]:
        """R^2(n) of Sec. II.B for n = 0..n_max: the mean squared chain vector between beads of
        one polymer n bonds apart, over all such pairs, and the number of pairs behind each."""
        r2 = np.zeros(int(n_max) + 1)
        pairs = np.zeros(int(n_max) + 1, dtype=np.int64)
        _check(lib().ecmc_internal_distances(self.ctx, int(n_max), r2.ctypes.data, pairs.ctypes.data),
               "ecmc_internal_distances", self.ctx)
        return r2, pairs

    def internal_distances_noalloc(self, n_max: int) -> tuple[np.ndarray, np.ndarray]:
        """internal_distances with the partial sums in the library's static per-device array
        (no workspace, no allocation); calls that overlap on one device race."""
        r2 = np.zeros(int(n_max) + 1)
        pairs = np.zeros(int(n_max) + 1, dtype=np.int64)
        _check(lib().ecmc_internal_distances_noalloc(self.ctx, int(n_max), r2.ctypes.data, pairs.ctypes.data),
               "ecmc_internal_distances_noalloc", self.ctx)
        return r2, pairs

    def pair_histogram(self, nbins: int, r_max: float) -> np.ndarray:
        """Pair counts behind g(r): pairs i < j of a melt with r < r_max (<= the cell edge)."""
        h = np.zeros(int(nbins), dtype=np.int64)
        _check(lib().ecmc_pair_histogram(self.ctx, int(nbins), float(r_max), h.ctypes.data), "ecmc_pair_histogram",
               self.ctx)
        return h

    def pair_correlation(self, nbins: int, r_max: float) -> np.ndarray:
        """g(r) of the context's melts (pooled over a batch) for r < r_max (<= the cell edge):
        the GPU pair counts normalised by the library."""
        h = self.pair_histogram(nbins, r_max)
        infos = [self.melt_info(m) for m in range(self.n_melts)]
        return pair_correlation(h, r_max, [i["n_beads"] for i in infos], [i["box"] ** 3 for i in infos])

    def shape(self) -> dict:
        """Per polymer: gyration tensor [M, 6] (xx, yy, zz, xy, xz, yz), its eigenvalues [M, 3]
        (descending) and the image-unwrapped centre of mass [M, 3], computed on the GPU."""
        n_poly = ctypes.c_int64()
        M = self.n_poly
        gyr, eig, com = np.zeros((M, 6)), np.zeros((M, 3)), np.zeros((M, 3))
        _check(lib().ecmc_shape(self.ctx, gyr.ctypes.data, eig.ctypes.data, com.ctypes.data, ctypes.byref(n_poly)),
               "ecmc_shape", self.ctx)
        assert n_poly.value == M
        return {"gyr": gyr, "eig": eig, "com": com, "n_poly": M}


def shape_descriptors(eig) -> dict:
    """Ensemble shape descriptors (appendix, Table II) from per-polymer gyration eigenvalues
    (Melt.shape()["eig"]), computed by the library: <kappa^2>, the three ratios
    <I1 + I2 - I3>/<tr I>, <I1 - I2 + I3>/<tr I>, <-I1 + I2 + I3>/<tr I> and
    <4 b^2 + 3 c^2>/<tr I>^2 (I_i = tr G - l_i in descending order)."""
    lam = np.ascontiguousarray(eig, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(5)
    _check(lib().ecmc_shape_descriptors(lam.ctypes.data, lam.shape[0], out.ctypes.data), "ecmc_shape_descriptors")
    return {"kappa2": float(out[0]), "r_123": float(out[1]), "r_132": float(out[2]), "r_231": float(out[3]),
            "solc": float(out[4])}


def pair_correlation(hist, r_max: float, n_beads, volume) -> np.ndarray:
    """g(r) from pair counts (ecmc_pair_histogram), computed by the library: each bin divided by
    the ideal-gas count of its shell summed over the melts (n_beads and volume: one value per
    melt, or scalars for one melt)."""
    h = np.ascontiguousarray(hist, dtype=np.int64)
    nb = np.ascontiguousarray(np.atleast_1d(n_beads), dtype=np.int64)
    vol = np.ascontiguousarray(np.atleast_1d(volume), dtype=np.float64)
    if nb.shape != vol.shape:
        raise ValueError("one bead count and one volume per melt")
    g = np.zeros(h.shape[0])
    _check(lib().ecmc_pair_correlation(h.ctypes.data, h.shape[0], float(r_max), nb.shape[0], nb.ctypes.data,
                                       vol.ctypes.data, g.ctypes.data), "ecmc_pair_correlation")
    return g
