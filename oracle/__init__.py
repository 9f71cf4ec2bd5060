"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the serial FP64 CPU oracle.

The oracle is the plain reference implementation of the event-chain move for
tethered hard-sphere melts (Kampmann, Boltz, Kierfeld, arXiv:1502.06447,
Sec. II and II.A).  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the GPU library never
does.  It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecmc_oracle.c")
_LIB = os.environ.get("ECMC_ORACLE_LIB") or os.path.join(_HERE, "libecmc_oracle.so")

OK, E_ARG, E_OVERLAP, E_TETHER, E_BOX, E_CELL_OVERFLOW, E_STUCK, E_CHECK = 0, -1, -2, -3, -4, -5, -6, -9
EV_HS_LIFT, EV_TETHER_LIFT, EV_HS_REFLECT, EV_TETHER_REFLECT, EV_WALL, EV_END, EV_PERIOD, EV_CYCLE, EV_SWAP = range(9)
C_HS_LIFT, C_TETHER_LIFT, C_HS_REFLECT, C_TETHER_REFLECT, C_WALL, C_CROSS, C_EC, C_STEPS, C_PERIOD, C_CYCLE, C_SWAP = \
    range(11)
NCNT = 11

EVENT_DTYPE = np.dtype([
    ("sweep", "<u4"), ("domain", "<u4"), ("ec", "<u4"), ("step", "<u4"),
    ("pivot", "<i4"), ("target", "<i4"), ("kind", "<u4"), ("colour", "<u4"),
])


def build(force: bool = True) -> str:
    """Compile the oracle (IEEE binary64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        i64, i32, u32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_create.argtypes = [P(vp), dbl, dbl, dbl, ctypes.c_int, i64, vp, i64, vp]
        L.orc_create.restype = ctypes.c_int
        L.orc_create_overlapping.argtypes = [P(vp), dbl, dbl, dbl, ctypes.c_int, i64, vp, i64, vp]
        L.orc_create_overlapping.restype = ctypes.c_int
        L.orc_set_pushoff.argtypes = [vp, dbl]
        L.orc_set_pushoff.restype = ctypes.c_int
        L.orc_count_overlaps.argtypes = [vp, dbl]
        L.orc_count_overlaps.restype = i64
        L.orc_destroy.argtypes = [vp]
        L.orc_set_options.argtypes = [vp, i64, ctypes.c_int]
        L.orc_set_swap.argtypes = [vp, ctypes.c_int]
        L.orc_set_periodic_skip.argtypes = [vp, ctypes.c_int]
        L.orc_set_swap.restype = ctypes.c_int
        L.orc_set_spring.argtypes = [vp, dbl]
        L.orc_set_spring.restype = ctypes.c_int
        L.orc_bond_x.argtypes = [vp, dbl, dbl, dbl]
        L.orc_bond_x.restype = dbl
        L.orc_ln.argtypes = [dbl]
        L.orc_ln.restype = dbl
        L.orc_set_stream.argtypes = [vp, u32]
        L.orc_set_stream.restype = ctypes.c_int
        L.orc_set_log.argtypes = [vp, vp, i64]
        L.orc_log_count.argtypes = [vp]
        L.orc_log_count.restype = i64
        L.orc_sweep.argtypes = [vp, i64, dbl, u64, ctypes.c_int, ctypes.c_int, u32]
        L.orc_sweep.restype = ctypes.c_int
        L.orc_sweep_subset.argtypes = [vp, i64, dbl, u64, ctypes.c_int, u32, vp, i64]
        L.orc_sweep_subset.restype = ctypes.c_int
        L.orc_next_event.argtypes = [vp, i32, ctypes.c_int, ctypes.c_int, P(dbl), P(i32), P(ctypes.c_int), P(dbl)]
        L.orc_run_ec.argtypes = [vp, i32, ctypes.c_int, dbl]
        L.orc_observables.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, P(i64)]
        L.orc_pair_histogram.argtypes = [vp, ctypes.c_int, dbl, vp]
        L.orc_pair_histogram.restype = ctypes.c_int
        L.orc_end_to_end_histogram.argtypes = [vp, ctypes.c_int, dbl, vp]
        L.orc_end_to_end_histogram.restype = ctypes.c_int
        L.orc_internal_distances.argtypes = [vp, i64, vp, vp]
        L.orc_internal_distances.restype = ctypes.c_int
        L.orc_gyration.argtypes = [vp, i64, vp]
        L.orc_gyration.restype = None
        L.orc_shape.argtypes = [vp, vp, vp]
        L.orc_n_beads.argtypes = [vp]
        L.orc_n_beads.restype = i64
        L.orc_n_cells.argtypes = [vp]
        L.orc_cell_size.argtypes = [vp]
        L.orc_cell_size.restype = dbl
        L.orc_sweep_counter.argtypes = [vp]
        L.orc_sweep_counter.restype = u32
        for f in ("orc_get_positions", "orc_get_cells", "orc_get_images"):
            getattr(L, f).argtypes = [vp, vp]
            getattr(L, f).restype = None
        L.orc_counters.argtypes = [vp, vp, P(dbl)]
        L.orc_counters.restype = None
        L.orc_set_state.argtypes = [vp, vp, vp, vp, u32]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox4x32_10.restype = None
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def ln(u: float) -> float:
    """The oracle's natural logarithm (the one the spring draws use)."""
    return lib().orc_ln(float(u))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


class Oracle:
    """One melt held by the CPU oracle."""

    def __init__(self, L: float, sigma: float, b_max: float, positions, bonds, n_cells: int = 0,
                 event_cap: int = 0, check: int = 0, overlapping: bool = False):
        self._pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        self._bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
        h = ctypes.c_void_p()
        create = lib().orc_create_overlapping if overlapping else lib().orc_create
        st = create(ctypes.byref(h), float(L), float(sigma), float(b_max), int(n_cells),
                    self._pos.shape[0], self._pos.ctypes.data, self._bonds.shape[0],
                    self._bonds.ctypes.data if self._bonds.size else None)
        if st != OK:
            raise OracleError(st, "orc_create")
        self._h = h
        self.L, self.sigma, self.b_max = float(L), float(sigma), float(b_max)
        self.n_beads = self._pos.shape[0]
        self._log = None
        lib().orc_set_options(self._h, int(event_cap), int(check))

    @classmethod
    def from_melt(cls, melt, **kw):
        return cls(melt.L, melt.sigma, melt.b_max, melt.positions, melt.bonds, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    @property
    def n_cells(self) -> int:
        return lib().orc_n_cells(self._h)

    @property
    def h(self) -> float:
        return lib().orc_cell_size(self._h)

    @property
    def sweep_counter(self) -> int:
        return lib().orc_sweep_counter(self._h)

    def set_options(self, event_cap: int = 0, check: int = 0):
        lib().orc_set_options(self._h, int(event_cap), int(check))

    def shape(self) -> dict:
        """Per polymer: gyration tensor [n, 6] (xx, yy, zz, xy, xz, yz), its eigenvalues [n, 3]
        in descending order (numpy's symmetric eigensolver), unwrapped centre of mass [n, 3]."""
        n = self.observables(nbins=1)["n_poly"]
        gyr = np.zeros((n, 6))
        com = np.zeros((n, 3))
        st = lib().orc_shape(self._h, gyr.ctypes.data, com.ctypes.data)
        if st != OK:
            raise OracleError(st, "orc_shape")
        return {"gyr": gyr, "eig": tensor_eigenvalues(gyr), "com": com, "n_poly": n}

    def set_swap(self, on: bool = True):
        """Swap moves at hard-sphere contacts (Sec. II.C) for the following ECs."""
        if lib().orc_set_swap(self._h, 1 if on else 0) != OK:
            raise ValueError("swap moves cannot be combined with springs")

    def set_periodic_skip(self, on: bool = True):
        """Whole periods of an EC dropped after its second reflection (the default), or the plain
        loop of Sec. II steps 1-4 that runs every bounce until x_max is used up."""
        lib().orc_set_periodic_skip(self._h, 1 if on else 0)

    def set_pushoff(self, d: float):
        """Push-off (Sec. II.B) at working diameter d for the following sweeps (d = 0: off)."""
        if lib().orc_set_pushoff(self._h, float(d)) != OK:
            raise ValueError(f"push-off diameter {d!r} refused")

    def count_overlaps(self, d: float) -> int:
        """Pairs closer than d (squared distance below d^2 (1 - 1e-9))."""
        return int(lib().orc_count_overlaps(self._h, float(d)))

    def set_spring(self, k: float):
        """Bonds as harmonic springs of constant k (Eq. (2), k_B T / sigma^2), capped at b_max;
        k = 0 gives tethers."""
        if lib().orc_set_spring(self._h, float(k)) != OK:
            raise ValueError(f"spring constant {k!r} refused")

    def bond_x(self, dpar: float, dperp2: float, g: float) -> float:
        """Bond candidate for a partner at (d_par, d_perp^2); g = 2 dE / k, or < 0 for the tether."""
        return lib().orc_bond_x(self._h, float(dpar), float(dperp2), float(g))

    def set_stream(self, m: int):
        """Random stream m: the draws of melt m of a batch (Philox counter word 3 = 2 m, 2 m + 1)."""
        if lib().orc_set_stream(self._h, int(m)) != 0:
            raise ValueError(f"stream index {m} out of range")

    def enable_log(self, capacity: int):
        self._log = np.zeros(int(capacity), dtype=EVENT_DTYPE)
        lib().orc_set_log(self._h, self._log.ctypes.data, self._log.shape[0])

    def event_log(self) -> np.ndarray:
        if self._log is None:
            return np.zeros(0, dtype=EVENT_DTYPE)
        n = lib().orc_log_count(self._h)
        if n > self._log.shape[0]:
            raise OracleError(E_ARG, f"event log overflow ({n} > {self._log.shape[0]})")
        return self._log[:n].copy()

    def sweep(self, n_ec: int, ell: float, seed: int, tiling: int = 0, D: int = 1,
              colour_mask: int = 0xFF):
        st = lib().orc_sweep(self._h, int(n_ec), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF,
                             int(tiling), int(D), int(colour_mask))
        if st != OK:
            raise OracleError(st, "orc_sweep")

    def sweep_subset(self, n_ec: int, ell: float, seed: int, D: int, colour_mask: int, domains):
        d = np.ascontiguousarray(np.sort(np.asarray(domains, dtype=np.uint32)))
        st = lib().orc_sweep_subset(self._h, int(n_ec), float(ell), int(seed) & 0xFFFFFFFFFFFFFFFF, int(D),
                                    int(colour_mask), d.ctypes.data, d.shape[0])
        if st != OK:
            raise OracleError(st, "orc_sweep_subset")

    def run_ec(self, pivot: int, direction: int, ell: float):
        st = lib().orc_run_ec(self._h, int(pivot), int(direction), float(ell))
        if st != OK:
            raise OracleError(st, "orc_run_ec")

    def next_event(self, pivot: int, axis: int, sgn: int):
        x = ctypes.c_double()
        j = ctypes.c_int32()
        k = ctypes.c_int()
        xc = ctypes.c_double()
        st = lib().orc_next_event(self._h, int(pivot), int(axis), int(sgn), ctypes.byref(x),
                                  ctypes.byref(j), ctypes.byref(k), ctypes.byref(xc))
        if st != OK:
            raise OracleError(st, "orc_next_event")
        return x.value, j.value, k.value, xc.value

    def positions(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3))
        lib().orc_get_positions(self._h, out.ctypes.data)
        return out

    def cells(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3), dtype=np.int32)
        lib().orc_get_cells(self._h, out.ctypes.data)
        return out

    def images(self) -> np.ndarray:
        out = np.zeros((self.n_beads, 3), dtype=np.int32)
        lib().orc_get_images(self._h, out.ctypes.data)
        return out

    def counters(self):
        c = np.zeros(NCNT, dtype=np.uint64)
        d = ctypes.c_double()
        lib().orc_counters(self._h, c.ctypes.data, ctypes.byref(d))
        return c, d.value

    def set_state(self, pos, cells, img, sweep_ctr: int):
        p = np.ascontiguousarray(pos, dtype=np.float64)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        i = np.ascontiguousarray(img, dtype=np.int32)
        st = lib().orc_set_state(self._h, p.ctypes.data, c.ctypes.data, i.ctypes.data, int(sweep_ctr))
        if st != OK:
            raise OracleError(st, "orc_set_state")

    def pair_histogram(self, nbins: int, r_max: float) -> np.ndarray:
        """Pair counts (i < j, minimum image, r < r_max) in nbins bins of width r_max / nbins."""
        h = np.zeros(int(nbins), dtype=np.int64)
        st = lib().orc_pair_histogram(self._h, int(nbins), float(r_max), h.ctypes.data)
        if st != OK:
            raise OracleError(st, "orc_pair_histogram")
        return h

    def end_to_end_histogram(self, nbins: int, r_max: float) -> np.ndarray:
        """W(R): polymers per bin of |R| (width r_max / nbins; |R| >= r_max in the last bin)."""
        h = np.zeros(int(nbins), dtype=np.int64)
        st = lib().orc_end_to_end_histogram(self._h, int(nbins), float(r_max), h.ctypes.data)
        if st != OK:
            raise OracleError(st, "orc_end_to_end_histogram")
        return h

    def internal_distances(self, n_max: int) -> tuple[np.ndarray, np.ndarray]:
        """R^2(n) of Sec. II.B: the mean squared chain vector between two beads of one polymer n
        bonds apart (summed bond by bond), over all such pairs, for n = 0..n_max, and the number of
        pairs behind each mean (a mean with no pairs is 0)."""
        n_max = int(n_max)
        s = np.zeros(n_max + 1)
        c = np.zeros(n_max + 1, dtype=np.int64)
        st = lib().orc_internal_distances(self._h, n_max, s.ctypes.data, c.ctypes.data)
        if st != OK:
            raise OracleError(st, "orc_internal_distances")
        return np.divide(s, c, out=np.zeros_like(s), where=c > 0), c

    def snapshot(self) -> np.ndarray:
        """Per polymer: the middle bead floor(N/2) and the centre of mass, both image-unwrapped,
        as [n_poly, 6] (the quantities whose displacements g1 and g2 of Sec. IV.A average)."""
        return np.concatenate([self.observables(nbins=1)["mid"], self.shape()["com"]], axis=1)

    def observables(self, nbins: int = 20):
        n_poly = ctypes.c_int64()
        lib().orc_observables(self._h, 0, None, None, None, None, ctypes.byref(n_poly))
        M = n_poly.value
        r2 = np.zeros(M)
        rg2 = np.zeros(M)
        hist = np.zeros(max(nbins, 1), dtype=np.int64)
        mid = np.zeros((M, 3))
        lib().orc_observables(self._h, int(nbins), r2.ctypes.data, rg2.ctypes.data, hist.ctypes.data,
                              mid.ctypes.data, ctypes.byref(n_poly))
        return {"r2": r2, "rg2": rg2, "hist": hist[:nbins], "mid": mid, "n_poly": M}


def gyration(u) -> np.ndarray:
    """Gyration tensor (xx, yy, zz, xy, xz, yz) of one unwrapped chain u [n, 3]."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
    g = np.zeros(6)
    lib().orc_gyration(u.ctypes.data, u.shape[0], g.ctypes.data)
    return g


def tensor_eigenvalues(g) -> np.ndarray:
    """Eigenvalues, descending, of symmetric 3 x 3 tensors given as [..., 6] (xx, yy, zz, xy, xz, yz)."""
    g = np.asarray(g, dtype=np.float64)
    m = np.empty(g.shape[:-1] + (3, 3))
    m[..., 0, 0], m[..., 1, 1], m[..., 2, 2] = g[..., 0], g[..., 1], g[..., 2]
    m[..., 0, 1] = m[..., 1, 0] = g[..., 3]
    m[..., 0, 2] = m[..., 2, 0] = g[..., 4]
    m[..., 1, 2] = m[..., 2, 1] = g[..., 5]
    return np.linalg.eigvalsh(m)[..., ::-1]


def shape_descriptors(eig) -> dict:
    """Appendix (moment of inertia tensor) from gyration eigenvalues l1 >= l2 >= l3 per polymer,
    with the inertia eigenvalues I_i = tr G - l_i taken in descending order (I1 >= I2 >= I3:
    the order that makes b, c >= 0 and gives the printed infinite-chain limits): kappa^2 =
    4 (1 - 3 (I1 I2 + I2 I3 + I3 I1) / (tr I)^2), the ratios <I1 + I2 - I3> / <tr I> etc.,
    and <4 b^2 + 3 c^2> / <tr I>^2 with b = (I1 + I2)/2 - I3, c = I1 - I2."""
    eig = np.asarray(eig, dtype=np.float64)
    S = eig.sum(axis=-1, keepdims=True)
    I = np.sort(S - eig, axis=-1)[..., ::-1]
    tr = I.sum(axis=-1)
    k2 = 4.0 * (1.0 - 3.0 * (I[..., 0] * I[..., 1] + I[..., 1] * I[..., 2] + I[..., 2] * I[..., 0]) / tr ** 2)
    b = 0.5 * (I[..., 0] + I[..., 1]) - I[..., 2]
    c = I[..., 0] - I[..., 1]
    return {"kappa2": float(k2.mean()),
            "r_123": float((I[..., 0] + I[..., 1] - I[..., 2]).mean() / tr.mean()),
            "r_132": float((I[..., 0] - I[..., 1] + I[..., 2]).mean() / tr.mean()),
            "r_231": float((-I[..., 0] + I[..., 1] + I[..., 2]).mean() / tr.mean()),
            "solc": float((4 * b ** 2 + 3 * c ** 2).mean() / tr.mean() ** 2)}


def msd_series(snaps) -> tuple[np.ndarray, np.ndarray]:
    """Mean-square displacements of Sec. IV.A from a time series of snapshots [T, n_poly, 6]
    (middle bead r_{N/2}, centre of mass R, both unwrapped), averaged over polymers and over
    every time origin t: for each lag d = 0..T-1,
      g1(d) = < |r_{N/2}(t + d) - r_{N/2}(t)|^2 >,
      g2(d) = < |(r_{N/2} - R)(t + d) - (r_{N/2} - R)(t)|^2 >."""
    s = np.asarray(snaps, dtype=np.float64)
    T = s.shape[0]
    mid = s[:, :, 0:3]
    rel = s[:, :, 0:3] - s[:, :, 3:6]
    g1 = np.zeros(T)
    g2 = np.zeros(T)
    for d in range(1, T):
        g1[d] = np.mean(np.sum((mid[d:] - mid[:-d]) ** 2, axis=2))
        g2[d] = np.mean(np.sum((rel[d:] - rel[:-d]) ** 2, axis=2))
    return g1, g2
