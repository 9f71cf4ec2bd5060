"""Seeded synthetic starting configurations for tethered hard-sphere melts.

This module only builds inputs: bead positions, bond lists and box edges. It
holds none of the event-chain arithmetic, and both the GPU library and the
CPU oracle take their starting states from it.

The model is the one of Kampmann, Boltz and Kierfeld (arXiv:1502.06447,
Sec. II, Eq. (1) and the tether variant that follows Eq. (2)): M linear
chains of N hard spheres of diameter sigma, consecutive beads joined by
tethers of maximal length b_max, in a periodic cube.  The packing fraction is
eta = M N (pi/6) sigma^3 / L^3 (Sec. II, the definition of Systems I-III).

Recipes (all draws from ``numpy.random.default_rng(seed)``):

* ``saw_chains``   - chains grown as self-avoiding random walks with a fixed
  bond length (default 1.2 sigma); the small parity melt.
* ``lattice_chains`` - dense melts: the smallest simple-cubic lattice with at
  least M N sites and spacing a = L / n_l >= sigma, walked by a boustrophedon
  Hamiltonian path; chains are consecutive segments of that path, with the
  n_l^3 - M N vacancies spread evenly as gaps between chains.  A random lattice
  shift and axis permutation come from the seed, and every bead is jittered
  by up to 0.45 (a - sigma) / sqrt(3) per coordinate so that no bond is
  exactly parallel to an axis (exactly aligned, fully stretched bonds stall an
  axis-parallel event chain).
* ``hs_fluid``     - unbonded spheres on a lattice (pressure checks).
* ``isolated_chain`` / ``dimer`` - single short chains in a large box.
* ``batch_melts``  - many independent melts of mixed N, M and eta.
* ``phantom_chains`` - the start of the push-off (Sec. II.B): phantom non-reversal
  random walks with bond length sigma, each bond direction uniform on the cap
  within theta_max of the previous one, first beads uniform in the box; beads
  overlap freely until the push-off removes the overlaps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Melt",
    "box_for",
    "saw_chains",
    "lattice_chains",
    "hs_fluid",
    "isolated_chain",
    "dimer",
    "batch_melts",
    "phantom_chains",
    "theta_max_for",
]


@dataclass
class Melt:
    """One periodic melt: positions [n,3] in [0, L), bonds [m,2] (int32)."""

    L: float
    positions: np.ndarray
    bonds: np.ndarray
    sigma: float = 1.0
    b_max: float = 1.4
    n_poly: int = 0
    n_per: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_beads(self) -> int:
        return int(self.positions.shape[0])

    @property
    def eta(self) -> float:
        return self.n_beads * math.pi / 6.0 * self.sigma ** 3 / self.L ** 3


def box_for(n_beads: int, eta: float, sigma: float = 1.0) -> float:
    """Cube edge L with n_beads spheres at packing fraction eta."""
    return (n_beads * math.pi / 6.0 * sigma ** 3 / eta) ** (1.0 / 3.0)


def _chain_bonds(n_poly: int, n_per: int) -> np.ndarray:
    if n_per < 2:
        return np.zeros((0, 2), dtype=np.int32)
    base = (np.arange(n_poly, dtype=np.int64) * n_per)[:, None]
    i = base + np.arange(n_per - 1, dtype=np.int64)[None, :]
    return np.stack([i.ravel(), i.ravel() + 1], axis=1).astype(np.int32)


def _wrap(p: np.ndarray, L: float) -> np.ndarray:
    q = np.mod(p, L)
    q[q >= L] = 0.0
    return q


def _min_dist2(p: np.ndarray, others: np.ndarray, L: float) -> float:
    if others.shape[0] == 0:
        return np.inf
    d = others - p[None, :]
    d -= L * np.round(d / L)
    return float(np.min(np.einsum("ij,ij->i", d, d)))


def saw_chains(n_poly: int, n_per: int, eta: float, seed: int, bond: float = 1.2,
               sigma: float = 1.0, b_max: float = 1.4, tries: int = 512,
               max_backtrack: int = 100, margin: float = 1e-6) -> Melt:
    """Self-avoiding random-walk chains grown one after another.  The first bead
    is uniform in the box; each later bead sits at distance ``bond`` from the
    previous one along a uniform random direction.  A position closer than
    sigma (1 + margin) to any bead already placed (minimum image) is redrawn up to
    ``tries`` times; when every draw fails the walk steps back one bead and
    redraws that one (depth-first backtracking), and a chain that needs more than
    ``max_backtrack`` steps back is started again from a new first bead."""
    rng = np.random.default_rng(seed)
    n = n_poly * n_per
    L = box_for(n, eta, sigma)
    lim2 = (sigma * (1.0 + margin)) ** 2
    pos = np.zeros((n, 3))
    placed = 0
    for c in range(n_poly):
        start = placed
        backs = 0
        while placed < start + n_per:
            i = placed - start
            n_try = tries if i > 0 else 16 * tries
            if i == 0:
                cand = rng.uniform(0.0, L, (n_try, 3))
            else:
                v = rng.normal(size=(n_try, 3))
                v /= np.linalg.norm(v, axis=1)[:, None]
                cand = _wrap(pos[placed - 1][None, :] + bond * v, L)
            if placed:
                d = cand[:, None, :] - pos[None, :placed, :]
                d -= L * np.round(d / L)
                good = np.flatnonzero(np.einsum("ijk,ijk->ij", d, d).min(axis=1) >= lim2)
            else:
                good = np.arange(n_try)
            if good.size:
                pos[placed] = cand[good[0]]
                placed += 1
                continue
            backs += 1
            if i == 0 or backs > max_backtrack:
                if i == 0:
                    raise RuntimeError("saw_chains: no room for a new chain; lower eta")
                placed = start
                backs = 0
            else:
                placed -= 1
    return Melt(L=L, positions=_wrap(pos, L), bonds=_chain_bonds(n_poly, n_per),
                sigma=sigma, b_max=b_max, n_poly=n_poly, n_per=n_per,
                meta={"recipe": "saw", "seed": seed, "bond": bond, "eta": eta})


def _snake_sites(nl: int) -> np.ndarray:
    """Boustrophedon Hamiltonian path through an nl^3 simple-cubic lattice;
    consecutive entries are nearest neighbours."""
    out = np.empty((nl ** 3, 3), dtype=np.int64)
    k = 0
    row = 0
    for z in range(nl):
        ys = range(nl) if z % 2 == 0 else range(nl - 1, -1, -1)
        for y in ys:
            xs = np.arange(nl) if row % 2 == 0 else np.arange(nl - 1, -1, -1)
            out[k:k + nl, 0] = xs
            out[k:k + nl, 1] = y
            out[k:k + nl, 2] = z
            k += nl
            row += 1
    return out


def lattice_chains(n_poly: int, n_per: int, eta: float, seed: int, sigma: float = 1.0,
                   b_max: float = 1.4, L: float | None = None) -> Melt:
    """Dense start: chains laid along a Hamiltonian walk of a simple-cubic lattice of
    spacing a = L / n_l (sigma <= a <= b_max), n_l the smallest edge with n_l^3 >= M N
    (or floor(L / sigma) if that spacing would be below sigma)."""
    rng = np.random.default_rng(seed)
    n = n_poly * n_per
    if L is None:
        L = box_for(n, eta, sigma)
    nl = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while nl ** 3 < n:
        nl += 1
    if L / nl < sigma:
        nl = int(math.floor(L / sigma))
    a = L / nl
    if nl ** 3 < n:
        raise ValueError(f"lattice {nl}^3 too small for {n} beads")
    if not (sigma <= a <= b_max):
        raise ValueError(f"lattice spacing {a} outside [sigma, b_max]")
    sites = _snake_sites(nl)
    free = nl ** 3 - n
    start = np.arange(n_poly, dtype=np.int64) * n_per + (np.arange(n_poly, dtype=np.int64) * free) // max(n_poly, 1)
    idx = (start[:, None] + np.arange(n_per, dtype=np.int64)[None, :]).ravel()
    # for even n_l the walk closes on itself through the periodic boundary, so it may start
    # anywhere; for odd n_l it starts at site 0
    shift_path = int(rng.integers(0, nl ** 3)) if nl % 2 == 0 else 0
    sites = sites[(idx + shift_path) % (nl ** 3)]
    perm = rng.permutation(3)
    sites = sites[:, perm]
    shift = rng.uniform(0.0, a, 3)
    jit = 0.45 * (a - sigma) / math.sqrt(3.0)
    pos = sites.astype(np.float64) * a + shift[None, :] + rng.uniform(-jit, jit, (n, 3))
    pos = _wrap(pos, L)
    bonds = _chain_bonds(n_poly, n_per)
    if len(bonds):
        d = pos[bonds[:, 1]] - pos[bonds[:, 0]]
        d -= L * np.round(d / L)
        if np.einsum("ij,ij->i", d, d).max() > b_max * b_max:
            raise ValueError("a chain crosses the end of the lattice walk; use another seed")
    return Melt(L=L, positions=pos, bonds=bonds, sigma=sigma,
                b_max=b_max, n_poly=n_poly, n_per=n_per,
                meta={"recipe": "lattice", "seed": seed, "eta": eta, "a": a, "jitter": jit})


def hs_fluid(n: int, eta: float, seed: int, sigma: float = 1.0) -> Melt:
    """Unbonded spheres on a random subset of a simple-cubic lattice."""
    rng = np.random.default_rng(seed)
    L = box_for(n, eta, sigma)
    nl = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while nl ** 3 < n:
        nl += 1
    a = L / nl
    if a < sigma:
        raise ValueError("too dense for a lattice start")
    idx = np.sort(rng.choice(nl ** 3, size=n, replace=False))
    sites = np.stack([idx % nl, (idx // nl) % nl, idx // (nl * nl)], axis=1)
    pos = _wrap(sites * a + rng.uniform(0.0, a, 3)[None, :], L)
    return Melt(L=L, positions=pos, bonds=np.zeros((0, 2), dtype=np.int32), sigma=sigma,
                b_max=max(1.4 * sigma, sigma), n_poly=n, n_per=1,
                meta={"recipe": "hs_lattice", "seed": seed, "eta": eta})


def isolated_chain(n_per: int, L: float, seed: int, bond: float = 1.2, sigma: float = 1.0,
                   b_max: float = 1.4) -> Melt:
    """One straight chain (bond ``bond`` along a random axis) in a box of edge L."""
    rng = np.random.default_rng(seed)
    ax = int(rng.integers(0, 3))
    pos = np.zeros((n_per, 3))
    pos[:, ax] = np.arange(n_per) * bond
    pos += rng.uniform(0.0, L, 3)[None, :]
    return Melt(L=L, positions=_wrap(pos, L), bonds=_chain_bonds(1, n_per), sigma=sigma,
                b_max=b_max, n_poly=1, n_per=n_per, meta={"recipe": "isolated", "seed": seed})


def dimer(L: float, seed: int, r0: float = 1.2, sigma: float = 1.0, b_max: float = 1.4) -> Melt:
    return isolated_chain(2, L, seed, bond=r0, sigma=sigma, b_max=b_max)


def batch_melts(n_melts: int, seed: int, n_choices=(16, 32, 64, 128, 256),
                beads_range=(2048, 65536), eta_range=(0.35, 0.45), sigma: float = 1.0,
                b_max: float = 1.4) -> list[Melt]:
    """Independent melts: N uniform from ``n_choices``, bead count uniform in
    ``beads_range`` with M = round(beads / N), eta uniform in ``eta_range``;
    each laid out by ``lattice_chains``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_melts):
        N = int(rng.choice(np.asarray(n_choices)))
        beads = int(rng.integers(beads_range[0], beads_range[1] + 1))
        M = max(1, int(round(beads / N)))
        eta = float(rng.uniform(*eta_range))
        out.append(lattice_chains(M, N, eta, seed=int(rng.integers(0, 2 ** 31)), sigma=sigma,
                                  b_max=b_max))
    return out


def theta_max_for(c: float) -> float:
    """Opening angle theta_max (radians) of the non-reversal walk whose bonds are uniform on the cap
    within theta_max of the previous bond: <cos theta> = (1 + cos theta_max) / 2 = cos^2(theta_max / 2)
    (Sec. II.B), and c = (1 + <cos theta>) / (1 - <cos theta>) fixes <cos theta> = (c - 1) / (c + 1)."""
    mean_cos = (c - 1.0) / (c + 1.0)
    return 2.0 * math.acos(math.sqrt(mean_cos))


def phantom_chains(n_poly: int, n_per: int, eta: float, seed: int, c: float = 1.9, sigma: float = 1.0,
                   b_max: float = 1.4, L: float | None = None) -> Melt:
    """Phantom chains for the push-off (Sec. II.B): bond length sigma, vanishing excluded volume,
    grown as non-reversal random walks whose bond directions are uniform on the cap within
    theta_max of the previous bond (theta_max from c: 112.3 degrees for c = 1.9); the first bead
    of each chain and its first bond direction are uniform.  The box is sized for packing
    fraction eta at diameter sigma (or given as L)."""
    rng = np.random.default_rng(seed)
    n = n_poly * n_per
    if L is None:
        L = box_for(n, eta, sigma)
    cos_max = math.cos(theta_max_for(c))
    pos = np.zeros((n_poly, n_per, 3))
    pos[:, 0] = rng.uniform(0.0, L, size=(n_poly, 3))
    t = rng.normal(size=(n_poly, 3))
    t /= np.linalg.norm(t, axis=1)[:, None]
    for k in range(1, n_per):
        if k > 1:
            # a direction on the cap around t: cos uniform in [cos theta_max, 1], azimuth uniform
            ct = rng.uniform(cos_max, 1.0, size=n_poly)
            st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
            ph = rng.uniform(0.0, 2.0 * math.pi, size=n_poly)
            a = np.where(np.abs(t[:, 0:1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
            e1 = np.cross(t, a)
            e1 /= np.linalg.norm(e1, axis=1)[:, None]
            e2 = np.cross(t, e1)
            t = ct[:, None] * t + (st * np.cos(ph))[:, None] * e1 + (st * np.sin(ph))[:, None] * e2
            t /= np.linalg.norm(t, axis=1)[:, None]
        pos[:, k] = pos[:, k - 1] + sigma * t
    return Melt(L=L, positions=_wrap(pos.reshape(-1, 3), L), bonds=_chain_bonds(n_poly, n_per), sigma=sigma,
                b_max=b_max, n_poly=n_poly, n_per=n_per,
                meta={"recipe": "phantom", "seed": seed, "c": c, "theta_max": theta_max_for(c)})
