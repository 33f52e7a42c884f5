"""Seeded synthetic inputs for the entropic JKO flows.

This module only *draws* inputs: densities, obstacle masks, potentials,
capacity fields and coefficient fields, all in float64 numpy arrays.  It holds
none of the method's arithmetic (no Gibbs kernel, no proximal map, no scaling
update), so both the FP64 oracle and the HIP path can take their inputs from
here without sharing any computation.

Every generator takes an explicit ``seed`` and uses ``numpy.random.default_rng``
(PCG64).  Grids are cell-centred on the unit cube: along an axis of length n the
cell centres are ``(i + 0.5) / n``.  Array index ``(i0, i1[, i2])`` is the point
``(x1, x2[, x3])``; the last axis is contiguous in memory.

Workloads (synthetic stand-ins for the paper's figures, which print no data):

* ``crowd32``   -- 2D crowd motion with congestion (Section 4.2) on 32x32:
                   3 Gaussian bumps, scalar capacity, potential |x - exit|^2.
* ``crowd256``  -- 2D crowd motion on 256x256 with 6 rectangular obstacles
                   (capacity 0 inside), 8 bumps.
* ``porous512`` -- 2D nonlinear diffusion on 512x512 with
                   f(p) = sum c(x) p^m / (m - 1), m = 2 (Section 4.4), smoothed
                   uniform noise as initial density.
* ``crowd128c`` -- 3D crowd motion on 128^3 with 10 box obstacles, 16 bumps.
* ``gen512``    -- 2D nonlinear diffusion on 512x512 with the generalised
                   entropies of Section 4.4: weights b = 1 and exponents
                   m(x) = 1 + sin(pi x1) sin(pi x2) (1 at the boundary, 2 in the
                   centre, as in the paper's second nonlinear-diffusion
                   example), density units, the porous512 initial density,
                   3 steps of 300 iterations.
* ``crowd256_attraction`` -- the ``crowd256`` obstacles, capacity and bump
                   recipe under the Wasserstein attraction of Section 5.2, at
                   gamma = 1e-3, tau = 1e-2: the target r is p0 translated by
                   0.1 along the first axis (26 cells, the wrapped band set to
                   0), of the same mass; 3 steps of 300 iterations.  (The
                   second coupling carries every cell to its target in one hop:
                   its kernel entries stay representable in float32 while
                   displacement^2 / gamma stays well under 87.)
* ``heat100``   -- crowd motion on a 100x100 room with a wall, a door and
                   pillars under the heat-kernel Gibbs operator of Section 4.1
                   (L = 10 implicit steps; ``heat_room``), capacity max p0;
                   3 steps of 300 iterations.
* ``crowd256_binary`` -- ``crowd256`` under the non-convex binary constraint
                   {0, kappa} (Section 4.5): potential scaled to sigma w <= 1/2
                   (above 1 the binary prox empties every cell), initial density
                   binary (kappa where the projected p0 reaches kappa/2, else 0),
                   3 steps of 300 iterations.

The ``projected`` flag replaces p0 by min(c * p0, kappa) with the scalar c found
by bisection so that the total mass is one: the paper requires the capacity to
dominate the initial density (Section 4.2), which the raw bump mixtures do not.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "cell_centres", "gaussian_bumps", "box_obstacles",
    "project_capacity", "make_workload", "WORKLOADS", "small_case", "heat_room",
]


def cell_centres(n: int) -> np.ndarray:
    """Cell centres (i + 0.5) / n of a uniform grid on [0, 1]."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _mesh(shape):
    return np.meshgrid(*[cell_centres(n) for n in shape], indexing="ij")


def gaussian_bumps(shape, centres, sigma, weights) -> np.ndarray:
    """Sum of isotropic Gaussian bumps sampled at the cell centres, mass 1."""
    X = _mesh(shape)
    out = np.zeros(shape, dtype=np.float64)
    for c, wt in zip(centres, weights):
        r2 = sum((X[k] - c[k]) ** 2 for k in range(len(shape)))
        out += wt * np.exp(-r2 / (2.0 * sigma * sigma))
    return out / out.sum()


def box_obstacles(shape, corners, sides) -> np.ndarray:
    """Boolean mask of the cells whose centre lies in one of the boxes
    [corner, corner + side) (one box per row of ``corners``/``sides``)."""
    X = _mesh(shape)
    mask = np.zeros(shape, dtype=bool)
    for c, s in zip(corners, sides):
        inside = np.ones(shape, dtype=bool)
        for k in range(len(shape)):
            inside &= (X[k] >= c[k]) & (X[k] < c[k] + s[k])
        mask |= inside
    return mask


def squared_distance(shape, point) -> np.ndarray:
    X = _mesh(shape)
    return sum((X[k] - point[k]) ** 2 for k in range(len(shape)))


def project_capacity(p: np.ndarray, kappa: np.ndarray, iters: int = 90) -> np.ndarray:
    """Return min(c * p, kappa) with c > 0 chosen by bisection so the sum is 1.

    Requires sum(kappa) > 1 over the support of p.
    """
    kappa = np.broadcast_to(kappa, p.shape)
    lo, hi = 0.0, 1.0
    while np.minimum(hi * p, kappa).sum() < 1.0:
        hi *= 2.0
        if hi > 1e30:
            raise ValueError("capacity too small to hold unit mass")
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.minimum(mid * p, kappa).sum() < 1.0:
            lo = mid
        else:
            hi = mid
    out = np.minimum(hi * p, kappa)
    return out / out.sum()


@dataclass
class Workload:
    """One synthetic flow: grid, energy fields, solver parameters, p0."""
    name: str
    shape: tuple
    gamma: float
    tau: float
    kind: str                    # "congestion" | "binary_congestion" | "porous" | "entropy" | "gen_entropy" |
                                 # "attraction" | "zero"
    p0: np.ndarray
    w: Optional[np.ndarray] = None         # congestion potential (None = 0)
    kappa: Optional[np.ndarray] = None     # capacity field (None = kappa_scalar)
    kappa_scalar: float = math.inf
    coef: Optional[np.ndarray] = None      # porous / entropy coefficient c(x)
    coef_scalar: float = 1.0
    m: float = 2.0
    density_scale: float = 1.0
    m_field: Optional[np.ndarray] = None   # gen_entropy exponents per cell (None = m)
    target: Optional[np.ndarray] = None    # attraction target density r
    mask: Optional[np.ndarray] = None      # heat-kernel domain (True = free cell); None = Gaussian kernel
    heat_L: int = 10                       # implicit heat steps of the heat kernel
    n_steps: int = 1
    max_iters: int = 300
    tol: float = 0.0                       # 0 = fixed iteration count
    check_every: int = 10
    extras: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))

    def kappa_field(self) -> np.ndarray:
        if self.kappa is not None:
            return self.kappa
        return np.full(self.shape, self.kappa_scalar, dtype=np.float64)


def _crowd(name, shape, gamma, tau, n_bumps, n_boxes, centre_box, exit_pt,
           cap_factor, seed, projected, n_steps, max_iters, tol):
    rng = np.random.default_rng(seed)
    d = len(shape)
    N = int(np.prod(shape))
    X = _mesh(shape)
    exit_cell = tuple(min(int(exit_pt[k] * shape[k]), shape[k] - 1) for k in range(d))
    # obstacles: all sides, then all corners; redraw until feasible
    if n_boxes > 0:
        while True:
            sides = rng.uniform(0.05, 0.2, size=(n_boxes, d))
            corners = rng.uniform(0.0, 1.0 - sides)
            mask = box_obstacles(shape, corners, sides)
            free = 1.0 - mask.mean()
            if cap_factor * free >= 1.05 and not mask[exit_cell]:
                break
    else:
        sides = np.zeros((0, d))
        corners = np.zeros((0, d))
        mask = np.zeros(shape, dtype=bool)
    # bump centres by rejection outside the obstacles
    lo, hi = centre_box
    centres = []
    while len(centres) < n_bumps:
        c = rng.uniform(lo, hi)
        cell = tuple(min(int(c[k] * shape[k]), shape[k] - 1) for k in range(d))
        if not mask[cell]:
            centres.append(c)
    weights = rng.dirichlet(np.ones(n_bumps))
    p0 = gaussian_bumps(shape, centres, 0.05, weights)
    p0[mask] = 0.0
    p0 /= p0.sum()
    w = squared_distance(shape, exit_pt)
    if n_boxes > 0:
        kappa = np.where(mask, 0.0, cap_factor / N)
        kappa_scalar = math.inf
    else:
        kappa = None
        kappa_scalar = cap_factor / N
    if projected:
        p0 = project_capacity(p0, kappa if kappa is not None else kappa_scalar)
    return Workload(
        name=name, shape=tuple(shape), gamma=gamma, tau=tau, kind="congestion",
        p0=p0, w=w, kappa=kappa, kappa_scalar=kappa_scalar, n_steps=n_steps,
        max_iters=max_iters, tol=tol,
        extras=dict(mask=mask, corners=corners, sides=sides, centres=np.array(centres),
                    weights=weights, exit=np.array(exit_pt)),
    )


def _porous(name, shape, gamma, tau, m, seed, density_scaled, n_steps, max_iters, tol):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    noise = rng.uniform(0.5, 1.5, size=shape)
    # normalised separable Gaussian smoothing, std 0.02
    sm = noise
    for ax, n in enumerate(shape):
        x = cell_centres(n)
        G = np.exp(-((x[:, None] - x[None, :]) ** 2) / (2.0 * 0.02 ** 2))
        G /= G.sum(axis=1, keepdims=True)
        sm = np.moveaxis(np.tensordot(G, np.moveaxis(sm, ax, 0), axes=(1, 0)), 0, ax)
    p0 = sm / sm.sum()
    X = _mesh(shape)
    coef = 1.0 + 0.9 * np.sin(6 * np.pi * X[0]) * np.sin(6 * np.pi * X[1])
    return Workload(
        name=name, shape=tuple(shape), gamma=gamma, tau=tau, kind="porous", p0=p0,
        coef=coef, m=m, density_scale=float(N) if density_scaled else 1.0,
        n_steps=n_steps, max_iters=max_iters, tol=tol,
    )


def _geodesic_steps(mask: np.ndarray, goal) -> np.ndarray:
    """Length of the shortest 4-neighbour path inside ``mask`` from every
    cell to ``goal``, in cells (inf where unreachable)."""
    n0, n1 = mask.shape
    dist = np.full(mask.shape, np.inf)
    dist[goal] = 0.0
    frontier = [goal]
    while frontier:
        nxt = []
        for (i, j) in frontier:
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                a, b = i + di, j + dj
                if 0 <= a < n0 and 0 <= b < n1 and mask[a, b] and dist[a, b] == np.inf:
                    dist[a, b] = dist[i, j] + 1.0
                    nxt.append((a, b))
        frontier = nxt
    return dist


def heat_room(n0: int, n1: int, seed: int = 0, gamma=None, tau=None, L: int = 10,
              n_steps: int = 3, max_iters: int = 300, tol: float = 0.0) -> Workload:
    """Crowd motion on a non-convex room under the heat-kernel Gibbs operator
    (Section 4.1 and the obstacle-domain crowd example of Section 4.3):
    the unit square with a wall across the first axis at x0 = 0.55 pierced by
    a door of width 0.16 around x1 = 0.5, and three square pillars in the
    start region.  The crowd starts as 4 Gaussian bumps (std 0.05) in
    x0 < 0.45, their peaks cut to a plateau at a fifth of the highest one (mass
    kept at 1), the potential w is the geodesic distance (4-neighbour path
    length, in units of the longer axis) to an exit at (0.95, 0.5), and the
    capacity is kappa = max p0 (the paper's choice).  gamma defaults to
    L / max(n)^2 (one heat-step weight nu = 1 on the longer axis), tau to
    20 gamma."""
    rng = np.random.default_rng(seed)
    shape = (n0, n1)
    X = _mesh(shape)
    free = np.ones(shape, bool)
    wall = (X[0] >= 0.55) & (X[0] < 0.55 + max(0.03, 1.5 / n0))
    door = np.abs(X[1] - 0.5) < 0.08
    free &= ~(wall & ~door)
    for _ in range(3):
        c = rng.uniform([0.1, 0.1], [0.35, 0.8])
        free &= ~box_obstacles(shape, [c], [[0.08, 0.08]])
    centres = []
    while len(centres) < 4:
        c = rng.uniform([0.08, 0.1], [0.42, 0.9])
        cell = (min(int(c[0] * n0), n0 - 1), min(int(c[1] * n1), n1 - 1))
        if free[cell]:
            centres.append(c)
    p0 = gaussian_bumps(shape, centres, 0.05, rng.dirichlet(np.ones(4)))
    p0[~free] = 0.0
    p0 /= p0.sum()
    p0 = project_capacity(p0, 0.2 * p0.max())     # peaks flattened: the capacity max p0 binds
    exit_cell = (min(int(0.95 * n0), n0 - 1), min(int(0.5 * n1), n1 - 1))
    w = _geodesic_steps(free, exit_cell) / max(shape)
    w[~np.isfinite(w)] = 0.0          # cells cut off from the exit (none in this room) and obstacles
    if gamma is None:
        gamma = L / float(max(shape)) ** 2
    if tau is None:
        tau = 20.0 * gamma
    return Workload(name=f"heat{n0}x{n1}", shape=shape, gamma=gamma, tau=tau, kind="congestion",
                    p0=p0, w=w, kappa_scalar=float(p0.max()), n_steps=n_steps, max_iters=max_iters,
                    tol=tol, mask=free, heat_L=L, extras=dict(centres=np.array(centres), exit=exit_cell))


def make_workload(name: str, seed: int = 0, projected: bool = True, **over) -> Workload:
    """Build a named workload.  ``over`` overrides scalar solver parameters
    (n_steps, max_iters, tol, check_every)."""
    if name == "crowd32":
        wl = _crowd(name, (32, 32), 2e-3, 5e-3, 3, 0, ([0.1, 0.1], [0.5, 0.9]),
                    (0.9, 0.5), 1.5, seed, projected, 10, 300, 0.0)
    elif name == "crowd256":
        wl = _crowd(name, (256, 256), 2e-4, 2e-3, 8, 6, ([0.1, 0.1], [0.9, 0.9]),
                    (0.9, 0.5), 1.2, seed, projected, 50, 2000, 1e-6)
    elif name == "crowd256_fixed":
        wl = _crowd(name, (256, 256), 2e-4, 2e-3, 8, 6, ([0.1, 0.1], [0.9, 0.9]),
                    (0.9, 0.5), 1.2, seed, projected, 20, 300, 0.0)
    elif name == "porous512":
        wl = _porous(name, (512, 512), 1e-4, 1e-3, 2.0, seed, False, 40, 300, 1e-6)
    elif name == "porous512_scaled":
        wl = _porous(name, (512, 512), 1e-4, 1e-3, 2.0, seed, True, 40, 300, 1e-6)
    elif name == "crowd128c":
        wl = _crowd(name, (128, 128, 128), 5e-4, 2e-3, 16, 10,
                    ([0.1, 0.1, 0.1], [0.9, 0.9, 0.9]), (0.9, 0.5, 0.5), 1.2, seed,
                    projected, 20, 300, 0.0)
    elif name == "gen512":
        wl = _porous(name, (512, 512), 1e-4, 1e-3, 2.0, seed, True, 3, 300, 0.0)
        X = _mesh(wl.shape)
        wl.kind = "gen_entropy"
        wl.coef = None
        wl.coef_scalar = 1.0
        wl.m_field = 1.0 + np.sin(np.pi * X[0]) * np.sin(np.pi * X[1])
    elif name == "crowd256_attraction":
        wl = _crowd(name, (256, 256), 1e-3, 1e-2, 8, 6, ([0.1, 0.1], [0.9, 0.9]),
                    (0.9, 0.5), 1.2, seed, projected, 3, 300, 0.0)
        wl.kind = "attraction"
        wl.w = None
        r = np.roll(wl.p0, -26, axis=0)
        r[-26:, :] = 0.0
        wl.target = r * (wl.p0.sum() / r.sum())
    elif name == "crowd256_binary":
        wl = _crowd(name, (256, 256), 2e-4, 2e-3, 8, 6, ([0.1, 0.1], [0.9, 0.9]),
                    (0.9, 0.5), 1.2, seed, projected, 3, 300, 0.0)
        wl.kind = "binary_congestion"
        wl.w = wl.w * (0.5 / ((wl.tau / wl.gamma) * float(wl.w.max())))
        kap = wl.kappa_field()
        wl.p0 = np.where((kap > 0) & (wl.p0 >= 0.5 * kap), kap, 0.0)
    elif name == "heat100":
        wl = heat_room(100, 100, seed)
        wl.name = name
    else:
        raise KeyError(name)
    for k, v in over.items():
        if not hasattr(wl, k):
            raise KeyError(k)
        setattr(wl, k, v)
    return wl


WORKLOADS = ("crowd32", "crowd256", "crowd256_fixed", "crowd256_binary", "crowd256_attraction", "porous512",
             "porous512_scaled", "gen512",
             "crowd128c", "heat100")


def small_case(shape, kind="congestion", seed=0, gamma=None, tau=None, n_boxes=None,
               n_bumps=3, cap_factor=1.5, projected=True, **over) -> Workload:
    """A workload of arbitrary (possibly ragged) shape for parity tests.

    Same recipe as the named workloads; gamma defaults to a kernel width of a
    few cells, tau to 2.5 gamma.
    """
    d = len(shape)
    h = 1.0 / max(shape)
    if gamma is None:
        gamma = 2.0 * (2.0 * h) ** 2 * 2.0
    if tau is None:
        tau = 2.5 * gamma
    if kind == "congestion":
        nb = (0 if d == 1 else 2) if n_boxes is None else n_boxes
        lo = [0.15] * d
        hi = [0.85] * d
        wl = _crowd("small", tuple(shape), gamma, tau, n_bumps, nb, (lo, hi),
                    tuple([0.9] + [0.5] * (d - 1)), cap_factor, seed, projected, 2, 50, 0.0)
    elif kind in ("porous", "entropy", "zero"):
        rng = np.random.default_rng(seed)
        centres = rng.uniform(0.25, 0.75, size=(n_bumps, d))
        weights = rng.dirichlet(np.ones(n_bumps))
        p0 = gaussian_bumps(shape, centres, 0.08, weights)
        coef = 1.0 + 0.5 * rng.uniform(size=shape)
        wl = Workload(name="small", shape=tuple(shape), gamma=gamma, tau=tau, kind=kind,
                      p0=p0, coef=coef if kind != "zero" else None, m=2.0,
                      n_steps=2, max_iters=50)
    else:
        raise KeyError(kind)
    for k, v in over.items():
        setattr(wl, k, v)
    return wl
