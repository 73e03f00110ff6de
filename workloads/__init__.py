"""Seeded synthetic inputs for the multigrid solver and for its reference checks.

This module only draws random numbers and lays them out; it holds none of the
solver's arithmetic.  Both the HIP library's tests/benchmarks and the CPU
reference consume these arrays, and nothing else is shared between the two.

Layout conventions (shared by every producer and consumer of these arrays):

* A level-``L`` regular grid of the unit cube ``(0,1)^d`` has ``n = 3**L`` cells
  per axis (tripartitioned spacetree, every cell refined down to level ``L``).
* ``eps`` holds one diffusion coefficient per finest cell, shape ``(n,)*d``,
  C order with x fastest, i.e. ``eps[z, y, x]`` (``eps[y, x]`` in 2D).
* ``f`` holds one source value per interior vertex, shape ``(n-1,)*d``, again x
  fastest.  Interior vertex ``(i, j[, k])`` with ``1 <= i,j,k <= n-1`` sits at
  ``x = i/n`` and is stored at ``f[k-1, j-1, i-1]``.

The problems follow the paper's setups (Table "parameters", Sect. 7): zero
Dirichlet boundary, piecewise-constant coefficients (and, for ``circle``,
velocities) per cell.
The concrete random fields stand in for the paper's analytic setups; no data set
is involved.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


@dataclasses.dataclass
class Problem:
    """One solve request: grid size, coefficient field and right-hand side."""
    name: str
    dim: int
    level: int
    eps: np.ndarray        # (n,)*dim float64, one value per finest cell
    f: np.ndarray          # (n-1,)*dim float64, one value per interior vertex
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return 3 ** self.level

    @property
    def n_unknowns(self) -> int:
        return (self.n - 1) ** self.dim


def _uniform_f(rng: np.random.Generator, dim: int, level: int) -> np.ndarray:
    n = 3 ** level
    return rng.uniform(-1.0, 1.0, size=(n - 1,) * dim)


def _block_index(dim: int, level: int, blocks: int) -> List[np.ndarray]:
    """Per axis, the index of the ``blocks``-wide coarse block each finest cell
    centre falls into (``floor(blocks * x_centre)``)."""
    n = 3 ** level
    centres = (np.arange(n) + 0.5) / n
    b = np.floor(blocks * centres).astype(np.int64)
    grids = np.meshgrid(*([b] * dim), indexing="ij")
    return grids[::-1]  # returned as (x, y[, z]) index arrays shaped like eps[z, y, x]


def poisson(dim: int, level: int, seed: int, name: str = "poisson") -> Problem:
    """Constant coefficient (eps = 1) and f ~ U[-1, 1] i.i.d. per unknown."""
    rng = np.random.default_rng(seed)
    n = 3 ** level
    eps = np.ones((n,) * dim)
    f = _uniform_f(rng, dim, level)
    return Problem(name, dim, level, eps, f, {"seed": seed, "eps": "1"})


def random_checkerboard(dim: int, level: int, seed: int, values=(1.0, 1.0e4),
                        blocks: int = 9, name: str = "jump") -> Problem:
    """Coefficient piecewise constant on a ``blocks^d`` array of equal boxes;
    each box draws one of ``values`` i.i.d. (box array drawn first, C order),
    then f ~ U[-1, 1] per unknown."""
    rng = np.random.default_rng(seed)
    table = rng.choice(np.asarray(values, dtype=np.float64), size=(blocks,) * dim)
    idx = _block_index(dim, level, blocks)          # x, y[, z]
    eps = table[tuple(idx[::-1])]                   # table indexed [z, y, x]
    f = _uniform_f(rng, dim, level)
    return Problem(name, dim, level, eps, f,
                   {"seed": seed, "eps": f"random {blocks}^d boxes of {values}"})


def alternating_checkerboard(dim: int, level: int, contrast: float, seed: int,
                             blocks: int = 9, name: str = "checker") -> Problem:
    """Coefficient 1 / ``contrast`` alternating on a ``blocks^d`` box array
    (parity of the box index sum), f ~ U[-1, 1] per unknown."""
    rng = np.random.default_rng(seed)
    idx = _block_index(dim, level, blocks)
    parity = sum(idx) % 2
    eps = np.where(parity == 0, 1.0, float(contrast))
    f = _uniform_f(rng, dim, level)
    return Problem(name, dim, level, eps, f,
                   {"seed": seed, "eps": f"alternating {blocks}^d, contrast {contrast:g}"})


def sin_source(dim: int, level: int) -> Problem:
    """The paper's validation setup with eps = 1 and a sine source whose exact
    solution is prod_i sin(pi x_i); f = d*pi^2*prod_i sin(pi x_i) (the printed
    2*pi^2 is the d = 2 instance)."""
    n = 3 ** level
    x = np.arange(1, n) / n
    s = np.sin(np.pi * x)
    grids = np.meshgrid(*([s] * dim), indexing="ij")
    prod = np.ones_like(grids[0])
    for g in grids:
        prod = prod * g
    f = dim * np.pi ** 2 * prod
    return Problem("sin", dim, level, np.ones((n,) * dim), f, {"exact": prod})


def material_jump(dim: int, level: int) -> Problem:
    """The paper's ``jump`` setup (Table "parameters"): eps = 1 where the first
    coordinate of the cell centre is below 0.5, 0.1 elsewhere (a jump that no
    cell face of any level meets), f = 1."""
    n = 3 ** level
    xc = (np.arange(n) + 0.5) / n
    eps = np.broadcast_to(np.where(xc < 0.5, 1.0, 0.1), (n,) * dim).copy()
    return Problem(f"jump{dim}d-L{level}", dim, level, eps, np.ones((n - 1,) * dim),
                   {"eps": "1 | 0.1 at x = 0.5"})


def circle(dim: int, level: int, eps_small: float, seed: int = 0) -> Problem:
    """The paper's ``circle`` setup (Table "parameters"): a recirculating flow
    v = (sin(pi(y - 1/2)) cos(pi(x - 1/2)), -cos(pi(y - 1/2)) sin(pi(x - 1/2)), 0)
    sampled at cell centres, eps = eps_small (1 in 3D where z > 1/2).  The
    paper's inflow boundary data are replaced by zero Dirichlet values and a
    seeded f ~ U[-1, 1], which leaves the operator unchanged.  ``meta["v"]``
    holds the velocities, shape (dim,) + (n,)*dim."""
    n = 3 ** level
    xc = (np.arange(n) + 0.5) / n
    grids = np.meshgrid(*([xc] * dim), indexing="ij")   # axis order (z,) y, x
    x, y = grids[-1], grids[-2]
    v = np.zeros((dim,) + (n,) * dim)
    v[0] = np.sin(np.pi * (y - 0.5)) * np.cos(np.pi * (x - 0.5))
    v[1] = -np.cos(np.pi * (y - 0.5)) * np.sin(np.pi * (x - 0.5))
    eps = np.full((n,) * dim, float(eps_small))
    if dim == 3:
        eps = np.where(grids[0] > 0.5, 1.0, eps)
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, (n - 1,) * dim)
    return Problem(f"circle{dim}d-L{level}-eps{eps_small:g}", dim, level, eps, f, {"v": v})


# --------------------------------------------------------------------------
# Named workloads: a small 2D Poisson problem; the 2D jumping coefficient on
# 729^2 cells; a stream of mixed 2D/3D checkerboard requests.
# --------------------------------------------------------------------------

def poisson2d_l4(seed: int = 0) -> Problem:
    """2D Poisson, 81^2 cells (80^2 unknowns), eps = 1, f ~ U[-1, 1]."""
    return poisson(2, 4, seed, name="poisson2d-L4")


def checkerboard2d(seed: int = 0, level: int = 6) -> Problem:
    """2D jumping coefficient: random 9x9 checkerboard of {1, 1e4} on 3^level
    cells per axis (729^2 by default), f ~ U[-1, 1]."""
    return random_checkerboard(2, level, seed, name=f"checkerboard2d-L{level}")


def jump3d(level: int, seed: int = 0) -> Problem:
    """3D analogue of checkerboard2d: random 9^3 boxes with values {1, 1e4}."""
    return random_checkerboard(3, level, seed, name=f"jump3d-L{level}")


# --------------------------------------------------------------------------
# Adaptive spacetrees.  A problem is (base level, max level, refinement flags
# per level) plus coefficient and source *fields* that each side evaluates at
# its own leaf cells and unknowns, so that no side needs the other's numbering.
# --------------------------------------------------------------------------

def _cell_boxes(dim, level):
    n = 3 ** level
    idx = np.stack(np.meshgrid(*([np.arange(n)] * dim), indexing="ij"), -1)[..., ::-1]  # x first
    lo = idx / n
    return lo, lo + 1.0 / n


def ball_flags(dim, base, level, centres, radius):
    """Refine a cell when its closed box comes closer than ``radius`` to any
    centre (levels base..level-1)."""
    flags = {}
    for l in range(base, level):
        lo, hi = _cell_boxes(dim, l)
        f = np.zeros((3 ** l,) * dim, dtype=bool)
        for c in np.atleast_2d(centres):
            gap = np.maximum(np.maximum(lo - c, 0.0), np.maximum(c - hi, 0.0))
            f |= np.sqrt((gap ** 2).sum(-1)) < radius
        flags[l] = f
    return flags


def rff_field(dim, seed, n_features, length):
    """Random-Fourier-feature Gaussian field g(x) = sqrt(2/M) sum cos(k_m.x + p_m),
    k_m ~ N(0, length^-2 I), p_m ~ U[0, 2pi): zero mean, unit variance,
    covariance exp(-|r|^2 / (2 length^2)).  The callable carries its
    parameters as attributes ``k`` (M, dim; x first), ``p`` (M) and ``scale``."""
    rng = np.random.default_rng(seed)
    k = rng.normal(0.0, 1.0 / length, size=(n_features, dim))
    p = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    scale = np.sqrt(2.0 / n_features)

    def g(x):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        out = np.empty(len(x))
        for c0 in range(0, len(x), 1 << 16):
            xs = x[c0:c0 + (1 << 16)]
            out[c0:c0 + len(xs)] = scale * np.cos(xs @ k.T + p).sum(axis=1)
        return out
    g.k, g.p, g.scale = k, p, scale
    return g


# Region kinds of the library's grid description (refine the cells that meet
# the region); the parameter layouts are those of the C header.
REGION_BALL, REGION_LEVELSET_BAND, REGION_CELL_LIST = 0, 1, 2


def ball_regions(centres, radius, level):
    """One ball region per centre: params (centre x first, radius)."""
    return [(REGION_BALL, level, np.concatenate([np.asarray(c, np.float64), [radius]]))
            for c in np.atleast_2d(centres)]


def band_region(phi, tau, level):
    """The band |phi| < tau (or a sign change) of an RFF level set: params
    (tau, scale, M, k (M x dim, x first, row by row), phases (M))."""
    k, p = np.asarray(phi.k, np.float64), np.asarray(phi.p, np.float64)
    return [(REGION_LEVELSET_BAND, level,
             np.concatenate([[tau, phi.scale, float(len(p))], k.ravel(), p]))]


def uniform_hash(seed, level, idx):
    """Counter-based U[-1, 1) value per (seed, level, lattice index) from the
    SplitMix64 finaliser (Steele, Lea, Flood 2014): the source value of an
    unknown depends only on its level and position."""
    idx = np.atleast_2d(np.asarray(idx, dtype=np.uint64))
    with np.errstate(over="ignore"):
        z = np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(level + 1)
        for c in range(idx.shape[1]):
            z = (z ^ idx[:, c]) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(c + 1)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 2.0 ** 53) - 1.0


@dataclasses.dataclass
class AdaptiveProblem:
    name: str
    dim: int
    base: int
    level: int
    flags_fn: object            # () -> {level: bool array over the level's cells (NumPy axes z,y,x)}
    eps_at: object              # callable: cell centres (m, dim) x-first -> eps (m,)
    f_seed: int                 # source of unknown (level l, vertex i,j,k) = uniform_hash(f_seed, l, (i,j,k))
    meta: dict = dataclasses.field(default_factory=dict)
    regions: list = dataclasses.field(default_factory=list)   # the same refinement as region descriptions
    mark: object = None         # (level, cells (m, dim) int x-first) -> bool: the region meets the cell
    _flags: dict = None

    @property
    def flags(self):
        """Refinement flags per level, evaluated here (NumPy) on first use."""
        if self._flags is None:
            self._flags = self.flags_fn()
        return self._flags

    def f_at(self, level, coords_xfirst):
        """Source values at unknowns of one level given their coordinates."""
        n = 3 ** level
        idx = np.rint(np.asarray(coords_xfirst) * n).astype(np.int64)
        return uniform_hash(self.f_seed, level, idx)


def adaptive_balls(dim=3, base=3, level=5, n_balls=4, radius=0.2, seed=0, contrast_field=True,
                   name="adaptive-balls3d"):
    """Refined to ``level`` within ``radius`` of ``n_balls`` seeded points,
    ``base`` everywhere; eps = exp(g) with g a unit-variance RFF field of
    correlation length 0.1 (M = 1024) at leaf-cell centres."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_balls, dim))
    g = rff_field(dim, seed + 1000, 1024, 0.1) if contrast_field else (lambda x: np.zeros(len(x)))
    def mark(l, cells_xfirst):
        n = 3 ** l
        lo = np.atleast_2d(cells_xfirst) / n
        hi = lo + 1.0 / n
        f = np.zeros(len(lo), dtype=bool)
        for c in np.atleast_2d(centres):
            gap = np.maximum(np.maximum(lo - c, 0.0), np.maximum(c - hi, 0.0))
            f |= np.sqrt((gap ** 2).sum(-1)) < radius
        return f
    return AdaptiveProblem(name, dim, base, level, lambda: ball_flags(dim, base, level, centres, radius),
                           lambda x: np.exp(g(x)), seed + 2000,
                           {"centres": centres, "radius": radius, "seed": seed},
                           ball_regions(centres, radius, level), mark)


def adaptive_band(dim=3, base=3, level=6, seed=0, fraction=0.10, n_cubes=64, n_features=64,
                  name="adaptive-band3d"):
    """Refined to ``level`` around the zero set of an RFF level set phi
    (length 0.2): a cell is refined where |phi| < tau at one of its 3^d sample
    points or phi changes sign there, tau being the ``fraction`` quantile of
    |phi| on 10^6 seeded points.  eps = 1e6 inside ``n_cubes`` random cubes
    (centres U[0,1]^3, sides U[0.05, 0.15]), 1 outside."""
    rng = np.random.default_rng(seed)
    phi = rff_field(dim, seed + 3000, n_features, 0.2)
    tau = float(np.quantile(np.abs(phi(rng.uniform(0.0, 1.0, size=(10 ** 6, dim)))), fraction))
    centres = rng.uniform(0.0, 1.0, size=(n_cubes, dim))
    sides = rng.uniform(0.05, 0.15, size=n_cubes)

    def mark(l, cells_xfirst):
        """Does the band meet these cells of level l (integer indices, x first)?"""
        n = 3 ** l
        lo = np.atleast_2d(cells_xfirst) / n
        pts = []
        for o in np.ndindex(*([3] * dim)):
            pts.append(lo + (np.array(o) * 0.5) / n)
        vals = np.stack([phi(pp) for pp in pts], 1)
        return (np.abs(vals).min(1) < tau) | (vals.min(1) < 0) & (vals.max(1) > 0)

    def flags_fn():
        flags = {}
        exist = None
        for l in range(base, level):
            n = 3 ** l
            cells = np.argwhere(np.ones((n,) * dim, bool) if exist is None else exist)  # numpy order
            f = np.zeros((n,) * dim, dtype=bool)
            if len(cells):
                f[tuple(cells.T)] = mark(l, cells[:, ::-1])
            flags[l] = f
            exist = np.repeat(np.repeat(np.repeat(f, 3, 0), 3, 1), 3, 2) if dim == 3 else \
                np.repeat(np.repeat(f, 3, 0), 3, 1)
        return flags

    def eps_at(x):
        x = np.atleast_2d(x)
        inside = np.zeros(len(x), dtype=bool)
        for c, s in zip(centres, sides):
            inside |= np.all(np.abs(x - c) <= s / 2, axis=1)
        return np.where(inside, 1e6, 1.0)
    return AdaptiveProblem(name, dim, base, level, flags_fn, eps_at, seed + 4000,
                           {"tau": tau, "seed": seed, "centres": centres, "sides": sides},
                           band_region(phi, tau, level), mark)


@dataclasses.dataclass
class Request:
    problem: Problem
    arrival: float       # seconds after stream start


def request_stream(seed: int = 0, n_requests: int = 256, rate: float = 100.0,
                levels_2d=(3, 6), levels_3d=(2, 4)) -> List[Request]:
    """Served stream: each request draws d in {2,3} with p = 1/2, a level
    uniformly in ``levels_2d`` / ``levels_3d`` (inclusive), a contrast 10^c with
    c ~ U[0, 4] and its own f; arrivals are a Poisson process of ``rate``/s."""
    rng = np.random.default_rng(seed)
    out: List[Request] = []
    t = 0.0
    for k in range(n_requests):
        dim = 2 if rng.uniform() < 0.5 else 3
        lo, hi = levels_2d if dim == 2 else levels_3d
        level = int(rng.integers(lo, hi + 1))
        c = float(rng.uniform(0.0, 4.0))
        sub_seed = int(rng.integers(0, 2 ** 31 - 1))
        t += float(rng.exponential(1.0 / rate))
        p = alternating_checkerboard(dim, level, 10.0 ** c, sub_seed,
                                     name=f"stream-req{k}-d{dim}-L{level}")
        out.append(Request(p, t))
    return out


__all__ = ["Problem", "Request", "poisson", "random_checkerboard",
           "alternating_checkerboard", "sin_source", "poisson2d_l4", "checkerboard2d", "jump3d",
           "request_stream", "ball_flags", "rff_field", "uniform_hash", "AdaptiveProblem",
           "adaptive_balls", "adaptive_band", "material_jump", "circle", "ball_regions", "band_region",
           "REGION_BALL", "REGION_LEVELSET_BAND", "REGION_CELL_LIST"]
