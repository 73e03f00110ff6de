"""Adaptive spacetrees: composite system and FAS V-cycle (oracle, FP64).

Paper passages followed (Sect. 3):

* A cell is refined independently of its neighbours; level l holds the cells
  of depth l, so each level is a ragged Cartesian grid.
* A vertex of level l is hanging if fewer than 2^d level-l cells touch it,
  refined if all its level-l cells are refined (a non-hanging copy then exists
  on level l+1), unrefined otherwise.
* A refined vertex holds the value of the vertex at the same position on the
  finer level (injection I); a hanging vertex holds the d-linear interpolant of
  the coarser level; every level uses the same discretisation.
* FAS/HTMG: the coarse equation of a refined vertex has the right-hand side
  R (b - A u) + A_{l-1} I u; unrefined vertices keep the PDE right-hand side.

Readings (the paper is silent or its Alg. 1 is garbled here; see the design
notes):

* Levels 0..base are complete; refinement flags are given for levels
  base..L-1 (a flag on a cell that does not exist is ignored).
* The unknowns are the unrefined non-hanging interior vertices of levels
  base..L ("leaves"), numbered level by level, x fastest within a level.  Leaf
  cells (cells that exist and are not refined) carry the coefficients; a
  refined cell's coefficient is the mean of its 3^d children.
* Leaf v of level l satisfies sum_w a_l(v,w) u_bar(w) = h_l^d f_v, with a_l the
  level-l rediscretised stencil and u_bar the composite value: the unknown for
  a leaf, the finer copy for a refined vertex, the d-linear interpolant of the
  coarser level for a hanging vertex, zero on the boundary.
* The cycle on adaptive levels is the textbook FAS V-cycle (smooth all
  non-hanging vertices of the level with hanging values frozen, inject, FAS
  right-hand side on refined coarse vertices, recurse, correct with
  P (u_{l-1} - I u_l), re-interpolate hanging vertices); at the complete base
  level it continues as the regular correction-scheme cycle.  The paper's code
  additionally smooths coarser unrefined regions while finer levels are
  active; that changes iterates, not the fixed point.  Iterate parity is
  therefore pinned only against this reading; the fixed point is pinned by the
  composite system.
* Coarse stencils of refined vertices are Galerkin products with the d-linear
  P (the hanging interpolation uses the same weights), or rediscretised for the
  geometric variant.
* BoxMG on adaptive levels (Sect. 4.4, the passage on spacetree grids): P is
  built per refined coarse cell only (a patch), from the level's stencils.  At
  hanging vertices, whose rows the collapsed systems of the patch faces need,
  the paper takes stencils obtained from the coarser level by d-linear
  interpolation.  Reading: the hanging vertex's row is rediscretised on its
  level from its 2^d cells, a cell that does not exist taking the coefficient
  of the leaf cell that covers it (the coarse data prolongated to the missing
  fine cells).  Interpolating the parents' stencil entries themselves breaks
  down where a parent is a Dirichlet vertex (it has no stencil), and this
  reading keeps the invariant that a constant coefficient gives d-linear BoxMG
  weights.  The value of a hanging vertex is the BoxMG interpolant
  P u_{l-1} (not the geometric one), so the composite system of the BoxMG
  variant has BoxMG constraints at hanging vertices.  A point shared by
  several refined patches takes the value of the one whose orthant has + signs
  on the most significant shared axes (the lowest rank below); the others must
  agree (rounding aside).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import itertools
from typing import Dict

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import (geometric_stencil, offsets, shifted, csr_to_stencil, stencil_to_csr,
                  interior_mask, corners, corner_index, element_matrix, apply_dirichlet)
from .transfer import (dlinear_P, boxmg_P, boxmg_reference_stepwise, _gather_reference, _points,
                       shared_entry_tolerance, unique_shared_entries)
from .fem import _unknown_numbering
from .galerkin import rap, definiteness_violations
from . import solver as S

OUT, LEAF, REFINED, HANGING = 0, 1, 2, 3


def _children(a, d):
    """Each cell value repeated on its 3^d children (lattice cell arrays)."""
    out = a
    for ax in range(d):
        out = np.repeat(out, 3, axis=ax)
    return out


class AdaptiveGrid:
    """Levels 0..L of a tripartitioned spacetree with refinement flags for
    levels base..L-1 (``flags[l]``: bool array (3^l,)*d over cells, NumPy axes
    z, y, x)."""

    def __init__(self, d, base, L, flags: Dict[int, np.ndarray]):
        self.d, self.base, self.L = d, base, L
        self.exist, self.refined, self.vtype = {}, {}, {}
        for l in range(0, L + 1):
            n = 3 ** l
            if l <= base:
                self.exist[l] = np.ones((n,) * d, dtype=bool)
            else:
                self.exist[l] = _children(self.refined[l - 1], d)
            if l < base:
                self.refined[l] = np.ones((n,) * d, dtype=bool)
            elif l < L:
                self.refined[l] = self.exist[l] & np.asarray(flags.get(l, np.zeros((n,) * d, bool)), bool)
            else:
                self.refined[l] = np.zeros((n,) * d, dtype=bool)
            self.vtype[l] = self._classify(l)

    def _classify(self, l):
        d = self.d
        n = 3 ** l
        cnt = np.zeros((n + 1,) * d, dtype=np.int64)
        nref = np.zeros((n + 1,) * d, dtype=np.int64)
        ex = np.pad(self.exist[l].astype(np.int64), 1)
        rf = np.pad(self.refined[l].astype(np.int64), 1)
        for s in itertools.product((0, 1), repeat=d):
            sl = tuple(slice(1 - si, 1 - si + n + 1) for si in s)   # cell (v - s), axes z,y,x
            cnt += ex[sl]
            nref += rf[sl]
        t = np.full((n + 1,) * d, OUT, dtype=np.int8)
        inner = interior_mask(d, l) > 0
        full = cnt == 2 ** d
        t[inner & full & (nref == 2 ** d)] = REFINED
        t[inner & full & (nref < 2 ** d)] = LEAF
        t[inner & (cnt > 0) & ~full] = HANGING
        return t

    # -- numbering -------------------------------------------------------------
    def leaves(self):
        """(level, lattice index tuple in NumPy order) of every unknown."""
        out = []
        for l in range(self.base, self.L + 1):
            idx = np.argwhere(self.vtype[l] == LEAF)
            out += [(l, tuple(i)) for i in idx]
        return out

    def leaf_cells(self):
        out = []
        for l in range(self.base, self.L + 1):
            idx = np.argwhere(self.exist[l] & ~self.refined[l])
            out += [(l, tuple(i)) for i in idx]
        return out

    def n_unknowns(self):
        return sum(int((self.vtype[l] == LEAF).sum()) for l in range(self.base, self.L + 1))

    def level_eps(self, eps_leaf):
        """Cell coefficients of every level from the leaf-cell values (in
        ``leaf_cells`` order): leaf cells keep theirs, refined cells take the
        mean of their children, non-existing cells 0."""
        d = self.d
        eps = {l: np.zeros((3 ** l,) * d) for l in range(self.L + 1)}
        for k, (l, c) in enumerate(self.leaf_cells()):
            eps[l][c] = eps_leaf[k]
        for l in range(self.L - 1, -1, -1):
            n = 3 ** l
            ch = eps[l + 1].reshape(sum(((n, 3) for _ in range(d)), ()))
            mean = ch.mean(axis=tuple(2 * i + 1 for i in range(d)))
            eps[l] = np.where(self.refined[l], mean, eps[l])
        return eps

    def cell_centres(self):
        """Centres of the leaf cells in ``leaf_cells`` order, x first."""
        out = []
        for l in range(self.base, self.L + 1):
            idx = np.argwhere(self.exist[l] & ~self.refined[l])
            out.append((idx[:, ::-1] + 0.5) * 3.0 ** -l)
        return np.concatenate(out)

    def unknown_coords(self):
        """Positions of the unknowns in ``leaves`` order, x first."""
        out = []
        for l in range(self.base, self.L + 1):
            idx = np.argwhere(self.vtype[l] == LEAF)
            out.append(idx[:, ::-1] * 3.0 ** -l)
        return np.concatenate(out)


# ---------------------------------------------------------------------------
# Composite system (the plain definition of the result)
# ---------------------------------------------------------------------------

class _CompositeValues:
    """u_bar(l, v) of the composite system as {unknown: weight}: the unknown
    for a leaf, the finer copy for a refined vertex, the interpolant of the
    coarser level for a hanging vertex (d-linear, or the rows of the given
    prolongations ``P[l]``), nothing on the boundary."""

    def __init__(self, G: AdaptiveGrid, P=None):
        self.G = G
        self.P = P
        self.num = {lv: k for k, lv in enumerate(G.leaves())}
        self.memo = {}

    def __call__(self, l, v):
        G, d = self.G, self.G.d
        key = (l, v)
        if key in self.memo:
            return self.memo[key]
        t = G.vtype[l][v]
        if t == LEAF:
            res = {self.num[key]: 1.0}
        elif t == REFINED:
            res = self(l + 1, tuple(3 * vi for vi in v))
        elif t == HANGING and self.P is not None:
            res = {}
            n = 3 ** l
            Pl = self.P[l]
            row = _unknown_numbering(d, l)[v]
            numc = 3 ** (l - 1) - 1
            for jj in range(Pl.indptr[row], Pl.indptr[row + 1]):
                c = Pl.indices[jj]
                par = tuple(reversed([c // numc ** i % numc + 1 for i in range(d)]))   # numpy order
                for j, cw in self(l - 1, par).items():
                    res[j] = res.get(j, 0.0) + Pl.data[jj] * cw
        elif t == HANGING:
            res = {}
            q = [vi // 3 for vi in v]
            r = [vi - 3 * qi for vi, qi in zip(v, q)]
            for kap in itertools.product((0, 1), repeat=d):
                w = 1.0
                for ri, ki in zip(r, kap):
                    w *= (1.0 - ri / 3.0) if ki == 0 else (ri / 3.0)
                if w == 0.0:
                    continue
                par = tuple(qi + ki for qi, ki in zip(q, kap))
                for j, c in self(l - 1, par).items():
                    res[j] = res.get(j, 0.0) + w * c
        else:
            res = {}
        self.memo[key] = res
        return res


def composite_system(G: AdaptiveGrid, eps_leaf, f_leaf, P=None):
    """Sparse composite matrix over the leaf unknowns and its right-hand side
    (hanging constraints d-linear, or from the prolongations ``P``)."""
    d = G.d
    value = _CompositeValues(G, P)
    num = value.num
    N = len(num)
    eps = G.level_eps(eps_leaf)
    rows, cols, vals = [], [], []
    b = np.zeros(N)
    stencils = {l: geometric_stencil(eps[l], d, l) for l in range(G.base, G.L + 1)}
    offs = offsets(d)
    for (l, v), k in num.items():
        S_l = stencils[l]
        for e, o in enumerate(offs):
            a = S_l[(e,) + v]
            if a == 0.0:
                continue
            w = tuple(vi + oi for vi, oi in zip(v, reversed(o)))   # v is (z,y,x)
            for j, c in value(l, w).items():
                rows.append(k)
                cols.append(j)
                vals.append(a * c)
        b[k] = (3.0 ** -l) ** d * f_leaf[k]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    return A, b


def composite_residual_rows(G: AdaptiveGrid, eps_leaf, f_leaf, u_leaf, sample, P=None):
    """b_k - (A u)_k of the composite system at the unknowns ``sample``, each
    row assembled on its own: the element matrices (Sect. 3, Q1) of the 2^d
    cells around the leaf, applied to the composite values of their corners.
    Usable on grids far too large for ``composite_system``."""
    d = G.d
    value = _CompositeValues(G, P)
    leaves = G.leaves()
    eps = G.level_eps(eps_leaf)
    cs = corners(d)
    out = np.zeros(len(sample))
    for q, k in enumerate(sample):
        l, v = leaves[k]
        h = 3.0 ** -l
        acc = 0.0
        for s in cs:                               # v is corner s of cell v - s
            cell = tuple(vi - si for vi, si in zip(v, reversed(s)))
            K = element_matrix(d, h, eps[l][cell])
            ia = corner_index(s)
            for ib, w in enumerate(cs):
                corner = tuple(ci + wi for ci, wi in zip(cell, reversed(w)))
                for j, c in value(l, corner).items():
                    acc += K[ia, ib] * c * u_leaf[j]
        out[q] = h ** d * f_leaf[k] - acc
    return out


# ---------------------------------------------------------------------------
# FAS V-cycle on the adaptive levels
# ---------------------------------------------------------------------------

class AdaptiveHierarchy:
    pass


def virtual_eps(G: AdaptiveGrid, eps):
    """Cell coefficients of every level where a cell that does not exist takes
    the coefficient of the leaf cell covering it (base level up)."""
    d = G.d
    out = {G.base: eps[G.base]}
    for l in range(G.base + 1, G.L + 1):
        out[l] = np.where(G.exist[l], eps[l], _children(out[l - 1], d))
    return out


def hanging_stencils(G: AdaptiveGrid, eps):
    """Rows of the hanging vertices of levels base+1..L for the collapsed BoxMG
    systems, rediscretised from the virtual coefficients (zero elsewhere)."""
    d = G.d
    ev = virtual_eps(G, eps)
    out = {}
    for l in range(G.base + 1, G.L + 1):
        out[l] = geometric_stencil(ev[l], d, l) * (G.vtype[l] == HANGING)[None]
    return out


def hanging_stencils_parents(G: AdaptiveGrid, eps):
    """Rows of the hanging vertices of levels base+1..L for the collapsed BoxMG
    systems read as the paper's d-linear interpolation of the parent
    stencils: the rediscretised level-(l-1) rows of the coarse vertices
    spanning the hanging vertex's coarse face or edge, weighted by its
    d-linear weights.  A Dirichlet parent has no stencil; the weights of the
    interior parents are renormalised to sum one.  The parents' rows are
    taken whole (entries towards Dirichlet vertices kept) and the entries of
    the interpolated row that point at Dirichlet vertices from the hanging
    vertex are dropped, as for every row.  A parent that is itself hanging
    has no stencil of its own either; parents' rows are rediscretised from
    the virtual coefficients (a missing cell takes the leaf cell covering
    it), which for a hanging parent is the interpolation of its own parents'
    rows when the coefficient is constant.  (A row's scale does not change
    the collapsed systems, each row being one equation.)"""
    d = G.d
    ev = virtual_eps(G, eps)
    out = {}
    for l in range(G.base + 1, G.L + 1):
        n = 3 ** l
        nc = n // 3
        Sc = geometric_stencil(ev[l - 1], d, l - 1, dirichlet=False)
        grids = np.meshgrid(*([np.arange(n + 1)] * d), indexing="ij")      # axes z,y,x
        acc = np.zeros((3 ** d,) + (n + 1,) * d)
        wsum = np.zeros((n + 1,) * d)
        for kap in itertools.product((0, 1), repeat=d):                    # NumPy order
            w = np.ones((n + 1,) * d)
            par = []
            for ax in range(d):
                q = grids[ax] // 3
                r = grids[ax] - 3 * q
                w = w * (np.where(kap[ax] == 0, 1.0 - r / 3.0, r / 3.0))
                par.append(np.minimum(q + kap[ax], nc))
            inner = np.ones((n + 1,) * d, bool)
            for ax in range(d):
                inner &= (par[ax] >= 1) & (par[ax] <= nc - 1)
            w = np.where(inner, w, 0.0)
            acc += w[None] * Sc[(slice(None),) + tuple(par)]
            wsum += w
        hv = G.vtype[l] == HANGING
        rows = apply_dirichlet(acc / np.where(wsum > 0, wsum, 1.0)[None], d, l)
        out[l] = np.where(hv[None] & (wsum > 0)[None], rows, 0.0)
    return out


def boxmg_adaptive_P(G: AdaptiveGrid, S_full, l, check=True):
    """BoxMG prolongation from level l-1 to level l computed on the refined
    coarse cells only (Sect. 4.4 per patch and corner), from the level's
    stencil array ``S_full`` (rows of leaf, refined and hanging vertices).
    Sparse, fine interior unknowns x coarse interior unknowns; rows of fine
    vertices outside every refined cell are empty."""
    d = G.d
    nf = 3 ** l
    nc = nf // 3
    numf = _unknown_numbering(d, l)
    numc = _unknown_numbering(d, l - 1)
    Vall = np.array(list(itertools.product(range(1, nc), repeat=d)))[:, ::-1]   # x first
    ref = G.refined[l - 1]
    rows, cols, ranks, vals = [], [], [], []
    for sigma in itertools.product((1, -1), repeat=d):
        sigma = tuple(reversed(sigma))
        sig = np.array(sigma)
        cell = Vall + (sig - 1) // 2                       # the orthant's coarse cell, x first
        ok = ref[tuple(cell[:, i] for i in reversed(range(d)))]
        V = Vall[ok]
        if len(V) == 0:
            continue
        p = boxmg_reference_stepwise(_gather_reference(S_full, d, V, sigma), d)
        c = numc[tuple(V[:, i] for i in reversed(range(d)))]
        for j, y in enumerate(_points(d, 3)):
            # a point on the patch's own axes is shared with the orthants that
            # differ there; rank orders those (+ first, axis i weighing 2^i)
            rank = sum(1 << i for i in range(d) if y[i] == 0 and sigma[i] < 0)
            F = 3 * V + sig * np.array(y)
            rows.append(numf[tuple(F[:, i] for i in reversed(range(d)))])
            cols.append(c)
            ranks.append(np.full(len(V), rank))
            vals.append(p[:, j])
    Nf, Nc = (nf - 1) ** d, (nc - 1) ** d
    if not rows:
        return sp.csr_matrix((Nf, Nc))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    ranks, vals = np.concatenate(ranks), np.concatenate(vals)
    uniq, v, dis = unique_shared_entries(rows, cols, vals, Nc, ranks)
    if check and dis > shared_entry_tolerance(S_full, d):
        raise AssertionError("adaptive BoxMG: neighbouring patches disagree on a shared entry")
    return sp.csr_matrix((v, (uniq // Nc, uniq % Nc)), shape=(Nf, Nc))


def build_adaptive(G: AdaptiveGrid, eps_leaf, transfer="galerkin", omega=0.6, mu_pre=2, mu_post=2,
                   lc=1, check_definite=False, direct_max=S.COARSE_DIRECT_MAX, hanging_rows="covering",
                   multiscale=False):
    """Operators of every level: rediscretised rows for unrefined vertices,
    Galerkin rows P^T A P (d-linear or BoxMG P) or rediscretised rows for
    refined ones; prolongations ``H.P[l]`` (also used for the hanging values);
    the levels up to the base level form a regular hierarchy below.

    ``check_definite``: the definiteness check of Sect. 4.3 on the Galerkin
    operators of the complete levels below the base level (a row with a
    non-positive diagonal or without diagonal dominance); the first level
    whose coarser operator fails becomes the coarsest level, which is at most
    the base level (the levels above it hold unknowns).  ``direct_max``: the
    largest coarsest level solved exactly (see ``solver.factor_coarse``).
    ``hanging_rows`` (BoxMG): "covering", the rows of hanging vertices
    rediscretised from the leaf cells covering the missing cells (this
    build's reading), or "parents", the paper's d-linear interpolation of the
    parent stencils (``hanging_stencils_parents``).  ``multiscale``: the FAS
    cycle also smooths the leaves of the coarser levels while a finer level
    is smoothed (see ``fas_cycle``)."""
    if transfer not in ("geometric", "galerkin", "boxmg"):
        raise ValueError(transfer)
    d = G.d
    eps = G.level_eps(eps_leaf)
    H = AdaptiveHierarchy()
    H.G, H.d, H.base, H.L = G, d, G.base, G.L
    H.omega, H.mu_pre, H.mu_post = omega, mu_pre, mu_post
    H.eps = eps
    H.transfer = transfer
    geo = {l: geometric_stencil(eps[l], d, l) for l in range(lc, G.L + 1)}
    act = {l: np.isin(G.vtype[l], (LEAF, REFINED)) for l in range(lc, G.L + 1)}
    if hanging_rows not in ("covering", "parents"):
        raise ValueError(hanging_rows)
    H.multiscale = bool(multiscale)
    Hs = {}
    if transfer == "boxmg":
        Hs = hanging_stencils(G, eps) if hanging_rows == "covering" else hanging_stencils_parents(G, eps)
    H.S = {G.L: geo[G.L] * act[G.L][None]}
    H.P = {}
    lc_used = lc
    for l in range(G.L, lc, -1):
        if transfer == "boxmg":
            H.P[l] = boxmg_adaptive_P(G, H.S[l] + Hs[l], l) if l > G.base else boxmg_P(H.S[l], d, l)
        else:
            H.P[l] = dlinear_P(d, l)
        if transfer == "geometric":
            Sc = geo[l - 1]
        else:
            gal = csr_to_stencil(rap(stencil_to_csr(H.S[l], d, l), H.P[l]), d, l - 1)
            Sc = np.where((G.vtype[l - 1] == REFINED)[None], gal, geo[l - 1])
        if (check_definite and transfer != "geometric" and l - 1 < G.base
                and len(definiteness_violations(stencil_to_csr(Sc, d, l - 1))) > 0):
            del H.P[l]
            lc_used = l
            break
        # rows only for leaf and refined vertices
        H.S[l - 1] = Sc * act[l - 1][None]
    # regular hierarchy from the base level down (correction scheme)
    lc = lc_used
    A = {l: stencil_to_csr(H.S[l], d, l) for l in range(lc, G.base + 1)}
    P = {l: H.P[l] for l in range(lc + 1, G.base + 1)}
    Hr = S.Hierarchy(d, G.base, lc, transfer, A, P, {l: eps[l] for l in range(lc, G.base + 1)},
                     omega, mu_pre, mu_post, direct_max=direct_max)
    Hr.coarse_lu = S.factor_coarse(A[lc], direct_max)
    H.regular = Hr
    H.lc = lc
    return H


def hanging_constraints(H):
    """The prolongations that define hanging values in the composite system
    (None: d-linear)."""
    return H.P if H.transfer == "boxmg" else None


def _apply(Sl, u, d):
    """(A u) on a lattice array from a stencil array."""
    out = np.zeros_like(u)
    for e, o in enumerate(offsets(d)):
        out += Sl[e] * shifted(u, o)
    return out


def _dlin_weights(d, l):
    """Per fine lattice vertex of level l, the d-linear weights of its parents
    floor(v/3) + kappa, as a list over kappa of (kappa, weight array)."""
    n = 3 ** l
    grids = np.meshgrid(*([np.arange(n + 1)] * d), indexing="ij")   # axes z,y,x
    out = []
    for kap in itertools.product((0, 1), repeat=d):                # kap in NumPy order
        w = np.ones((n + 1,) * d)
        for ax in range(d):
            r = grids[ax] % 3
            w = w * (np.where(kap[ax] == 0, 1.0 - r / 3.0, r / 3.0))
        out.append((kap, w))
    return out


def _from_coarse(uc, d, l):
    """d-linear interpolation of the level l-1 lattice array to level l."""
    n = 3 ** l
    grids = np.meshgrid(*([np.arange(n + 1)] * d), indexing="ij")
    res = np.zeros((n + 1,) * d)
    ucp = np.pad(uc, [(0, 1)] * d)
    for kap, w in _dlin_weights(d, l):
        idx = tuple(g // 3 + k for g, k in zip(grids, kap))
        res += w * ucp[idx]
    return res


def _restrict_dlin(r, d, l):
    """P^T r from level l to level l-1 (d-linear, all coarse lattice points)."""
    nc = 3 ** (l - 1)
    out = np.zeros((nc + 1,) * d)
    rp = np.pad(r, [(2, 2)] * d)
    for o in itertools.product(range(-2, 3), repeat=d):
        w = np.prod([1.0 - abs(oi) / 3.0 for oi in o])
        sl = tuple(slice(2 + oi, 2 + oi + 3 * nc + 1, 3) for oi in o)
        out += w * rp[sl]
    return out


def _prolong(H, uc, l):
    """P u_{l-1} on the level-l lattice: d-linear, or the BoxMG rows."""
    if H.transfer != "boxmg":
        return _from_coarse(uc, H.d, l)
    d = H.d
    out = np.zeros((3 ** l + 1,) * d)
    out[(slice(1, 3 ** l),) * d] = (H.P[l] @ uc[(slice(1, 3 ** (l - 1)),) * d].ravel()).reshape((3 ** l - 1,) * d)
    return out


def _restrict(H, r, l):
    """P^T r on the level l-1 lattice: d-linear, or the BoxMG columns."""
    if H.transfer != "boxmg":
        return _restrict_dlin(r, H.d, l)
    d = H.d
    out = np.zeros((3 ** (l - 1) + 1,) * d)
    out[(slice(1, 3 ** (l - 1)),) * d] = (H.P[l].T @ r[(slice(1, 3 ** l),) * d].ravel()).reshape(
        (3 ** (l - 1) - 1,) * d)
    return out


def hang(H, u, l):
    """Hanging vertices of level l take the interpolant of level l-1."""
    G = H.G
    hv = G.vtype[l] == HANGING
    u[l] = np.where(hv, _prolong(H, u[l - 1], l), u[l])


def inject(H, u, l):
    """Refined vertices of level l-1 take the value of their copy on level l."""
    G = H.G
    ref = G.vtype[l - 1] == REFINED
    sl = (slice(None, None, 3),) * H.d
    u[l - 1] = np.where(ref, u[l][sl], u[l - 1])


def _jacobi_masked(H, l, u, b):
    d = H.d
    act = np.isin(H.G.vtype[l], (LEAF, REFINED))
    Sl = H.S[l]
    c = (3 ** d) // 2
    diag = np.where(act, Sl[c], 1.0)
    new = u + H.omega * (b - _apply(Sl, u, d)) / diag
    return np.where(act, new, u)


def _smooth_multiscale(H, l, u, b):
    """One smoothing step of Alg. 1 with level l active: the refined vertices
    of the coarser levels first take their finer copies (injection), then
    one damped Jacobi step updates the non-hanging vertices of level l and,
    from the same old values, the leaves of every coarser level (base..l-1),
    which see the finer solution through their refined neighbours."""
    d, G = H.d, H.G
    for m in range(l, H.base, -1):
        inject(H, u, m)
    c = (3 ** d) // 2
    new = {}
    for m in range(H.base, l):
        lf = G.vtype[m] == LEAF
        Sm = H.S[m]
        diag = np.where(lf, Sm[c], 1.0)
        new[m] = np.where(lf, u[m] + H.omega * (b[m] - _apply(Sm, u[m], d)) / diag, u[m])
    u[l] = _jacobi_masked(H, l, u[l], b[l])
    for m, v in new.items():
        u[m] = v
    for m in range(H.base + 1, l + 1):
        hang(H, u, m)


def fas_cycle(H, l, u, b):
    """One FAS V-cycle from level l (u, b: dicts of lattice arrays, changed in
    place).  At the base level the regular correction-scheme cycle runs on the
    base lattice.  With ``H.multiscale`` every smoothing step of an adaptive
    level also smooths the coarser levels' leaves (``_smooth_multiscale``),
    as Alg. 1 does while a finer level is active."""
    d = H.d
    G = H.G
    if l == H.base:
        ub = u[l][(slice(1, 3 ** l),) * d].ravel()
        bb = b[l][(slice(1, 3 ** l),) * d].ravel()
        ub = S.vcycle(H.regular, l, ub, bb)
        u[l][(slice(1, 3 ** l),) * d] = ub.reshape((3 ** l - 1,) * d)
        return
    ms = getattr(H, "multiscale", False)
    act = np.isin(G.vtype[l], (LEAF, REFINED))
    hang(H, u, l)
    for _ in range(H.mu_pre):
        if ms:
            _smooth_multiscale(H, l, u, b)
        else:
            u[l] = _jacobi_masked(H, l, u[l], b[l])
    r = np.where(act, b[l] - _apply(H.S[l], u[l], d), 0.0)
    inject(H, u, l)
    saved = u[l - 1].copy()
    ref = G.vtype[l - 1] == REFINED
    b[l - 1] = np.where(ref, _restrict(H, r, l) + _apply(H.S[l - 1], u[l - 1], d), b[l - 1])
    fas_cycle(H, l - 1, u, b)
    corr = _prolong(H, u[l - 1] - saved, l)
    u[l] = np.where(act, u[l] + corr, u[l])
    hang(H, u, l)
    for _ in range(H.mu_post):
        if ms:
            _smooth_multiscale(H, l, u, b)
        else:
            u[l] = _jacobi_masked(H, l, u[l], b[l])


def composite_state(H, u):
    """Make refined and hanging values consistent with the leaves: inject from
    the finest level down, then interpolate hanging vertices from the base up."""
    for l in range(H.L, H.base, -1):
        inject(H, u, l)
    for l in range(H.base + 1, H.L + 1):
        hang(H, u, l)


def leaf_vector(H, u):
    return np.concatenate([u[l][H.G.vtype[l] == LEAF] for l in range(H.base, H.L + 1)])


def composite_residual(H, u, b):
    """Residual of the composite equations at the leaves (after
    ``composite_state``), level by level in unknown order."""
    out = []
    for l in range(H.base, H.L + 1):
        lf = H.G.vtype[l] == LEAF
        r = b[l] - _apply(H.S[l], u[l], H.d)
        out.append(r[lf])
    return np.concatenate(out)


def initial_state(H, f_leaf):
    """Zero iterate; PDE right-hand side h^d f at the leaves of every level."""
    d = H.d
    u = {l: np.zeros((3 ** l + 1,) * d) for l in range(1, H.L + 1)}
    b = {l: np.zeros((3 ** l + 1,) * d) for l in range(1, H.L + 1)}
    k = 0
    for l in range(H.base, H.L + 1):
        lf = H.G.vtype[l] == LEAF
        m = int(lf.sum())
        b[l][lf] = (3.0 ** -l) ** d * np.asarray(f_leaf[k:k + m])
        k += m
    return u, b


def solve_adaptive(H, f_leaf, tol=1e-8, max_cycles=200, cycles=None, stagnation=0.0):
    """FAS V-cycles from zero; returns (leaf values, relres history).  With
    ``stagnation`` > 0 the coarsest level of the regular levels moves up (to
    the base level at most) after a cycle that reduced the composite residual
    by less than that factor (Sect. 4.3)."""
    u, b = initial_state(H, f_leaf)
    b0 = {l: v.copy() for l, v in b.items()}
    bl = np.concatenate([b0[l][H.G.vtype[l] == LEAF] for l in range(H.base, H.L + 1)])
    nb = np.linalg.norm(bl)
    hist = []
    prev = 1.0
    n = cycles if cycles is not None else max_cycles
    for k in range(n):
        fas_cycle(H, H.L, u, b)
        composite_state(H, u)
        # leaf right-hand sides are the PDE ones (FAS only rewrites refined rows)
        hist.append(float(np.linalg.norm(composite_residual(H, u, b0)) / nb))
        if cycles is None and hist[-1] <= tol:
            break
        if k + 1 < n and S.stagnated(hist[-1], prev, stagnation, tol):
            S.raise_coarsest(H.regular, top=min(H.base, H.L - 1))
        prev = hist[-1]
    return leaf_vector(H, u), hist


def solve_composite_direct(G, eps_leaf, f_leaf, P=None):
    A, b = composite_system(G, eps_leaf, f_leaf, P)
    return spla.spsolve(sp.csc_matrix(A), b), A, b


# ---------------------------------------------------------------------------
# Spacetrees too large to lay out: classes and composite rows decided locally
# ---------------------------------------------------------------------------

class LocalSpacetree:
    """The spacetree of Sect. 3 decided cell by cell for grids too large for
    ``AdaptiveGrid``: levels 0..base are complete; a cell of level base..L-1
    is refined when it exists and the refinement predicate ``mark(l, cells)``
    holds; a cell of a finer level exists when its parent is refined.  Vertex
    classes follow the same definitions as ``AdaptiveGrid`` (hanging: fewer
    than 2^d cells of its level; refined: all 2^d cells refined; leaf: the
    other interior vertices).  Positions are x-first integer tuples."""

    def __init__(self, d, base, L, mark):
        self.d, self.base, self.L, self.mark = d, base, L, mark
        self._ref = {}

    def exists(self, l, c):
        n = 3 ** l
        if any(ci < 0 or ci >= n for ci in c):
            return False
        return l <= self.base or self.refined(l - 1, tuple(ci // 3 for ci in c))

    def refined(self, l, c):
        if l >= self.L:
            return False
        if l < self.base:
            return self.exists(l, c)
        key = (l, c)
        if key not in self._ref:
            self._ref[key] = bool(self.exists(l, c) and self.mark(l, np.array([c]))[0])
        return self._ref[key]

    def vclass(self, l, v):
        n = 3 ** l
        if any(vi <= 0 or vi >= n for vi in v):
            return OUT
        cnt = nref = 0
        for s in corners(self.d):
            c = tuple(vi - si for vi, si in zip(v, s))
            if self.exists(l, c):
                cnt += 1
                nref += self.refined(l, c)
        if cnt == 2 ** self.d:
            return REFINED if nref == 2 ** self.d else LEAF
        return HANGING if cnt > 0 else OUT

    def cell_eps(self, l, c, eps_at):
        """Coefficient of an existing cell: its own for a leaf cell (at its
        centre), the mean of its 3^d children for a refined one."""
        if not self.refined(l, c):
            x = (np.array(c, dtype=np.float64) + 0.5) * 3.0 ** -l
            return float(eps_at(x[None, :])[0])
        kids = [tuple(3 * ci + oi for ci, oi in zip(c, o)) for o in itertools.product(range(3), repeat=self.d)]
        return float(np.mean([self.cell_eps(l + 1, k, eps_at) for k in kids]))


def local_composite_rows(T: LocalSpacetree, eps_at, f_at, u_of, samples):
    """b - A u of the composite system (Sect. 3) at leaf unknowns given as
    (level, x-first position) pairs, each row assembled on its own from the
    element matrices of the 2^d cells around the vertex (coefficients from
    ``eps_at``, the source from ``f_at(level, coords)``) and the composite
    values of their corners: ``u_of(level, position)`` for a leaf, the finest
    copy for a refined vertex, zero on the boundary.  A row that needs a
    hanging value (an interpolant of the coarser level) is returned as NaN.
    Also returns, per row, sum |K| |u| (the scale of the row's rounding)."""
    d = T.d
    cs = corners(d)
    out = np.full(len(samples), np.nan)
    scale = np.zeros(len(samples))

    def value(l, w):
        t = T.vclass(l, w)
        if t == LEAF:
            return u_of(l, w)
        if t == REFINED:
            return value(l + 1, tuple(3 * wi for wi in w))
        if t == HANGING:
            return None
        return 0.0

    for q, (l, v) in enumerate(samples):
        if T.vclass(l, v) != LEAF:
            raise AssertionError(f"sample {l} {v} is not a leaf vertex")
        h = 3.0 ** -l
        acc, sc, ok = 0.0, 0.0, True
        for s in cs:                                   # v is corner s of cell v - s
            cell = tuple(vi - si for vi, si in zip(v, s))
            K = element_matrix(d, h, T.cell_eps(l, cell, eps_at))
            ia = corner_index(s)
            for ib, w in enumerate(cs):
                uw = value(l, tuple(ci + wi for ci, wi in zip(cell, w)))
                if uw is None:
                    ok = False
                    break
                acc += K[ia, ib] * uw
                sc += abs(K[ia, ib] * uw)
            if not ok:
                break
        if ok:
            x = np.array(v, dtype=np.float64) * h
            bq = h ** d * float(f_at(l, x[None, :])[0])
            out[q] = bq - acc
            scale[q] = sc + abs(bq)
    return out, scale
