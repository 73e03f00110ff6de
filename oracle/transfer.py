"""Inter-grid transfer operators (oracle, FP64).

* d-linear prolongation (Sect. 4.3 "Galerkin multigrid variants"): the weight
  of coarse vertex V at fine vertex 3V + o is prod_i (1 - |o_i|/3), |o_i| <= 2.
* BoxMG prolongation for tripartitioning (Sect. 4.4 and the appendix "BoxMG
  realisation as one linear equation system solve"): per coarse cell (patch of
  4^d fine vertices) and per patch corner, mirror the patch so that the corner
  is the reference (lower-left) vertex, then

  1. p = 1 at the c-point (the corner itself);
  2. points on coarse-grid lines (gamma points) use their stencils collapsed
     along the line (all offsets perpendicular to the line summed), giving a
     2x2 system per line;
  3. in 3D, points on coarse-grid faces use their stencils collapsed along the
     face normal, giving a 4x4 system per face;
  4. the interior (iota) points use their full stencils: a 4x4 (2D) or 8x8
     (3D) system;
  5. the right-hand sides are zero (b_gamma = b_iota = 0) and p vanishes at the
     opposite side of the patch (that region belongs to other coarse vertices);
  6. mirror back.

Both forms the paper describes are implemented: the stepwise solve (steps 2-4
in sequence) and the single system C(s) p = e_0 of the appendix.  They must
agree; a test checks that.

Readings: the appendix's right-hand side says "i = 1" although it enumerates
from 0 and prints (1, 0, 0)^T; it is read as e_0.  Row 5 of the printed 2D C(s)
lacks one column separator; it is read as the nine entries s_{5,0..8}.

Mirroring is expressed with an orthant sign sigma in {-1,+1}^d: the reference
point y in {0..3}^d of coarse vertex V is fine vertex 3V + sigma*y and the
mirrored stencil offset o' is the true offset sigma*o'.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .fem import offsets, flat_offset, _unknown_numbering


def _points(d, m):
    """All y in {0..m-1}^d, x fastest."""
    return [tuple(reversed(t)) for t in itertools.product(range(m), repeat=d)]


def _idx(y, m):
    return sum(yi * m ** i for i, yi in enumerate(y))


def dlinear_P(d, level_f):
    """d-linear prolongation from level_f-1 to level_f as a sparse matrix
    (fine interior unknowns x coarse interior unknowns)."""
    nf = 3 ** level_f
    nc = nf // 3
    numf = _unknown_numbering(d, level_f)
    numc = _unknown_numbering(d, level_f - 1)
    Vs = np.array(list(itertools.product(range(1, nc), repeat=d)))[:, ::-1]  # x first
    rows, cols, vals = [], [], []
    for o in offsets(d, 2):
        w = np.prod([1.0 - abs(oi) / 3.0 for oi in o])
        F = 3 * Vs + np.array(o)
        r = numf[tuple(F[:, i] for i in reversed(range(d)))]
        c = numc[tuple(Vs[:, i] for i in reversed(range(d)))]
        ok = r >= 0
        rows.append(r[ok])
        cols.append(c[ok])
        vals.append(np.full(ok.sum(), w))
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=((nf - 1) ** d, (nc - 1) ** d))
    return P


def injection_R(d, level_f):
    """Injection from level_f to level_f-1 (Petrov-Galerkin R = I of the
    convection results): coarse vertex V takes the fine value at 3V.  Sparse,
    coarse interior unknowns x fine interior unknowns."""
    nf = 3 ** level_f
    nc = nf // 3
    numf = _unknown_numbering(d, level_f)
    numc = _unknown_numbering(d, level_f - 1)
    Vs = np.array(list(itertools.product(range(1, nc), repeat=d)))[:, ::-1]  # x first
    r = numc[tuple(Vs[:, i] for i in reversed(range(d)))]
    c = numf[tuple(3 * Vs[:, i] for i in reversed(range(d)))]
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=((nc - 1) ** d, (nf - 1) ** d))


def aggregation_R(d, level_f):
    """Aggregation restriction from level_f to level_f-1: coarse vertex V sums
    the fine values of its aggregate, the 3^d fine vertices within 1 of 3V
    (unit weights; the aggregates partition the fine vertices, those next to
    the boundary belong to boundary vertices and drop out).  Sparse, coarse
    interior unknowns x fine interior unknowns."""
    nf = 3 ** level_f
    nc = nf // 3
    numf = _unknown_numbering(d, level_f)
    numc = _unknown_numbering(d, level_f - 1)
    Vs = np.array(list(itertools.product(range(1, nc), repeat=d)))[:, ::-1]  # x first
    r = numc[tuple(Vs[:, i] for i in reversed(range(d)))]
    rows, cols = [], []
    for o in offsets(d, 1):
        F = 3 * Vs + np.array(o)
        rows.append(r)
        cols.append(numf[tuple(F[:, i] for i in reversed(range(d)))])
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=((nc - 1) ** d, (nf - 1) ** d))


def boxmg_reference_matrix(t, d):
    """C(s) of the reference corner.  ``t`` has shape (batch, 4^d, 3^d): the
    mirrored stencils of the patch points y in {0..3}^d (x fastest).  Returns
    (batch, 3^d, 3^d) over the unknowns p(y), y in {0,1,2}^d.  Row y collapses
    the stencil onto the axes where y is non-zero (none: the c-point row is the
    identity; one: a coarse-grid line; two in 3D: a face; all: interior)."""
    B = t.shape[0]
    n3 = 3 ** d
    C = np.zeros((B, n3, n3))
    offs = offsets(d)
    for y in _points(d, 3):
        iy = _idx(y, 3)
        if not any(y):
            C[:, iy, iy] = 1.0
            continue
        keep = [i for i in range(d) if y[i] != 0]
        for k, o in enumerate(offs):
            w = tuple(y[i] + (o[i] if i in keep else 0) for i in range(d))
            if any(wi == 3 for wi in w):
                continue                         # p vanishes on the far side
            C[:, iy, _idx(w, 3)] += t[:, _idx(y, 4), k]
    return C


def boxmg_reference_Cs(t, d):
    """Solve C(s) p = e_0 in one dense solve (appendix form)."""
    C = boxmg_reference_matrix(t, d)
    rhs = np.zeros(C.shape[:2])
    rhs[:, 0] = 1.0
    return np.linalg.solve(C, rhs[..., None])[..., 0]


def boxmg_reference_stepwise(t, d):
    """Stepwise BoxMG (Sect. 4.4 steps): c-point, then each coarse-grid line
    (2x2), then each face in 3D (4x4), then the interior (2^d x 2^d).  Each
    group only couples to itself and to groups solved before it."""
    B = t.shape[0]
    p = np.zeros((B, 4 ** d))                      # over y in {0..3}^d; y_i = 3 stays 0
    p[:, 0] = 1.0
    offs = offsets(d)
    subsets = [s for r in range(1, d + 1) for s in itertools.combinations(range(d), r)]
    for S in subsets:
        group = [y for y in _points(d, 3) if tuple(i for i in range(d) if y[i]) == S]
        gidx = {y: j for j, y in enumerate(group)}
        m = len(group)
        M = np.zeros((B, m, m))
        rhs = np.zeros((B, m))
        for j, y in enumerate(group):
            for k, o in enumerate(offs):
                w = tuple(y[i] + (o[i] if i in S else 0) for i in range(d))
                coef = t[:, _idx(y, 4), k]
                if w in gidx:
                    M[:, j, gidx[w]] += coef
                else:
                    rhs[:, j] -= coef * p[:, _idx(w, 4)]
        sol = np.linalg.solve(M, rhs[..., None])[..., 0]
        for j, y in enumerate(group):
            p[:, _idx(y, 4)] = sol[:, j]
    keep = [_idx(y, 4) for y in _points(d, 3)]
    return p[:, keep]


def _gather_reference(S_lat, d, V, sigma):
    """Mirrored patch stencils t[b, y, o'] = S[sigma*o'] at fine vertex
    3V + sigma*y, for coarse vertices V (batch, d; x first)."""
    offs = offsets(d)
    B = V.shape[0]
    t = np.zeros((B, 4 ** d, 3 ** d))
    sig = np.array(sigma)
    for y in _points(d, 4):
        F = 3 * V + sig * np.array(y)
        sel = tuple(F[:, i] for i in reversed(range(d)))
        for k, o in enumerate(offs):
            ko = flat_offset(tuple(sig[i] * o[i] for i in range(d)))
            t[:, _idx(y, 4), k] = S_lat[ko][sel]
    return t


def shared_entry_tolerance(S_lat, d):
    """Largest disagreement allowed between two patches' copies of a shared
    BoxMG entry, relative to max(1, |entry|): rounding amplified by the
    coefficient contrast, 16 kappa 2^-52 with kappa the ratio of the largest
    to the smallest non-zero diagonal entry of the stencils (for piecewise
    constant eps, the contrast).  On random two-valued checkerboards of
    contrast 1e2 to 1e6 (d = 2 and 3) the copies differ by at most
    0.7 kappa 2^-52, and for constant eps not at all."""
    diag = np.abs(np.asarray(S_lat)[(3 ** d) // 2])
    nz = diag[diag > 0]
    kappa = float(nz.max() / nz.min()) if nz.size else 1.0
    return 16.0 * max(1.0, kappa) * 2.0 ** -52


def unique_shared_entries(rows, cols, vals, Nc, ranks=None):
    """Sorts the computed copies of every (row, col) entry (by the copy's rank
    when given, else in computation order) and returns the distinct keys, the
    first copy of each, and the largest disagreement of any copy with it
    relative to max(1, |first|)."""
    key = rows * Nc + cols
    order = np.argsort(key, kind="stable") if ranks is None else np.lexsort((ranks, key))
    key, vals = key[order], vals[order]
    uniq, first = np.unique(key, return_index=True)
    grp = np.repeat(np.arange(len(uniq)), np.diff(np.append(first, len(key))))
    ref = vals[first][grp]
    dis = float((np.abs(vals - ref) / np.maximum(1.0, np.abs(ref))).max()) if len(vals) else 0.0
    return uniq, vals[first], dis


def boxmg_P(S_fine, d, level_f, solver=boxmg_reference_stepwise, chunk=16384, check=True, info=None):
    """BoxMG prolongation from level_f-1 to level_f (sparse, fine x coarse)
    from the fine stencil array ``S_fine`` (lattice form).  Entries shared by
    neighbouring patches (c-points, line and face points) are computed by each
    of them; with ``check`` they must agree to rounding amplified by the
    coefficient contrast (``shared_entry_tolerance``); the copy of the orthant
    with + signs on the axes where the point lies is kept.  ``info`` (a dict)
    receives the largest disagreement as "shared_disagreement"."""
    nf = 3 ** level_f
    nc = nf // 3
    numf = _unknown_numbering(d, level_f)
    numc = _unknown_numbering(d, level_f - 1)
    Vall = np.array(list(itertools.product(range(1, nc), repeat=d)))[:, ::-1]  # x first
    pts3 = _points(d, 3)
    rows, cols, vals = [], [], []
    for sigma in itertools.product((1, -1), repeat=d):
        sigma = tuple(reversed(sigma))
        for c0 in range(0, len(Vall), chunk):
            V = Vall[c0:c0 + chunk]
            t = _gather_reference(S_fine, d, V, sigma)
            p = solver(t, d)
            c = numc[tuple(V[:, i] for i in reversed(range(d)))]
            for j, y in enumerate(pts3):
                F = 3 * V + np.array(sigma) * np.array(y)
                rows.append(numf[tuple(F[:, i] for i in reversed(range(d)))])
                cols.append(c)
                vals.append(p[:, j])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Nc = (nc - 1) ** d
    uniq, v, dis = unique_shared_entries(rows, cols, vals, Nc)
    if info is not None:
        info["shared_disagreement"] = dis
    if check and dis > shared_entry_tolerance(S_fine, d):
        raise AssertionError("BoxMG: neighbouring patches disagree on a shared entry")
    P = sp.csr_matrix((v, (uniq // Nc, uniq % Nc)), shape=((nf - 1) ** d, Nc))
    return P
