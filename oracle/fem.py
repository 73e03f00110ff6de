"""d-linear (Q1) finite elements on tripartitioned levels (oracle, FP64).

Paper passages followed:

* Eq. (1) of the introduction: -div(eps grad u) + (v . grad) u = f on the unit
  cube, eps a diagonal tensor, v a velocity field.
* Sect. 3 (spacetree, vertex classes, d-linear shape functions on every level)
  and Sect. 4, eq. "03_solver:stencils": a vertex's stencil is the sum of the
  contributions of its 2^d adjacent cells.

Readings (the paper is silent on these):

* The element matrix of cell c is the Q1 stiffness of the diagonal tensor eps_c
  that is constant on the cell.  In tensor-product form
  ``K_c(a,b) = h^(d-2) sum_i eps_{c,i} k(a_i,b_i) prod_{j!=i} m(a_j,b_j)``
  with the 1D stiffness ``k = [[1,-1],[-1,1]]`` and mass ``m = [[1/3,1/6],[1/6,1/3]]``.
* The convection term is the plain Galerkin one (no upwinding; the paper
  names none) with v constant on each cell: the element matrix is
  ``C_c(a,b) = h^(d-1) sum_i v_{c,i} g(a_i,b_i) prod_{j!=i} m(a_j,b_j)`` with
  ``g(a,b) = int_0^1 phi_b' phi_a = [[-1/2, 1/2], [-1/2, 1/2]]`` (row a = the
  test function's corner).
* The right-hand side is lumped: ``b_v = h^d f_v``.
* Zero Dirichlet boundary: boundary vertices carry no row, and stencil entries
  that point at boundary vertices are dropped.

Lattice arrays of level ``l`` have shape ``(n+1,)*d`` with ``n = 3**l`` and
NumPy axes ordered (z, y, x), so x is the fastest index.  Stencil arrays have a
leading axis of length 3^d; entry ``k`` belongs to offset ``o`` (coordinate
order x, y, z) with ``k = sum_i (o_i + 1) 3^i``.  Interior unknowns are the
interior lattice vertices, numbered with x fastest.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

K1D = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1D = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


def corners(d):
    """All a in {0,1}^d in lexicographic order with a[0] (x) fastest."""
    return [tuple(reversed(t)) for t in itertools.product((0, 1), repeat=d)]


def offsets(d, r=1):
    """All o in {-r..r}^d with o[0] (x) fastest; position = flat stencil index."""
    rng = range(-r, r + 1)
    return [tuple(reversed(t)) for t in itertools.product(rng, repeat=d)]


def flat_offset(o, r=1):
    w = 2 * r + 1
    return sum((oi + r) * w ** i for i, oi in enumerate(o))


def corner_index(a):
    return sum(ai << i for i, ai in enumerate(a))


def element_matrix(d, h, eps_c):
    """Q1 element stiffness of one cell (Sect. 3, d-linear shape functions) for
    the diagonal coefficient ``eps_c`` (scalar or length-d).  Rows and columns
    are the cell's corners in ``corners(d)`` order."""
    eps_c = np.broadcast_to(np.asarray(eps_c, dtype=np.float64), (d,))
    cs = corners(d)
    K = np.zeros((2 ** d, 2 ** d))
    for ia, a in enumerate(cs):
        for ib, b in enumerate(cs):
            tot = 0.0
            for i in range(d):
                term = eps_c[i] * K1D[a[i], b[i]]
                for j in range(d):
                    if j != i:
                        term *= M1D[a[j], b[j]]
                tot += term
            K[ia, ib] = h ** (d - 2) * tot
    return K


G1D = np.array([[-0.5, 0.5], [-0.5, 0.5]])


def convection_element_matrix(d, h, v_c):
    """Q1 element matrix of (v . grad) u on one cell for constant ``v_c``
    (length d): entry (a, b) integrates (v . grad phi_b) phi_a, a and b the
    cell's corners in ``corners(d)`` order."""
    v_c = np.asarray(v_c, dtype=np.float64)
    cs = corners(d)
    C = np.zeros((2 ** d, 2 ** d))
    for ia, a in enumerate(cs):
        for ib, b in enumerate(cs):
            tot = 0.0
            for i in range(d):
                term = v_c[i] * G1D[a[i], b[i]]
                for j in range(d):
                    if j != i:
                        term *= M1D[a[j], b[j]]
                tot += term
            C[ia, ib] = h ** (d - 1) * tot
    return C


def convection_stencil(v, d, level):
    """Stencils of the convection term on a regular level from per-cell
    velocities ``v`` (shape ``(d,) + (n,)*d``, component i along axis i), by
    the same sum over the 2^d cells around each vertex as
    ``geometric_stencil``; Dirichlet rows/entries removed."""
    n = 3 ** level
    h = 1.0 / n
    v = np.asarray(v, dtype=np.float64)
    if v.shape != (d,) + (n,) * d:
        raise ValueError(f"v must have shape {(d,) + (n,) * d}; got {v.shape}")
    padded = [np.pad(v[i], 1) for i in range(d)]
    cref = []
    for i in range(d):
        e = np.zeros(d)
        e[i] = 1.0
        cref.append(convection_element_matrix(d, h, e))
    S = np.zeros((3 ** d,) + (n + 1,) * d)
    for s in corners(d):
        sl = tuple(slice(1 - s[i], 1 - s[i] + n + 1) for i in reversed(range(d)))
        cell = [p[sl] for p in padded]
        for w in corners(d):
            o = tuple(w[i] - s[i] for i in range(d))
            k = flat_offset(o)
            ia, ib = corner_index(s), corner_index(w)
            for i in range(d):
                S[k] += cell[i] * cref[i][ia, ib]
    return apply_dirichlet(S, d, level)


def shifted(a, o):
    """``b[v] = a[v + o]`` for a lattice array (NumPy axes z, y, x); zero where
    ``v + o`` leaves the array."""
    d = a.ndim
    b = np.zeros_like(a)
    src = [slice(None)] * d
    dst = [slice(None)] * d
    for i, oi in enumerate(o):
        ax = d - 1 - i
        m = a.shape[ax]
        if oi >= 0:
            dst[ax] = slice(0, m - oi)
            src[ax] = slice(oi, m)
        else:
            dst[ax] = slice(-oi, m)
            src[ax] = slice(0, m + oi)
    b[tuple(dst)] = a[tuple(src)]
    return b


def interior_mask(d, level):
    n = 3 ** level
    m = np.zeros((n + 1,) * d)
    m[(slice(1, n),) * d] = 1.0
    return m


def _eps_components(eps, d):
    eps = np.asarray(eps, dtype=np.float64)
    n = eps.shape[-1]
    if eps.ndim == d:
        return [eps] * d
    if eps.ndim == d + 1 and eps.shape[0] == d:
        return [eps[i] for i in range(d)]
    raise ValueError(f"eps must have shape (n,)*{d} or ({d},)+(n,)*{d}; got {eps.shape} (n={n})")


def geometric_stencil(eps, d, level, dirichlet=True):
    """Stencils of all vertices of a regular level from per-cell coefficients
    (eq. "03_solver:stencils": the row of vertex v is the sum over the 2^d
    cells around v of that cell's element-matrix row).  Returns a stencil array
    of shape ``(3^d,) + (n+1,)*d`` with Dirichlet rows/entries removed
    (``dirichlet=False``: kept, the rows of interior vertices whole)."""
    n = 3 ** level
    h = 1.0 / n
    comps = _eps_components(eps, d)
    padded = [np.pad(c, 1) for c in comps]          # cell c at padded index c+1
    # per-axis reference matrices: element_matrix with unit coefficient on one axis
    kref = []
    for i in range(d):
        e = np.zeros(d)
        e[i] = 1.0
        kref.append(element_matrix(d, h, e))
    S = np.zeros((3 ** d,) + (n + 1,) * d)
    for s in corners(d):                 # v sits at corner s of cell (v - s)
        sl = tuple(slice(1 - s[i], 1 - s[i] + n + 1) for i in reversed(range(d)))
        cell = [p[sl] for p in padded]   # coefficient of cell (v - s) at every v
        for w in corners(d):
            o = tuple(w[i] - s[i] for i in range(d))
            k = flat_offset(o)
            ia, ib = corner_index(s), corner_index(w)
            for i in range(d):
                S[k] += cell[i] * kref[i][ia, ib]
    return apply_dirichlet(S, d, level) if dirichlet else S


def apply_dirichlet(S, d, level):
    mask = interior_mask(d, level)
    out = S.copy()
    for k, o in enumerate(offsets(d, stencil_radius(S, d))):
        out[k] *= mask * shifted(mask, o)
    return out


def _unknown_numbering(d, level):
    n = 3 ** level
    idx = -np.ones((n + 1,) * d, dtype=np.int64)
    inner = (slice(1, n),) * d
    idx[inner] = np.arange((n - 1) ** d).reshape((n - 1,) * d)
    return idx


def stencil_radius(S, d):
    w = int(round(S.shape[0] ** (1.0 / d)))
    assert w ** d == S.shape[0] and w % 2 == 1
    return (w - 1) // 2


def stencil_to_csr(S, d, level):
    """Sparse matrix over the interior unknowns from a stencil array."""
    n = 3 ** level
    r = stencil_radius(S, d)
    num = _unknown_numbering(d, level)
    rows, cols, vals = [], [], []
    for k, o in enumerate(offsets(d, r)):
        nbv = shifted(num + 1, o) - 1          # -1 outside or on the boundary
        valid = (num >= 0) & (nbv >= 0)
        rows.append(num[valid])
        cols.append(nbv[valid])
        vals.append(S[k][valid])
    N = (n - 1) ** d
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    return A


def csr_to_stencil(A, d, level, r=1):
    """Stencil array (radius r) of a sparse matrix over the interior unknowns.
    Entries outside the radius-r window are not representable and must be 0."""
    n = 3 ** level
    num = _unknown_numbering(d, level)
    A = sp.csr_matrix(A)
    S = np.zeros(((2 * r + 1) ** d,) + (n + 1,) * d)
    valid_rows = num >= 0
    for k, o in enumerate(offsets(d, r)):
        nbv = shifted(num + 1, o) - 1
        valid = valid_rows & (nbv >= 0)
        vals = np.asarray(A[num[valid], nbv[valid]]).ravel()
        S[k][valid] = vals
    return S


def lattice_from_unknowns(x, d, level):
    n = 3 ** level
    out = np.zeros((n + 1,) * d)
    out[(slice(1, n),) * d] = np.asarray(x).reshape((n - 1,) * d)
    return out


def unknowns_from_lattice(a, d, level):
    n = 3 ** level
    return np.ascontiguousarray(a[(slice(1, n),) * d]).ravel()


def coarsen_eps(eps, d):
    """Coefficient of a level-(l-1) cell = mean of its 3^d children.  The paper
    rediscretises on every level (Sect. 3, item 3) without fixing how eps is
    sampled there; averaging is a reading of the paper."""
    comps = np.asarray(eps, dtype=np.float64)
    lead = comps.ndim - d
    n = comps.shape[-1]
    shape = comps.shape[:lead]
    for _ in range(d):
        shape = shape + (n // 3, 3)
    r = comps.reshape(shape)
    axes = tuple(lead + 2 * i + 1 for i in range(d))
    return r.mean(axis=axes)


def rhs_from_f(f, d, level):
    """Lumped right-hand side b_v = h^d f_v over the interior unknowns."""
    h = 1.0 / 3 ** level
    return (h ** d) * np.asarray(f, dtype=np.float64).ravel()
