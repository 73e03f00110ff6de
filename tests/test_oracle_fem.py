"""Pins of the oracle's finite-element layer against closed forms, quadrature,
tensor-product assembly and the paper's stencil splitting."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import fem


def _quadrature_element(d, h, eps_diag):
    """Element stiffness by 2-point Gauss quadrature per axis of
    int eps_i d_i phi_a d_i phi_b over [0,h]^d (exact for Q1)."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]) * h
    wq = h / 2.0
    cs = fem.corners(d)

    def phi_grad(a, x):
        vals = [(x[i] / h) if a[i] else (1.0 - x[i] / h) for i in range(d)]
        ders = [(1.0 / h) if a[i] else (-1.0 / h) for i in range(d)]
        out = []
        for i in range(d):
            t = ders[i]
            for j in range(d):
                if j != i:
                    t *= vals[j]
            out.append(t)
        return np.array(out)

    K = np.zeros((2 ** d, 2 ** d))
    for q in itertools.product(range(2), repeat=d):
        x = np.array([g[qi] for qi in q])
        w = wq ** d
        for ia, a in enumerate(cs):
            ga = phi_grad(a, x)
            for ib, b in enumerate(cs):
                gb = phi_grad(b, x)
                K[ia, ib] += w * np.sum(np.asarray(eps_diag) * ga * gb)
    return K


@pytest.mark.parametrize("d", [1, 2, 3])
def test_element_matrix_matches_quadrature(d):
    rng = np.random.default_rng(1)
    h = 1.0 / 27
    eps = rng.uniform(0.1, 10.0, size=d)
    np.testing.assert_allclose(fem.element_matrix(d, h, eps), _quadrature_element(d, h, eps),
                               rtol=1e-13, atol=1e-15)


def test_closed_form_stencils():
    S2 = O.geometric_stencil(np.ones((9, 9)), 2, 2)
    np.testing.assert_allclose(S2[:, 4, 4], np.array([-1, -1, -1, -1, 8, -1, -1, -1, -1]) / 3.0,
                               rtol=1e-15)
    h = 1.0 / 9
    S3 = O.geometric_stencil(np.ones((9, 9, 9)), 3, 2)
    want = []
    for o in fem.offsets(3):
        nz = sum(1 for oi in o if oi)
        want.append({0: 8.0 / 3, 1: 0.0, 2: -1.0 / 6, 3: -1.0 / 12}[nz] * h)
    np.testing.assert_allclose(S3[:, 4, 4, 4], want, rtol=1e-14, atol=1e-17)


def _kron_assembly(d, level):
    """Constant-coefficient Q1 matrix as sum_i (M x .. x K x .. x M) over the
    interior (1D stiffness K/h and mass M*h, Dirichlet rows/columns removed)."""
    n = 3 ** level
    h = 1.0 / n
    m = n - 1
    K = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]) / h
    M = sp.diags([np.ones(m - 1) / 6, 4 * np.ones(m) / 6, np.ones(m - 1) / 6], [-1, 0, 1]) * h
    A = None
    for i in range(d):          # axis i = x, y, z; kron order is (z, y, x) with x fastest
        mats = [K if j == i else M for j in reversed(range(d))]
        T = mats[0]
        for Mt in mats[1:]:
            T = sp.kron(T, Mt)
        A = T if A is None else A + T
    return sp.csr_matrix(A)


@pytest.mark.parametrize("d,level", [(2, 2), (2, 3), (3, 2)])
def test_tensor_product_assembly(d, level):
    n = 3 ** level
    A = O.stencil_to_csr(O.geometric_stencil(np.ones((n,) * d), d, level), d, level)
    B = _kron_assembly(d, level)
    assert abs(A - B).max() < 1e-13 * abs(B).max()


@pytest.mark.parametrize("d", [2, 3])
def test_elementwise_assembly_variable_eps(d):
    """Scatter of quadrature element matrices over all cells == stencil rows."""
    level = 1 if d == 3 else 2
    n = 3 ** level
    h = 1.0 / n
    rng = np.random.default_rng(7)
    eps = rng.uniform(0.5, 5.0, size=(d,) + (n,) * d)  # diagonal tensor per cell
    N = (n - 1) ** d
    A = np.zeros((N, N))
    cs = fem.corners(d)

    def num(v):
        if any(vi <= 0 or vi >= n for vi in v):
            return -1
        return sum((v[i] - 1) * (n - 1) ** i for i in range(d))

    for c in itertools.product(range(n), repeat=d):
        c = tuple(reversed(c))
        e = [eps[i][tuple(reversed(c))] for i in range(d)]
        K = _quadrature_element(d, h, e)
        for ia, a in enumerate(cs):
            ra = num(tuple(c[i] + a[i] for i in range(d)))
            if ra < 0:
                continue
            for ib, b in enumerate(cs):
                rb = num(tuple(c[i] + b[i] for i in range(d)))
                if rb >= 0:
                    A[ra, rb] += K[ia, ib]
    S = O.geometric_stencil(eps, d, level)
    B = O.stencil_to_csr(S, d, level).toarray()
    np.testing.assert_allclose(B, A, rtol=1e-12, atol=1e-14)


def test_stencil_split_into_cell_parts():
    """Eq. "03_solver:stencils": for constant coefficients the row of the
    element matrix of each of the four cells around v is the printed cell part
    (corner entries full, edge entries halved, centre quartered)."""
    h = 1.0 / 9
    S = O.geometric_stencil(np.full((9, 9), 2.5), 2, 2)[:, 4, 4]
    s = S.reshape(3, 3)   # s[oy+1, ox+1]
    K = fem.element_matrix(2, h, 2.5)
    cs = fem.corners(2)
    total = np.zeros((3, 3))
    for sx, sy in [(1, 0), (0, 0), (0, 1), (1, 1)]:      # v is corner (sx, sy) of the cell
        part = np.zeros((3, 3))
        ia = cs.index((sx, sy))
        for ib, (bx, by) in enumerate(cs):
            part[by - sy + 1, bx - sx + 1] = K[ia, ib]
        want = np.zeros((3, 3))
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                inside = (0 <= sx + ox <= 1) and (0 <= sy + oy <= 1)
                if not inside:
                    continue
                shared = 2 ** ((ox == 0) + (oy == 0))          # cells sharing that entry
                want[oy + 1, ox + 1] = s[oy + 1, ox + 1] / shared
        np.testing.assert_allclose(part, want, rtol=1e-14, atol=1e-16)
        total += part
    np.testing.assert_allclose(total, s, rtol=1e-14)


@pytest.mark.parametrize("d,levels", [(2, (2, 3, 4, 5)), (3, (1, 2, 3))])
def test_manufactured_solution_second_order(d, levels):
    import workloads as W
    errs = []
    for L in levels:
        p = W.sin_source(d, L)
        A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
        u = O.direct_solve(A, O.rhs_from_f(p.f, d, L))
        errs.append(np.max(np.abs(u - p.meta["exact"].ravel())))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios[1:] if d == 3 else ratios:
        assert 7.5 <= r <= 10.5, (errs, ratios)


def test_coarsen_eps_brute_force():
    rng = np.random.default_rng(3)
    e = rng.uniform(size=(9, 9, 9))
    c = fem.coarsen_eps(e, 3)
    for k, j, i in itertools.product(range(3), repeat=3):
        assert abs(c[k, j, i] - e[3 * k:3 * k + 3, 3 * j:3 * j + 3, 3 * i:3 * i + 3].mean()) < 1e-15


def test_rows_annihilate_constants_away_from_boundary():
    rng = np.random.default_rng(4)
    eps = rng.uniform(1, 100, size=(27, 27))
    S = O.geometric_stencil(eps, 2, 3)
    rows = S.sum(axis=0)[2:-2, 2:-2]
    assert np.abs(rows).max() < 1e-12 * np.abs(S).max()
