"""Pins of the oracle's convection-diffusion operator (eq. (1) with v != 0)
and of the Petrov-Galerkin injection: quadrature of the element matrix,
skew symmetry for constant v, exactness on linear functions, and the
convergence behaviour the paper reports for the circle setup."""
import itertools

import numpy as np
import pytest

import oracle as O
import oracle.fem as F
import workloads as W


def _basis(corner, xi):
    """Bilinear/trilinear basis of the unit cell at points xi (npts, d)."""
    val = np.ones(len(xi))
    for i, a in enumerate(corner):
        val *= xi[:, i] if a else 1.0 - xi[:, i]
    return val


def _basis_grad(corner, xi, axis):
    g = np.ones(len(xi))
    for i, a in enumerate(corner):
        if i == axis:
            g *= 1.0 if a else -1.0
        else:
            g *= xi[:, i] if a else 1.0 - xi[:, i]
    return g


@pytest.mark.parametrize("d", [2, 3])
def test_element_matrix_by_gauss_quadrature(d):
    """Two-point Gauss quadrature per axis integrates (v . grad phi_b) phi_a
    exactly (degree <= 2 per axis); h enters as h^(d-1)."""
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    pts = np.array(list(itertools.product(gp, repeat=d)))
    wts = np.full(len(pts), 0.5 ** d)
    v = np.array([0.7, -1.3, 0.4][:d])
    h = 1.0 / 27
    cs = F.corners(d)
    C = np.zeros((2 ** d, 2 ** d))
    for ia, a in enumerate(cs):
        for ib, b in enumerate(cs):
            conv = sum(v[i] * _basis_grad(b, pts, i) for i in range(d)) / h
            C[ia, ib] = h ** d * np.sum(wts * conv * _basis(a, pts))
    np.testing.assert_allclose(F.convection_element_matrix(d, h, v), C, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,L", [(2, 3), (3, 2)])
def test_constant_velocity_is_skew(d, L):
    """With v constant and zero boundary values, integration by parts makes the
    convection matrix skew: C + C^T = 0 on the interior unknowns."""
    n = 3 ** L
    v = np.stack([np.full((n,) * d, c) for c in (0.8, -0.5, 0.3)[:d]])
    C = O.stencil_to_csr(F.convection_stencil(v, d, L), d, L)
    assert abs(C + C.T).max() <= 1e-15
    assert abs(C).max() > 1e-3


@pytest.mark.parametrize("d", [2, 3])
def test_linear_functions(d):
    """Away from the boundary, the convection stencil maps u = a . x to
    (v . a) h^d (the integral of a basis function is h^d) and the diffusion
    stencil maps it to zero; constants map to zero for any v."""
    L = 2 if d == 3 else 3
    n = 3 ** L
    h = 1.0 / n
    rng = np.random.default_rng(2)
    vc = rng.uniform(-1, 1, d)
    v = np.stack([np.full((n,) * d, c) for c in vc])
    a = rng.uniform(-1, 1, d)
    coords = np.meshgrid(*([np.arange(n + 1) * h] * d), indexing="ij")  # (z,) y, x
    u = sum(a[i] * coords[d - 1 - i] for i in range(d))
    S = F.convection_stencil(v, d, L)
    G = O.geometric_stencil(np.full((n,) * d, 2.5), d, L)
    far = (slice(2, n - 1),) * d
    for stencil, want in ((S, np.dot(vc, a) * h ** d), (G, 0.0)):
        out = sum(stencil[k] * F.shifted(u, o) for k, o in enumerate(F.offsets(d)))
        np.testing.assert_allclose(out[far], want, rtol=0, atol=1e-13)
    vr = rng.uniform(-1, 1, (d,) + (n,) * d)
    rows = F.convection_stencil(vr, d, L).sum(axis=0)
    assert np.abs(rows[far]).max() <= 1e-15


@pytest.mark.parametrize("d,l", [(2, 3), (3, 2)])
def test_injection_picks_the_coincident_vertex(d, l):
    """R = I keeps the fine value at 3V: R P = identity (P injects at
    c-points), and the Petrov-Galerkin coarse equation at V is the fine
    equation at 3V applied to the prolongated coarse vector."""
    R = O.transfer.injection_R(d, l)
    P = O.dlinear_P(d, l)
    assert abs(R @ P - np.eye(P.shape[1])).max() == 0.0
    rng = np.random.default_rng(3)
    n = 3 ** l
    v = rng.uniform(-1, 1, (d,) + (n,) * d)
    A = O.stencil_to_csr(O.geometric_stencil(np.ones((n,) * d), d, l) + F.convection_stencil(v, d, l), d, l)
    Ac = O.rap(A, P, R)
    ec = rng.normal(size=P.shape[1])
    fine = A @ (P @ ec)
    np.testing.assert_allclose(Ac @ ec, fine[O.cpoint_positions(d, l)], rtol=0, atol=1e-14)


def test_circle_convergence_behaviour():
    """eps = 0.1 (the paper's case without any coarse-level increase): BoxMG
    with R = P^T converges to the direct solution with the coarsest level kept
    at 1 even with the stagnation check on; injection is the slowest."""
    p = W.circle(2, 4, 0.1)
    b = O.rhs_from_f(p.f, 2, 4)
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", v=p.meta["v"])
    assert H.lc == 1
    u, h = O.solve(H, b, tol=1e-10, max_cycles=100, stagnation=0.9)
    assert H.lc == 1 and h[-1] <= 1e-10 and len(h) <= 30
    ustar = O.direct_solve(H.A[4], b)
    assert np.linalg.norm(u - ustar) <= 1e-8 * np.linalg.norm(ustar)
    Hi = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", v=p.meta["v"], restriction="injection")
    _, hi = O.solve(Hi, b, cycles=len(h))
    assert hi[-1] > 100 * h[-1]
    # the operator is not symmetric
    A = H.A[4]
    assert abs(A - A.T).max() > 1e-3


@pytest.mark.parametrize("d,l", [(2, 3), (3, 2)])
def test_aggregates_partition_the_fine_vertices(d, l):
    """Aggregation: every fine vertex away from the boundary belongs to exactly
    one aggregate (the coarse vertex nearest to it), and the coarse equation
    at V is the sum of the fine equations of its aggregate applied to the
    prolongated coarse vector."""
    R = O.aggregation_R(d, l)
    n = 3 ** l
    cover = np.asarray(R.sum(axis=0)).ravel().reshape((n - 1,) * d)
    inner = (slice(1, n - 2),) * d          # lattice 2..n-2
    assert (cover[inner] == 1).all() and cover.max() == 1
    assert (np.asarray(R.sum(axis=1)).ravel() == 3 ** d).all()
    rng = np.random.default_rng(4)
    v = rng.uniform(-1, 1, (d,) + (n,) * d)
    A = O.stencil_to_csr(O.geometric_stencil(np.ones((n,) * d), d, l) + F.convection_stencil(v, d, l), d, l)
    P = O.dlinear_P(d, l)
    ec = rng.normal(size=P.shape[1])
    fine = O.fem.lattice_from_unknowns(A @ (P @ ec), d, l)
    box = sum(F.shifted(fine, o) for o in F.offsets(d))       # sum over the 3^d box around each vertex
    coarse_pts = (slice(3, n - 2, 3),) * d
    np.testing.assert_allclose(O.rap(A, P, R) @ ec, box[coarse_pts].ravel(), rtol=0, atol=1e-13)


def test_aggregation_converges_like_galerkin():
    """On the circle setup with eps = 0.1 the aggregation restriction with the
    BoxMG prolongation converges at nearly the rate of R = P^T (the paper
    finds them close), while injection is far slower."""
    p = W.circle(2, 4, 0.1, seed=5)
    b = O.rhs_from_f(p.f, 2, 4)
    counts = {}
    for r in ("transpose", "aggregation", "injection"):
        H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", v=p.meta["v"], restriction=r)
        _, h = O.solve(H, b, tol=1e-10, max_cycles=400)
        counts[r] = len(h)
    assert counts["aggregation"] <= counts["transpose"] + 3
    assert counts["injection"] > 5 * counts["transpose"]
