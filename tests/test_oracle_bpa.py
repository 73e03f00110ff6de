"""Pins of the oracle's bpa codec (Sect. 5, stencil compression): values
worked out by hand, a brute-force search over exponents, exactness at eight
bytes, minimality of the chosen width, and the solver behaviour the paper
reports for eps_mf = 1e-8."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_hand_worked_values():
    """0.3 with one mantissa byte: 0.3 * 2^8 = 76.8 fits (|m| <= 127) but
    0.3 * 2^9 = 153.6 does not, so e = -8, m = 77; with two bytes
    0.3 * 2^16 = 19660.8 -> 19661 (|m| <= 32767)."""
    q, e, m = O.bpa_value(np.array([0.3, -0.3, 1.0, 0.0]), 2)
    assert list(e) == [-8, -8, -6, 0] and list(m) == [77, -77, 64, 0]
    assert q[0] == 77 / 256 and q[1] == -77 / 256 and q[2] == 1.0 and q[3] == 0.0
    q, e, m = O.bpa_value(np.array([0.3]), 3)
    assert e[0] == -16 and m[0] == 19661 and q[0] == 19661 / 65536
    # per vertex (columns): {0.3, 0.001} needs one mantissa byte at eps 1e-2
    # (0.3 -> 77/256, error 7.8e-4), and 0.001 is coded at the vertex's width:
    # 0.001 * 2^16 = 65.536 -> 66; {0.001, 0} lies within eps of zero: bpa 0
    dq, w = O.bpa_encode(np.array([[0.3, 1e-3], [0.001, 0.0]]), 1e-2)
    assert list(w) == [2, 0]
    assert dq[0, 0] == 77 / 256 and dq[1, 0] == 66 / 65536
    assert dq[0, 1] == 0.0 and dq[1, 1] == 0.0


@pytest.mark.parametrize("bpa", [2, 3, 4])
def test_exponent_is_the_smallest_that_fits(bpa):
    """Brute force: scan e upwards from far below and take the first e with
    |rint(x / 2^e)| <= 2^(8(bpa-1)-1) - 1."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal(300) * 10.0 ** rng.uniform(-12, 3, 300)
    x[:3] = [2.0 ** -5, -(2.0 ** 7 - 0.4), 127.5]          # powers of two and rounding edges
    mmax = 2 ** (8 * (bpa - 1) - 1) - 1
    q, e, m = O.bpa_value(x, bpa)
    for i, xi in enumerate(x):
        ee = -200
        while abs(np.rint(xi / 2.0 ** ee)) > mmax:
            ee += 1
        assert e[i] == ee, (xi, e[i], ee)
        assert m[i] == int(np.rint(xi / 2.0 ** ee))
        assert q[i] == m[i] * 2.0 ** ee


def test_eight_bytes_are_exact_and_errors_are_bounded():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(2000) * 10.0 ** rng.uniform(-15, 4, 2000)
    assert np.array_equal(O.bpa_value(x, 8)[0], x)
    for bpa in range(2, 8):
        q, e, m = O.bpa_value(x, bpa)
        assert np.all(np.abs(q - x) <= np.ldexp(1.0, e - 1))
        assert np.all(np.abs(m) <= 2 ** (8 * (bpa - 1) - 1) - 1)
        # sign symmetry and invariance under powers of two
        assert np.array_equal(O.bpa_value(-x, bpa)[0], -q)
        assert np.array_equal(O.bpa_value(x * 2.0 ** 5, bpa)[0], q * 2.0 ** 5)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_width_is_minimal(eps):
    """Every vertex meets eps at its width and misses it at every smaller
    width of the set {0, 2, ..., 8}."""
    rng = np.random.default_rng(5)
    scale = 10.0 ** rng.uniform(-10, 1, 400)
    delta = rng.standard_normal((9, 400)) * scale
    q, w = O.bpa_encode(delta, eps, axis=0)
    widths = (0, 2, 3, 4, 5, 6, 7, 8)
    for v in range(400):
        assert np.max(np.abs(q[:, v] - delta[:, v])) <= eps
        for smaller in widths[:widths.index(w[v])]:
            assert np.max(np.abs(O.bpa_value(delta[:, v], smaller)[0] - delta[:, v])) > eps
    assert len(set(w.tolist())) >= 3          # the sample spans several widths


def test_constant_coefficients_compress_to_nothing():
    """eps = 1 (the sine setup): BoxMG and Galerkin reproduce the d-linear and
    rediscretised operators, so every vertex of every stored level is bpa 0."""
    p = W.sin_source(2, 4)
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    Hq = O.solver.quantised_hierarchy(H, "bpa", eps_mf=1e-8)
    for l in H.A:
        assert abs(Hq.A[l] - O.stencil_to_csr(O.geometric_stencil(H.eps[l], 2, l), 2, l)).max() == 0.0
    for l in H.P:
        assert abs(Hq.P[l] - O.dlinear_P(2, l)).max() == 0.0


def test_eps_1e8_keeps_the_solver_semantics():
    """With eps_mf = 1e-8 the compressed FP64 hierarchy solves a per-cell
    random coefficient setup (BoxMG and Galerkin far from d-linear and
    rediscretised on every level) with the uncompressed cycle count and nearly
    the same residual history; eps_mf = 1e-2 still converges to the same
    solution."""
    p = W.random_checkerboard(2, 5, seed=7, values=(1.0, 10.0), blocks=243)
    b = O.rhs_from_f(p.f, 2, 5)
    H = O.build_hierarchy(p.eps, 2, 5, transfer="boxmg", check_definite=False)
    assert H.lc == 1
    assert min(abs(H.P[l] - O.dlinear_P(2, l)).max() for l in H.P) > 1e-2
    u0, h0 = O.solve(H, b, tol=1e-10, max_cycles=200)
    Hq = O.solver.quantised_hierarchy(H, "bpa", eps_mf=1e-8)
    assert Hq.dtype == np.float64
    u1, h1 = O.solve(Hq, b, tol=1e-10, max_cycles=200)
    assert len(h1) == len(h0)
    np.testing.assert_allclose(h1, h0, rtol=1e-5)
    assert abs(Hq.P[5] - H.P[5]).max() <= 1e-8 and abs(Hq.A[4] - H.A[4]).max() <= 1e-8
    Hc = O.solver.quantised_hierarchy(H, "bpa", eps_mf=1e-2)
    u2, h2 = O.solve(Hc, b, tol=1e-10, max_cycles=400)
    assert h2[-1] <= 1e-10
    assert np.linalg.norm(u2 - u0) <= 1e-8 * np.linalg.norm(u0)
    # the loose codec changes the operators measurably
    assert abs(Hc.P[5] - H.P[5]).max() > 1e-3 and abs(Hc.A[4] - H.A[4]).max() > 1e-3
