"""Pins of the oracle's V-cycle and outer loops: convergence to the direct
solution, monotone energy error, h-independence, mixed precision."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W


@pytest.mark.parametrize("d,L,transfer", [(2, 3, "boxmg"), (2, 3, "geometric"),
                                          (3, 2, "boxmg"), (3, 2, "galerkin")])
def test_vcycles_converge_to_direct_solution(d, L, transfer):
    p = W.random_checkerboard(d, L, seed=3, values=(1.0, 100.0), blocks=3) \
        if transfer != "geometric" else W.poisson(d, L, 3)
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer)
    b = O.rhs_from_f(p.f, d, L)
    ustar = O.direct_solve(H.A[L], b)
    u, hist = O.solve(H, b, tol=1e-15, max_cycles=200)
    assert np.linalg.norm(u - ustar) <= 1e-13 * np.linalg.norm(ustar) * 10


def test_energy_error_decreases_every_cycle():
    p = W.random_checkerboard(2, 4, seed=5, values=(1.0, 1e4))
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    b = O.rhs_from_f(p.f, 2, 4)
    A = H.A[4]
    ustar = O.direct_solve(A, b)
    u = np.zeros_like(b)
    prev = np.inf
    for _ in range(15):
        u = O.vcycle(H, 4, u, b)
        e = u - ustar
        en = float(e @ (A @ e))
        assert en < prev
        prev = en


def test_poisson_convergence_factor_h_independent():
    rho = []
    for L in (3, 4, 5, 6):
        p = W.poisson(2, L, 0)
        H = O.build_hierarchy(p.eps, 2, L, transfer="geometric")
        b = O.rhs_from_f(p.f, 2, L)
        _, hist = O.solve(H, b, cycles=10)
        rho.append(hist[-1] / hist[-2])
    assert max(rho) - min(rho) <= 0.05, rho
    assert max(rho) < 0.5


def test_boxmg_equals_geometric_for_constant_eps():
    p = W.poisson2d_l4(0)
    b = O.rhs_from_f(p.f, 2, 4)
    Hg = O.build_hierarchy(p.eps, 2, 4, transfer="geometric")
    Hb = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    ug, _ = O.solve(Hg, b, cycles=5)
    ub, _ = O.solve(Hb, b, cycles=5)
    A = Hg.A[4]
    assert np.linalg.norm(A @ (ug - ub)) <= 1e-13 * np.linalg.norm(b)


def test_indefinite_coarse_raises_coarsest_level():
    """A planted indefinite Galerkin operator moves the coarsest level up."""
    import oracle.solver as S
    import oracle.galerkin as G
    p = W.poisson(2, 4, 0)
    orig = G.definiteness_violations
    calls = []

    def planted(Ac):
        calls.append(Ac.shape[0])
        return np.array([0]) if Ac.shape[0] == (3 ** 2 - 1) ** 2 else orig(Ac)

    S.definiteness_violations = planted
    try:
        H = O.build_hierarchy(p.eps, 2, 4, transfer="galerkin")
    finally:
        S.definiteness_violations = orig
    assert H.lc == 3
    b = O.rhs_from_f(p.f, 2, 4)
    u, hist = O.solve(H, b, tol=1e-10)
    assert hist[-1] <= 1e-10


@pytest.mark.parametrize("fmt", ["fp32", "bf16", "fp16"])
def test_mixed_precision_reaches_tolerance(fmt):
    p = W.random_checkerboard(2, 4, seed=1, values=(1.0, 1e4))
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    Hq = O.solver.quantised_hierarchy(H, fmt)
    b = O.rhs_from_f(p.f, 2, 4)
    x, hist = O.mixed_solve(H, Hq, b, tol=1e-8)
    assert hist[-1] <= 1e-8
    u64, h64 = O.solve(H, b, tol=1e-8)
    assert len(hist) - 1 <= 1.5 * len(h64) + 2


# ---------------------------------------------------------------------------
# Dynamic coarsest level (Sect. 4.3): raise between cycles on stagnation
# ---------------------------------------------------------------------------

def _two_grid_cycle(A, P, Ac, b, u, omega, mu_pre, mu_post):
    """Textbook two-grid cycle with dense linear algebra: damped Jacobi
    pre-smoothing, exact coarse correction with R = P^T, post-smoothing."""
    A = A.toarray()
    P = P.toarray()
    D = np.diag(A)
    for _ in range(mu_pre):
        u = u + omega * (b - A @ u) / D
    u = u + P @ np.linalg.solve(Ac.toarray(), P.T @ (b - A @ u))
    for _ in range(mu_post):
        u = u + omega * (b - A @ u) / D
    return u


@pytest.mark.parametrize("transfer", ["galerkin", "boxmg", "geometric"])
def test_raise_to_top_gives_the_two_grid_cycle(transfer):
    """Raised to L - 1, a V-cycle is the two-grid cycle with an exact coarse
    solve of level L - 1's operator."""
    d, L = 2, 3
    p = W.random_checkerboard(d, L, seed=2, values=(1.0, 100.0), blocks=3)
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, check_definite=False)
    assert H.lc == 1
    assert O.raise_coarsest(H) and H.lc == 2
    assert not O.raise_coarsest(H) and H.lc == 2      # L - 1 is the top
    b = O.rhs_from_f(p.f, d, L)
    rng = np.random.default_rng(0)
    u0 = rng.uniform(-1, 1, size=b.shape) * 1e-2
    u1 = O.vcycle(H, L, u0.copy(), b)
    ref = _two_grid_cycle(H.A[L], H.P[L], H.A[L - 1], b, u0, H.omega, H.mu_pre, H.mu_post)
    np.testing.assert_allclose(u1, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_raised_level_is_solved_with_its_own_operator():
    """After one raise the cycle equals that of a hierarchy built with the
    higher coarsest level from the start."""
    p = W.random_checkerboard(2, 4, seed=4, values=(1.0, 1e3))
    b = O.rhs_from_f(p.f, 2, 4)
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", check_definite=False)
    O.raise_coarsest(H)
    H2 = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", lc=2, check_definite=False)
    u = np.zeros_like(b)
    np.testing.assert_allclose(O.vcycle(H, 4, u, b), O.vcycle(H2, 4, u, b), rtol=1e-13, atol=0)


def test_threshold_above_every_ratio_changes_nothing():
    p = W.random_checkerboard(2, 4, seed=1, values=(1.0, 1e4))
    b = O.rhs_from_f(p.f, 2, 4)
    H0 = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    _, h0 = O.solve(H0, b, tol=1e-8)
    ratios = np.array(h0) / np.array([1.0] + h0[:-1])
    H1 = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    _, h1 = O.solve(H1, b, tol=1e-8, stagnation=2.0 * ratios.max())
    assert h1 == h0 and H1.lc == H0.lc == 1


def test_tiny_threshold_raises_after_every_cycle_up_to_the_top():
    p = W.random_checkerboard(2, 4, seed=1, values=(1.0, 1e4))
    b = O.rhs_from_f(p.f, 2, 4)
    lcs = []
    for k in range(1, 5):
        H = O.build_hierarchy(p.eps, 2, 4, transfer="galerkin", check_definite=False)
        O.solve(H, b, cycles=k, stagnation=1e-12)
        lcs.append(H.lc)
    # the check runs between cycles only: k cycles leave k - 1 raises
    assert lcs == [1, 2, 3, 3]


def test_jump_setup_growth_triggers_raise():
    """The paper's jump setup with geometric V(1,1) cycles: the residual grows
    over the first cycles (the coarse corrections' d-linear interpolation
    across the jump); raising the coarsest level on growth keeps the solve
    convergent and does not take more cycles (the behaviour reported with
    the dynamic coarsest level)."""
    p = W.material_jump(2, 5)
    b = O.rhs_from_f(p.f, 2, 5)
    H0 = O.build_hierarchy(p.eps, 2, 5, transfer="geometric", omega=0.9, mu_pre=1, mu_post=1)
    _, h0 = O.solve(H0, b, tol=1e-8, max_cycles=300)
    assert max(np.array(h0) / np.array([1.0] + h0[:-1])) > 1.0
    H1 = O.build_hierarchy(p.eps, 2, 5, transfer="geometric", omega=0.9, mu_pre=1, mu_post=1)
    _, h1 = O.solve(H1, b, tol=1e-8, max_cycles=300, stagnation=1.0)
    assert H1.lc > 1 and h1[-1] <= 1e-8 and len(h1) <= len(h0)
    # the raise happened exactly after the cycles whose residual grew
    grow = [k for k in range(len(h1) - 1) if h1[k] > (h1[k - 1] if k else 1.0)]
    assert H1.lc == 1 + len(grow)


# ---------------------------------------------------------------------------
# Block Jacobi (Sect. "Spacetree block smoothers")
# ---------------------------------------------------------------------------

def _level_system(d, L, seed=5):
    p = W.random_checkerboard(d, L, seed=seed, values=(1.0, 30.0), blocks=3)
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
    rng = np.random.default_rng(seed)
    return A, rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])


@pytest.mark.parametrize("d", [2, 3])
def test_block_jacobi_on_one_patch_is_gauss_seidel(d):
    """On level 1 the only patch holds every unknown, all of them
    iota-vertices: BJ(1) is one lexicographic Gauss-Seidel sweep, i.e. the
    forward substitution (D + L) u' = b - U u, and many sweeps reach the
    exact solution."""
    import scipy.linalg as sla
    A, b, u0 = _level_system(d, 1)
    Ad = A.toarray()
    D = A.diagonal()
    lower = np.tril(Ad)
    ref = sla.solve_triangular(lower, b - np.triu(Ad, 1) @ u0, lower=True)
    np.testing.assert_allclose(O.block_jacobi(A, D, u0, b, 0.6, 1, d, 1), ref, rtol=0, atol=1e-13)
    many = O.block_jacobi(A, D, u0, b, 0.6, 200, d, 1)
    np.testing.assert_allclose(many, np.linalg.solve(Ad, b), rtol=0, atol=1e-12)


@pytest.mark.parametrize("d,sweeps", [(2, 1), (2, 3), (3, 1)])
def test_block_jacobi_by_patch_blocks(d, sweeps):
    """Level 2, written per patch with dense blocks: each patch's iota block
    takes `sweeps` forward substitutions against its own lower triangle with
    every other value held; then the remaining vertices take damped Jacobi
    from the updated iterate."""
    import scipy.linalg as sla
    L = 2
    A, b, u0 = _level_system(d, L)
    Ad = A.toarray()
    D = A.diagonal()
    n = 3 ** L
    coords = np.array(list(np.ndindex(*((n - 1,) * d))))[:, ::-1] + 1   # x first, unknown order
    iota = np.all(coords % 3 != 0, axis=1)
    patch = [tuple(c) for c in (coords // 3)]
    u = u0.copy()
    for key in sorted(set(pk for pk, io in zip(patch, iota) if io)):
        idx = np.array([k for k in range(len(u)) if iota[k] and patch[k] == key])
        order = np.lexsort(coords[idx].T)          # x fastest: last key is the slowest axis
        idx = idx[order]
        rest = np.setdiff1d(np.arange(len(u)), idx)
        Aii = Ad[np.ix_(idx, idx)]
        for _ in range(sweeps):
            rhs = b[idx] - Ad[np.ix_(idx, rest)] @ u[rest] - np.triu(Aii, 1) @ u[idx]
            u[idx] = sla.solve_triangular(np.tril(Aii), rhs, lower=True)
    ref = u + 0.6 * (b - Ad @ u) / D
    ref[iota] = u[iota]
    got = O.block_jacobi(A, D, u0, b, 0.6, sweeps, d, L)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_block_jacobi_cycles_converge_faster():
    """The block smoother cuts the cycle count of V(2,2) cycles (the paper
    reports up to twice as fast convergence) and still reaches the direct
    solution."""
    p = W.random_checkerboard(2, 4, seed=1, values=(1.0, 1e3))
    b = O.rhs_from_f(p.f, 2, 4)
    H0 = O.build_hierarchy(p.eps, 2, 4, transfer="galerkin")
    _, h0 = O.solve(H0, b, tol=1e-10, max_cycles=400)
    H1 = O.build_hierarchy(p.eps, 2, 4, transfer="galerkin", smoother="block", bj_sweeps=3)
    u1, h1 = O.solve(H1, b, tol=1e-10, max_cycles=400)
    assert h1[-1] <= 1e-10 and len(h1) < len(h0)
    ustar = O.direct_solve(H1.A[4], b)
    assert np.linalg.norm(u1 - ustar) <= 1e-8 * np.linalg.norm(ustar)


# ---------------------------------------------------------------------------
# Additive cycles (Alg. 2, additive multigrid appendix)
# ---------------------------------------------------------------------------

def test_additive_two_level_closed_form():
    """Two levels with an exact coarse solve: u + omega D^-1 r + P A_c^-1 P^T r."""
    p = W.random_checkerboard(2, 2, seed=3, values=(1.0, 20.0), blocks=3)
    H = O.build_hierarchy(p.eps, 2, 2, transfer="galerkin")
    assert H.lc == 1 and H.coarse_lu is not None
    b = O.rhs_from_f(p.f, 2, 2)
    u0 = np.random.default_rng(1).normal(size=b.shape)
    A = H.A[2].toarray()
    P = H.P[2].toarray()
    r = b - A @ u0
    want = u0 + 0.6 * r / np.diag(A) + P @ np.linalg.solve(H.A[1].toarray(), P.T @ r)
    np.testing.assert_allclose(O.additive_cycle(H, u0, b), want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("damping", ["exp", "const"])
def test_additive_operator_is_symmetric(damping):
    """u -> additive_cycle(0, b) is the linear map B = sum_l P omega_l D_l^-1 P^T
    (plus P A_c^-1 P^T): symmetric for R = P^T, checked column by column."""
    p = W.random_checkerboard(2, 3, seed=2, values=(1.0, 10.0), blocks=3)
    H = O.build_hierarchy(p.eps, 2, 3, transfer="boxmg")
    n = H.A[3].shape[0]
    B = np.column_stack([O.additive_cycle(H, np.zeros(n), np.eye(n)[:, j], damping) for j in range(n)])
    assert np.abs(B - B.T).max() <= 1e-14 * np.abs(B).max()
    assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0


def test_additive_exponential_damping_converges():
    """With omega = 0.8 the undamped sum of level corrections diverges in 2D;
    exponential damping converges to the direct solution."""
    p = W.sin_source(2, 4)
    b = O.rhs_from_f(p.f, 2, 4)
    H = O.build_hierarchy(p.eps, 2, 4, transfer="geometric", omega=0.8)
    u, h = O.solve_additive(H, b, tol=1e-10, max_cycles=400, damping="exp")
    assert h[-1] <= 1e-10
    ustar = O.direct_solve(H.A[4], b)
    assert np.linalg.norm(u - ustar) <= 1e-8 * np.linalg.norm(ustar)
    _, hc = O.solve_additive(H, b, cycles=60, damping="const")
    assert hc[-1] > 1.0


# ---------------------------------------------------------------------------
# BPX cycles (Alg. 3, additive multigrid appendix)
# ---------------------------------------------------------------------------

def _injection_from_P(P):
    """Injection to the coarse vertices found from P alone: the fine row of
    coarse vertex j is the one whose only entry is P[i, j] = 1."""
    P = sp.csr_matrix(P)
    nnz = np.diff(P.indptr)
    I = np.zeros((P.shape[1], P.shape[0]))
    for i in np.nonzero(nnz == 1)[0]:
        j = P.indices[P.indptr[i]]
        if abs(P.data[P.indptr[i]] - 1.0) < 1e-12:
            I[j, i] = 1.0
    assert (I.sum(axis=1) == 1).all()
    return I


@pytest.mark.parametrize("d,l", [(2, 2), (2, 3), (3, 2)])
def test_cpoint_positions_are_the_unit_rows_of_P(d, l):
    """The c-point of every coarse vertex is the fine row of P that injects it."""
    P = O.dlinear_P(d, l)
    I = _injection_from_P(P)
    np.testing.assert_array_equal(np.argmax(I, axis=1), O.cpoint_positions(d, l))


def test_bpx_two_level_closed_form():
    """Two levels with an exact coarse solve: the fine level adds only the
    surplus (I - P I_c) omega D^-1 r of its Jacobi step to P A_c^-1 P^T r."""
    p = W.random_checkerboard(2, 2, seed=3, values=(1.0, 20.0), blocks=3)
    H = O.build_hierarchy(p.eps, 2, 2, transfer="galerkin")
    assert H.lc == 1 and H.coarse_lu is not None
    b = O.rhs_from_f(p.f, 2, 2)
    u0 = np.random.default_rng(1).normal(size=b.shape)
    A = H.A[2].toarray()
    P = H.P[2].toarray()
    Ic = _injection_from_P(P)
    r = b - A @ u0
    d = 0.6 * r / np.diag(A)
    want = u0 + d - P @ (Ic @ d) + P @ np.linalg.solve(H.A[1].toarray(), P.T @ r)
    np.testing.assert_allclose(O.bpx_cycle(H, u0, b), want, rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("damping", ["const", "exp"])
def test_bpx_operator_is_the_level_sum(damping):
    """Three levels: u -> bpx_cycle(0, b) is the map
    sum_l P_{L<-l} (I - P_l I_l) omega_l D_l^-1 P_{L<-l}^T plus the coarsest
    term, assembled here from dense matrices level by level."""
    p = W.random_checkerboard(2, 3, seed=2, values=(1.0, 10.0), blocks=3)
    H = O.build_hierarchy(p.eps, 2, 3, transfer="boxmg", lc=1)
    L, lc = 3, H.lc
    assert lc == 1
    n = H.A[L].shape[0]
    Pc = {L: np.eye(n)}                     # P_{L<-l}
    for l in range(L, lc, -1):
        Pc[l - 1] = Pc[l] @ H.P[l].toarray()
    def om(l):
        return 0.6 ** (L - l + 1) if damping == "exp" else 0.6
    if H.coarse_lu is not None:
        want = Pc[lc] @ np.linalg.solve(H.A[lc].toarray(), Pc[lc].T)
    else:
        want = Pc[lc] @ np.diag(om(lc) / H.A[lc].diagonal()) @ Pc[lc].T
    for l in range(lc + 1, L + 1):
        P = H.P[l].toarray()
        S = np.eye(P.shape[0]) - P @ _injection_from_P(P)
        want += Pc[l] @ S @ np.diag(om(l) / H.A[l].diagonal()) @ Pc[l].T
    B = np.column_stack([O.bpx_cycle(H, np.zeros(n), np.eye(n)[:, j], damping) for j in range(n)])
    np.testing.assert_allclose(B, want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_bpx_coarse_vertices_take_the_coarsest_correction():
    """Every vertex is updated by the coarsest level holding it: at the
    vertices of the coarsest level the fine correction equals the coarse
    solve of the restricted residual (the additive cycle adds the finer
    levels' Jacobi steps there too)."""
    p = W.random_checkerboard(2, 4, seed=5, values=(1.0, 100.0), blocks=9)
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    b = O.rhs_from_f(p.f, 2, 4)
    L, lc = H.L, H.lc
    assert H.coarse_lu is not None and lc < L - 1
    e = O.bpx_cycle(H, np.zeros_like(b), b)
    rc, pos = b, np.arange(len(b))
    for l in range(L, lc, -1):
        rc = H.P[l].T @ rc
        pos = pos[O.cpoint_positions(2, l)]
    ec = np.linalg.solve(H.A[lc].toarray(), rc)
    np.testing.assert_allclose(e[pos], ec, rtol=0, atol=1e-12 * np.abs(ec).max())
    ea = O.additive_cycle(H, np.zeros_like(b), b, "const")
    assert np.abs(ea[pos] - ec).max() > 1e-3 * np.abs(ec).max()


def test_bpx_constant_omega_converges():
    """omega = 0.8 on every level: BPX converges to the direct solution on
    the sine setup, where the additive cycle with the same damping diverges,
    and its cycle count grows only mildly from level 3 to level 5."""
    counts = []
    for L in (3, 5):
        p = W.sin_source(2, L)
        b = O.rhs_from_f(p.f, 2, L)
        H = O.build_hierarchy(p.eps, 2, L, transfer="geometric", omega=0.8)
        u, h = O.solve_additive(H, b, tol=1e-10, max_cycles=200, damping="const", bpx=True)
        assert h[-1] <= 1e-10
        counts.append(len(h))
        if L == 5:
            ustar = O.direct_solve(H.A[L], b)
            assert np.linalg.norm(u - ustar) <= 1e-8 * np.linalg.norm(ustar)
    assert counts[1] <= 1.5 * counts[0]


# ---------------------------------------------------------------------------
# Quantised hierarchy (the inner hierarchy of the mixed loop)
# ---------------------------------------------------------------------------

# unit roundoff of each delta format (FP16 per-vertex scaled: below the
# normal range its absolute error is bounded by 2^-25 of the vertex maximum)
_U = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


@pytest.mark.parametrize("fmt", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_quantised_hierarchy_within_the_format_rounding(fmt, d, L):
    """Every stored operator of the quantised hierarchy is the rediscretised
    stencil plus its hierarchical delta rounded to the format, then rounded
    to FP32: |A_q - A| <= u_fmt |delta| + 2^-25 max_vertex |delta| +
    2^-24 |A| + 2^-40 max_vertex |A_geom| entry by entry (the last term: a
    vertex whose deltas are all below 2^-40 of its reference row stores
    none), and the prolongations likewise against the d-linear weights.  A
    dropped or sign-flipped delta fails it."""
    n = 3 ** L
    eps = np.exp(np.random.default_rng(2).normal(size=(n,) * d))   # every delta non-zero
    H = O.build_hierarchy(eps, d, L, transfer="boxmg", check_definite=False)
    Hq = O.solver.quantised_hierarchy(H, fmt)
    u = _U[fmt]
    for l in range(H.lc, L):
        S = O.csr_to_stencil(H.A[l], d, l)
        Sq = O.csr_to_stencil(sp.csr_matrix(Hq.A[l], dtype=np.float64), d, l)
        G = O.geometric_stencil(H.eps[l], d, l)
        dl = S - G
        vmax = np.max(np.abs(dl), axis=0)[None]
        gmax = np.max(np.abs(G), axis=0)[None]
        bound = u * np.abs(dl) + 2.0 ** -25 * vmax + 2.0 ** -24 * np.abs(S) + 2.0 ** -40 * gmax + 1e-300
        assert (np.abs(Sq - S) <= bound).all(), l
    for l in range(H.lc + 1, L + 1):
        Pd = O.dlinear_P(d, l).toarray()
        Pf = H.P[l].toarray()
        Pq = Hq.P[l].astype(np.float64).toarray()
        dP = Pf - Pd
        rmax = np.max(np.abs(dP), axis=1)[:, None]
        pmax = np.max(np.abs(Pd), axis=1)[:, None]
        bound = u * np.abs(dP) + 2.0 ** -25 * rmax + 2.0 ** -24 * np.abs(Pf) + 2.0 ** -40 * pmax + 1e-300
        assert (np.abs(Pq - Pf) <= bound).all(), l


@pytest.mark.parametrize("fmt", ["fp32", "bf16", "fp16"])
def test_quantised_hierarchy_of_constant_eps_is_the_fp32_reference(fmt):
    """Constant eps: every delta counts as zero, so the quantised hierarchy is
    exactly the FP32 rounding of the rediscretised operators and of the
    d-linear prolongations."""
    d, L = 2, 4
    n = 3 ** L
    H = O.build_hierarchy(np.full((n,) * d, 3.0), d, L, transfer="boxmg")
    Hq = O.solver.quantised_hierarchy(H, fmt)
    for l in range(H.lc, L + 1):
        G = O.stencil_to_csr(O.geometric_stencil(H.eps[l], d, l), d, l).astype(np.float32)
        assert (Hq.A[l] != G).nnz == 0, l
    for l in range(H.lc + 1, L + 1):
        assert (Hq.P[l] != O.dlinear_P(d, l).astype(np.float32)).nnz == 0, l


@pytest.mark.parametrize("fmt,bound", [("fp32", 1e-5), ("fp16", 1e-4), ("bf16", 2e-3)])
def test_mixed_outer_iterations_track_the_fp64_cycles(fmt, bound):
    """One outer iteration of the defect correction (FP64 residual, one FP32
    V-cycle from zero on the residual equation, FP64 update) is, in exact
    arithmetic with the same hierarchy, one V-cycle x + B (b - A x): the
    cycle is affine and consistent.  So the mixed residual history follows
    the FP64 V-cycle history iteration by iteration, apart from the inner
    hierarchy's quantisation (FP32 entries, or FP16/BF16 deltas) and FP32
    arithmetic: relative gaps measured at most 5e-7 (FP32), 1.5e-5 (FP16) and
    3e-4 (BF16) over the first 30 iterations.  A subtracted correction, a
    residual not recomputed or a second inner cycle moves it by O(1)."""
    p = W.random_checkerboard(2, 4, 3, values=(1.0, 1e3))
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg")
    b = O.rhs_from_f(p.f, 2, 4)
    _, hist_mixed = O.mixed_solve(H, O.solver.quantised_hierarchy(H, fmt), b, tol=1e-8, max_outer=31)
    _, hist_64 = O.solve(H, b, cycles=30)
    gaps = [abs(hist_mixed[k + 1] - hist_64[k]) / hist_64[k] for k in range(30)]
    assert hist_mixed[0] == 1.0 and max(gaps) < bound, max(gaps)
