"""Pins of the oracle's V-cycle and outer loops: convergence to the direct
solution, monotone energy error, h-independence, mixed precision."""
import numpy as np
import pytest

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
    p = W.cfg1(0)
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
