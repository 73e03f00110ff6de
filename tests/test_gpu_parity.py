"""Parity of the HIP path against the CPU oracle, step by step and end to end.

Every comparison uses the same seeded inputs on both sides; sizes span several
64 x 4 tiles with ragged tails (n + 1 = 28, 82, 244, 730 slots per row)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import require_gpu, announce, lattice_of_unknowns, unknowns_of_lattice, weights_to_csr
from noise_floor import iterate_tolerances, operator_tolerance

pytestmark = pytest.mark.gpu

RTOL64 = 1e-13


def _grid(qmg, p, transfer="boxmg", store="hier64", **kw):
    g = qmg.Grid(p.dim, p.level, qmg.make_opts(transfer, store, **kw))
    g.set_coefficients(p.eps, p.f)
    return g


@pytest.mark.parametrize("d,L", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_finest_operator_rediscretised(d, L):
    qmg = require_gpu()
    announce(f"finest operator d={d} L={L}")
    p = W.random_checkerboard(d, L, seed=1, values=(0.5, 30.0), blocks=3)
    g = _grid(qmg, p, "geometric", "hier64")
    S = g.operator(L)
    g.close()
    R = O.geometric_stencil(p.eps, d, L)
    assert np.abs(S - R).max() <= RTOL64 * np.abs(R).max()


@pytest.mark.parametrize("d,L,store", [(2, 4, "hier64"), (2, 4, "plain64"), (3, 3, "hier64")])
def test_single_steps_on_finest_level(d, L, store):
    qmg = require_gpu()
    announce(f"single steps d={d} L={L} {store}")
    p = W.random_checkerboard(d, L, seed=2, values=(1.0, 1e3), blocks=9 if L > 2 else 3)
    g = _grid(qmg, p, "boxmg", store)
    g.build()
    rng = np.random.default_rng(5)
    x = lattice_of_unknowns(rng.normal(size=p.n_unknowns), d, L)
    b = lattice_of_unknowns(rng.normal(size=p.n_unknowns), d, L)
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
    xu, bu = unknowns_of_lattice(x, d, L), unknowns_of_lattice(b, d, L)
    mv = unknowns_of_lattice(g.apply(qmg.OP_MATVEC, L, x), d, L)
    np.testing.assert_allclose(mv, A @ xu, rtol=0, atol=RTOL64 * np.abs(A @ xu).max())
    rs = unknowns_of_lattice(g.apply(qmg.OP_RESIDUAL, L, x, b), d, L)
    np.testing.assert_allclose(rs, bu - A @ xu, rtol=0, atol=RTOL64 * np.abs(bu - A @ xu).max())
    jac = unknowns_of_lattice(g.apply(qmg.OP_JACOBI, L, x, b), d, L)
    want = O.jacobi(A, A.diagonal(), xu, bu, 0.6)
    np.testing.assert_allclose(jac, want, rtol=0, atol=RTOL64 * np.abs(want).max())
    g.close()


@pytest.mark.parametrize("d,L", [(2, 3), (2, 5), (3, 2), (3, 3)])
def test_boxmg_prolongation_and_galerkin_operators(d, L):
    qmg = require_gpu()
    announce(f"boxmg+rap d={d} L={L}")
    p = W.random_checkerboard(d, L, seed=3, values=(1.0, 1e4), blocks=9 if L > 2 else 3)
    g = _grid(qmg, p, "boxmg", "hier64")
    info = g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    assert info["coarsest_level_used"] == H.lc
    # below the finest level both sides start from Galerkin operators that
    # already differ by rounding: bounds come from the oracle's own one-ulp
    # sensitivity (the finest-level P depends on rediscretised stencils only)
    tolP, tolA = operator_tolerance(p, "boxmg", H)
    for l in range(H.lc + 1, L + 1):
        tol = 1e-13 if l == L else tolP[l]
        Wg = g.prolongation(l)
        Wo = O.P_to_parent_weights(H.P[l], d, l)
        assert np.abs(Wg - Wo).max() <= tol, (l, np.abs(Wg - Wo).max(), tol)
    for l in range(H.lc, L):
        Sg = g.operator(l)
        So = O.csr_to_stencil(H.A[l], d, l)
        assert np.abs(Sg - So).max() <= tolA[l] * np.abs(So).max(), (l, np.abs(Sg - So).max(), tolA[l])
    g.close()


@pytest.mark.parametrize("d,L,contrast", [(2, 4, 1e4), (2, 5, 1e4), (3, 3, 1e4), (3, 3, 10.0)])
def test_boxmg_and_rap_steps_on_gpu_inputs(d, L, contrast):
    """Each construction step on the same input: the oracle's BoxMG applied to
    the GPU's level operator must give the GPU's weights, and the oracle's
    P^T A P of the GPU's A and P must give the GPU's coarse operator."""
    qmg = require_gpu()
    announce(f"boxmg/rap steps d={d} L={L} contrast={contrast:g}")
    p = W.random_checkerboard(d, L, seed=12, values=(1.0, contrast), blocks=9 if L > 2 else 3)
    g = _grid(qmg, p, "boxmg", "plain64")
    info = g.build()
    lc = info["coarsest_level_used"]
    for l in range(L, lc, -1):
        S = g.operator(l)
        Wg = g.prolongation(l)
        Wo = O.P_to_parent_weights(O.boxmg_P(S, d, l), d, l)
        assert np.abs(Wg - Wo).max() <= 1e-11, (l, np.abs(Wg - Wo).max())
        Ag = O.stencil_to_csr(S, d, l)
        Ac = O.csr_to_stencil(O.rap(Ag, weights_to_csr(Wg, d, l)), d, l - 1)
        Sc = g.operator(l - 1)
        assert np.abs(Sc - Ac).max() <= 1e-13 * np.abs(Ac).max(), (l, np.abs(Sc - Ac).max())
    g.close()


@pytest.mark.parametrize("transfer,store", [("galerkin", "hier64"), ("galerkin", "plain64"),
                                            ("geometric", "plain64"), ("boxmg", "plain64")])
def test_operators_other_transfers(transfer, store):
    qmg = require_gpu()
    announce(f"operators {transfer} {store}")
    d, L = 2, 4
    p = W.random_checkerboard(d, L, seed=4, values=(1.0, 50.0))
    g = _grid(qmg, p, transfer, store)
    g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer)
    for l in range(H.lc, L + 1):
        Sg, So = g.operator(l), O.csr_to_stencil(H.A[l], d, l)
        assert np.abs(Sg - So).max() <= 1e-11 * np.abs(So).max(), l
    for l in range(H.lc + 1, L + 1):
        assert np.abs(g.prolongation(l) - O.P_to_parent_weights(H.P[l], d, l)).max() <= 1e-11
    g.close()


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_restrict_and_prolong(d, L):
    qmg = require_gpu()
    announce(f"transfer ops d={d} L={L}")
    p = W.random_checkerboard(d, L, seed=6, values=(1.0, 1e4), blocks=3)
    g = _grid(qmg, p, "boxmg", "hier64")
    g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    rng = np.random.default_rng(7)
    r = rng.normal(size=p.n_unknowns)
    bc = unknowns_of_lattice(g.apply(qmg.OP_RESTRICT, L, lattice_of_unknowns(r, d, L)), d, L - 1)
    want = H.P[L].T @ r
    np.testing.assert_allclose(bc, want, rtol=0, atol=1e-13 * np.abs(want).max())
    e = rng.normal(size=H.P[L].shape[1])
    base = rng.normal(size=p.n_unknowns)
    up = unknowns_of_lattice(g.apply(qmg.OP_PROLONG, L, lattice_of_unknowns(e, d, L - 1),
                                     lattice_of_unknowns(base, d, L)), d, L)
    want = base + H.P[L] @ e
    np.testing.assert_allclose(up, want, rtol=0, atol=1e-13 * np.abs(want).max())
    g.close()


def _check_history(rr, hist, tols):
    """The two relative residuals of a cycle differ by at most the iterate
    bound of that cycle (triangle inequality on ||b - A u||)."""
    gap = np.abs(np.asarray(rr, dtype=np.float64) - np.asarray(hist))
    print("history gap per cycle", " ".join(f"{g:.1e}/{t:.1e}" for g, t in zip(gap, tols)))
    assert len(rr) == len(hist) and np.all(gap <= tols)


@pytest.mark.parametrize("d,L,transfer,store", [
    (2, 4, "geometric", "plain64"),   # small 2D Poisson shape of the first workload
    (2, 4, "boxmg", "hier64"),
    (2, 5, "boxmg", "plain64"),
    (3, 3, "boxmg", "hier64"),
    (3, 3, "galerkin", "hier64"),
])
def test_vcycle_iterates_match_oracle(d, L, transfer, store):
    qmg = require_gpu()
    announce(f"vcycles d={d} L={L} {transfer} {store}")
    if transfer == "geometric":
        p = W.poisson(d, L, seed=0)
    else:
        p = W.random_checkerboard(d, L, seed=8, values=(1.0, 1e4), blocks=9 if L > 2 else 3)
    k = 6
    g = _grid(qmg, p, transfer, store)
    g.build()
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer)
    b = O.rhs_from_f(p.f, d, L)
    uo, hist = O.solve(H, b, cycles=k)
    A = H.A[L]
    tols, _ = iterate_tolerances(p, transfer, H, k)
    diff = np.linalg.norm(A @ (u - uo)) / np.linalg.norm(b)
    print(f"iterate measure {diff:.3e} (bound {tols[-1]:.3e})")
    assert diff <= tols[-1]
    _check_history(rr, hist, tols)


def test_checkerboard2d_level6_full_size_cycles_and_solve():
    """The 729^2-cell jumping-coefficient workload at full size: 4 cycles match
    the oracle's iterate; the solve reaches 1e-8 by the oracle's own FP64
    recomputation of the residual; continued to 1e-13, the FP64 solution
    matches the oracle's direct solve of the fine system within 1e-12
    relative residual, ||A (u - u*)|| / ||b||."""
    qmg = require_gpu()
    announce("2D checkerboard level 6 full size")
    p = W.checkerboard2d(0)
    g = _grid(qmg, p, "boxmg", "hier64")
    g.build()
    rr = g.vcycle(4)
    u4 = g.solution()
    H = O.build_hierarchy(p.eps, 2, 6, transfer="boxmg")
    b = O.rhs_from_f(p.f, 2, 6)
    uo, hist = O.solve(H, b, cycles=4)
    A = H.A[6]
    tols, _ = iterate_tolerances(p, "boxmg", H, 4)
    diff = np.linalg.norm(A @ (u4 - uo)) / np.linalg.norm(b)
    print(f"iterate measure {diff:.3e} (bound {tols[-1]:.3e})")
    assert diff <= tols[-1]
    _check_history(rr, hist, tols)
    rep, _ = g.solve(1e-8, 400)
    u = g.solution()
    assert rep["status"] == "QMG_OK"
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8
    rep, _ = g.solve(1e-13, 400)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    ustar = O.direct_solve(A, b)
    dres = np.linalg.norm(A @ (u - ustar)) / np.linalg.norm(b)
    print(f"converged FP64 solution against the direct solve: {dres:.3e}")
    assert dres <= 1e-12


@pytest.mark.parametrize("store", ["hier32", "bf16", "hier16"])
def test_mixed_precision_reaches_tolerance(store):
    qmg = require_gpu()
    announce(f"mixed {store}")
    d, L = 2, 5
    p = W.random_checkerboard(d, L, seed=9, values=(1.0, 1e4))
    g = _grid(qmg, p, "boxmg", store)
    g.build()
    rep, hist = g.solve(1e-8, 400)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    b = O.rhs_from_f(p.f, d, L)
    A = H.A[L]
    assert rep["status"] == "QMG_OK"
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8
    ustar = O.direct_solve(A, b)
    u64, h64 = O.solve(H, b, tol=1e-8)
    err64 = np.linalg.norm(u64 - ustar) / np.linalg.norm(ustar)
    err = np.linalg.norm(u - ustar) / np.linalg.norm(ustar)
    assert err <= 10 * max(err64, 1e-12)
    assert rep["cycles"] <= 1.5 * len(h64) + 3


def test_constant_coefficient_store_is_empty():
    qmg = require_gpu()
    announce("constant eps store")
    p = W.poisson(2, 5, seed=1)
    g = _grid(qmg, p, "boxmg", "hier64")
    info = g.build()
    g.close()
    assert info["zero_delta_fraction"] == 1.0


def test_raised_coarsest_level_and_errors():
    qmg = require_gpu()
    announce("coarsest level 2, error paths")
    p = W.random_checkerboard(2, 4, seed=10, values=(1.0, 10.0))
    g = _grid(qmg, p, "boxmg", "hier64", coarsest_level=2)
    info = g.build()
    assert info["coarsest_level_used"] == 2
    rep, _ = g.solve(1e-10, 200)
    assert rep["status"] == "QMG_OK"
    g.close()
    with pytest.raises(qmg.QmgError):
        qmg.Grid(2, 4, qmg.make_opts(omega=2.5))
    with pytest.raises(qmg.QmgError):      # BPX takes one Jacobi step per level
        qmg.Grid(2, 4, qmg.make_opts(cycle="bpx", smoother="block"))
    with pytest.raises(qmg.QmgError):
        qmg.Grid(2, 4, qmg.make_opts(cycle=3))
    g = qmg.Grid(2, 3, qmg.make_opts())
    with pytest.raises(qmg.QmgError):      # solve before build
        g.solve()
    bad = np.ones((27, 27))
    bad[3, 3] = -1.0
    with pytest.raises(qmg.QmgError):
        g.set_coefficients(bad, np.zeros(26 * 26))
    g.close()


def test_device_inputs_match_host_inputs():
    """Coefficients handed over in device memory give bitwise the result of
    the host hand-over; bad device values are rejected and leave the grid
    without coefficients."""
    import torch
    qmg = require_gpu()
    announce("device-resident inputs")
    p = W.checkerboard2d(0, level=4)
    res = []
    for dev in (False, True):
        g = qmg.Grid(p.dim, p.level, qmg.make_opts())
        if dev:
            g.set_coefficients(torch.from_numpy(p.eps.ravel()).cuda(), torch.from_numpy(p.f.ravel()).cuda())
        else:
            g.set_coefficients(p.eps, p.f)
        g.build()
        rr = g.vcycle(4)
        res.append((rr, g.solution()))
        g.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    g = qmg.Grid(p.dim, p.level, qmg.make_opts())
    bad = torch.from_numpy(p.eps.ravel()).cuda()
    bad[17] = float("nan")
    with pytest.raises(qmg.QmgError):
        g.set_coefficients(bad, torch.from_numpy(p.f.ravel()).cuda())
    with pytest.raises(qmg.QmgError):      # no coefficients: build is refused
        g.build()
    g.close()


def test_profiling_and_graphs_leave_results_unchanged():
    """Event timing of the finest sweeps and graph replay of the cycles change
    neither the iterates nor the residual history."""
    qmg = require_gpu()
    announce("profiling strides and graph replay")
    p = W.checkerboard2d(0, level=4)
    out = []
    for every, graphs in ((0, True), (0, False), (1, True), (3, False)):
        g = qmg.Grid(p.dim, p.level, qmg.make_opts(graphs=graphs))
        g.set_coefficients(p.eps, p.f)
        g.profile(every)
        g.build()
        rep, hist = g.solve(1e-8, 200)
        n, ms = g.profile_read()
        if every:
            assert n > 0 and ms > 0.0
        else:
            assert n == 0
        out.append((hist, g.solution()))
        g.close()
    for hist, u in out[1:]:
        assert np.array_equal(hist, out[0][0]) and np.array_equal(u, out[0][1])


@pytest.mark.parametrize("d,L,mu,omega,lc", [
    (2, 4, (1, 1), 0.6, 1),     # single-sweep passes
    (2, 4, (2, 1), 0.6, 1),     # odd sweep count per cycle: eager launches
    (2, 5, (3, 3), 0.8, 1),     # a pass of two sweeps then one of one
    (2, 4, (2, 2), 0.6, 2),     # coarsest level 2: 64 unknowns, exact solve
    (3, 3, (1, 2), 0.7, 1),
    (3, 3, (2, 2), 0.6, 2),     # 3D coarsest level 2: 512 unknowns
])
def test_cycle_options_match_oracle(d, L, mu, omega, lc):
    """Smoothing counts, damping and coarsest level other than the defaults:
    iterates and residual histories against the oracle (Galerkin, moderate
    contrast, so rounding stays far below the tolerance)."""
    qmg = require_gpu()
    announce(f"cycle options d={d} L={L} mu={mu} omega={omega} lc={lc}")
    p = W.random_checkerboard(d, L, seed=3, values=(1.0, 10.0))
    g = qmg.Grid(d, L, qmg.make_opts("galerkin", "hier64", mu=mu, omega=omega, coarsest_level=lc))
    g.set_coefficients(p.eps, p.f)
    info = g.build()
    assert info["coarsest_level_used"] == lc
    k = 5
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer="galerkin", lc=lc, omega=omega, mu_pre=mu[0], mu_post=mu[1])
    b = O.rhs_from_f(p.f, d, L)
    uo, hist = O.solve(H, b, cycles=k)
    np.testing.assert_allclose(rr, hist, rtol=1e-10, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-11 * np.abs(uo).max()


@pytest.mark.parametrize("store", ["hier32", "bf16"])
def test_mixed_inner_cycles(store):
    """Two FP32 inner cycles per FP64 outer iteration: fewer outer iterations,
    the same FP64 tolerance (recomputed by the oracle)."""
    qmg = require_gpu()
    announce(f"mixed inner cycles 2 {store}")
    p = W.random_checkerboard(2, 5, seed=4, values=(1.0, 1e3))
    out = {}
    for inner in (1, 2):
        g = qmg.Grid(2, 5, qmg.make_opts("boxmg", store, inner_cycles=inner))
        g.set_coefficients(p.eps, p.f)
        g.build()
        rep, _ = g.solve(1e-8, 300)
        assert rep["status"] == "QMG_OK"
        out[inner] = (rep, g.solution())
        g.close()
    H = O.build_hierarchy(p.eps, 2, 5, transfer="boxmg")
    b = O.rhs_from_f(p.f, 2, 5)
    for inner, (rep, u) in out.items():
        rr = np.linalg.norm(b - H.A[5] @ u) / np.linalg.norm(b)
        assert rr <= 1e-8 * (1 + 1e-6)
    assert out[2][0]["outer_iters"] < out[1][0]["outer_iters"]
    assert out[2][0]["cycles"] == 2 * (out[2][0]["outer_iters"] - 1)


# ---------------------------------------------------------------------------
# Dynamic coarsest level (Sect. 4.3): raise between cycles on stagnation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("transfer,store", [("geometric", "hier64"), ("geometric", "plain64"),
                                            ("galerkin", "hier64"), ("galerkin", "plain64")])
def test_stagnation_raise_on_jump_matches_oracle(transfer, store):
    """The paper's jump setup (eps 1 | 0.1 at x = 0.5, f = 1) with V(1,1)
    cycles, omega 0.9: the residual grows over the first cycles, the
    coarsest level moves up after each of them (threshold 1: growth only),
    and the solve converges.  Cycle count, raised level, residual history and
    iterate against the oracle; every decision's ratio lies at least 1e-3
    from the threshold, so rounding cannot flip one.""" 
    qmg = require_gpu()
    announce(f"stagnation raise jump 2D L5 {transfer} {store}")
    p = W.material_jump(2, 5)
    H = O.build_hierarchy(p.eps, 2, 5, transfer=transfer, omega=0.9, mu_pre=1, mu_post=1,
                          check_definite=False)
    b = O.rhs_from_f(p.f, 2, 5)
    uo, ho = O.solve(H, b, tol=1e-8, max_cycles=300, stagnation=1.0)
    ratios = np.array(ho) / np.array([1.0] + ho[:-1])
    assert np.abs(ratios - 1.0).min() > 1e-3
    assert H.lc > 1 and ho[-1] <= 1e-8
    g = qmg.Grid(2, 5, qmg.make_opts(transfer, store, mu=(1, 1), omega=0.9, check_definite=False,
                                     stagnation=1.0))
    g.set_coefficients(p.eps, p.f)
    g.build()
    rep, hist = g.solve(1e-8, 300)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    assert rep["coarsest_level_used"] == H.lc
    assert rep["cycles"] == len(ho)
    # the residual norm of an FP64 iterate carries ~1e-14 of rounding relative
    # to ||b|| (f = 1 gives |u| ~ 0.1 against |b| ~ 1e-3 per vertex)
    np.testing.assert_allclose(hist, ho, rtol=1e-9, atol=1e-13)
    assert np.abs(u - uo).max() <= 1e-10 * np.abs(uo).max()


@pytest.mark.parametrize("d,L,transfer,store", [(2, 4, "boxmg", "hier64"), (2, 5, "boxmg", "hier64"),
                                                (2, 4, "boxmg", "plain64"), (3, 3, "boxmg", "hier64"),
                                                (3, 3, "galerkin", "hier64")])
def test_raise_after_every_cycle_matches_oracle(d, L, transfer, store):
    """A threshold no cycle meets moves the coarsest level up after every
    cycle until L - 1: each raised level's stored operator is decoded for its
    exact solve (or smoothed when larger than 1024 unknowns, level 4 in 2D),
    and the fused coarse levels are rebuilt.  History and iterate against the
    oracle."""
    qmg = require_gpu()
    announce(f"raise every cycle d={d} L={L} {transfer} {store}")
    p = W.random_checkerboard(d, L, seed=6, values=(1.0, 10.0), blocks=9 if L > 3 else 3)
    k = L + 1
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, check_definite=False)
    b = O.rhs_from_f(p.f, d, L)
    uo, ho = O.solve(H, b, tol=1e-30, max_cycles=k, stagnation=1e-12)
    assert H.lc == L - 1
    g = qmg.Grid(d, L, qmg.make_opts(transfer, store, check_definite=False, stagnation=1e-12))
    g.set_coefficients(p.eps, p.f)
    g.build()
    rep, hist = g.solve(1e-30, k)
    u = g.solution()
    assert rep["coarsest_level_used"] == L - 1 and rep["cycles"] == k
    np.testing.assert_allclose(hist, ho, rtol=1e-10, atol=0)
    assert np.abs(u - uo).max() <= 1e-11 * np.abs(uo).max()
    # a new build starts again from the requested coarsest level
    info = g.build()
    assert info["coarsest_level_used"] == 1
    g.close()


@pytest.mark.parametrize("store", ["hier32", "bf16"])
def test_raise_with_fp32_iterates(store):
    """Raises between FP64 outer iterations: the inner FP32 cycles continue
    on the raised hierarchy and the FP64 tolerance is reached (the oracle
    recomputes the residual)."""
    qmg = require_gpu()
    announce(f"raise every outer iteration {store}")
    p = W.random_checkerboard(2, 4, seed=4, values=(1.0, 1e3))
    g = qmg.Grid(2, 4, qmg.make_opts("boxmg", store, check_definite=False, stagnation=1e-12))
    g.set_coefficients(p.eps, p.f)
    g.build()
    rep, _ = g.solve(1e-8, 300)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK" and rep["coarsest_level_used"] == 3
    H = O.build_hierarchy(p.eps, 2, 4, transfer="boxmg", check_definite=False)
    b = O.rhs_from_f(p.f, 2, 4)
    assert np.linalg.norm(b - H.A[4] @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)


def test_3d_level5_single_steps_full_size():
    """The 3D levels large enough for the plane-marching kernel (level 5 and
    up: 64 x 8 tiles marching over 32-plane chunks): matrix-vector product,
    residual, Jacobi sweep and the sweep from a zero iterate on a 3D level-5
    grid (242^3 unknowns; the tiles are ragged on every axis), on the whole
    lattice against the oracle's rediscretised operator."""
    from oracle import adaptive as AD
    qmg = require_gpu()
    announce("3D level 5 single steps (marching kernel)")
    d, L = 3, 5
    p = W.random_checkerboard(d, L, seed=7, values=(1.0, 1e3))
    g = _grid(qmg, p, "geometric", "hier64")
    rng = np.random.default_rng(8)
    x = lattice_of_unknowns(rng.normal(size=p.n_unknowns), d, L)
    b = lattice_of_unknowns(rng.normal(size=p.n_unknowns), d, L)
    S = O.geometric_stencil(p.eps, d, L)
    Ax = AD._apply(S, x, d)
    del S
    inner = (slice(1, 3 ** L),) * d
    D = O.geometric_stencil(p.eps, d, L)[(3 ** d) // 2]

    def close(got, want):
        tol = RTOL64 * np.abs(want[inner]).max()
        assert np.abs(got[inner] - want[inner]).max() <= tol

    close(g.apply(qmg.OP_MATVEC, L, x), Ax)
    close(g.apply(qmg.OP_RESIDUAL, L, x, b), b - Ax)
    jac = np.zeros_like(x)
    jac[inner] = x[inner] + 0.6 * (b[inner] - Ax[inner]) / D[inner]
    close(g.apply(qmg.OP_JACOBI, L, x, b), jac)
    zero = np.zeros_like(x)
    zero[inner] = 0.6 * b[inner] / D[inner]
    close(g.apply(qmg.OP_JACOBI, L, None, b), zero)
    g.close()
    # block Jacobi (one Gauss-Seidel sweep): the oracle's step on lattice
    # arrays, the patch positions in lexicographic order taken as masks
    g = qmg.Grid(d, L, qmg.make_opts("geometric", "hier64", smoother="block", bj_sweeps=1))
    g.set_coefficients(p.eps, p.f)
    S = O.geometric_stencil(p.eps, d, L)
    idx = np.arange(3 ** L + 1)
    want = x.copy()
    iota = np.zeros(x.shape, dtype=bool)
    for q in range(2 ** d):
        loc = [1 + ((q >> a) & 1) for a in range(d)]          # x, y, z offsets in the patch
        m = np.ones(x.shape, dtype=bool)
        for a in range(d):
            ax = (idx % 3 == loc[a]) & (idx > 0) & (idx < 3 ** L)
            shape = [1] * d
            shape[d - 1 - a] = -1
            m &= ax.reshape(shape)
        want[m] = want[m] + (b[m] - AD._apply(S, want, d)[m]) / D[m]
        iota |= m
    jb = want + 0.6 * (b - AD._apply(S, want, d)) / np.where(D != 0, D, 1.0)
    jb[iota] = want[iota]
    del S
    close(g.apply(qmg.OP_SMOOTH, L, x, b), jb)
    g.close()


# ---------------------------------------------------------------------------
# Block Jacobi smoother
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,transfer,store,sweeps", [(2, 4, "galerkin", "hier64", 1), (2, 4, "boxmg", "plain64", 3),
                                                       (3, 3, "boxmg", "hier64", 2), (2, 5, "galerkin", "hier64", 4)])
def test_block_jacobi_step_matches_oracle(d, L, transfer, store, sweeps):
    """One block Jacobi step (Gauss-Seidel on every patch's iota-vertices,
    damped Jacobi on the rest) on the finest level (rediscretised or plain
    rows) and on the next coarser level (stored Galerkin rows)."""
    qmg = require_gpu()
    announce(f"block jacobi step d={d} L={L} {transfer} {store} sweeps={sweeps}")
    p = W.random_checkerboard(d, L, seed=9, values=(1.0, 1e3), blocks=9 if L > 2 else 3)
    g = _grid(qmg, p, transfer, store, smoother="block", bj_sweeps=sweeps, check_definite=False)
    g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, check_definite=False)
    rng = np.random.default_rng(10)
    for l in (L, L - 1):
        x = rng.normal(size=(3 ** l - 1) ** d)
        b = rng.normal(size=(3 ** l - 1) ** d)
        got = unknowns_of_lattice(g.apply(qmg.OP_SMOOTH, l, lattice_of_unknowns(x, d, l),
                                          lattice_of_unknowns(b, d, l)), d, l)
        A = H.A[l]
        want = O.block_jacobi(A, A.diagonal(), x, b, 0.6, sweeps, d, l)
        tol = 1e-12 if l == L else 1e-10
        assert np.abs(got - want).max() <= tol * np.abs(want).max(), (l, np.abs(got - want).max())
    g.close()


@pytest.mark.parametrize("d,L,transfer,store,sweeps", [(2, 4, "galerkin", "hier64", 1), (2, 5, "boxmg", "hier64", 3),
                                                       (3, 3, "boxmg", "hier64", 1), (2, 4, "geometric", "plain64", 2)])
def test_block_jacobi_cycles_match_oracle(d, L, transfer, store, sweeps):
    """V(2,2) cycles with the block smoother on every level (the coarse
    levels inside the fused LDS kernel): residual history and iterate
    against the oracle."""
    qmg = require_gpu()
    announce(f"block jacobi cycles d={d} L={L} {transfer} {store} sweeps={sweeps}")
    p = W.random_checkerboard(d, L, seed=11, values=(1.0, 1e2), blocks=9 if L > 3 else 3)
    g = _grid(qmg, p, transfer, store, smoother="block", bj_sweeps=sweeps, check_definite=False)
    g.build()
    k = 5
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, check_definite=False, smoother="block",
                          bj_sweeps=sweeps)
    uo, hist = O.solve(H, O.rhs_from_f(p.f, d, L), cycles=k)
    np.testing.assert_allclose(rr, hist, rtol=1e-10, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-11 * np.abs(uo).max()


@pytest.mark.parametrize("store", ["hier64", "bf16"])
def test_block_jacobi_solve_fewer_cycles(store):
    """To the same tolerance (recomputed by the oracle), the block smoother
    needs fewer cycles than point Jacobi, in FP64 and with FP32 iterates."""
    qmg = require_gpu()
    announce(f"block jacobi solve {store}")
    p = W.random_checkerboard(2, 5, seed=4, values=(1.0, 1e4))
    reps = {}
    for sm in ("jacobi", "block"):
        g = _grid(qmg, p, "boxmg", store, smoother=sm, bj_sweeps=3)
        g.build()
        rep, _ = g.solve(1e-8, 500)
        assert rep["status"] == "QMG_OK"
        u = g.solution()
        g.close()
        H = O.build_hierarchy(p.eps, 2, 5, transfer="boxmg")
        b = O.rhs_from_f(p.f, 2, 5)
        assert np.linalg.norm(b - H.A[5] @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
        reps[sm] = rep
    assert reps["block"]["outer_iters"] < reps["jacobi"]["outer_iters"]


# ---------------------------------------------------------------------------
# Additive cycles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,transfer,store,omega,damping", [
    (2, 4, "geometric", "hier64", 0.8, "exp"), (2, 5, "boxmg", "hier64", 0.6, "const"),
    (3, 3, "galerkin", "hier64", 0.8, "exp"), (2, 4, "boxmg", "plain64", 0.6, "exp")])
def test_additive_cycles_match_oracle(d, L, transfer, store, omega, damping):
    """Additive cycles (restricted fine residual, one damped Jacobi step from
    zero per level, prolongated sum of corrections): residual history and
    iterate against the oracle."""
    qmg = require_gpu()
    announce(f"additive cycles d={d} L={L} {transfer} {store} omega={omega} {damping}")
    p = W.random_checkerboard(d, L, seed=13, values=(1.0, 1e2), blocks=9 if L > 3 else 3)
    g = _grid(qmg, p, transfer, store, omega=omega, cycle="add", damping=damping, check_definite=False)
    g.build()
    k = 6
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, omega=omega, check_definite=False)
    uo, hist = O.solve_additive(H, O.rhs_from_f(p.f, d, L), damping=damping, cycles=k)
    np.testing.assert_allclose(rr, hist, rtol=1e-10, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-11 * np.abs(uo).max()


@pytest.mark.parametrize("store", ["hier64", "bf16"])
def test_additive_solve_sine_setup(store):
    """The paper's sin setup with omega = 0.8 and exponential damping, solved
    to 1e-8 (the oracle recomputes the residual), in FP64 and with FP32 inner
    cycles; the FP64 run takes the oracle's cycle count."""
    qmg = require_gpu()
    announce(f"additive solve sin {store}")
    p = W.sin_source(2, 5)
    g = _grid(qmg, p, "geometric", store, omega=0.8, cycle="add")
    g.build()
    rep, _ = g.solve(1e-8, 600)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    H = O.build_hierarchy(p.eps, 2, 5, transfer="geometric", omega=0.8)
    b = O.rhs_from_f(p.f, 2, 5)
    assert np.linalg.norm(b - H.A[5] @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    if store == "hier64":
        _, hist = O.solve_additive(H, b, tol=1e-8, max_cycles=600)
        assert abs(rep["cycles"] - len(hist)) <= 1   # the batched loop may stop one cycle late


# ---------------------------------------------------------------------------
# BPX cycles
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,transfer,store,omega,damping", [
    (2, 4, "geometric", "hier64", 0.8, "const"), (2, 5, "boxmg", "hier64", 0.6, "exp"),
    (3, 3, "galerkin", "hier64", 0.8, "const"), (2, 5, "boxmg", "plain64", 0.8, "const")])
def test_bpx_cycles_match_oracle(d, L, transfer, store, omega, damping):
    """BPX cycles (each level adds only the hierarchical surplus of its Jacobi
    step): residual history and iterate against the oracle."""
    qmg = require_gpu()
    announce(f"bpx cycles d={d} L={L} {transfer} {store} omega={omega} {damping}")
    p = W.random_checkerboard(d, L, seed=17, values=(1.0, 1e2), blocks=9 if L > 3 else 3)
    g = _grid(qmg, p, transfer, store, omega=omega, cycle="bpx", damping=damping, check_definite=False)
    g.build()
    k = 6
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, omega=omega, check_definite=False)
    uo, hist = O.solve_additive(H, O.rhs_from_f(p.f, d, L), damping=damping, cycles=k, bpx=True)
    np.testing.assert_allclose(rr, hist, rtol=1e-10, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-11 * np.abs(uo).max()


@pytest.mark.parametrize("store", ["hier64", "bf16"])
def test_bpx_solve_sine_constant_omega(store):
    """The sin setup with omega = 0.8 on every level (where the additive cycle
    diverges) solved to 1e-8 by BPX cycles, in FP64 and with FP32 inner
    cycles; the FP64 run takes the oracle's cycle count."""
    qmg = require_gpu()
    announce(f"bpx solve sin {store}")
    p = W.sin_source(2, 5)
    g = _grid(qmg, p, "geometric", store, omega=0.8, cycle="bpx", damping="const")
    g.build()
    rep, _ = g.solve(1e-8, 600)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    H = O.build_hierarchy(p.eps, 2, 5, transfer="geometric", omega=0.8)
    b = O.rhs_from_f(p.f, 2, 5)
    assert np.linalg.norm(b - H.A[5] @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    if store == "hier64":
        _, hist = O.solve_additive(H, b, tol=1e-8, max_cycles=600, damping="const", bpx=True)
        assert abs(rep["cycles"] - len(hist)) <= 1   # the batched loop may stop one cycle late


# ---------------------------------------------------------------------------
# The bpa store (the paper's codec)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,eps_mf", [(2, 5, 1e-2), (2, 5, 1e-8), (3, 3, 1e-4)])
def test_bpa_operators_and_cycles_match_oracle(d, L, eps_mf):
    """Per-cell random coefficients (BoxMG and Galerkin deltas on every
    level): the decoded operators and weights equal the oracle's bpa
    hierarchy, lie within eps_mf of the uncompressed FP64 store, and six
    cycles give the oracle's residual history and iterate."""
    qmg = require_gpu()
    announce(f"bpa store d={d} L={L} eps_mf={eps_mf:g}")
    p = W.random_checkerboard(d, L, seed=21, values=(1.0, 10.0), blocks=3 ** L)
    ref = _grid(qmg, p, "boxmg", "hier64", check_definite=False)
    ref.build()
    g = _grid(qmg, p, "boxmg", "bpa", eps_mf=eps_mf, check_definite=False)
    info = g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg", check_definite=False)
    Hq = O.solver.quantised_hierarchy(H, "bpa", eps_mf=eps_mf)
    assert info["coarsest_level_used"] == H.lc
    _, tolA = operator_tolerance(p, "boxmg", H, check_definite=False)
    for l in range(H.lc, L):
        Sg, Sr = g.operator(l), ref.operator(l)
        # the coarsest level's exact solve keeps the full FP64 operator
        So = O.csr_to_stencil((H if l == H.lc else Hq).A[l], d, l)
        assert np.abs(Sg - Sr).max() <= eps_mf * (1 + 1e-9), l
        assert np.abs(Sg - So).max() <= tolA[l] * np.abs(So).max(), (l, np.abs(Sg - So).max())
    for l in range(H.lc + 1, L + 1):
        Wg, Wr = g.prolongation(l), ref.prolongation(l)
        Wo = O.P_to_parent_weights(Hq.P[l], d, l)
        assert np.abs(Wg - Wr).max() <= eps_mf * (1 + 1e-9), l
        assert np.abs(Wg - Wo).max() <= 1e-11, (l, np.abs(Wg - Wo).max())
    rr = g.vcycle(6)
    u = g.solution()
    g.close()
    ref.close()
    uo, hist = O.solve(Hq, O.rhs_from_f(p.f, d, L), cycles=6)
    np.testing.assert_allclose(rr, hist, rtol=1e-9, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-10 * np.abs(uo).max()


def test_bpa_store_sizes():
    """Constant coefficients compress to nothing (every delta block dropped);
    on the per-cell random setup a loose eps_mf stores fewer bytes than a
    tight one, and both fewer than the FP64 deltas.  eps_mf outside (0, 1]
    and the bpa store on an adaptive grid are rejected."""
    qmg = require_gpu()
    announce("bpa store sizes")
    p = W.sin_source(2, 5)
    g = _grid(qmg, p, "boxmg", "bpa")
    info = g.build()
    g.close()
    assert info["zero_delta_fraction"] == 1.0
    p = W.random_checkerboard(2, 5, seed=21, values=(1.0, 10.0), blocks=243)
    sizes = {}
    for store, eps in (("hier64", 1e-8), ("bpa", 1e-8), ("bpa", 1e-2)):
        g = _grid(qmg, p, "boxmg", store, eps_mf=eps, check_definite=False)
        sizes[(store, eps)] = g.build()["bytes_operators"]
        g.close()
    assert sizes[("bpa", 1e-2)] < sizes[("bpa", 1e-8)] < sizes[("hier64", 1e-8)]
    for bad in (0.0, -1.0, 2.0):
        with pytest.raises(qmg.QmgError):
            qmg.Grid(2, 4, qmg.make_opts("boxmg", "bpa", eps_mf=bad))
    P = W.adaptive_balls(dim=2, base=2, level=3, n_balls=1)
    with pytest.raises(qmg.QmgError):
        qmg.Grid(2, 3, qmg.make_opts("boxmg", "bpa"), base_level=2, refine=P.flags)


# ---------------------------------------------------------------------------
# Convection-diffusion (the circle setup) and Petrov-Galerkin injection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,transfer,restriction", [
    (2, 4, "boxmg", "transpose"), (2, 5, "galerkin", "injection"),
    (3, 3, "boxmg", "transpose"), (2, 4, "boxmg", "injection"),
    (2, 5, "boxmg", "aggregation"), (3, 3, "galerkin", "aggregation")])
def test_convection_operators_and_cycles_match_oracle(d, L, transfer, restriction):
    """The circle flow with eps = 0.1 (1 above z = 1/2 in 3D): the finest
    operator with its convection term, the BoxMG weights, the (Petrov-)
    Galerkin coarse operators and six cycles against the oracle.  In 3D the
    convection entries on the face neighbours (zero in the Q1 diffusion
    stencil) break diagonal dominance on every level, so the check is off."""
    qmg = require_gpu()
    announce(f"convection d={d} L={L} {transfer} R={restriction}")
    p = W.circle(d, L, 0.1, seed=5)
    chk = d == 2
    g = qmg.Grid(d, L, qmg.make_opts(transfer, "plain64", restriction=restriction, check_definite=chk))
    g.set_coefficients(p.eps, p.f, v=p.meta["v"])
    info = g.build()
    H = O.build_hierarchy(p.eps, d, L, transfer=transfer, v=p.meta["v"], restriction=restriction,
                          check_definite=chk)
    assert info["coarsest_level_used"] == H.lc
    for l in range(H.lc, L + 1):
        Sg, So = g.operator(l), O.csr_to_stencil(H.A[l], d, l)
        tol = 1e-13 if l == L else 1e-11
        assert np.abs(Sg - So).max() <= tol * np.abs(So).max(), (l, np.abs(Sg - So).max())
    for l in range(H.lc + 1, L + 1):
        assert np.abs(g.prolongation(l) - O.P_to_parent_weights(H.P[l], d, l)).max() <= 1e-11, l
    rr = g.vcycle(6)
    u = g.solution()
    g.close()
    uo, hist = O.solve(H, O.rhs_from_f(p.f, d, L), cycles=6)
    np.testing.assert_allclose(rr, hist, rtol=1e-9, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-10 * np.abs(uo).max()


def test_convection_circle_full_solve_and_errors():
    """The 2D circle setup at level 6 (728^2 unknowns) with BoxMG solved to
    1e-8 (residual recomputed by the oracle), and the restrictions of the
    convection input and of injection."""
    qmg = require_gpu()
    announce("convection circle 2D L6 solve")
    p = W.circle(2, 6, 0.1, seed=5)
    g = qmg.Grid(2, 6, qmg.make_opts("boxmg", "plain64"))
    g.set_coefficients(p.eps, p.f, v=p.meta["v"])
    g.build()
    rep, _ = g.solve(1e-8, 200)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, 2, 6) + O.convection_stencil(p.meta["v"], 2, 6), 2, 6)
    b = O.rhs_from_f(p.f, 2, 6)
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    g = qmg.Grid(2, 3, qmg.make_opts("boxmg", "hier64"))
    q = W.circle(2, 3, 0.1)
    with pytest.raises(qmg.QmgError):      # convection needs the plain store
        g.set_coefficients(q.eps, q.f, v=q.meta["v"])
    g.close()
    with pytest.raises(qmg.QmgError):      # injection is a Petrov-Galerkin restriction
        qmg.Grid(2, 3, qmg.make_opts("geometric", "plain64", restriction="injection"))
    with pytest.raises(qmg.QmgError):
        qmg.Grid(2, 3, qmg.make_opts("boxmg", "plain64", restriction="injection", cycle="add"))
    g = qmg.Grid(2, 3, qmg.make_opts("boxmg", "plain64"))
    bad = q.meta["v"].copy()
    bad[1, 2, 3] = np.inf
    with pytest.raises(qmg.QmgError):
        g.set_coefficients(q.eps, q.f, v=bad)
    g.close()


# ---------------------------------------------------------------------------
# Refinement criterion (dynamic adaptivity)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,L,fraction", [(2, 5, 0.1), (2, 4, 0.3), (3, 3, 0.1)])
def test_refine_flags_match_oracle(d, L, fraction):
    """A seeded iterate (smooth field, bumps and noise) on a checkerboard
    setup: the cells flagged by the mean-difference criterion with ten bins
    equal the oracle's, for a residual threshold between two of the oracle's
    residual magnitudes near their median."""
    qmg = require_gpu()
    announce(f"refine flags d={d} L={L} fraction={fraction}")
    p = W.random_checkerboard(d, L, seed=8, values=(1.0, 10.0), blocks=9 if L > 3 else 3)
    g = _grid(qmg, p, "boxmg", "hier64")
    g.build()
    n = 3 ** L
    rng = np.random.default_rng(31)
    x = np.meshgrid(*([np.arange(1, n) / n] * d), indexing="ij")
    u = np.prod([np.sin(np.pi * xi) for xi in x], axis=0)
    u = u + 0.01 * rng.normal(size=u.shape)
    idx = rng.integers(0, n - 1, size=(6, d))
    u[tuple(idx.T)] += 0.5
    u = u.ravel()
    g.set_solution(u)
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
    b = O.rhs_from_f(p.f, d, L)
    r = b - A @ u
    s = np.sort(np.abs(r))
    k = len(s) // 2
    while s[k + 1] - s[k] <= 1e-9 * s[k]:
        k += 1
    res_tol = 0.5 * (s[k] + s[k + 1])
    flags = g.refine_flags(res_tol, fraction)
    g.close()
    want = O.refine.refinement_flags(O.fem.lattice_from_unknowns(u, d, L),
                                     O.fem.lattice_from_unknowns(r, d, L), d, res_tol, fraction)
    assert want.any() and not want.all()
    assert np.array_equal(flags, want), (int(flags.sum()), int(want.sum()))


# ---------------------------------------------------------------------------
# Smallest grids and degenerate settings of the optional paths
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("case", ["bpx", "bpa_loose", "convection_injection", "convection_aggregation"])
def test_optional_paths_on_the_smallest_grid(d, case):
    """Level 2 (two levels, an exact level-1 solve): BPX cycles, the bpa store
    with eps_mf = 1 (every delta codes to zero, so the operators are the
    rediscretised ones plus nothing), and the Petrov-Galerkin convection
    variants, each against the oracle over four cycles."""
    qmg = require_gpu()
    announce(f"smallest grid d={d} {case}")
    L = 2
    if case.startswith("convection"):
        r = case.split("_")[1]
        p = W.circle(d, L, 0.1, seed=2)
        g = qmg.Grid(d, L, qmg.make_opts("boxmg", "plain64", restriction=r, check_definite=False))
        g.set_coefficients(p.eps, p.f, v=p.meta["v"])
        H = O.build_hierarchy(p.eps, d, L, transfer="boxmg", v=p.meta["v"], restriction=r,
                              check_definite=False)
        step = lambda: O.solve(H, O.rhs_from_f(p.f, d, L), cycles=4)
    else:
        p = W.random_checkerboard(d, L, seed=4, values=(1.0, 30.0), blocks=3)
        if case == "bpx":
            g = _grid(qmg, p, "boxmg", "hier64", cycle="bpx", damping="const")
            H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
            step = lambda: O.solve_additive(H, O.rhs_from_f(p.f, d, L), damping="const", cycles=4, bpx=True)
        else:
            g = _grid(qmg, p, "boxmg", "bpa", eps_mf=1.0)
            H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
            Hq = O.solver.quantised_hierarchy(H, "bpa", eps_mf=1.0)
            step = lambda: O.solve(Hq, O.rhs_from_f(p.f, d, L), cycles=4)
    info = g.build()
    rr = g.vcycle(4)
    u = g.solution()
    g.close()
    uo, hist = step()
    assert info["coarsest_level_used"] == 1
    np.testing.assert_allclose(rr, hist, rtol=1e-9, atol=1e-14)
    assert np.abs(u - uo).max() <= 1e-10 * np.abs(uo).max()


def test_refine_flags_degenerate_settings():
    """No candidate (threshold below every residual): nothing is flagged;
    fraction 1: every candidate is chosen, as in the oracle."""
    qmg = require_gpu()
    announce("refine flags degenerate")
    d, L = 2, 3
    p = W.random_checkerboard(d, L, seed=9, values=(1.0, 5.0), blocks=3)
    g = _grid(qmg, p, "boxmg", "hier64")
    g.build()
    n = 3 ** L
    u = np.random.default_rng(5).normal(size=(n - 1) ** d)
    g.set_solution(u)
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
    r = O.rhs_from_f(p.f, d, L) - A @ u
    tiny = 0.5 * np.abs(r).min()
    assert not g.refine_flags(tiny, 0.1).any()
    big = 2.0 * np.abs(r).max()
    flags = g.refine_flags(big, 1.0)
    g.close()
    want = O.refine.refinement_flags(O.fem.lattice_from_unknowns(u, d, L),
                                     O.fem.lattice_from_unknowns(r, d, L), d, big, 1.0)
    assert np.array_equal(flags, want) and want.all()


# ---------------------------------------------------------------------------
# The timed variants at their full size
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["additive_exp", "bpx_const", "bpa_checkerboard"])
def test_timed_variants_full_size(case):
    """The level-6 workloads the benchmark times besides the main one: the
    sine setup under additive (exponential damping) and BPX (omega on every
    level) cycles, and the 729^2-cell checkerboard with the bpa store at
    eps_mf = 1e-8; each solve reaches 1e-8 by the oracle's FP64 recomputation
    of the residual, and the bpa solve takes the FP64 store's cycle count."""
    qmg = require_gpu()
    announce(f"timed variant full size {case}")
    if case == "bpa_checkerboard":
        p = W.checkerboard2d(0)
        g = _grid(qmg, p, "boxmg", "bpa", eps_mf=1e-8)
        ref = _grid(qmg, p, "boxmg", "hier64")
        ref.build()
        rref, _ = ref.solve(1e-8, 400)
        ref.close()
        A = O.stencil_to_csr(O.geometric_stencil(p.eps, 2, 6), 2, 6)
    else:
        p = W.sin_source(2, 6)
        kw = dict(cycle="add", damping="exp") if case == "additive_exp" else dict(cycle="bpx", damping="const")
        g = _grid(qmg, p, "geometric", "hier64", omega=0.8, **kw)
        A = O.stencil_to_csr(O.geometric_stencil(p.eps, 2, 6), 2, 6)
    g.build()
    rep, _ = g.solve(1e-8, 1000)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK"
    b = O.rhs_from_f(p.f, 2, 6)
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8 * (1 + 1e-6)
    if case == "bpa_checkerboard":
        assert rep["cycles"] == rref["cycles"]


def test_fp32_iterates_on_the_fp64_store_reach_tolerance():
    """iterate = FP32 with HIER_FP64 deltas: FP32 cycles inside the FP64 defect
    correction on exact deltas reach 1e-8, recomputed by the oracle in FP64;
    the error against the direct solution stays within 10x the FP64 path's."""
    qmg = require_gpu()
    announce("fp32 iterates, hier64 store")
    d, L = 2, 5
    p = W.random_checkerboard(d, L, seed=9, values=(1.0, 1e4))
    g = _grid(qmg, p, "boxmg", "hier64", iterate="fp32")
    g.build()
    rep, hist = g.solve(1e-8, 400)
    u = g.solution()
    g.close()
    assert rep["status"] == "QMG_OK" and rep["outer_iters"] > 0
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    b = O.rhs_from_f(p.f, d, L)
    A = H.A[L]
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8
    ustar = O.direct_solve(A, b)
    u64, _ = O.solve(H, b, tol=1e-8)
    err64 = np.linalg.norm(u64 - ustar) / np.linalg.norm(ustar)
    assert np.linalg.norm(u - ustar) / np.linalg.norm(ustar) <= 10 * max(err64, 1e-12)


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_coarse_sweeps_match_oracle(d, L):
    """coarse_solver = sweeps: the coarsest level takes mu_pre + mu_post Jacobi
    sweeps from zero instead of the exact solve, as in the oracle with no
    direct coarse solve."""
    qmg = require_gpu()
    announce(f"coarse sweeps d={d} L={L}")
    p = W.random_checkerboard(d, L, seed=4, values=(1.0, 100.0))
    k = 4
    g = _grid(qmg, p, "boxmg", "hier64", coarse_solver="sweeps")
    g.build()
    rr = g.vcycle(k)
    u = g.solution()
    g.close()
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg", direct_max=0)
    assert H.coarse_lu is None
    b = O.rhs_from_f(p.f, d, L)
    uo, ho = O.solve(H, b, cycles=k)
    np.testing.assert_allclose(rr, ho, rtol=1e-9)
    assert np.linalg.norm(H.A[L] @ (u - uo)) / np.linalg.norm(b) <= 1e-12
    Hd = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    _, hd = O.solve(Hd, b, cycles=k)
    assert abs(hd[-1] - ho[-1]) > 1e-3 * hd[-1]          # the exact solve is a different cycle


def test_eps_zero_threshold_drops_small_deltas():
    """A larger zero-delta threshold stores fewer blocks; the solve still
    reaches the tolerance (the dropped deltas only change the coarse
    operators).  A smooth coefficient 1 + 0.3 sin(2 pi x) sin(2 pi y) on
    level 5: the oracle's level-4 deltas all lie between 2^-40 and 10^-3 of
    the rediscretised rows, so the 10^-3 threshold drops every level-4 block
    the default keeps.  (A checkerboard of 9^2 blocks has no such deltas: it
    is constant on the level-2 cells.)"""
    qmg = require_gpu()
    announce("eps_zero threshold")
    d, L = 2, 5
    n = 3 ** L
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="ij")
    eps = 1.0 + 0.3 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    H = O.build_hierarchy(eps, d, L, transfer="boxmg")
    G = O.geometric_stencil(H.eps[4], d, 4)
    rel = np.abs(O.solver.csr_to_stencil(H.A[4], d, 4) - G).max(axis=0)
    rel = rel[np.abs(G).max(axis=0) > 0] / np.abs(G).max(axis=0)[np.abs(G).max(axis=0) > 0]
    assert (rel > 2.0 ** -40).all() and (rel < 1e-3).all()
    f = W.poisson(d, L, seed=3).f
    fr = []
    for ez in (0.0, 1e-3):
        g = qmg.Grid(d, L, qmg.make_opts("boxmg", "hier64", eps_zero=ez))
        g.set_coefficients(eps, f)
        info = g.build()
        rep, _ = g.solve(1e-8, 400)
        assert rep["status"] == "QMG_OK"
        fr.append(info["zero_delta_fraction"])
        g.close()
    assert fr[1] > fr[0]
