"""Adaptive spacetrees on the GPU against the adaptive oracle: numbering of
unknowns and leaf cells, the operators of every level, FAS V-cycle iterates
and residual histories, and the composite fixed point."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive as AD
from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


def _problem(d, base, L, seed=0, r=0.2, n_balls=2):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, size=(n_balls, d))
    flags = W.ball_flags(d, base, L, c, r)
    G = AD.AdaptiveGrid(d, base, L, flags)
    eps = rng.uniform(0.5, 2.0, size=len(G.leaf_cells()))
    f = rng.uniform(-1.0, 1.0, size=G.n_unknowns())
    return flags, G, eps, f


def _grid(qmg, d, base, L, flags, transfer="galerkin", store="hier64", **kw):
    return qmg.Grid(d, L, qmg.make_opts(transfer=transfer, store=store, **kw), base_level=base,
                    refine=flags)


def _contrast_tol(eps):
    """Bound for the relative gaps of BoxMG cycles (iterates and residual
    histories): rounding amplified by the coefficient contrast kappa, as for
    the entries that neighbouring BoxMG patches share, with 4x more room for
    the levels and cycles it passes through: 64 kappa 2^-52."""
    return 64.0 * float(np.max(eps) / np.min(eps)) * 2.0 ** -52


def _print_gaps(rr, hist_o, u, u_o):
    rel = np.abs(np.asarray(rr) - np.asarray(hist_o)) / np.abs(np.asarray(hist_o))
    print(f"history gap (relative, worst cycle) {rel.max():.2e}; "
          f"iterate gap {np.abs(u - u_o).max() / np.abs(u_o).max():.2e}")


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (2, 1, 5), (3, 1, 3)])
def test_numbering_matches_oracle(d, base, L):
    qmg = require_gpu()
    announce(f"adaptive numbering d={d} base={base} L={L}")
    flags, G, _, _ = _problem(d, base, L)
    g = _grid(qmg, d, base, L, flags)
    assert g.n_unknowns == G.n_unknowns()
    assert g.n_cells == len(G.leaf_cells())
    xyz, lev = g.unknown_coords()
    np.testing.assert_allclose(xyz, G.unknown_coords(), rtol=0, atol=1e-14)
    assert lev.tolist() == [l for l, _ in G.leaves()]
    np.testing.assert_allclose(g.cell_centres(), G.cell_centres(), rtol=0, atol=1e-14)
    g.close()


@pytest.mark.parametrize("d,base,L,transfer", [(2, 2, 4, "galerkin"), (2, 1, 4, "galerkin"),
                                               (3, 1, 3, "galerkin"), (2, 2, 4, "geometric")])
def test_level_operators_match_oracle(d, base, L, transfer):
    """Rows of leaf and refined vertices of every adaptive level (and the full
    rows of the complete levels below) equal the oracle's stencils."""
    qmg = require_gpu()
    announce(f"adaptive operators d={d} base={base} L={L} {transfer}")
    flags, G, eps, f = _problem(d, base, L)
    H = AD.build_adaptive(G, eps, transfer=transfer)
    g = _grid(qmg, d, base, L, flags, transfer=transfer)
    g.set_coefficients(eps, f)
    rep = g.build()
    assert rep["coarsest_level_used"] == 1
    for l in range(2, L + 1):
        S_gpu = g.operator(l)
        act = np.isin(G.vtype[l], (AD.LEAF, AD.REFINED))
        ref = H.S[l]
        scale = np.abs(ref).max()
        diff = np.abs(S_gpu[:, act] - ref[:, act]).max()
        assert diff <= 1e-13 * scale, (l, diff / scale)
    g.close()


CYCLE_CASES = [
    (2, 2, 4, "galerkin", "hier64"),
    (2, 2, 4, "geometric", "hier64"),
    (2, 2, 4, "galerkin", "plain64"),
    (2, 1, 5, "galerkin", "hier64"),
    (3, 1, 3, "galerkin", "hier64"),
    (3, 1, 3, "geometric", "plain64"),
]


@pytest.mark.parametrize("d,base,L,transfer,store", CYCLE_CASES)
def test_fas_cycles_match_oracle(d, base, L, transfer, store):
    """Iterates and residual histories of the first cycles agree with the
    oracle's FAS V-cycle (same composite state after every cycle)."""
    qmg = require_gpu()
    announce(f"adaptive cycles d={d} base={base} L={L} {transfer} {store}")
    flags, G, eps, f = _problem(d, base, L)
    H = AD.build_adaptive(G, eps, transfer=transfer)
    k = 6
    u_o, hist_o = AD.solve_adaptive(H, f, cycles=k)
    g = _grid(qmg, d, base, L, flags, transfer=transfer, store=store)
    g.set_coefficients(eps, f)
    g.build()
    rr = g.vcycle(k)
    u = g.solution()
    _print_gaps(rr, hist_o, u, u_o)
    np.testing.assert_allclose(rr, hist_o, rtol=1e-9, atol=1e-14)
    assert np.abs(u - u_o).max() <= 1e-11 * np.abs(u_o).max()
    g.close()


@pytest.mark.parametrize("d,base,L,transfer", [(2, 2, 4, "galerkin"), (3, 1, 3, "galerkin"),
                                               (2, 1, 5, "geometric")])
def test_solve_reaches_composite_solution(d, base, L, transfer):
    qmg = require_gpu()
    announce(f"adaptive solve d={d} base={base} L={L} {transfer}")
    flags, G, eps, f = _problem(d, base, L)
    ustar, A, b = AD.solve_composite_direct(G, eps, f)
    g = _grid(qmg, d, base, L, flags, transfer=transfer)
    g.set_coefficients(eps, f)
    g.build()
    rep, hist = g.solve(tol=1e-11, max_cycles=200)
    assert rep["status"] == "QMG_OK", rep
    u = g.solution()
    # the reported residual is the composite residual of the returned solution
    rr = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    assert rr <= 1e-11 * (1 + 1e-6)
    assert abs(rr - rep["relres"]) <= 1e-14 + 1e-6 * rr
    assert np.linalg.norm(u - ustar) <= 1e-9 * np.linalg.norm(ustar)
    g.close()


def test_warm_start_resumes_the_cycle():
    """set_solution of the oracle's k-cycle iterate, then one GPU cycle, equals
    k+1 oracle cycles."""
    qmg = require_gpu()
    d, base, L = 2, 2, 4
    announce("adaptive warm start")
    flags, G, eps, f = _problem(d, base, L)
    H = AD.build_adaptive(G, eps, transfer="galerkin")
    u3, _ = AD.solve_adaptive(H, f, cycles=3)
    u4, h4 = AD.solve_adaptive(H, f, cycles=4)
    g = _grid(qmg, d, base, L, flags)
    g.set_coefficients(eps, f)
    g.build()
    g.set_solution(u3)
    rr = g.vcycle(1)
    np.testing.assert_allclose(rr[0], h4[-1], rtol=1e-9)
    assert np.abs(g.solution() - u4).max() <= 1e-11 * np.abs(u4).max()
    g.close()


def test_no_refinement_equals_regular_grid():
    """Flags that refine nothing beyond the base level give the regular grid of
    the base level on the finest lattice (no adaptive level has a leaf)."""
    qmg = require_gpu()
    announce("adaptive without refinement")
    d, base, L = 2, 3, 4
    flags = {3: np.zeros((27, 27), bool)}
    G = AD.AdaptiveGrid(d, base, L, flags)
    rng = np.random.default_rng(5)
    eps = rng.uniform(0.5, 2.0, size=len(G.leaf_cells()))
    f = rng.uniform(-1, 1, size=G.n_unknowns())
    ustar, A, b = AD.solve_composite_direct(G, eps, f)
    g = _grid(qmg, d, base, L, flags)
    assert g.n_unknowns == 26 * 26
    g.set_coefficients(eps, f)
    g.build()
    rep, _ = g.solve(tol=1e-11, max_cycles=100)
    assert rep["status"] == "QMG_OK"
    assert np.linalg.norm(g.solution() - ustar) <= 1e-9 * np.linalg.norm(ustar)
    g.close()


def test_adaptive_rejected_by_server():
    qmg = require_gpu()
    flags, G, eps, f = _problem(2, 2, 4)
    srv = qmg.Server(1 << 30, max_slots=2)
    desc = qmg.GridDesc(2, 4, 2, qmg.pack_refine(2, 2, 4, flags).ctypes.data_as(qmg.C.c_void_p))
    t = qmg.C.c_uint64(0)
    rc = srv.lib.qmg_server_submit(srv.h, qmg.C.byref(desc), qmg.C.byref(qmg.make_opts(transfer="galerkin")),
                                   qmg._ptr(eps), qmg._ptr(f), 1e-8, 100, -1.0, qmg.C.byref(t))
    assert rc == qmg.QMG_EINVAL
    srv.close()


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
@pytest.mark.parametrize("store", ["hier32", "bf16", "hier16"])
def test_mixed_precision_reaches_composite_solution(d, base, L, store):
    """FP32 inner FAS cycles on reduced-precision stores inside the FP64
    composite defect correction: the oracle recomputes the final relative
    residual in FP64, and the error against the directly solved composite
    system stays within 10x that of the FP64 path stopped at the same
    tolerance."""
    qmg = require_gpu()
    announce(f"adaptive mixed d={d} base={base} L={L} {store}")
    flags, G, eps, f = _problem(d, base, L)
    ustar, A, b = AD.solve_composite_direct(G, eps, f)
    errs, cyc = {}, {}
    for st in ("hier64", store):
        g = _grid(qmg, d, base, L, flags, store=st)
        g.set_coefficients(eps, f)
        g.build()
        rep, hist = g.solve(tol=1e-8, max_cycles=300)
        assert rep["status"] == "QMG_OK", rep
        u = g.solution()
        rr = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
        assert rr <= 1e-8 * (1 + 1e-6)
        assert abs(rr - rep["relres"]) <= 1e-6 * rr
        errs[st] = np.linalg.norm(u - ustar) / np.linalg.norm(ustar)
        cyc[st] = rep["cycles"]
        g.close()
    print(f"[adaptive mixed] {store}: err {errs[store]:.2e} (fp64 {errs['hier64']:.2e}), "
          f"cycles {cyc[store]} (fp64 {cyc['hier64']})")
    assert errs[store] <= 10 * errs["hier64"]


def _workload_inputs(P, G):
    eps = P.eps_at(G.cell_centres())
    X = G.unknown_coords()
    levels = np.concatenate([np.full(int((G.vtype[l] == AD.LEAF).sum()), l)
                             for l in range(G.base, G.L + 1)])
    f = np.empty(len(X))
    for l in range(G.base, G.L + 1):
        m = levels == l
        f[m] = P.f_at(l, X[m])
    return eps, f


def test_balls_midsize_cycles_match_oracle():
    """The 3D four-ball workload (smooth log-normal eps) at base 2, level 4:
    FAS cycle iterates against the oracle."""
    qmg = require_gpu()
    announce("adaptive balls 3D base2 L4 cycles")
    P = W.adaptive_balls(dim=3, base=2, level=4)
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    H = AD.build_adaptive(G, eps, transfer="galerkin")
    k = 4
    u_o, hist_o = AD.solve_adaptive(H, f, cycles=k)
    g = _grid(qmg, 3, P.base, P.level, P.flags)
    g.set_coefficients(eps, f)
    g.build()
    rr = g.vcycle(k)
    u = g.solution()
    _print_gaps(rr, hist_o, u, u_o)
    np.testing.assert_allclose(rr, hist_o, rtol=1e-9)
    assert np.abs(u - u_o).max() <= 1e-11 * np.abs(u_o).max()
    g.close()


def test_balls_full_size_solve_sampled_rows():
    """The 3D four-ball workload at full size (base 3, level 5, about 1.3e6
    unknowns): the GPU reaches 1e-8 and the composite residual of its solution,
    assembled row by row by the oracle at sampled unknowns of every level,
    agrees with that."""
    qmg = require_gpu()
    announce("adaptive balls 3D base3 L5 full size")
    P = W.adaptive_balls()
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    # 3D Galerkin coarse stencils of a variable scalar eps carry small positive
    # face entries: SPD, but not diagonally dominant, so the check would raise
    # the coarsest level to the base level (Jacobi there); it is off here, as
    # in the oracle's adaptive hierarchy
    g = _grid(qmg, 3, P.base, P.level, P.flags, check_definite=False)
    assert g.n_unknowns == G.n_unknowns()
    g.set_coefficients(eps, f)
    info = g.build()
    assert info["coarsest_level_used"] == 1
    rep, hist = g.solve(tol=1e-8, max_cycles=100)
    assert rep["status"] == "QMG_OK", rep
    u = g.solution()
    levels = np.concatenate([np.full(int((G.vtype[l] == AD.LEAF).sum()), l)
                             for l in range(G.base, G.L + 1)])
    b = f * (3.0 ** -levels.astype(float)) ** 3
    nb = np.linalg.norm(b)
    rng = np.random.default_rng(11)
    sample = np.concatenate([rng.choice(np.flatnonzero(levels == l), 100, replace=False)
                             for l in range(G.base, G.L + 1)])
    r = AD.composite_residual_rows(G, eps, f, u, sample)
    assert np.abs(r).max() <= 1e-8 * nb * (1 + 1e-6)
    # the sampled rows estimate the full residual norm (level-stratified)
    est = 0.0
    for l in range(G.base, G.L + 1):
        m = levels[sample] == l
        est += (levels == l).sum() * np.mean(r[m] ** 2)
    assert np.sqrt(est) <= 10 * rep["relres"] * nb
    g.close()


def test_balls_full_size_mixed_bf16_sampled_rows():
    """The 3D four-ball workload at full size in its mixed form: BF16 deltas,
    FP32 inner cycles, FP64 composite defect correction to 1e-8; the oracle
    recomputes the composite residual at sampled unknowns of every level."""
    qmg = require_gpu()
    announce("adaptive balls 3D base3 L5 full size, bf16 mixed")
    P = W.adaptive_balls()
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    g = _grid(qmg, 3, P.base, P.level, P.flags, store="bf16", check_definite=False)
    g.set_coefficients(eps, f)
    g.build()
    rep, hist = g.solve(tol=1e-8, max_cycles=200)
    assert rep["status"] == "QMG_OK", rep
    u = g.solution()
    g.close()
    levels = np.concatenate([np.full(int((G.vtype[l] == AD.LEAF).sum()), l)
                             for l in range(G.base, G.L + 1)])
    b = f * (3.0 ** -levels.astype(float)) ** 3
    nb = np.linalg.norm(b)
    rng = np.random.default_rng(12)
    sample = np.concatenate([rng.choice(np.flatnonzero(levels == l), 100, replace=False)
                             for l in range(G.base, G.L + 1)])
    r = AD.composite_residual_rows(G, eps, f, u, sample)
    assert np.abs(r).max() <= 1e-8 * nb * (1 + 1e-6)
    est = sum((levels == l).sum() * np.mean(r[levels[sample] == l] ** 2) for l in range(G.base, G.L + 1))
    assert np.sqrt(est) <= 10 * rep["relres"] * nb
    print(f"[balls3d bf16] outer iterations {rep['outer_iters']}, relres {rep['relres']:.2e}")


# ---------------------------------------------------------------------------
# BoxMG on adaptive levels
# ---------------------------------------------------------------------------

def _checker(G, seed, values=(1.0, 1e3)):
    rng = np.random.default_rng(seed)
    table = rng.choice(np.asarray(values), size=(9,) * G.d)
    idx = np.minimum((G.cell_centres() * 9).astype(int), 8)
    return table[tuple(idx[:, i] for i in reversed(range(G.d)))]


BOX_CASES = [(2, 2, 4), (2, 1, 5), (3, 1, 3)]


@pytest.mark.parametrize("d,base,L", BOX_CASES)
def test_boxmg_operators_and_prolongations_match_oracle(d, base, L):
    qmg = require_gpu()
    from gpu_util import weights_to_csr
    announce(f"adaptive boxmg operators d={d} base={base} L={L}")
    flags, G, _, f = _problem(d, base, L, seed=8)
    eps = _checker(G, 8)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    g = _grid(qmg, d, base, L, flags, transfer="boxmg")
    g.set_coefficients(eps, f)
    assert g.build()["coarsest_level_used"] == 1
    for l in range(2, L + 1):
        act = np.isin(G.vtype[l], (AD.LEAF, AD.REFINED))
        S_gpu = g.operator(l)
        scale = np.abs(H.S[l]).max()
        assert np.abs(S_gpu[:, act] - H.S[l][:, act]).max() <= 1e-11 * scale, l
        # prolongation rows of fine vertices in refined patches (all rows below the base level)
        Pg = weights_to_csr(g.prolongation(l), d, l).toarray()
        Po = H.P[l].toarray()
        rows = np.abs(Po).sum(axis=1) > 0
        assert np.abs(Pg[rows] - Po[rows]).max() <= 1e-11, l
    g.close()


@pytest.mark.parametrize("d,base,L", BOX_CASES)
def test_boxmg_fas_cycles_match_oracle(d, base, L):
    qmg = require_gpu()
    announce(f"adaptive boxmg cycles d={d} base={base} L={L}")
    flags, G, _, f = _problem(d, base, L, seed=8)
    eps = _checker(G, 8)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    k = 6
    u_o, hist_o = AD.solve_adaptive(H, f, cycles=k)
    g = _grid(qmg, d, base, L, flags, transfer="boxmg")
    g.set_coefficients(eps, f)
    g.build()
    rr = g.vcycle(k)
    u = g.solution()
    _print_gaps(rr, hist_o, u, u_o)
    tol = _contrast_tol(eps)
    np.testing.assert_allclose(rr, hist_o, rtol=tol)
    assert np.abs(u - u_o).max() <= tol * np.abs(u_o).max()
    g.close()


@pytest.mark.parametrize("store", ["hier64", "bf16"])
@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_boxmg_solve_reaches_composite_solution(d, base, L, store):
    """BoxMG hanging constraints: the solution (FP64, or BF16 deltas with FP32
    inner cycles) solves the composite system the oracle assembles with its
    own BoxMG prolongations."""
    qmg = require_gpu()
    announce(f"adaptive boxmg solve d={d} base={base} L={L} {store}")
    flags, G, _, f = _problem(d, base, L, seed=8)
    eps = _checker(G, 8)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    ustar, A, b = AD.solve_composite_direct(G, eps, f, AD.hanging_constraints(H))
    g = _grid(qmg, d, base, L, flags, transfer="boxmg", store=store)
    g.set_coefficients(eps, f)
    g.build()
    rep, _ = g.solve(tol=1e-10, max_cycles=400)
    assert rep["status"] == "QMG_OK", rep
    u = g.solution()
    rr = np.linalg.norm(b - A @ u) / np.linalg.norm(b)
    # the FP64 residual at 1e-10 carries ~1e-14 of cancellation noise
    assert rr <= 1e-10 + 1e-13
    assert abs(rr - rep["relres"]) <= 1e-13 + 1e-5 * rr
    assert np.linalg.norm(u - ustar) <= 1e-7 * np.linalg.norm(ustar)
    g.close()


def test_boxmg_balls_midsize_cycles_match_oracle():
    """The 3D four-ball workload at base 2, level 4 with BoxMG: FAS iterates
    against the oracle."""
    qmg = require_gpu()
    announce("adaptive balls 3D base2 L4 boxmg cycles")
    P = W.adaptive_balls(dim=3, base=2, level=4)
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    k = 4
    u_o, hist_o = AD.solve_adaptive(H, f, cycles=k)
    # as in the oracle's adaptive hierarchy the coarsest level stays at 1 (3D
    # Galerkin rows of a variable coefficient are not diagonally dominant)
    g = _grid(qmg, 3, P.base, P.level, P.flags, transfer="boxmg", check_definite=False)
    g.set_coefficients(eps, f)
    assert g.build()["coarsest_level_used"] == 1
    rr = g.vcycle(k)
    u = g.solution()
    _print_gaps(rr, hist_o, u, u_o)
    tol = _contrast_tol(eps)
    np.testing.assert_allclose(rr, hist_o, rtol=tol)
    assert np.abs(u - u_o).max() <= tol * np.abs(u_o).max()
    g.close()


def test_boxmg_balls_full_size_mixed():
    """The 3D four-ball workload at full size in the configured form: BoxMG +
    Galerkin, BF16 deltas, FP32 inner cycles, FP64 defect correction to 1e-8.
    The FP64 BoxMG solve of the same system (the oracle cannot assemble it at
    this size) bounds the error: both stop at 1e-8, so they agree within the
    conditioning bound."""
    qmg = require_gpu()
    announce("adaptive balls 3D base3 L5 full size, boxmg bf16 mixed")
    P = W.adaptive_balls()
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    sol = {}
    for store in ("hier64", "bf16"):
        g = _grid(qmg, 3, P.base, P.level, P.flags, transfer="boxmg", store=store, check_definite=False)
        g.set_coefficients(eps, f)
        g.build()
        rep, _ = g.solve(tol=1e-8, max_cycles=300)
        assert rep["status"] == "QMG_OK", (store, rep)
        sol[store] = g.solution()
        print(f"[balls3d boxmg {store}] cycles {rep['cycles']}, outer {rep['outer_iters']}, relres {rep['relres']:.2e}")
        g.close()
    rel = np.linalg.norm(sol["bf16"] - sol["hier64"]) / np.linalg.norm(sol["hier64"])
    print(f"[balls3d boxmg] bf16 vs fp64 solution: {rel:.2e}")
    assert rel <= 1e-5
    # the oracle recomputes the composite residual of each solution at sampled
    # unknowns, row by row; rows that need a hanging value (a BoxMG
    # interpolant) are skipped, the others do not depend on P
    from gpu_util import sampled_local_rows
    levels = np.concatenate([np.full(int((G.vtype[l] == AD.LEAF).sum()), l)
                             for l in range(G.base, G.L + 1)])
    nb = np.linalg.norm(f * (3.0 ** -levels.astype(float)) ** 3)
    xyz = G.unknown_coords()
    for store, u in sol.items():
        pick, rows, scale = sampled_local_rows(P, xyz, levels, u, 300, seed=21)
        ok = ~np.isnan(rows)
        assert ok.sum() >= 100, ok.sum()
        print(f"[balls3d boxmg {store}] {ok.sum()} rows, max |r| / ||b|| = {np.abs(rows[ok]).max() / nb:.2e}")
        assert np.abs(rows[ok]).max() <= 1e-8 * nb * (1 + 1e-6)


def test_band_midsize_boxmg_cycles_match_oracle():
    """The level-set band workload with 1e6 cube inclusions (base 2, level 4):
    the first BoxMG FAS cycles against the oracle.  With V(2,2) damped Jacobi
    this coefficient field makes the cycle diverge, on both sides alike; the
    comparison is of the iterates, relative to their size."""
    qmg = require_gpu()
    announce("adaptive band 3D base2 L4 boxmg cycles")
    P = W.adaptive_band(dim=3, base=2, level=4)
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    k = 3
    u_o, hist_o = AD.solve_adaptive(H, f, cycles=k)
    g = _grid(qmg, 3, P.base, P.level, P.flags, transfer="boxmg", check_definite=False)
    g.set_coefficients(eps, f)
    assert g.build()["coarsest_level_used"] == 1
    rr = g.vcycle(k)
    u = g.solution()
    _print_gaps(rr, hist_o, u, u_o)
    tol = _contrast_tol(eps)
    np.testing.assert_allclose(rr, hist_o, rtol=tol)
    assert np.abs(u - u_o).max() <= tol * np.abs(u_o).max()
    g.close()


def test_band_full_size_grid_from_region_and_residual_rows():
    """The 3D band workload at full size (base 3, level 6, 4.5e7 unknowns): the
    grid is built from the band region inside the library; after two BoxMG
    FAS cycles in FP64 the library's composite residual equals, row by row,
    the oracle's rows assembled at sampled unknowns from the same iterate
    (rows that need a hanging value are left to the mid-size tests); every
    sampled unknown is a leaf vertex of the oracle's spacetree."""
    qmg = require_gpu()
    from gpu_util import band_inputs_on_device, sampled_local_rows
    announce("adaptive band 3D base3 L6 full size, hier64, two cycles")
    P = W.adaptive_band(dim=3, base=3, level=6)
    g = qmg.Grid(3, 6, qmg.make_opts("boxmg", "hier64", check_definite=False, graphs=False), base_level=3,
                 regions=P.regions)
    assert g.n_unknowns > 4e7
    eps, f, xyz, lev = band_inputs_on_device(g, P)
    g.set_coefficients(eps, f)
    assert g.build()["coarsest_level_used"] == 1
    rr = g.vcycle(2)
    assert np.all(np.isfinite(rr))
    u = g.solution()
    r = g.residual()
    g.close()
    fh = f.cpu().numpy()
    assert abs(np.linalg.norm(r) / np.linalg.norm(fh * (3.0 ** -lev.astype(float)) ** 3) - rr[-1]) <= 1e-9 * rr[-1]
    pick, rows, scale = sampled_local_rows(P, xyz, lev, u, 200, seed=5)
    ok = ~np.isnan(rows)
    assert ok.sum() >= 100, ok.sum()
    err = np.abs(rows[ok] - r[pick][ok]) / scale[ok]
    print(f"[band3d L6] {ok.sum()} rows, max |r_gpu - r_oracle| / sum|K||u| = {err.max():.2e}")
    assert err.max() <= 1e-13


def test_stagnation_raise_to_base_matches_oracle():
    """Dynamic coarsest level on an adaptive grid: a threshold no cycle meets
    moves the regular levels' coarsest level up to the base level (676
    unknowns, solved exactly); FAS cycle history and leaf values against the
    oracle."""
    qmg = require_gpu()
    announce("adaptive stagnation raise 2D base3 L5")
    flags, G, eps, f = _problem(2, 3, 5)
    k = 4
    H = AD.build_adaptive(G, eps, transfer="galerkin")
    u_o, hist_o = AD.solve_adaptive(H, f, tol=0.0, max_cycles=k, stagnation=1e-12)
    assert H.regular.lc == 3
    g = _grid(qmg, 2, 3, 5, flags, check_definite=False, stagnation=1e-12)
    g.set_coefficients(eps, f)
    g.build()
    rep, hist = g.solve(1e-30, k)
    u = g.solution()
    g.close()
    assert rep["coarsest_level_used"] == 3 and rep["cycles"] == k
    np.testing.assert_allclose(hist, hist_o, rtol=1e-9, atol=0)
    assert np.abs(u - u_o).max() <= 1e-10 * np.abs(u_o).max()


def test_repeated_coefficients_equal_a_fresh_grid():
    """A second set_coefficients on the same adaptive grid (new coefficients
    and source) clears only the active tiles; its build and cycles must equal
    those of a fresh grid given the same inputs, bit for bit."""
    qmg = require_gpu()
    announce("adaptive repeated set_coefficients")
    P = W.adaptive_band(dim=3, base=1, level=3, seed=0)
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    eps, f = _workload_inputs(P, G)
    rng = np.random.default_rng(4)
    eps2 = eps * rng.uniform(0.5, 2.0, size=eps.shape)
    f2 = rng.uniform(-1.0, 1.0, size=f.shape)
    for transfer, store in (("boxmg", "bf16"), ("galerkin", "hier64")):
        kw = dict(check_definite=False)
        g = _grid(qmg, 3, P.base, P.level, P.flags, transfer=transfer, store=store, **kw)
        g.set_coefficients(eps, f)
        g.build()
        g.solve(0.0, 2)
        g.set_coefficients(eps2, f2)
        g.build()
        rep, hist = g.solve(0.0, 2)
        u = g.solution()
        g.close()
        h = _grid(qmg, 3, P.base, P.level, P.flags, transfer=transfer, store=store, **kw)
        h.set_coefficients(eps2, f2)
        h.build()
        rep_h, hist_h = h.solve(0.0, 2)
        u_h = h.solution()
        h.close()
        assert np.array_equal(hist, hist_h), (transfer, hist, hist_h)
        assert np.array_equal(u, u_h), transfer
