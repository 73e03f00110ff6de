"""Pins of the adaptive oracle: the composite system against the regular
system in the limiting cases, d-linear reproduction at hanging vertices,
and FAS V-cycles against the directly solved composite system."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from boxmg_equations import worst_defining_equation
from oracle import adaptive as AD


def _problem(d, base, L, seed=0, r=0.2):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, size=(2, d))
    G = AD.AdaptiveGrid(d, base, L, W.ball_flags(d, base, L, c, r))
    eps = rng.uniform(0.5, 2.0, size=len(G.leaf_cells()))
    f = rng.uniform(-1.0, 1.0, size=G.n_unknowns())
    return G, eps, f


def test_vertex_classes():
    G, _, _ = _problem(2, 2, 4)
    for l in range(G.base + 1, G.L + 1):
        t = G.vtype[l]
        assert (t == AD.HANGING).any() and (t == AD.LEAF).any()
        # a refined vertex has a non-hanging copy on the next level
        for v in np.argwhere(t == AD.REFINED):
            assert G.vtype[l + 1][tuple(3 * v)] in (AD.LEAF, AD.REFINED)
    assert not (G.vtype[G.L] == AD.REFINED).any()
    assert not (G.vtype[G.base] == AD.HANGING).any()


@pytest.mark.parametrize("d", [2, 3])
def test_no_refinement_is_the_regular_system(d):
    base = 2 if d == 2 else 1
    n = 3 ** base
    G = AD.AdaptiveGrid(d, base, base + 2, {})
    rng = np.random.default_rng(1)
    eps = rng.uniform(0.5, 2.0, size=n ** d)
    f = rng.uniform(-1, 1, size=G.n_unknowns())
    A, b = AD.composite_system(G, eps, f)
    Ar = O.stencil_to_csr(O.geometric_stencil(eps.reshape((n,) * d), d, base), d, base)
    assert abs(A - Ar).max() < 1e-14 * abs(Ar).max()
    np.testing.assert_allclose(b, O.rhs_from_f(f, d, base))


def test_full_refinement_is_the_regular_fine_system():
    d, base, L = 2, 1, 3
    flags = {l: np.ones((3 ** l,) * d, bool) for l in range(base, L)}
    G = AD.AdaptiveGrid(d, base, L, flags)
    n = 3 ** L
    assert G.n_unknowns() == (n - 1) ** d
    rng = np.random.default_rng(2)
    eps = rng.uniform(0.5, 2.0, size=n ** d)
    f = rng.uniform(-1, 1, size=G.n_unknowns())
    A, b = AD.composite_system(G, eps, f)
    Ar = O.stencil_to_csr(O.geometric_stencil(eps.reshape((n,) * d), d, L), d, L)
    assert abs(A - Ar).max() < 1e-14 * abs(Ar).max()


def test_hanging_values_reproduce_dlinear_functions():
    """With leaves holding a d-linear function, injection and interpolation
    give every vertex of every level that function's value."""
    d = 2
    # refinement away from the boundary, where Dirichlet zeros would enter
    G = AD.AdaptiveGrid(d, 2, 4, W.ball_flags(d, 2, 4, np.array([[0.5, 0.5]]), 0.2))
    eps = np.ones(len(G.leaf_cells()))
    f = np.zeros(G.n_unknowns())
    H = AD.build_adaptive(G, eps, transfer="geometric")
    fun = lambda x, y: 0.3 + 1.5 * x - 0.7 * y + 2.0 * x * y
    u, _ = AD.initial_state(H, f)
    for l in range(G.base, G.L + 1):
        n = 3 ** l
        yy, xx = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n, indexing="ij")
        u[l] = np.where(G.vtype[l] == AD.LEAF, fun(xx, yy), 0.0)
    AD.composite_state(H, u)
    for l in range(G.base, G.L + 1):
        n = 3 ** l
        yy, xx = np.meshgrid(np.arange(n + 1) / n, np.arange(n + 1) / n, indexing="ij")
        live = G.vtype[l] != AD.OUT
        np.testing.assert_allclose(u[l][live], fun(xx, yy)[live], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
@pytest.mark.parametrize("transfer", ["galerkin", "geometric"])
def test_fas_cycles_converge_to_composite_solution(d, base, L, transfer):
    G, eps, f = _problem(d, base, L)
    ustar, A, b = AD.solve_composite_direct(G, eps, f)
    H = AD.build_adaptive(G, eps, transfer=transfer)
    u, hist = AD.solve_adaptive(H, f, tol=1e-12, max_cycles=100)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(u - ustar) <= 1e-10 * np.linalg.norm(ustar)
    # the cycle's own residual equals the independently assembled one
    assert abs(np.linalg.norm(b - A @ u) / np.linalg.norm(b) - hist[-1]) <= 1e-14
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))


def test_adaptive_manufactured_solution_improves_with_refinement():
    """sin source, exact solution prod sin(pi x_i): refining a region (the
    whole domain in the limit) reduces the nodal error at the leaves."""
    d = 2
    errs = []
    for L in (3, 4):
        flags = {l: np.ones((3 ** l,) * d, bool) for l in range(2, L)}
        G = AD.AdaptiveGrid(d, 2, L, flags)
        X = G.unknown_coords()
        f = d * np.pi ** 2 * np.prod(np.sin(np.pi * X), axis=1)
        u, _, _ = AD.solve_composite_direct(G, np.ones(len(G.leaf_cells())), f)
        errs.append(np.max(np.abs(u - np.prod(np.sin(np.pi * X), axis=1))))
    assert 7.5 <= errs[0] / errs[1] <= 10.5


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_residual_rows_assembled_one_by_one(d, base, L):
    """Rows evaluated on their own from element matrices equal the rows of the
    assembled composite system (so they can stand in for it on large grids)."""
    G, eps, f = _problem(d, base, L, seed=3)
    A, b = AD.composite_system(G, eps, f)
    u = np.random.default_rng(4).uniform(-1, 1, size=G.n_unknowns())
    sample = np.arange(0, G.n_unknowns(), 7)
    rows = AD.composite_residual_rows(G, eps, f, u, sample)
    ref = (b - A @ u)[sample]
    np.testing.assert_allclose(rows, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------------------
# BoxMG on adaptive levels
# ---------------------------------------------------------------------------

def _checkerboard_eps(G, seed, values=(1.0, 1e3)):
    """Leaf-cell coefficients from a random 9^d table (jumps on level-2 faces)."""
    rng = np.random.default_rng(seed)
    table = rng.choice(np.asarray(values), size=(9,) * G.d)
    idx = np.minimum((G.cell_centres() * 9).astype(int), 8)
    return table[tuple(idx[:, i] for i in reversed(range(G.d)))]


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_boxmg_constant_coefficient_is_dlinear(d, base, L):
    """For constant eps BoxMG reproduces d-linear weights, also at hanging
    vertices (whose interpolated stencils are then proportional to the
    rediscretised ones), so every operator, every prolongation and the
    composite system equal those of the d-linear Galerkin variant."""
    G, _, f = _problem(d, base, L, seed=5)
    eps = np.full(len(G.leaf_cells()), 2.5)
    Hb = AD.build_adaptive(G, eps, transfer="boxmg")
    Hg = AD.build_adaptive(G, eps, transfer="galerkin")
    for l in range(2, L + 1):
        np.testing.assert_allclose(Hb.P[l].toarray(), Hg.P[l].toarray()[:, :] * (abs(Hb.P[l]).toarray() > 0),
                                   atol=1e-12)
        act = np.isin(G.vtype[l], (AD.LEAF, AD.REFINED))
        np.testing.assert_allclose(Hb.S[l][:, act], Hg.S[l][:, act], atol=1e-12 * abs(Hg.S[l]).max())
    Ab, bb = AD.composite_system(G, eps, f, AD.hanging_constraints(Hb))
    Ag, bg = AD.composite_system(G, eps, f)
    assert abs(Ab - Ag).max() <= 1e-12 * abs(Ag).max()


def test_boxmg_full_refinement_is_the_regular_boxmg():
    """Refining every cell leaves no hanging vertex: the adaptive BoxMG of each
    level equals the regular BoxMG of the same stencils."""
    d, base, L = 2, 1, 3
    flags = {l: np.ones((3 ** l,) * d, bool) for l in range(base, L)}
    G = AD.AdaptiveGrid(d, base, L, flags)
    rng = np.random.default_rng(7)
    eps = rng.choice([1.0, 100.0], size=len(G.leaf_cells()))
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    for l in range(base + 1, L + 1):
        Pr = O.boxmg_P(H.S[l], d, l)
        assert abs(H.P[l] - Pr).max() <= 1e-12
        assert H.P[l].nnz == Pr.nnz


def test_boxmg_hanging_stencils_from_covering_cells():
    """A hanging vertex's row is the rediscretised row of its level with the
    missing cells carrying the coefficient of the leaf cell that covers them:
    check one hanging vertex by hand from the element matrices."""
    d, base, L = 2, 2, 4
    G, _, _ = _problem(d, base, L, seed=6)
    rng = np.random.default_rng(9)
    eps_leaf = rng.uniform(0.5, 2.0, size=len(G.leaf_cells()))
    eps = G.level_eps(eps_leaf)
    Hs = AD.hanging_stencils(G, eps)
    l = 3
    v = tuple(np.argwhere(G.vtype[l] == AD.HANGING)[0])      # numpy order (y, x)
    h = 3.0 ** -l
    row = np.zeros(9)
    for s in O.corners(d):                                    # v is corner s of cell v - s
        cell = tuple(vi - si for vi, si in zip(v, reversed(s)))
        if G.exist[l][cell]:
            e = eps[l][cell]
        else:                                                  # covered by a level-2 leaf cell
            e = eps[l - 1][tuple(c // 3 for c in cell)]
        K = O.element_matrix(d, h, e)
        for ib, w in enumerate(O.corners(d)):
            o = tuple(wi - si for wi, si in zip(w, s))        # x first
            row[O.fem.flat_offset(o)] += K[O.fem.corner_index(s), ib]
    n = 3 ** l
    for k, o in enumerate(O.offsets(d)):                       # Dirichlet entries dropped
        nb = (v[0] + o[1], v[1] + o[0])
        if not (0 < nb[0] < n and 0 < nb[1] < n):
            row[k] = 0.0
    np.testing.assert_allclose(Hs[l][(slice(None),) + v], row, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_boxmg_fas_cycles_converge_to_composite_solution(d, base, L):
    """A random 9^d checkerboard of {1, 1e3} (jumps on level-2 faces): the
    BoxMG FAS cycle converges to the directly solved composite system with
    BoxMG hanging constraints."""
    G, _, f = _problem(d, base, L, seed=8)
    eps = _checkerboard_eps(G, seed=8)
    H = AD.build_adaptive(G, eps, transfer="boxmg")
    ustar, A, b = AD.solve_composite_direct(G, eps, f, AD.hanging_constraints(H))
    u, hist = AD.solve_adaptive(H, f, tol=1e-12, max_cycles=300)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(u - ustar) <= 1e-9 * np.linalg.norm(ustar)
    assert abs(np.linalg.norm(b - A @ u) / np.linalg.norm(b) - hist[-1]) <= 1e-14
    rows = AD.composite_residual_rows(G, eps, f, u, np.arange(0, G.n_unknowns(), 11),
                                      AD.hanging_constraints(H))
    np.testing.assert_allclose(rows, (b - A @ u)[::11], atol=1e-13 * np.abs(b).max())


def test_stagnation_raise_moves_coarsest_level_to_the_base():
    """Dynamic coarsest level on an adaptive grid: with a threshold no cycle
    meets, the regular levels' coarsest level moves up after every cycle and
    stops at the base level; the first cycle is the one of the unraised
    hierarchy, and the raised solve still converges to the composite
    solution."""
    G, eps, f = _problem(2, 3, 5)
    H = AD.build_adaptive(G, eps, transfer="galerkin")
    _, h = AD.solve_adaptive(H, f, cycles=4, stagnation=1e-12)
    assert H.regular.lc == G.base
    H0 = AD.build_adaptive(G, eps, transfer="galerkin")
    _, h0 = AD.solve_adaptive(H0, f, cycles=1)
    assert h[0] == h0[0] and H0.regular.lc == 1
    H1 = AD.build_adaptive(G, eps, transfer="galerkin")
    u, h1 = AD.solve_adaptive(H1, f, tol=1e-10, max_cycles=200, stagnation=1e-12)
    ustar, _, _ = AD.solve_composite_direct(G, eps, f)
    assert h1[-1] <= 1e-10
    assert np.linalg.norm(u - ustar) <= 1e-8 * np.linalg.norm(ustar)


@pytest.mark.parametrize("d,base,L", [(3, 2, 3), (2, 2, 5)])
def test_local_spacetree_matches_the_laid_out_grid(d, base, L):
    """The spacetree decided cell by cell (for grids too large to lay out)
    has the vertex classes of the laid-out grid at every vertex, and its
    composite rows equal the assembled composite system's rows wherever no
    hanging value is needed (the band workload's refinement and coefficient
    contrast 10^6, random iterate)."""
    P = W.adaptive_band(dim=d, base=base, level=L)
    G = AD.AdaptiveGrid(d, base, L, P.flags)
    T = AD.LocalSpacetree(d, base, L, P.mark)
    rng = np.random.default_rng(3)
    for l in range(base, L + 1):
        n = 3 ** l
        idx = rng.integers(0, n + 1, size=(300, d))
        leaves = np.argwhere(G.vtype[l] == AD.LEAF)[:, ::-1]
        idx = np.concatenate([idx, leaves[rng.choice(len(leaves), min(200, len(leaves)), replace=False)]])
        for v in idx:
            assert T.vclass(l, tuple(int(x) for x in v)) == G.vtype[l][tuple(v[::-1])]
    eps = P.eps_at(G.cell_centres())
    xyz = G.unknown_coords()
    lv = np.array([l for l, _ in G.leaves()])
    f = np.concatenate([P.f_at(l, xyz[lv == l]) for l in range(base, L + 1)])
    u = rng.uniform(-1, 1, size=G.n_unknowns())
    A, b = AD.composite_system(G, eps, f)
    r_full = b - A @ u
    leaves = G.leaves()
    pos = {(l, tuple(int(x) for x in v[::-1])): k for k, (l, v) in enumerate(leaves)}
    pick = rng.choice(G.n_unknowns(), 300, replace=False)
    samples = [(leaves[k][0], tuple(int(x) for x in leaves[k][1][::-1])) for k in pick]
    rows, scale = AD.local_composite_rows(T, P.eps_at, P.f_at, lambda l, w: u[pos[(l, w)]], samples)
    ok = ~np.isnan(rows)
    assert ok.sum() > 100
    np.testing.assert_allclose(rows[ok], r_full[pick][ok], rtol=0, atol=1e-13 * scale[ok].max())
    # the rows it declines are exactly those touching a hanging vertex
    for (l, v), good in zip(samples, ok):
        nb = [tuple(vi + oi - 1 for vi, oi in zip(v, o)) for o in np.ndindex(*([3] * d))]
        hang = any(T.vclass(l, w) == AD.HANGING for w in nb)
        assert good != hang


@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_parent_interpolated_hanging_rows_keep_dlinear_for_constant_eps(d, base, L):
    """The paper's reading of BoxMG rows at hanging vertices (d-linear
    interpolation of the parent stencils): for constant eps the parents'
    stencils are all one stencil up to scale and truncation at the boundary,
    so BoxMG still reproduces the d-linear weights and the operators of the
    d-linear Galerkin variant."""
    G, _, f = _problem(d, base, L, seed=5)
    eps = np.full(len(G.leaf_cells()), 2.5)
    Hb = AD.build_adaptive(G, eps, transfer="boxmg", hanging_rows="parents")
    Hg = AD.build_adaptive(G, eps, transfer="galerkin")
    for l in range(2, L + 1):
        np.testing.assert_allclose(Hb.P[l].toarray(), Hg.P[l].toarray() * (abs(Hb.P[l]).toarray() > 0),
                                   atol=1e-12)
        act = np.isin(G.vtype[l], (AD.LEAF, AD.REFINED))
        np.testing.assert_allclose(Hb.S[l][:, act], Hg.S[l][:, act], atol=1e-12 * abs(Hg.S[l]).max())


def test_parent_interpolated_hanging_rows_interpolate_the_parents():
    """Each hanging row is the weighted mean of its interior parents' rows:
    a hanging vertex on a coarse edge midpoint-third takes (2/3, 1/3)."""
    G, eps, _ = _problem(2, 2, 4, seed=2)
    e = G.level_eps(eps)
    Hs = AD.hanging_stencils_parents(G, e)
    Sc = O.geometric_stencil(AD.virtual_eps(G, e)[3], 2, 3, dirichlet=False)
    hv = np.argwhere(G.vtype[4] == AD.HANGING)
    checked = 0
    for v in hv:                                     # numpy order (y, x)
        y, x = v
        if x % 3 == 0 and y % 3 == 1:                # on a vertical coarse edge, one third up
            p0, p1 = (y // 3, x // 3), (y // 3 + 1, x // 3)
            if all(1 <= c <= 26 for c in p0 + p1) and 2 <= x <= 79 and 2 <= y <= 79:
                np.testing.assert_allclose(Hs[4][:, y, x], (2 / 3) * Sc[:, p0[0], p0[1]] + (1 / 3) * Sc[:, p1[0], p1[1]],
                                           rtol=1e-14, atol=1e-14)
                checked += 1
    assert checked > 0


@pytest.mark.parametrize("hanging_rows", ["covering", "parents"])
def test_multiscale_smoothing_keeps_the_composite_fixed_point(hanging_rows):
    """Alg. 1's smoothing of the coarser levels' leaves while a finer level is
    active changes the iterates, not the fixed point: the cycle converges to
    the directly solved composite system (d-linear Galerkin), and with BoxMG
    to the composite system of its own hanging constraints."""
    G, eps, f = _problem(2, 2, 4)
    ustar, A, b = AD.solve_composite_direct(G, eps, f)
    H = AD.build_adaptive(G, eps, transfer="galerkin", multiscale=True)
    u, hist = AD.solve_adaptive(H, f, tol=1e-12, max_cycles=100)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(u - ustar) <= 1e-10 * np.linalg.norm(ustar)
    H0 = AD.build_adaptive(G, eps, transfer="galerkin")
    _, hist0 = AD.solve_adaptive(H0, f, cycles=3)
    _, hist1 = AD.solve_adaptive(H, f, cycles=3)
    assert hist0 != hist1                           # the iterates do change
    Hb = AD.build_adaptive(G, eps, transfer="boxmg", hanging_rows=hanging_rows, multiscale=True)
    ub, histb = AD.solve_adaptive(Hb, f, tol=1e-11, max_cycles=200)
    us, Ab, bb = AD.solve_composite_direct(G, eps, f, AD.hanging_constraints(Hb))
    assert np.linalg.norm(ub - us) <= 1e-9 * np.linalg.norm(us)


@pytest.mark.parametrize("d,base,L,transfer", [(2, 1, 3, "galerkin"), (2, 2, 4, "boxmg"), (3, 1, 3, "galerkin")])
def test_full_refinement_fas_cycles_are_the_regular_v_cycles(d, base, L, transfer):
    """Every cell refined down to level L: the FAS V-cycle on the linear
    problem is the correction-scheme V-cycle of the regular hierarchy (same
    Galerkin operators, smoother and transfers), iterate for iterate, so the
    residual histories and the solutions after six cycles agree to rounding."""
    flags = {l: np.ones((3 ** l,) * d, bool) for l in range(base, L)}
    G = AD.AdaptiveGrid(d, base, L, flags)
    n = 3 ** L
    rng = np.random.default_rng(3)
    eps = rng.uniform(0.5, 2.0, size=n ** d)
    f = rng.uniform(-1, 1, size=G.n_unknowns())
    ua, ha = AD.solve_adaptive(AD.build_adaptive(G, eps, transfer=transfer), f, cycles=6)
    Hr = O.build_hierarchy(eps.reshape((n,) * d), d, L, transfer=transfer, check_definite=False)
    _, b = AD.composite_system(G, eps, f)
    ur, hr = O.solve(Hr, b, cycles=6)
    assert max(abs(x - y) / y for x, y in zip(ha, hr)) <= 1e-11
    assert np.abs(ua - ur).max() <= 1e-12 * np.abs(ur).max()


@pytest.mark.parametrize("d,base,L,hanging_rows", [(2, 2, 4, "covering"), (2, 2, 4, "parents"),
                                                   (3, 1, 3, "covering"), (3, 1, 3, "parents")])
def test_adaptive_boxmg_columns_satisfy_the_collapsed_fine_equations(d, base, L, hanging_rows):
    """On every adaptive level, inside the closed refined coarse cells (where
    the level's BoxMG prolongation is formed), each column satisfies the
    collapsed fine equations that define BoxMG (Sect. 4.4) with the level's
    rows, hanging rows included, under either reading of those rows: two
    balls, a checkerboard of contrast 1e3, held to 16 kappa 2^-52 (measured
    at most 5e-14); d-linear weights miss it by O(1)."""
    P = W.adaptive_balls(dim=d, base=base, level=L, n_balls=2, radius=0.25, seed=0)
    G = AD.AdaptiveGrid(d, base, L, P.flags)
    rng = np.random.default_rng(0)
    contrast = 1e3
    eps = np.where(rng.random(len(G.leaf_cells())) < 0.5, 1.0, contrast)
    H = AD.build_adaptive(G, eps, transfer="boxmg", hanging_rows=hanging_rows)
    hang_rows = AD.hanging_stencils if hanging_rows == "covering" else AD.hanging_stencils_parents
    Hs = hang_rows(G, H.eps)
    for l in range(base + 1, L + 1):
        S = H.S[l] + Hs[l]
        nf = 3 ** l
        region = np.zeros((nf + 1,) * d, dtype=bool)
        for C in np.argwhere(G.refined[l - 1]):                     # lattice axes (z, y, x)
            region[tuple(slice(3 * c, 3 * c + 4) for c in C)] = True
        assert region.any()
        cols = range(H.P[l].shape[1])
        assert worst_defining_equation(S, H.P[l], d, l, cols, region) < 16 * contrast * 2.0 ** -52
        assert worst_defining_equation(S, O.dlinear_P(d, l), d, l, cols, region) > 0.1



def _asymptotic_rate(hist):
    return (hist[-1] / hist[-5]) ** 0.25


@pytest.mark.parametrize("transfer", ["galerkin", "boxmg"])
@pytest.mark.parametrize("d,base,L", [(2, 2, 4), (3, 1, 3)])
def test_adaptive_fas_converges_at_the_regular_rate(d, base, L, transfer):
    """With constant eps and d-linear transfers (or BoxMG, whose weights are
    d-linear for constant eps), the FAS cycle on a spacetree refined around
    two balls (hanging vertices present) contracts the composite residual
    per cycle at the rate of the regular V(2,2) cycle on
    the finest level, within 15 % (measured 1.07x in 2D, 0.96x in 3D).
    Planted on the CPU: a halved coarse correction, a missing FAS coarse term
    A u, hanging values left stale after the correction (2D) or one
    pre-smoothing step instead of two each push the rate past it."""
    P = W.adaptive_balls(dim=d, base=base, level=L, n_balls=2, radius=0.25, seed=0,
                         contrast_field=False)
    G = AD.AdaptiveGrid(d, base, L, P.flags)
    assert (G.vtype[L] == AD.HANGING).any()
    H = AD.build_adaptive(G, np.ones(len(G.leaf_cells())), transfer=transfer)
    n = sum(int((G.vtype[l] == AD.LEAF).sum()) for l in range(base, L + 1))
    f = np.random.default_rng(0).uniform(-1.0, 1.0, n)
    _, hist_ad = AD.solve_adaptive(H, f, cycles=12)
    p = W.random_checkerboard(d, L, 0, values=(1.0, 1.0))
    Hr = O.build_hierarchy(p.eps, d, L, transfer="galerkin")
    _, hist_reg = O.solve(Hr, O.rhs_from_f(p.f, d, L), cycles=12)
    assert _asymptotic_rate(hist_ad) <= 1.15 * _asymptotic_rate(hist_reg)
