"""Pins of the oracle's transfer operators: d-linear hat functions, the
printed BoxMG systems, closed forms and the invariants the paper states."""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from boxmg_equations import worst_defining_equation
from oracle import fem, transfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d,Lf", [(1, 2), (2, 2), (3, 2)])
def test_dlinear_columns_are_coarse_hat_functions(d, Lf):
    """Column V of P = the coarse d-linear basis function of V sampled at the
    fine vertices (tensor product of 1D hats of width 1/3^(Lf-1))."""
    P = O.dlinear_P(d, Lf).toarray()
    nf = 3 ** Lf
    nc = nf // 3
    fine = list(itertools.product(range(1, nf), repeat=d))
    coarse = list(itertools.product(range(1, nc), repeat=d))
    for jc, Vr in enumerate(coarse):
        V = Vr[::-1]
        col = np.zeros(len(fine))
        for jf, Fr in enumerate(fine):
            F = Fr[::-1]
            val = 1.0
            for i in range(d):
                val *= max(0.0, 1.0 - abs(F[i] / nf - V[i] / nc) * nc)
            col[jf] = val
        np.testing.assert_allclose(P[:, jc], col, atol=1e-15)


def test_boxmg_1d_golden():
    line = [l for l in open(os.path.join(GOLDEN, "boxmg_1d.txt")) if not l.startswith("#")][0]
    st, pv = line.split("|")
    st = np.array([float(x) for x in st.split()])
    want = np.array([float(x) for x in pv.split()])
    t = np.tile(st, (1, 4, 1))
    for solver in (O.boxmg_reference_stepwise, O.boxmg_reference_Cs):
        np.testing.assert_allclose(solver(t, 1)[0], want, rtol=1e-15)


def test_boxmg_1d_variable_coefficient_is_harmonic():
    """1D FEM stencils of cell coefficients e1, e2, e3 inside the patch: the
    prolongation is p(1) = 1 - (1/e1)/S, p(2) = (1/e3)/S with S = sum 1/e_i
    (flux continuity)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        e = rng.uniform(0.01, 100.0, size=3)         # cells [0,1], [1,2], [2,3] of the patch
        t = np.zeros((1, 4, 3))
        for y in (1, 2):
            t[0, y] = [-e[y - 1], e[y - 1] + e[y], -e[y]]
        S = np.sum(1.0 / e)
        p = O.boxmg_reference_stepwise(t, 1)[0]
        np.testing.assert_allclose(p, [1.0, 1.0 - (1.0 / e[0]) / S, (1.0 / e[2]) / S], rtol=1e-13)


def test_boxmg_2d_reference_matrix_equals_printed():
    rows = []
    for line in open(os.path.join(GOLDEN, "boxmg_Cs_2d.txt")):
        if line.startswith("#") or not line.strip():
            continue
        pv, rest = line.split("|")
        rows.append((int(pv), rest.split()))
    rng = np.random.default_rng(11)
    t = rng.normal(size=(3, 16, 9))
    C = O.boxmg_reference_matrix(t, 2)
    for pv, entries in rows:
        y = (pv % 4, pv // 4)
        r = y[0] + 3 * y[1]
        want = np.zeros((3, 9))
        if entries == ["id"]:
            want[:, r] = 1.0
        else:
            for e in entries:
                col, terms = e.split(":")
                for k in terms.split("+"):
                    want[:, int(col)] += t[:, pv, int(k)]
        np.testing.assert_allclose(C[:, r, :], want, rtol=1e-15, atol=0)
    assert len(rows) == 9


@pytest.mark.parametrize("d", [2, 3])
def test_stepwise_equals_single_system(d):
    rng = np.random.default_rng(12)
    B = 50
    t = rng.uniform(-1.0, -0.01, size=(B, 4 ** d, 3 ** d))
    centre = (3 ** d) // 2
    t[:, :, centre] = -t.sum(axis=2) + t[:, :, centre] + rng.uniform(0.0, 0.5, size=(B, 4 ** d))
    a = O.boxmg_reference_stepwise(t, d)
    b = O.boxmg_reference_Cs(t, d)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("d,Lf", [(2, 3), (3, 2)])
def test_boxmg_constant_eps_is_dlinear(d, Lf):
    n = 3 ** Lf
    S = O.geometric_stencil(np.full((n,) * d, 3.7), d, Lf)
    Pb = O.boxmg_P(S, d, Lf)
    Pd = O.dlinear_P(d, Lf)
    assert abs(Pb - Pd).max() < 1e-14


def test_boxmg_layered_eps_edges_follow_1d_formula():
    """eps = eps(x) constant in y: collapsing the 2D Q1 stencil over y gives the
    1D stiffness of eps(x) (times h-independent factors), so the weights on
    x-lines through coarse vertices follow the 1D harmonic formula."""
    Lf = 3
    n = 3 ** Lf
    rng = np.random.default_rng(8)
    ex = rng.uniform(0.1, 10.0, size=n)
    eps = np.tile(ex, (n, 1))
    P = O.boxmg_P(O.geometric_stencil(eps, 2, Lf), 2, Lf)
    W = O.P_to_parent_weights(P, 2, Lf)
    nc = n // 3
    for Vx in range(1, nc):
        for Vy in range(1, nc):
            for sgn in (1, -1):
                cells = [3 * Vx + (k if sgn > 0 else -k - 1) for k in range(3)]
                e = ex[cells]
                S = np.sum(1.0 / e)
                for t_, want in ((1, 1.0 - (1.0 / e[0]) / S), (2, (1.0 / e[2]) / S)):
                    fx, fy = 3 * Vx + sgn * t_, 3 * Vy
                    kappa_x = 0 if fx // 3 == Vx else 1
                    got = W[kappa_x, fy, fx]
                    assert abs(got - want) < 1e-13, (Vx, Vy, sgn, t_, got, want)


def test_boxmg_mirror_equivariance():
    Lf = 3
    n = 3 ** Lf
    rng = np.random.default_rng(9)
    eps = rng.uniform(0.1, 10.0, size=(n, n))
    P1 = O.P_to_parent_weights(O.boxmg_P(O.geometric_stencil(eps, 2, Lf), 2, Lf), 2, Lf)
    P2 = O.P_to_parent_weights(O.boxmg_P(O.geometric_stencil(eps[:, ::-1], 2, Lf), 2, Lf), 2, Lf)
    # weight of coarse vertex V at fine f  ==  weight of mirrored V at mirrored f
    nc = n // 3
    for fy in range(1, n):
        for fx in range(1, n):
            for kx in (0, 1):
                for ky in (0, 1):
                    Vx, Vy = fx // 3 + kx, fy // 3 + ky
                    if not (1 <= Vx < nc and 1 <= Vy < nc):
                        continue
                    mfx, mVx = n - fx, nc - Vx
                    mkx = mVx - mfx // 3
                    if mkx not in (0, 1):
                        assert P1[kx + 2 * ky, fy, fx] == 0.0
                        continue
                    a = P1[kx + 2 * ky, fy, fx]
                    b = P2[mkx + 2 * ky, fy, mfx]
                    assert abs(a - b) < 1e-13


@pytest.mark.parametrize("d", [2, 3])
def test_boxmg_ignores_patch_corner_stencils(d):
    rng = np.random.default_rng(13)
    t = rng.uniform(-1.0, -0.01, size=(4, 4 ** d, 3 ** d))
    t[:, :, (3 ** d) // 2] = 3 ** d
    p0 = O.boxmg_reference_stepwise(t, d)
    t2 = t.copy()
    for y in itertools.product((0, 3), repeat=d):
        t2[:, sum(yi * 4 ** i for i, yi in enumerate(y))] = rng.normal(size=(4, 3 ** d))
    np.testing.assert_array_equal(O.boxmg_reference_stepwise(t2, d), p0)


def test_boxmg_locality():
    """Perturbing a stencil outside coarse vertex V's 5^d neighbourhood leaves
    V's prolongation entries unchanged (no P entry depends on a stencil outside
    its patch)."""
    Lf = 3
    n = 3 ** Lf
    rng = np.random.default_rng(10)
    eps = rng.uniform(0.1, 10.0, size=(n, n))
    S = O.geometric_stencil(eps, 2, Lf)
    P1 = O.boxmg_P(S, 2, Lf).toarray()
    S2 = S.copy()
    S2[:, 20, 20] *= 1.7                  # one fine vertex (x=20, y=20)
    P2 = O.boxmg_P(S2, 2, Lf).toarray()
    nc = n // 3
    changed = np.nonzero(np.abs(P1 - P2).max(axis=0) > 0)[0]
    for c in changed:
        Vx, Vy = c % (nc - 1) + 1, c // (nc - 1) + 1
        assert abs(3 * Vx - 20) <= 3 and abs(3 * Vy - 20) <= 3, (Vx, Vy)
    assert len(changed) > 0


def test_boxmg_rows_partition_unity_inside():
    """Interior fine rows of P sum to one (collapsed stencils keep the zero row
    sum, so constants are interpolated exactly) away from the boundary."""
    Lf = 3
    n = 3 ** Lf
    rng = np.random.default_rng(14)
    eps = rng.choice([1.0, 1e4], size=(n, n))
    P = O.boxmg_P(O.geometric_stencil(eps, 2, Lf), 2, Lf)
    s = np.asarray(P.sum(axis=1)).reshape(n - 1, n - 1)
    np.testing.assert_allclose(s[3:-3, 3:-3], 1.0, rtol=1e-10)  # contrast 1e4 amplifies rounding


@pytest.mark.parametrize("d,Lf", [(2, 3), (3, 2)])
def test_boxmg_shared_entries_agree_exactly_for_constant_eps(d, Lf):
    """Neighbouring patches compute their shared entries (c-points, line and
    face points) alike: for constant eps the copies are identical."""
    n = 3 ** Lf
    S = O.geometric_stencil(np.full((n,) * d, 2.5), d, Lf)
    info = {}
    transfer.boxmg_P(S, d, Lf, info=info)
    assert info["shared_disagreement"] == 0.0


@pytest.mark.parametrize("d,Lf", [(2, 3), (3, 2)])
@pytest.mark.parametrize("contrast", [1e2, 1e4, 1e6])
def test_boxmg_shared_entries_agree_to_contrast_rounding(d, Lf, contrast):
    """For a two-valued checkerboard the copies of a shared entry differ by
    rounding amplified by the contrast: within the check's bound of
    16 kappa 2^-52, where kappa, the diagonal ratio, is the contrast within a
    factor of a few."""
    n = 3 ** Lf
    rng = np.random.default_rng(5)
    eps = np.where(rng.random((n,) * d) < 0.5, 1.0, contrast)
    S = O.geometric_stencil(eps, d, Lf)
    info = {}
    transfer.boxmg_P(S, d, Lf, info=info)
    tol = transfer.shared_entry_tolerance(S, d)
    assert info["shared_disagreement"] <= tol
    kappa = tol / (16.0 * 2.0 ** -52)
    assert contrast / 8 <= kappa <= 8 * contrast


def test_unique_shared_entries_reports_the_largest_disagreement():
    """Copies of (row, col) entries: the first copy is kept and the largest
    relative deviation of any other copy is reported (a planted 3e-7 on an
    entry of size 2 gives 1.5e-7); ranks decide which copy comes first."""
    rows = np.array([0, 0, 1, 1, 1, 2])
    cols = np.array([0, 0, 1, 1, 1, 0])
    vals = np.array([0.5, 0.5, 2.0, 2.0 + 3e-7, 2.0, 7.0])
    uniq, first, dis = transfer.unique_shared_entries(rows, cols, vals, 4)
    assert list(uniq) == [0, 5, 8]
    assert list(first) == [0.5, 2.0, 7.0]
    assert abs(dis - 1.5e-7) < 1e-15
    ranks = np.array([0, 0, 1, 0, 2, 0])
    _, first, dis = transfer.unique_shared_entries(rows, cols, vals, 4, ranks)
    assert first[1] == 2.0 + 3e-7 and abs(dis - 3e-7 / (2.0 + 3e-7)) < 1e-15


def _harmonic_weight(e, t):
    """Weight of a coarse vertex at fine distance t (0..2) towards the three
    fine cells e (in order away from it): the 1D solution of -(eps u')' = 0
    with u = 1 at the vertex and 0 at the next one."""
    return 1.0 - np.sum(1.0 / e[:t]) / np.sum(1.0 / e)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_boxmg_3d_layered_eps_is_harmonic_times_linear(axis):
    """eps varying along one axis only: every BoxMG weight of the orthant
    regions, interior points included, is the 1D harmonic weight along that
    axis times the linear weights along the other two (the local problems
    separate); a mixed-up axis or collapsed entry in the 3D patch systems
    breaks it."""
    Lf = 2
    n = 3 ** Lf
    rng = np.random.default_rng(8 + axis)
    e1 = rng.uniform(0.1, 10.0, size=n)
    shape = [1, 1, 1]
    shape[2 - axis] = n                       # lattice axes are (z, y, x)
    eps = np.broadcast_to(e1.reshape(shape), (n, n, n)).copy()
    W = O.P_to_parent_weights(O.boxmg_P(O.geometric_stencil(eps, 3, Lf), 3, Lf), 3, Lf)
    nc = n // 3
    worst = 0.0
    for V in itertools.product(range(1, nc), repeat=3):            # (Vx, Vy, Vz)
        for s in itertools.product((1, -1), repeat=3):
            for t in itertools.product(range(3), repeat=3):
                f = [3 * V[a] + s[a] * t[a] for a in range(3)]
                kap = [0 if f[a] // 3 == V[a] else 1 for a in range(3)]
                want = 1.0
                for a in range(3):
                    if a == axis:
                        cells = [3 * V[a] + (k if s[a] > 0 else -k - 1) for k in range(3)]
                        want *= _harmonic_weight(e1[cells], t[a])
                    else:
                        want *= 1.0 - t[a] / 3.0
                got = W[kap[0] + 2 * kap[1] + 4 * kap[2], f[2], f[1], f[0]]
                worst = max(worst, abs(got - want))
    assert worst < 1e-13


@pytest.mark.parametrize("seed,contrast", [(3, 10.0), (3, 1e4), (4, 1e4)])
def test_boxmg_3d_eps_constant_along_z_is_2d_weight_times_linear(seed, contrast):
    """eps varying along x and y only, two-valued at the given contrast: collapsing
    the 3D Q1 stencil along z gives h times the 2D Q1 stencil of the
    cross-section, and a Q1 z-stiffness annihilates linear functions, so every
    3D BoxMG weight (line, face and interior points) is the 2D BoxMG weight of
    the cross-section (itself pinned to the printed C(s) system and the 1D
    harmonic formula) times the linear weight along z.  Both sides solve
    their patch systems in floating point, so they agree to the rounding
    amplified by the contrast kappa: held to 16 kappa 2^-52, the shared-entry
    bound (measured at most 5 kappa 2^-52).  A dropped mass term or an axis
    mix-up in the 3D face or volume systems moves weights by 1e-2 or more."""
    Lf = 2
    n = 3 ** Lf
    rng = np.random.default_rng(seed)
    e2 = np.where(rng.random((n, n)) < 0.5, 1.0, contrast)      # (y, x)
    eps = np.broadcast_to(e2[None, :, :], (n, n, n)).copy()   # (z, y, x)
    W3 = O.P_to_parent_weights(O.boxmg_P(O.geometric_stencil(eps, 3, Lf), 3, Lf), 3, Lf)
    W2 = O.P_to_parent_weights(O.boxmg_P(O.geometric_stencil(e2, 2, Lf), 2, Lf), 2, Lf)
    nc = n // 3
    worst = 0.0
    for V in itertools.product(range(1, nc), repeat=3):            # (Vx, Vy, Vz)
        for s in itertools.product((1, -1), repeat=3):
            for t in itertools.product(range(3), repeat=3):
                f = [3 * V[a] + s[a] * t[a] for a in range(3)]
                kap = [0 if f[a] // 3 == V[a] else 1 for a in range(3)]
                want = W2[kap[0] + 2 * kap[1], f[1], f[0]] * (1.0 - t[2] / 3.0)
                got = W3[kap[0] + 2 * kap[1] + 4 * kap[2], f[2], f[1], f[0]]
                worst = max(worst, abs(got - want))
    assert worst < 16 * contrast * 2.0 ** -52, worst / (contrast * 2.0 ** -52)


@pytest.mark.parametrize("d,Lf,contrast,field", [(2, 3, 1e2, "smooth"), (2, 3, 1e4, "checker"),
                                                 (3, 2, 1e4, "smooth"), (3, 2, 1e4, "checker"),
                                                 (3, 3, 1e4, "checker")])
def test_boxmg_columns_satisfy_the_collapsed_fine_equations(d, Lf, contrast, field):
    """For eps varying along every axis (the case no closed form covers), each
    prolongated coarse hat function satisfies, on the whole fine lattice, the
    equations that define BoxMG (Sect. 4.4): the full fine stencil at points
    inside a coarse cell, the stencil collapsed onto the face in 3D, onto the
    line on coarse-grid lines.  This holds the lattice form (patch gather,
    mirroring, assembly of P) to the definition, to 16 kappa 2^-52 for kappa
    the contrast; d-linear interpolation misses it by O(1)."""
    n = 3 ** Lf
    rng = np.random.default_rng(31 + d + Lf)
    if field == "smooth":
        eps = np.exp(rng.uniform(0.0, np.log(contrast), size=(n,) * d))
    else:
        eps = np.where(rng.random((n,) * d) < 0.5, 1.0, contrast)
    S = O.geometric_stencil(eps, d, Lf)
    P = O.boxmg_P(S, d, Lf)
    ncol = P.shape[1]
    cols = range(ncol) if ncol <= 64 else np.random.default_rng(5).choice(ncol, 24, replace=False)
    bound = 16 * contrast * 2.0 ** -52
    assert worst_defining_equation(S, P, d, Lf, cols) < bound
    assert worst_defining_equation(S, O.dlinear_P(d, Lf), d, Lf, cols) > 0.1
