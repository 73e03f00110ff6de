"""The refinement criterion's entry point that allocates nothing: its flags
and counts equal those of the allocating entry point (and the oracle's), on
two calls in a row whose second input is smaller, so the scratch array
shared by the calls must be re-initialised by each."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _seeded_iterate(d, L, seed):
    n = 3 ** L
    rng = np.random.default_rng(seed)
    x = np.meshgrid(*([np.arange(1, n) / n] * d), indexing="ij")
    u = np.prod([np.sin(np.pi * xi) for xi in x], axis=0)
    u = u + 0.01 * rng.normal(size=u.shape)
    idx = rng.integers(0, n - 1, size=(6, d))
    u[tuple(idx.T)] += 0.5
    return u.ravel()


def _median_gap_threshold(r):
    s = np.sort(np.abs(r))
    k = len(s) // 2
    while s[k + 1] - s[k] <= 1e-9 * s[k]:
        k += 1
    return 0.5 * (s[k] + s[k + 1])


def _case(qmg, d, L, fraction, seed):
    p = W.random_checkerboard(d, L, seed=seed, values=(1.0, 10.0), blocks=9 if L > 3 else 3)
    g = qmg.Grid(d, L, qmg.make_opts("boxmg", "hier64"))
    g.set_coefficients(p.eps, p.f)
    g.build()
    u = _seeded_iterate(d, L, seed + 20)
    g.set_solution(u)
    A = O.stencil_to_csr(O.geometric_stencil(p.eps, d, L), d, L)
    r = O.rhs_from_f(p.f, d, L) - A @ u
    return g, u, r, _median_gap_threshold(r)


def _raw_call(qmg, g, name, res_tol, fraction):
    n = 3 ** g.level
    out = np.zeros((n,) * g.dim, dtype=np.uint8)
    cnt = C.c_int64(-1)
    rc = getattr(g.lib, name)(g.h, C.c_double(res_tol), C.c_double(fraction),
                              out.ctypes.data_as(C.c_void_p), C.byref(cnt))
    return rc, out, int(cnt.value)


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    qmg = require_gpu()
    # first call on the larger input, second on a smaller one; the no-alloc
    # call runs first on each grid, before the allocating one has made its
    # own buffer
    for d, L, fraction, seed in [(2, 5, 0.1, 8), (2, 4, 0.3, 3)]:
        announce(f"no-alloc refine flags d={d} L={L} fraction={fraction}")
        g, u, r, res_tol = _case(qmg, d, L, fraction, seed)
        rc0, f0, n0 = _raw_call(qmg, g, "qmg_refine_flags_noalloc", res_tol, fraction)
        rc1, f1, n1 = _raw_call(qmg, g, "qmg_refine_flags", res_tol, fraction)
        g.close()
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(f0, f1)
        assert n0 == n1 == int(f0.sum())
        want = O.refine.refinement_flags(O.fem.lattice_from_unknowns(u, d, L),
                                         O.fem.lattice_from_unknowns(r, d, L), d, res_tol, fraction)
        assert want.any() and not want.all()
        assert np.array_equal(f0.astype(bool), want)


def test_noalloc_degenerate_and_error_paths():
    """No candidate after a call that had many (the scratch keeps the last
    call's extrema, so this checks it is re-initialised), fraction 1 on a 3D
    grid, and the argument checks of the allocating entry point."""
    qmg = require_gpu()
    announce("no-alloc refine flags degenerate")
    g, u, r, res_tol = _case(qmg, 3, 3, 0.1, 4)
    f_many = g.refine_flags(res_tol, 0.1, noalloc=True)
    assert f_many.any()
    tiny = 0.5 * np.abs(r).min()
    rc, f, n = _raw_call(qmg, g, "qmg_refine_flags_noalloc", tiny, 0.1)
    assert rc == 0 and n == 0 and not f.any()
    big = 2.0 * np.abs(r).max()
    f_all = g.refine_flags(big, 1.0, noalloc=True)
    assert np.array_equal(f_all, g.refine_flags(big, 1.0))
    for tol, frac in [(0.0, 0.1), (1e-2, 0.0), (1e-2, 1.5)]:
        rc_a, _, _ = _raw_call(qmg, g, "qmg_refine_flags", tol, frac)
        rc_n, _, _ = _raw_call(qmg, g, "qmg_refine_flags_noalloc", tol, frac)
        assert rc_a == rc_n and rc_n != 0
    g.close()
