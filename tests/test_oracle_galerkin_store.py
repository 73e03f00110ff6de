"""Pins of the oracle's Galerkin operators, definiteness check and delta store."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle import galerkin, store


@pytest.mark.parametrize("d,Lf", [(2, 3), (2, 4), (3, 2)])
def test_galerkin_dlinear_equals_rediscretisation(d, Lf):
    """Constant eps, d-linear P, R = P^T: P^T A_h P = A_H (nested Q1 spaces)."""
    n = 3 ** Lf
    eps = np.full((n,) * d, 2.0)
    Af = O.stencil_to_csr(O.geometric_stencil(eps, d, Lf), d, Lf)
    Ac = O.rap(Af, O.dlinear_P(d, Lf))
    Ag = O.stencil_to_csr(O.geometric_stencil(np.full((n // 3,) * d, 2.0), d, Lf - 1), d, Lf - 1)
    assert abs(Ac - Ag).max() <= 4e-15 * abs(Ag).max()


def test_rap_symmetric_and_rows_sum_zero_inside():
    Lf = 4
    n = 3 ** Lf
    rng = np.random.default_rng(21)
    eps = rng.choice([1.0, 1e4], size=(n, n))
    Af = O.stencil_to_csr(O.geometric_stencil(eps, 2, Lf), 2, Lf)
    P = O.boxmg_P(O.csr_to_stencil(Af, 2, Lf), 2, Lf)
    Ac = O.rap(Af, P)
    assert abs(Ac - Ac.T).max() <= 1e-12 * abs(Ac).max()
    S = O.csr_to_stencil(Ac, 2, Lf - 1)
    rows = S.sum(axis=0)[3:-3, 3:-3]
    assert np.abs(rows).max() <= 1e-10 * np.abs(S).max()
    # SPD: smallest eigenvalue positive
    w = np.linalg.eigvalsh(Ac.toarray())
    assert w.min() > 0


def test_rap_brute_force_entries():
    """A_c(V,W) = sum_i sum_j P(i,V) a(i,j) P(j,W) by explicit loops."""
    Lf = 2
    n = 9
    rng = np.random.default_rng(22)
    eps = rng.uniform(0.5, 2.0, size=(n, n))
    Af = O.stencil_to_csr(O.geometric_stencil(eps, 2, Lf), 2, Lf).toarray()
    P = O.boxmg_P(O.csr_to_stencil(sp.csr_matrix(Af), 2, Lf), 2, Lf).toarray()
    Ac = O.rap(sp.csr_matrix(Af), sp.csr_matrix(P)).toarray()
    for V in range(P.shape[1]):
        for Wc in range(P.shape[1]):
            s = 0.0
            for i in range(P.shape[0]):
                if P[i, V] == 0.0:
                    continue
                for j in range(P.shape[0]):
                    s += P[i, V] * Af[i, j] * P[j, Wc]
            assert abs(s - Ac[V, Wc]) <= 1e-14 * np.abs(Ac).max()


def test_definiteness_check():
    Lf = 3
    n = 27
    Af = O.stencil_to_csr(O.geometric_stencil(np.ones((n, n)), 2, Lf), 2, Lf)
    Ac = O.rap(Af, O.dlinear_P(2, Lf))
    assert len(O.definiteness_violations(Ac)) == 0
    bad = Ac.tolil()
    bad[5, 5] = -bad[5, 5]
    assert list(O.definiteness_violations(bad.tocsr())) == [5]
    weak = Ac.tolil()
    weak[27, 27] = 0.9 * weak[27, 27]     # interior row (3,3) loses diagonal dominance
    assert list(O.definiteness_violations(weak.tocsr())) == [27]


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
@pytest.mark.parametrize("transfer", ["galerkin", "boxmg"])
def test_constant_eps_deltas_vanish(d, L, transfer):
    n = 3 ** L
    H = O.build_hierarchy(np.full((n,) * d, 5.0), d, L, transfer=transfer)
    for l in range(H.lc, L):
        S = O.csr_to_stencil(H.A[l], d, l)
        G = O.geometric_stencil(H.eps[l], d, l)
        zero = O.delta_zero(O.hier_deltas(S, G), G)
        inner = (slice(1, 3 ** l),) * d
        assert zero[inner].all(), (l, transfer)
    for l, P in H.P.items():
        assert abs(P - O.dlinear_P(d, l)).max() <= store.EPS_ZERO


def test_bf16_matches_library_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-20, 20, size=4000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.quantise(x, "bf16"), ref)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert O.quantise(np.array([1.0 + 2.0 ** -8]), "bf16")[0] == 1.0
    assert O.quantise(np.array([1.0 + 3 * 2.0 ** -8]), "bf16")[0] == 1.0 + 2.0 ** -6


def test_fp16_scale_rule():
    assert list(store.fp16_exponent(np.array([2.0 ** 15, 2.0 ** 15 + 1, 1.0, 3.0, 0.0]))) == [0, 1, -15, -13, 0]
    rng = np.random.default_rng(24)
    d = rng.normal(size=(9, 100)) * 10.0 ** rng.integers(-12, 6, size=100)
    q = O.quantise(d, "fp16", axis=0)
    rel = np.abs(q - d).max(axis=0) / np.abs(d).max(axis=0)
    assert rel.max() <= 2.0 ** -11 * 1.0001
    e = store.fp16_exponent(np.abs(d).max(axis=0))
    assert np.all(np.abs(d).max(axis=0) <= 2.0 ** (15 + e))
    assert np.all(np.abs(d).max(axis=0) > 2.0 ** (14 + e))
    # against the library half-precision conversion of the scaled value
    sc = np.ldexp(1.0, e)
    ref = (d / sc).astype(np.float32).astype(np.float16).astype(np.float64) * sc
    np.testing.assert_array_equal(q, ref)


def test_fp32_and_fp64_store():
    x = np.array([1.0 / 3.0, -2.0 ** -30 / 7.0])
    np.testing.assert_array_equal(O.quantise(x, "fp64"), x)
    np.testing.assert_array_equal(O.quantise(x, "fp32"), x.astype(np.float32).astype(np.float64))
