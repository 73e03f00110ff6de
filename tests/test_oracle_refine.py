"""Pins of the oracle's refinement criterion (Sect. 7, dynamic adaptivity):
brute-force mean differences, linear functions that change nothing, the
choice of about the top fraction through ten bins, and the cells around a
chosen vertex."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import refine as RF


@pytest.mark.parametrize("d", [2, 3])
def test_mean_difference_brute_force(d):
    rng = np.random.default_rng(1)
    n = 9 if d == 2 else 6
    u = rng.normal(size=(n + 1,) * d)
    got = RF.mean_difference(u, d)
    for v in itertools.product(range(1, n), repeat=d):
        nb = [u[tuple(v[i] + o[i] for i in range(d))]
              for o in itertools.product((-1, 0, 1), repeat=d) if any(o)]
        assert abs(got[v] - abs(np.mean(nb) - u[v])) <= 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_linear_iterates_choose_nothing(d):
    """A linear function equals the mean of its neighbours: every difference
    is zero (up to rounding far below any bin) and no cell is flagged."""
    n = 27 if d == 2 else 9
    x = np.meshgrid(*([np.arange(n + 1) / n] * d), indexing="ij")
    u = 0.3 + sum((i + 1) * xi for i, xi in enumerate(x))
    delta = RF.mean_difference(u, d)
    assert delta[(slice(1, n),) * d].max() <= 1e-14
    exact = RF.refinement_flags(np.round(u * n) / n * 0.0, np.zeros_like(u), d)
    assert not exact.any()


def test_top_fraction_through_bins():
    """Differences 0..999 (one per candidate): ten even bins of width 99.9
    take the top bin (candidates 900..999: 100 = 10 percent); asking for 25
    percent takes three bins (700..999)."""
    delta = np.arange(1000, dtype=np.float64)
    cand = np.ones(1000, dtype=bool)
    sel = RF.choose_vertices(delta, cand, 0.1)
    assert sel.sum() == 100 and sel[900:].all()
    sel = RF.choose_vertices(delta, cand, 0.25)
    assert sel.sum() == 300 and sel[700:].all()
    # non-candidates are never chosen, even with the largest difference
    cand2 = cand.copy()
    cand2[999] = False
    assert not RF.choose_vertices(delta, cand2, 0.1)[999]
    # equal differences: all candidates; all zero: none
    assert RF.choose_vertices(np.full(10, 2.0), np.ones(10, bool), 0.1).all()
    assert not RF.choose_vertices(np.zeros(10), np.ones(10, bool), 0.1).any()


def test_cells_around_a_chosen_vertex_and_residual_gate():
    """One bump at an interior vertex: its 2^d cells are flagged; with its
    residual above the threshold it is no candidate, and its eight
    neighbours (difference 1/8) are chosen instead: 4 x 4 cells."""
    d, n = 2, 27
    u = np.zeros((n + 1,) * d)
    u[10, 17] = 1.0                       # (y, x) = (10, 17)
    r = np.zeros_like(u)
    flags = RF.refinement_flags(u, r, d, fraction=0.001)
    # the bump and its 8 neighbours differ; the bump (|0.0 - 1|) is largest
    want = np.zeros((n, n), dtype=bool)
    want[9:11, 16:18] = True
    assert (flags == want).all()
    r[10, 17] = 0.5
    flags = RF.refinement_flags(u, r, d, fraction=0.001)
    assert flags.sum() == 16 and flags[8:12, 15:19].all()
