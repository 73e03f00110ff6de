"""Refinement criterion of the dynamically adaptive runs (oracle, FP64).

Sect. 7 (setups): per unrefined vertex, the absolute difference between the
vertex value and the mean of its 3^d - 1 neighbours; a vertex is a candidate
when it is unrefined and its residual is below a threshold (10^-2 in the
paper); about the 10 percent of the candidates with the largest differences
are refined, chosen through ten bins instead of a sort, and the region around
a chosen vertex is refined.

Readings (the paper gives the idea, not the arithmetic):

* Regular grids: every interior vertex is unrefined; boundary vertices hold
  zero and count as neighbours.
* The mean sums the neighbours in lattice order (x fastest, the centre
  skipped) and divides by 3^d - 1; the residual test is |r_v| < res_tol with
  r = b - A u.
* The ten bins split [lo, hi] (the smallest and largest candidate
  difference) evenly; a difference falls in bin min(9, floor((delta - lo) /
  ((hi - lo) / 10))), all of bin 9 when hi == lo.  Bins are taken from the top
  until they hold at least ``fraction`` of the candidates; every candidate in
  a taken bin is chosen.  Nothing is chosen when hi == 0.
* "The region around a vertex" is its 2^d adjacent cells: a cell is flagged
  when any of its corners is chosen.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import numpy as np

from .fem import offsets, shifted

NBINS = 10


def mean_difference(u_lat, d):
    """|mean of the 3^d - 1 neighbours - u| at every lattice vertex (lattice
    array, boundary entries meaningless)."""
    acc = np.zeros_like(u_lat)
    for o in offsets(d):
        if any(o):
            acc = acc + shifted(u_lat, o)
    return np.abs(acc / (3 ** d - 1) - u_lat)


def choose_vertices(delta, cand, fraction=0.1, nbins=NBINS):
    """Boolean mask of the chosen candidates (see module notes)."""
    chosen = np.zeros(delta.shape, dtype=bool)
    if not cand.any():
        return chosen
    dc = delta[cand]
    lo, hi = dc.min(), dc.max()
    if hi == 0.0:
        return chosen
    if hi > lo:
        width = (hi - lo) / nbins
        b = np.minimum(nbins - 1, np.floor((dc - lo) / width)).astype(np.int64)
    else:
        b = np.full(dc.shape, nbins - 1, dtype=np.int64)
    counts = np.bincount(b, minlength=nbins)
    need = fraction * len(dc)
    cum, kstar = 0, nbins - 1
    for k in range(nbins - 1, -1, -1):
        cum += counts[k]
        kstar = k
        if cum >= need:
            break
    sel = np.zeros(delta.shape, dtype=bool)
    sel[cand] = b >= kstar
    return sel


def refinement_flags(u_lat, r_lat, d, res_tol=1e-2, fraction=0.1):
    """Cell flags (shape (n,)*d, NumPy axes (z,) y, x) of one refinement step
    on a regular grid from the iterate and residual lattices."""
    level_n = u_lat.shape[0] - 1
    inner = np.zeros(u_lat.shape, dtype=bool)
    inner[(slice(1, level_n),) * d] = True
    delta = mean_difference(u_lat, d)
    cand = inner & (np.abs(r_lat) < res_tol)
    sel = choose_vertices(delta, cand, fraction)
    flags = np.zeros((level_n,) * d, dtype=bool)
    for s in offsets(d):
        if min(s) < 0:
            continue
        # cell c has corner c + s
        sl = tuple(slice(si, si + level_n) for si in reversed(s))
        flags |= sel[sl]
    return flags
