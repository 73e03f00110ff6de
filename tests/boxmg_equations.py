"""The equations that define BoxMG's prolongation (Sect. 4.4), checked on an
assembled P over the fine lattice: shared by the regular and adaptive oracle
pins."""
import itertools

import numpy as np

from oracle import fem
from oracle.fem import shifted


def worst_defining_equation(S, P, d, Lf, columns, region=None):
    """The largest relative residual of BoxMG's defining equations (Sect. 4.4)
    over the given coarse hat columns w = P e_V on the fine lattice: at a fine
    vertex that lies on the coarse planes of the axes in a set K (but not on
    all of them), the fine stencil collapsed along K (offsets along K set to
    zero, entries summed) annihilates w; interior points (K empty) take the
    stencil whole.  Each residual is relative to the sum of its terms'
    magnitudes.  ``region``: a lattice mask of the fine vertices checked
    (default: every interior vertex)."""
    nf = 3 ** Lf
    inner = (slice(1, nf),) * d
    ax = np.meshgrid(*[np.arange(nf + 1)] * d, indexing="ij")        # lattice axes (z, y, x)
    onplane = [ax[d - 1 - i] % 3 == 0 for i in range(d)]             # per axis, x first
    interior = np.zeros((nf + 1,) * d, dtype=bool)
    interior[inner] = True
    if region is not None:
        interior &= region
    Pc = P.tocsc()
    worst = 0.0
    for j in columns:
        if Pc[:, j].nnz == 0:
            continue
        w = np.zeros((nf + 1,) * d)
        w[inner] = Pc[:, j].toarray().reshape((nf - 1,) * d)
        for K in itertools.product((False, True), repeat=d):
            if all(K):
                continue                                             # c-points: unit rows
            sel = interior.copy()
            for i in range(d):
                sel &= onplane[i] if K[i] else ~onplane[i]
            eq = np.zeros_like(w)
            mag = np.zeros_like(w)
            for k, o in enumerate(fem.offsets(d)):
                t = S[k] * shifted(w, tuple(0 if K[i] else o[i] for i in range(d)))
                eq += t
                mag += np.abs(t)
            sel &= mag > 0
            if sel.any():
                worst = max(worst, float((np.abs(eq[sel]) / mag[sel]).max()))
    return worst
