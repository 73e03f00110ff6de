"""Galerkin coarse operators and the definiteness check (oracle, FP64).

* Sect. 4.3: A_{l-1} = R A_l P with R = P^T unless stated otherwise (Sect. 4.4).
  The oracle forms the plain definition, the sparse triple product, with a
  library sparse matrix product as the step.
* Sect. 4.3 (dynamic coarsest level): a coarse stencil with a non-positive
  diagonal, or that is no longer diagonally dominant, makes the solver use a
  finer coarsest level.  Reading: row V fails when a_VV <= 0 or
  a_VV < (1 - 1e-10) * sum_{W != V} |a_VW| (the slack absorbs rounding in rows
  that are exactly weakly dominant, such as the interior Laplacian).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DOMINANCE_SLACK = 1e-10


def rap(A, P, R=None):
    """R A P (sparse, interior unknowns); R = P^T unless given (Petrov-Galerkin,
    Sect. 4.3)."""
    R = P.T if R is None else R
    return sp.csr_matrix(R @ (A @ P))


def definiteness_violations(Ac):
    """Indices of coarse rows that fail the diagonal check."""
    Ac = sp.csr_matrix(Ac)
    diag = Ac.diagonal()
    absrow = np.asarray(abs(Ac).sum(axis=1)).ravel() - np.abs(diag)
    bad = (diag <= 0.0) | (diag < (1.0 - DOMINANCE_SLACK) * absrow)
    return np.nonzero(bad)[0]
