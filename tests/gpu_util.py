"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import sys

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1607_00648_amd import qmg
    qmg.load()  # raises when the library is missing: no fallback
    return qmg


def announce(msg):
    """Names the case on stdout before any GPU work (for post-mortems)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def lattice_of_unknowns(x, d, level):
    n = 3 ** level
    out = np.zeros((n + 1,) * d)
    out[(slice(1, n),) * d] = np.asarray(x).reshape((n - 1,) * d)
    return out


def unknowns_of_lattice(a, d, level):
    n = 3 ** level
    return np.ascontiguousarray(a[(slice(1, n),) * d]).ravel()


def weights_to_csr(W, d, level_f):
    """Sparse P (fine x coarse interior unknowns) from per-fine-vertex parent
    weights (2^d lattice arrays, as qmg_get_prolongation returns them)."""
    import itertools
    import scipy.sparse as sp
    nf = 3 ** level_f
    nc = nf // 3
    rows, cols, vals = [], [], []
    for c, kap in enumerate([tuple(reversed(t)) for t in itertools.product((0, 1), repeat=d)]):
        for idx in itertools.product(range(1, nf), repeat=d):
            f = idx[::-1]                       # x first
            V = tuple(f[i] // 3 + kap[i] for i in range(d))
            w = W[(c,) + idx]
            if w == 0.0:
                continue
            assert all(1 <= Vi <= nc - 1 for Vi in V), (f, V, w)
            rows.append(sum((f[i] - 1) * (nf - 1) ** i for i in range(d)))
            cols.append(sum((V[i] - 1) * (nc - 1) ** i for i in range(d)))
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=((nf - 1) ** d, (nc - 1) ** d))
