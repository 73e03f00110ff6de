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


def sampled_local_rows(P, xyz, lev, u, n_samples, seed):
    """The oracle's composite residual rows at sampled unknowns of a grid too
    large to lay out, from the library's unknown positions (xyz, level) and
    an FP64 solution u: rows assembled one by one from the spacetree decided
    cell by cell (rows that need a hanging value are NaN).  Returns (sample
    indices, rows, row scales)."""
    from oracle import adaptive as AD
    lev = np.asarray(lev, dtype=np.int64)
    ijk = np.rint(xyz * (3.0 ** lev)[:, None]).astype(np.int64)
    key = (lev << 40) | (ijk[:, 0] + 1024 * (ijk[:, 1] + 1024 * ijk[:, 2]))
    order = np.argsort(key)
    skey = key[order]

    def u_of(l, w):
        k = (l << 40) | (w[0] + 1024 * (w[1] + 1024 * w[2]))
        j = np.searchsorted(skey, k)
        assert j < len(skey) and skey[j] == k, f"no unknown at level {l} position {w}"
        return u[order[j]]

    rng = np.random.default_rng(seed)
    pick = rng.choice(len(lev), n_samples, replace=False)
    T = AD.LocalSpacetree(3, P.base, P.level, P.mark)
    samples = [(int(lev[k]), tuple(int(x) for x in ijk[k])) for k in pick]
    rows, scale = AD.local_composite_rows(T, P.eps_at, P.f_at, u_of, samples)
    return pick, rows, scale


def band_inputs_on_device(g, P):
    """eps of the band workload (1e6 inside the seeded cubes, 1 outside) at the
    library's leaf-cell centres, evaluated on the device with the generator's
    comparisons, and f at the library's unknowns (host, counter-based)."""
    import torch
    xc = torch.from_numpy(g.cell_centres()).cuda()
    c = torch.from_numpy(P.meta["centres"]).cuda()
    sd = torch.from_numpy(P.meta["sides"]).cuda()
    inside = torch.zeros(len(xc), dtype=torch.bool, device="cuda")
    for i in range(len(c)):
        inside |= torch.all(torch.abs(xc - c[i]) <= sd[i] / 2, dim=1)
    one = torch.ones((), dtype=torch.float64, device="cuda")
    eps = torch.where(inside, 1e6 * one, one).contiguous()
    xyz, lev = g.unknown_coords()
    f = np.empty(len(lev))
    for l in range(P.base, P.level + 1):
        m = lev == l
        f[m] = P.f_at(l, xyz[m])
    return eps, torch.from_numpy(f).cuda(), xyz, lev
