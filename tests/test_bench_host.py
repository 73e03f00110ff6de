"""Host logic of the benchmark's oracle checks (no GPU): the relative
residual it recomputes for regular-grid solutions, the sampled composite rows
of the four-ball workload and the served stream's per-request check, each on
solutions the oracle itself produced or on planted wrong ones."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from oracle import adaptive as AD  # noqa: E402


@pytest.mark.parametrize("d,L", [(2, 4), (3, 2)])
def test_oracle_relres_equals_the_assembled_residual(d, L):
    p = W.random_checkerboard(d, L, 0, values=(1.0, 1e4))
    H = O.build_hierarchy(p.eps, d, L, transfer="boxmg")
    b = O.rhs_from_f(p.f, d, L)
    u, hist = O.solve(H, b, tol=1e-8)
    rr, S = bench.oracle_relres(p, u)
    want = np.linalg.norm(b - H.A[L] @ u) / np.linalg.norm(b)
    assert abs(rr - want) <= 1e-12 * want and rr <= 1e-8
    # the stencil array is reused for a second solution of the same problem
    rr0, _ = bench.oracle_relres(p, np.zeros_like(u), S)
    assert rr0 == 1.0


def test_balls_rows_check_flags_a_perturbed_solution():
    P = W.adaptive_balls(dim=3, base=2, level=3, n_balls=1, radius=0.3)
    G = AD.AdaptiveGrid(P.dim, P.base, P.level, P.flags)
    xyz = G.unknown_coords()
    lev = np.concatenate([np.full(int((G.vtype[l] == AD.LEAF).sum()), l) for l in range(G.base, G.L + 1)])
    f = np.concatenate([P.f_at(l, xyz[lev == l]) for l in range(G.base, G.L + 1)])
    u, A, b = AD.solve_composite_direct(G, P.eps_at(G.cell_centres()), f)
    nb = np.linalg.norm(b)
    good = bench.balls_rows_check(P, xyz, lev, u, nb, n_samples=80)
    bad = bench.balls_rows_check(P, xyz, lev, u * 1.01, nb, n_samples=80)
    assert good["checked"] >= 20 and good["max_abs_row_over_norm_b"] < 1e-13
    assert bad["max_abs_row_over_norm_b"] > 1e-5


class _FakeServer:
    """Returns a fixed fraction of each request's direct solution, the same
    in every run, so the served-stream check sees known residuals."""
    scale = 1.0

    def __init__(self, budget, max_slots):
        self.out = []

    def submit(self, d, L, eps, f, opts, tol, t_arrival=0.0):
        A = O.stencil_to_csr(O.geometric_stencil(eps, d, L), d, L)
        self.out.append(self.scale * O.direct_solve(A, O.rhs_from_f(f, d, L)))
        return len(self.out) - 1

    def drain(self):
        pass

    def poll(self, t):
        return True, "QMG_OK", self.out[t], {"vertex_updates": 1}, 1e-3

    def stats(self):
        return {"hbm_peak": 0}

    def close(self):
        pass


class _FakeQmg:
    Server = _FakeServer

    @staticmethod
    def make_opts(*a, **k):
        return None


def test_served_stream_check_reports_the_worst_request(monkeypatch):
    import workloads
    small = workloads.request_stream(seed=0, n_requests=6, levels_2d=(2, 3), levels_3d=(1, 2))
    monkeypatch.setattr(workloads, "request_stream", lambda seed, n_requests: small)
    out = bench.serve_stream(_FakeQmg, n_requests=6, oracle_check=True)
    assert out["closed_loop"]["max_relres_by_oracle"] < 1e-13
    assert out["plain64_closed_loop"]["max_relres_by_oracle"] < 1e-13
    assert out["poisson_0.9"]["bitwise_equal_to_closed_loop"] is True
    monkeypatch.setattr(_FakeServer, "scale", 0.999)
    out = bench.serve_stream(_FakeQmg, n_requests=6, oracle_check=True)
    assert abs(out["closed_loop"]["max_relres_by_oracle"] - 1e-3) < 1e-9
