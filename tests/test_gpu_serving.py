"""Serving: each result is the same alone and in the mix; admission by HBM
budget queues requests; oversize requests are rejected without disturbing the
rest."""
import time

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _requests(n, seed=3, levels_2d=(3, 5), levels_3d=(2, 3)):
    reqs = W.request_stream(seed=seed, n_requests=n, levels_2d=levels_2d, levels_3d=levels_3d)
    return [r.problem for r in reqs]


def _alone(qmg, p, opts, tol):
    g = qmg.Grid(p.dim, p.level, opts)
    g.set_coefficients(p.eps, p.f)
    g.build()
    rep, _ = g.solve(tol, 1000)
    u = g.solution()
    g.close()
    return u, rep


@pytest.mark.parametrize("store,extra,shapes", [
    ("hier16", {}, "stream"), ("hier16", {}, "small"), ("hier64", {}, "small"), ("bpa", {}, "small"),
    ("hier64", {"smoother": "block", "bj_sweeps": 2}, "small")])
def test_results_identical_alone_and_in_mix(store, extra, shapes):
    """``stream``: the served stream's own level ranges (2D levels 3-6, 3D
    levels 2-4) and its store; ``small``: smaller grids for the other
    stores."""
    qmg = require_gpu()
    announce(f"serving mix {store} {extra} {shapes}")
    probs = _requests(12, seed=9, levels_2d=(3, 6), levels_3d=(2, 4)) if shapes == "stream" else _requests(12)
    if shapes == "stream":
        assert max(p.level for p in probs if p.dim == 2) == 6 and max(p.level for p in probs if p.dim == 3) == 4
    opts = qmg.make_opts("boxmg", store, **extra)
    alone = [_alone(qmg, p, opts, 1e-8) for p in probs]
    budget = 4 * max(qmg.workspace_bytes(p.dim, p.level, opts) for p in probs)
    srv = qmg.Server(budget, max_slots=6)
    tickets = [srv.submit(p.dim, p.level, p.eps, p.f, opts, 1e-8) for p in probs]
    srv.drain()
    for p, t, (ua, ra) in zip(probs, tickets, alone):
        done, status, u, rep, lat = srv.poll(t)
        assert done and status == "QMG_OK", (p.name, status)
        assert np.array_equal(u, ua), p.name          # bitwise: no cross-request arithmetic
        assert rep["cycles"] == ra["cycles"]
        assert lat > 0
        # the oracle's own FP64 residual of the served result
        A = O.stencil_to_csr(O.geometric_stencil(p.eps, p.dim, p.level), p.dim, p.level)
        b = O.rhs_from_f(p.f, p.dim, p.level)
        assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= 1e-8
    st = srv.stats()
    assert st["completed"] == len(probs) and st["failed"] == 0
    assert st["hbm_peak"] <= budget
    srv.close()


def test_admission_by_budget_queues_and_rejects_oversize():
    qmg = require_gpu()
    announce("serving admission")
    probs = _requests(8, seed=5)
    opts = qmg.make_opts("boxmg", "hier16")
    sizes = [qmg.workspace_bytes(p.dim, p.level, opts) for p in probs]
    budget = max(sizes)                      # at most one of the largest at a time
    srv = qmg.Server(budget, max_slots=8)
    big = W.poisson(2, 7, seed=1)            # needs more than the whole budget
    with pytest.raises(qmg.QmgError):
        srv.submit(big.dim, big.level, big.eps, big.f, opts, 1e-8)
    tickets = [srv.submit(p.dim, p.level, p.eps, p.f, opts, 1e-8) for p in probs]
    srv.drain()
    st = srv.stats()
    assert st["completed"] == len(probs) and st["failed"] == 0
    assert st["hbm_peak"] <= budget
    assert st["hbm_in_use"] == 0
    for t in tickets:
        done, status, u, rep, lat = srv.poll(t)
        assert done and status == "QMG_OK"
    # the requests could not all be resident at once, and some did wait
    assert sum(sizes) > budget
    assert st["deferred"] > 0
    srv.close()


def test_arrival_schedule_is_respected():
    """Requests handed over with future arrival times are not admitted before
    them; latency counts from arrival."""
    qmg = require_gpu()
    announce("serving arrival schedule")
    probs = _requests(6, seed=11)
    opts = qmg.make_opts("boxmg", "hier16")
    srv = qmg.Server(1 << 32, max_slots=4)
    gap = 0.05
    t0 = time.perf_counter()
    tickets = [srv.submit(p.dim, p.level, p.eps, p.f, opts, 1e-8, t_arrival=0.1 + gap * k)
               for k, p in enumerate(probs)]
    srv.drain()
    wall = time.perf_counter() - t0
    assert wall >= 0.1 + gap * (len(probs) - 1)
    for k, t in enumerate(tickets):
        done, status, u, rep, lat = srv.poll(t)
        assert done and status == "QMG_OK"
        assert 0 < lat < wall - (0.1 + gap * k) + 0.05
    assert srv.stats()["deferred"] == 0     # an idle server admits each at its arrival
    srv.close()


def test_destroy_with_requests_in_flight():
    qmg = require_gpu()
    announce("serving destroy in flight")
    probs = _requests(6, seed=7)
    opts = qmg.make_opts("boxmg", "hier16")
    srv = qmg.Server(1 << 34, max_slots=2)
    for p in probs:
        srv.submit(p.dim, p.level, p.eps, p.f, opts, 1e-8)
    time.sleep(0.01)
    srv.close()        # active requests finish, queued ones are dropped
