"""Benchmark: vertex updates/s, solves/s to 1e-8 and p50/p99 solve latency.

One step = the whole hot path for one request of the 2D jumping-coefficient
workload (729^2 cells, random 9x9 checkerboard of {1, 1e4}): set_coefficients,
build_operators (BoxMG P, Galerkin R A P with the definiteness check,
hierarchical FP64 delta store, coarsest LU) and V(2,2) cycles to a relative
residual of 1e-8, all in the HIP library on one GPU.  Inputs are seeded and
synthetic (workloads.checkerboard2d) and resident in HBM (torch tensors) before the
timed region; set_coefficients checks and scatters them on the device.  The
same steps with host-resident inputs (PCIe hand-over) are reported beside.

Prints one JSON line.  The dominant kernel (the finest-level pre-smoothing
pass) is timed with per-dispatch HIP events on the grid's stream around every
k-th of its launches during the timed steps; its algorithmic bytes per launch
give the roofline figure.  Beside the main line: build_operators timed on its
own, the other single-grid workloads (2D Poisson at level 4 in FP64 to 1e-10,
the 3D four-ball adaptive grid in BF16/FP32 under FP64 correction), the same
step with the plain FP64 and BF16 stores, a roofline sweep on grids larger
than the Infinity Cache, the served request stream (mixed precision, and plain
FP64 for the ratio) and the CPU baseline, which times the oracle (test
infrastructure) on one solve of the main workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "vertex updates/s + solves/s to 1e-8 rel residual; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0

# HBM traffic per launch of the timed kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated), keyed by
# (store, dim, level); the kernel summary under profiles/ gives the commands.
# An entry is removed whenever that kernel changes.
MEASURED_TRAFFIC = {("hier64", 2, 6): 6734.4 * 2.0 * 1024 + 8326.5 * 1.0 * 1024}

# Algorithmic bytes per finest vertex of one Jacobi sweep or one residual, each
# streamed on its own: eps, u, b read and u' (or r) written once, stencils
# rebuilt on the fly; the plain store reads its 3^d FP64 entries instead of eps.
OP_BYTES = {("hier64", 2): 32, ("plain64", 2): 96, ("hier32", 2): 16, ("hier16", 2): 16, ("bf16", 2): 16,
            ("hier64", 3): 32, ("plain64", 3): 240, ("hier32", 3): 16, ("hier16", 3): 16, ("bf16", 3): 16}
# The timed kernel: in 2D the finest-level pre-smoothing pass, which applies two
# Jacobi sweeps and the residual in one launch (k_pass2d): 3 operations per
# vertex; in 3D one Jacobi sweep (k_stencil).  Bytes the fused pass itself has
# to move (eps, u, b read; u'' and r written):
TIMED_OPS = {2: 3, 3: 1}
FUSED_MIN_BYTES = {("hier64", 2): 40, ("plain64", 2): 104, ("hier32", 2): 20, ("hier16", 2): 20, ("bf16", 2): 20}
TIMED_KERNEL = {2: "finest-level pre-smoothing pass: 2 Jacobi sweeps + residual in one launch (k_pass2d)",
                3: "finest-level Jacobi sweep (k_stencil mode 0)"}


def run_variant(qmg, problem, transfer, store, steps, warmup, tol=1e-8, profile=0, host_inputs=False,
                graphs=False, **opts_kw):
    import torch
    # one grid on its own stream: eager launches keep ahead of the device
    opts = qmg.make_opts(transfer, store, graphs=graphs, **opts_kw)
    g = qmg.Grid(problem.dim, problem.level, opts)
    if host_inputs:
        eps, f = problem.eps, problem.f
    else:   # inputs resident in HBM before the timed region
        eps = torch.from_numpy(np.ascontiguousarray(problem.eps).ravel()).cuda()
        f = torch.from_numpy(np.ascontiguousarray(problem.f).ravel()).cuda()
    if profile:
        g.profile(profile)
    lat = []
    updates = 0
    reps = []
    for it in range(warmup + steps):
        if it == warmup:
            torch.cuda.synchronize()
            if profile:
                g.profile_read()     # count the timed steps only
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        g.set_coefficients(eps, f)
        g.build()
        rep, _ = g.solve(tol, 2000)
        t1 = time.perf_counter()
        if rep["status"] != "QMG_OK":
            raise RuntimeError(f"solve did not converge: {rep}")
        if it >= warmup:
            lat.append(t1 - t0)
            updates += rep["vertex_updates"]
            reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    launches, ms = g.profile_read() if profile else (0, 0.0)
    u = g.solution()
    g.close()
    return {"elapsed": elapsed, "lat": lat, "updates": updates, "reps": reps,
            "kernel_launches": launches, "kernel_ms": ms, "u": u}


def time_solves(g, eps, f, tol, n, warmup=1, time_cap=20.0, v=None):
    """Repeated full solves (set_coefficients + build_operators + solve) of one
    grid: up to n timed solves, fewer if they exceed time_cap seconds.  ``v``:
    host velocities of a convection problem (handed over with eps)."""
    import torch
    lat, reps = [], []
    for it in range(warmup + n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if v is None:
            g.set_coefficients(eps, f)
        else:
            g.set_coefficients(eps, f, v=v)
        g.build()
        rep, _ = g.solve(tol, 2000)
        t1 = time.perf_counter()
        if rep["status"] != "QMG_OK":
            raise RuntimeError(f"solve did not converge: {rep}")
        if it >= warmup:
            lat.append(t1 - t0)
            reps.append(rep)
            if sum(lat) > time_cap:
                break
    lat = np.array(lat)
    return {"solves": len(lat), "solves_per_s": len(lat) / lat.sum(),
            "vertex_updates_per_s": sum(r["vertex_updates"] for r in reps) / lat.sum(),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "cycles_per_solve": reps[-1]["cycles"], "outer_iters": reps[-1].get("outer_iters"),
            "relres": reps[-1]["relres"]}


def time_build(g, eps, f, n=20):
    """build_operators on its own (after set_coefficients), synchronised."""
    import torch
    t = []
    for it in range(n + 1):
        g.set_coefficients(eps, f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.build()
        torch.cuda.synchronize()
        if it:
            t.append(time.perf_counter() - t0)
    return float(np.percentile(np.array(t), 50) * 1e3)


def other_workloads(qmg, n):
    """The 2D Poisson workload (level 4, FP64 plain store, geometric transfer,
    to 1e-10), the 2D sine workload under additive and BPX cycles, and the
    3D four-ball adaptive workload (base level 3, level 5,
    BoxMG + Galerkin, BF16 deltas and FP32 inner cycles under FP64 composite
    defect correction, to 1e-8), inputs generated at the library's own
    unknown and cell coordinates."""
    import torch
    import workloads as W
    out = {}
    p = W.poisson2d_l4(0)
    g = qmg.Grid(p.dim, p.level, qmg.make_opts("geometric", "plain64"))
    eps = torch.from_numpy(np.ascontiguousarray(p.eps).ravel()).cuda()
    f = torch.from_numpy(np.ascontiguousarray(p.f).ravel()).cuda()
    r = time_solves(g, eps, f, 1e-10, n, warmup=3)
    out["poisson2d_L4"] = dict(r, unknowns=p.n_unknowns, u=g.solution(),
                               workload="2D Poisson, 81^2 cells (80^2 unknowns), eps = 1, f~U[-1,1]; "
                                        "geometric V(2,2), omega 0.6, plain FP64 store, to 1e-10")
    g.close()
    p = W.sin_source(2, 6)
    g = qmg.Grid(p.dim, p.level, qmg.make_opts("geometric", "hier64", omega=0.8, cycle="add"))
    eps = torch.from_numpy(np.ascontiguousarray(p.eps).ravel()).cuda()
    f = torch.from_numpy(np.ascontiguousarray(p.f).ravel()).cuda()
    r = time_solves(g, eps, f, 1e-8, max(5, n // 5), warmup=1)
    out["additive2d_sin_L6"] = dict(r, unknowns=p.n_unknowns,
                                    workload="2D sine source (exact solution prod sin(pi x_i)), 729^2 cells; "
                                             "additive cycles with exponential damping, omega 0.8, "
                                             "geometric transfer, to 1e-8")
    g.close()
    g = qmg.Grid(p.dim, p.level, qmg.make_opts("geometric", "hier64", omega=0.8, cycle="bpx",
                                               damping="const"))
    r = time_solves(g, eps, f, 1e-8, max(5, n // 5), warmup=1)
    out["bpx2d_sin_L6"] = dict(r, unknowns=p.n_unknowns,
                               workload="2D sine source, 729^2 cells; BPX cycles, omega 0.8 on every "
                                        "level, geometric transfer, to 1e-8")
    g.close()
    # (injection, the other Petrov-Galerkin variant, needs about 2000 cycles here)
    p = W.circle(2, 6, 0.1, seed=5)
    for restriction, key, rname in (("transpose", "circle2d_L6_eps0.1", "R = P^T"),
                                    ("aggregation", "circle2d_L6_eps0.1_aggregation", "aggregation R")):
        g = qmg.Grid(p.dim, p.level, qmg.make_opts("boxmg", "plain64", restriction=restriction))
        r = time_solves(g, p.eps, p.f, 1e-8, max(5, n // 5), warmup=1, v=p.meta["v"])
        out[key] = dict(
            r, unknowns=p.n_unknowns,
            workload=f"2D convection-diffusion, recirculating flow, eps 0.1, 729^2 cells; BoxMG, {rname}, "
                     "plain FP64 store, to 1e-8 (eps, v and f handed over from host memory)")
        g.close()
    P = W.adaptive_balls()
    g = qmg.Grid(P.dim, P.level, qmg.make_opts("boxmg", "bf16", check_definite=False),
                 base_level=P.base, refine=P.flags)
    xyz, lev = g.unknown_coords()
    fa = np.empty(len(xyz))
    for l in range(P.base, P.level + 1):
        m = lev == l
        fa[m] = P.f_at(l, xyz[m])
    epsa = P.eps_at(g.cell_centres())
    epsa = torch.from_numpy(epsa).cuda()
    fa = torch.from_numpy(fa).cuda()
    r = time_solves(g, epsa, fa, 1e-8, n, warmup=1)
    out["adaptive3d_balls"] = dict(r, unknowns=g.n_unknowns, leaf_cells=g.n_cells,
                                   build_ms=time_build(g, epsa, fa, 5),
                                   workload="3D adaptive: level 3 everywhere, level 5 within 0.2 of 4 "
                                            "seeded points; eps = exp(g), g a unit-variance Gaussian "
                                            "field (correlation length 0.1); BoxMG + Galerkin, BF16 "
                                            "deltas, FP32 inner FAS cycles, FP64 composite defect "
                                            "correction to 1e-8")
    g.close()
    return out


def serve_stream(qmg, n_requests=256, seed=0, slots=16, budget=8 << 30):
    """Served stream of mixed 2D/3D checkerboard solves (FP16 deltas, FP32
    cycles under FP64 refinement to 1e-8): first closed loop (all requests at
    t = 0) for the saturated throughput, then Poisson arrivals at 0.9 of it."""
    import workloads as W
    mixed = qmg.make_opts("boxmg", "hier16")
    stream = W.request_stream(seed=seed, n_requests=n_requests)
    out = {"requests": n_requests, "store": "hier16", "slots": slots, "hbm_budget_bytes": budget}

    def run(arrivals, opts):
        srv = qmg.Server(budget, max_slots=slots)
        t0 = time.perf_counter()
        tickets = []
        for req, ta in zip(stream, arrivals):
            wait = ta - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            p = req.problem
            tickets.append(srv.submit(p.dim, p.level, p.eps, p.f, opts, 1e-8))
        srv.drain()
        wall = time.perf_counter() - t0
        lat, upd, bad = [], 0, 0
        for t in tickets:
            done, status, u, rep, l = srv.poll(t)
            bad += status != "QMG_OK"
            lat.append(l)
            upd += rep["vertex_updates"]
        st = srv.stats()
        srv.close()
        lat = np.array(lat)
        return {"wall_s": wall, "solves_per_s": len(tickets) / wall, "vertex_updates_per_s": upd / wall,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "failed": int(bad), "hbm_peak_bytes": int(st["hbm_peak"])}

    closed = run([0.0] * n_requests, mixed)
    rate = 0.9 * closed["solves_per_s"]
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    opened = run(list(arrivals), mixed)
    out["closed_loop"] = closed
    out["poisson_0.9"] = dict(opened, rate_per_s=rate)
    # the same stream served in plain FP64 (full stencils, FP64 cycles) to the
    # same tolerance, for the mixed-precision ratio
    plain = run([0.0] * n_requests, qmg.make_opts("boxmg", "plain64"))
    out["plain64_closed_loop"] = plain
    out["mixed_over_plain64"] = closed["solves_per_s"] / plain["solves_per_s"]
    return out


def cpu_baseline(problem):
    """The oracle (plain FP64 numpy/scipy) on one full solve of the workload."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        H = O.build_hierarchy(problem.eps, problem.dim, problem.level, transfer="boxmg")
        b = O.rhs_from_f(problem.f, problem.dim, problem.level)
        u, hist = O.solve(H, b, tol=1e-8, max_cycles=2000)
        dt = time.perf_counter() - t0
    per_cycle = sum(4 * (3 ** l - 1) ** problem.dim for l in range(H.lc + 1, problem.level + 1))
    upd = per_cycle * len(hist)
    return {"value": upd / dt, "unit": "vertex updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve (build + {len(hist)} V(2,2) cycles to 1e-8) of the benchmark "
                      f"workload, single thread, {dt:.1f} s; solves/s {1.0 / dt:.4f}",
            "solves_per_s": 1.0 / dt, "u": u}


def cpu_solution_poisson():
    """The oracle's solution of the 2D Poisson workload (level 4, geometric
    V(2,2) cycles to 1e-10)."""
    import oracle as O
    import workloads as W
    p = W.poisson2d_l4(0)
    H = O.build_hierarchy(p.eps, p.dim, p.level, transfer="geometric")
    u, _ = O.solve(H, O.rhs_from_f(p.f, p.dim, p.level), tol=1e-10, max_cycles=500)
    return u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=6)
    ap.add_argument("--store", default="hier64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time every k-th launch of the timed kernel with HIP events (0: none)")
    ap.add_argument("--sweep", default="2:8",
                    help="roofline sweep on larger regular grids, dim:level comma list ('' for none): "
                         "the same step for the hier64, plain64 and bf16 stores")
    ap.add_argument("--variants", default="plain64,bf16,bpa",
                    help="extra stores timed on the same workload (comma list, '' for none)")
    ap.add_argument("--others", type=int, default=50, metavar="N",
                    help="repeated solves of the 2D Poisson and 3D adaptive workloads (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver path is "
              f"single-GPU", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1607_00648_amd import qmg
    import workloads as W
    torch.cuda.set_device(0)
    qmg.load()
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {args.calibrate_copy} MiB read + written", file=sys.stderr)
        del src, dst
    p = W.checkerboard2d(0, level=args.level)
    # timed pass: every PROFILE_EVERY-th finest-level sweep carries per-dispatch
    # HIP events on the grid's stream
    res = run_variant(qmg, p, "boxmg", args.store, args.steps, args.warmup,
                      profile=args.profile_every)
    lat = np.array(res["lat"])
    vu = res["updates"] / res["elapsed"]
    n_int = p.n_unknowns
    bytes_per_launch = OP_BYTES[(args.store, p.dim)] * TIMED_OPS[p.dim] * n_int
    fused_bytes = FUSED_MIN_BYTES.get((args.store, p.dim), OP_BYTES[(args.store, p.dim)]) * n_int
    avg_s = res["kernel_ms"] / max(res["kernel_launches"], 1) / 1e3
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else None
    out = {
        "metric": METRIC,
        "value": vu,
        "unit": "vertex updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.store in ("hier64", "plain64") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"2D -div(eps grad u)=f, {p.n}^2 cells ({p.n - 1}^2 unknowns), "
                               f"eps random 9x9 checkerboard {{1,1e4}} (seed 0), f~U[-1,1]; "
                               f"BoxMG + Galerkin RAP, store {args.store}, V(2,2), omega 0.6, "
                               f"exact coarsest solve, to 1e-8 relative residual",
                   "step": "set_coefficients (inputs in HBM) + build_operators + solve",
                   "level": p.level, "unknowns": n_int},
        "solves_per_s": args.steps / res["elapsed"],
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "cycles_per_solve": res["reps"][-1]["cycles"],
        "relres": res["reps"][-1]["relres"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": MEASURED_TRAFFIC.get((args.store, p.dim, p.level)),
                     "kernel": TIMED_KERNEL[p.dim],
                     "bytes_per_launch": bytes_per_launch,
                     "bytes_per_launch_note": "per-operation figures (each sweep and the residual "
                                              "streamed on its own) x operations in the launch",
                     "fused_bytes_per_launch": fused_bytes,
                     "fused_gbs": fused_bytes / avg_s / 1e9 if avg_s > 0 else None,
                     "avg_launch_us": avg_s * 1e6, "timed_launches": res["kernel_launches"],
                     "timing": f"per-dispatch HIP events (hipExtLaunchKernelGGL) on the grid stream "
                               f"around every {args.profile_every}-th such launch of the timed steps"},
    }
    gb = qmg.Grid(p.dim, p.level, qmg.make_opts("boxmg", args.store))
    out["build_ms"] = time_build(gb, p.eps, p.f)
    out["build_note"] = "build_operators alone (BoxMG P, Galerkin RAP, delta store, coarsest inverse), p50"
    gb.close()
    hp = run_variant(qmg, p, "boxmg", args.store, max(3, args.steps // 2), 1, host_inputs=True)
    out["host_inputs"] = {"solves_per_s": len(hp["lat"]) / hp["elapsed"],
                          "p50_ms": float(np.percentile(hp["lat"], 50) * 1e3),
                          "note": "same step with eps and f handed over from host memory"}
    variants = {}
    for v in [s for s in args.variants.split(",") if s]:
        r = run_variant(qmg, p, "boxmg", v, max(3, args.steps // 2), 1)
        variants[v] = {"solves_per_s": len(r["lat"]) / r["elapsed"],
                       "vertex_updates_per_s": r["updates"] / r["elapsed"],
                       "cycles_per_solve": r["reps"][-1]["cycles"],
                       "relres": r["reps"][-1]["relres"],
                       "p50_ms": float(np.percentile(r["lat"], 50) * 1e3)}
    if args.variants:
        # the paper's block Jacobi smoother (3 Gauss-Seidel sweeps per patch)
        r = run_variant(qmg, p, "boxmg", args.store, max(3, args.steps // 2), 1, smoother="block", bj_sweeps=3)
        variants[f"{args.store}_block_jacobi3"] = {
            "solves_per_s": len(r["lat"]) / r["elapsed"],
            "vertex_updates_per_s": r["updates"] / r["elapsed"],
            "cycles_per_solve": r["reps"][-1]["cycles"], "relres": r["reps"][-1]["relres"],
            "p50_ms": float(np.percentile(r["lat"], 50) * 1e3)}
    if variants:
        out["variants"] = variants
    sweep = []
    for item in [s for s in args.sweep.split(",") if s]:
        dim, level = (int(x) for x in item.split(":"))
        q = W.random_checkerboard(dim, level, 0, name=f"jump{dim}d-L{level}")
        for store in ("hier64", "plain64", "bf16"):
            r = run_variant(qmg, q, "boxmg", store, 2, 1, profile=args.profile_every or 8)
            avg = r["kernel_ms"] / max(r["kernel_launches"], 1) / 1e3
            op_b = OP_BYTES[(store, dim)] * TIMED_OPS[dim] * q.n_unknowns
            fz_b = FUSED_MIN_BYTES.get((store, dim), OP_BYTES[(store, dim)]) * q.n_unknowns
            sweep.append({"dim": dim, "level": level, "unknowns": q.n_unknowns, "store": store,
                          "solves_per_s": len(r["lat"]) / r["elapsed"],
                          "vertex_updates_per_s": r["updates"] / r["elapsed"],
                          "cycles_per_solve": r["reps"][-1]["cycles"], "relres": r["reps"][-1]["relres"],
                          "kernel": TIMED_KERNEL[dim], "avg_launch_us": avg * 1e6,
                          # per-operation bytes (each sweep and the residual streamed on
                          # its own; above peak when fusion saves re-reads, as for the
                          # plain store's stencils) and the bytes the fused pass moves
                          "effective_gbs": op_b / avg / 1e9 if avg > 0 else None,
                          "effective_frac": op_b / avg / 1e9 / HBM_PEAK_GBS if avg > 0 else None,
                          "fused_bytes_per_launch": fz_b,
                          "fused_gbs": fz_b / avg / 1e9 if avg > 0 else None,
                          "fused_frac": fz_b / avg / 1e9 / HBM_PEAK_GBS if avg > 0 else None})
            print(f"sweep {dim}D L{level} {store}: {sweep[-1]['solves_per_s']:.2f} solves/s, "
                  f"{sweep[-1]['avg_launch_us']:.1f} us/launch", file=sys.stderr, flush=True)
        del q
    if sweep:
        out["roofline_sweep"] = sweep
    if args.others:
        out["other_workloads"] = other_workloads(qmg, args.others)
    if not args.no_serving:
        out["serving"] = serve_stream(qmg)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(p)
        ucpu = cb.pop("u")
        out["cpu_baseline"] = cb
        out["u_rel_diff_vs_oracle"] = float(np.linalg.norm(res["u"] - ucpu) / np.linalg.norm(ucpu))
    if args.others:
        ow = out["other_workloads"]["poisson2d_L4"]
        u1 = ow.pop("u")
        if not args.no_cpu_baseline:
            ucpu = cpu_solution_poisson()
            ow["u_rel_diff_vs_oracle"] = float(np.linalg.norm(u1 - ucpu) / np.linalg.norm(ucpu))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
