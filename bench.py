#!/usr/bin/env python3
"""Benchmark of the sparse grid characteristics method's hot path on one GPU.

One step = the whole hot path on one batch of synthetic input: solve the
characteristic BVP at every node of the level-4 Smolyak CGL grid of the 6-D
rigid-body attitude problem (1457 nodes, 256 trapezoidal intervals, Newton
to max|F| <= 1e-10), build the hierarchical-surplus interpolant of u(0), and
evaluate the feedback at 1e6 seeded uniform states.  Inputs are resident in
HBM before the timed region; W untimed warm-up steps, then exactly K timed
steps bracketed by synchronisation.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload full|small]
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

METRIC = "converged 6-D BVPs/s at tol 1e-10 + feedback evals/s; p50/p99 latency"
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector (and matrix) peak
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak

# Algorithmic FP64 work of the Newton solve (the counts are derived in the
# design notes):
#   per interval and linear solve: assembly of the 12 x 12 system and its
#   7 right-hand sides (S P_k, A_k^T P_k, S c_k, A_k^T c_k and the block sums:
#   1098), the solve itself counted as LU plus substitution (2/3 n^3 + 2 n^2 k
#   = 1152 + 2016 for n = 12, k = 7) and the forward pass with the update (156);
#   per mesh point and evaluation: Phi, A = df/dx and W (172) and the interval
#   residual (48).  Transcendentals (two sincos per point) are not counted.
#   The first (linearised) Newton step is formed from a solve plan, so a BVP
#   that takes iters Newton iterations does iters linear solves and iters + 1
#   evaluations (newton_flops_plan).
FLOPS_ASSEMBLY = 1098
FLOPS_PER_INTERVAL_SOLVE = FLOPS_ASSEMBLY + 1152 + 2016 + 156
FLOPS_PER_POINT_EVAL = 172 + 48


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_newton_full_L4_N256_counters.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1507_04769_amd", "csrc", "bvp.hip")


def measured_traffic() -> float | None:
    """HBM bytes per k_newton launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel source has changed since the counters
    were taken (the summary records the sha256 of the profiled source)."""
    import hashlib
    import re
    try:
        text = open(COUNTERS_FILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    h = re.search(r"sha256: ([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", text)
    if not h or not t or h.group(1) != src:
        return None
    return float(t.group(1))


# the first Newton step formed from a solve plan: a combination of six
# trajectories per mesh point and unknown (12 x 6 multiply-adds)
FLOPS_PER_POINT_PLAN_STEP = 12 * 6 * 2


def newton_flops_plan(N, iters: np.ndarray) -> float:
    """Flops of the same solves with a plan: the first step is formed from the
    plan (FLOPS_PER_POINT_PLAN_STEP per point) instead of solved, so there
    remain iters linear solves and (iters + 1) evaluations per BVP."""
    it = iters.astype(np.float64)
    N = np.asarray(N, dtype=np.float64) + 0 * it
    return float(np.sum(it * N * FLOPS_PER_INTERVAL_SOLVE + (it + 1) * (N + 1) * FLOPS_PER_POINT_EVAL
                        + (N + 1) * FLOPS_PER_POINT_PLAN_STEP))


def alu_roofline(kernel: str, flops: float, ms: float, peak: float) -> dict:
    achieved = flops / (ms / 1e3) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "algorithmic_flops_per_launch": flops}


def eval_flops_per_query(grid_keys: np.ndarray, level: int, m: int) -> float:
    """Algorithmic flops of one feedback evaluation: one FMA per node and
    output (2 m M), the partial products of the node trie, and the 1-D basis
    tables (prefix/suffix products, 3 flops per point of each X^i, plus one
    scale per new point) in every dimension."""
    M, d = grid_keys.shape
    prefixes = 0
    for k in range(1, d - 1):
        prefixes += len({tuple(r) for r in grid_keys[:, :k]})
    inner = len({tuple(r) for r in grid_keys[:, : d - 1]})
    basis = 0
    for i in range(2, level + 2):
        n = 2 ** (i - 1) + 1
        basis += 3 * n + 2 * (n // 2 if i > 2 else 2)
    return 2.0 * m * M + prefixes + 2.0 * m * inner + d * basis


def cpu_baseline(args, nodes: np.ndarray, xq: np.ndarray) -> dict:
    """The FP64 CPU oracle as it stands, on the host cores, on a bounded
    sample of the same workload: all BVPs of the grid, and a slice of the
    queries."""
    from oracle import oracle as O
    from paper_1507_04769_amd import workloads as W
    wl = W.FULL if args.workload == "full" else W.SMALL
    threads = O.default_threads()
    op = O.Problem(N=wl.n_intervals, T=wl.horizon)
    t0 = time.perf_counter()
    r = O.solve_bvps(op, nodes, nthreads=threads)
    t_solve = time.perf_counter() - t0
    conv = int(np.sum(r.status == O.CONVERGED))
    nq = min(len(xq), args.cpu_queries)
    w = O.build_surplus(6, wl.level, r.u0, nthreads=threads)
    t0 = time.perf_counter()
    O.eval_hier(6, wl.level, w, xq[:nq], W.BOX_LO, W.BOX_HI, nthreads=threads)
    t_eval = time.perf_counter() - t0
    return {"value": conv / t_solve, "unit": "BVPs/s", "cores": threads, "kind": "oracle",
            "sample": "all %d BVPs of the grid (N=%d) and %d of the %d queries" % (len(nodes), wl.n_intervals,
                                                                                nq, len(xq)),
            "feedback_evals_per_s": nq / t_eval, "solve_s": t_solve, "eval_s": t_eval}


def batched_leg(dev, reps: int) -> dict:
    """The mixed batch (3072 level-5 nodes + 1024 uniform states, N in
    {64..512}, T in {10, 20, 40}): one persistent launch with the autotuned
    schedule, captured in a HIP graph and replayed, against the same inputs
    solved unbatched (one launch per (N, T) group)."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import autotune as A
    order, slots, src = A.tuned_schedule()
    problem = A.batch_problem()
    x0h, N, T = A.batch_inputs()
    x0 = torch.tensor(x0h, device=dev)
    b = S.Batch(problem, N, T, order=order, slots_per_cu=slots)
    ws = S.batch_workspace(b, dev)
    n = b.n
    lam = torch.empty((n, 6), dtype=torch.float64, device=dev)
    u0 = torch.empty((n, b.m), dtype=torch.float64, device=dev)
    V = torch.empty((n,), dtype=torch.float64, device=dev)
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    it = torch.empty((n,), dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        S.sgcm_solve_bvps_batch(b, x0, lam, u0, V, st, it, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        S.sgcm_solve_bvps_batch(b, x0, lam, u0, V, st, it, ws)
    ms = A.time_ms(graph.replay, reps)
    converged = int((st == S.CONVERGED).sum().item())
    run, ngroups = A.unbatched_runner(problem, x0, N, T)
    ums = A.time_ms(run, reps)
    bms, ubms = float(np.median(ms)), float(np.median(ums))
    flops = newton_flops_plan(N, it.cpu().numpy())  # first steps from the batch's per-(N, T) steps
    return {"workload": "mixed batch: " + A.W.BATCH.name, "n_bvps": n, "converged": converged,
            "roofline": alu_roofline("k_newton_batch_grid<double>" if slots == 0 else "k_newton_batch<double>",
                                     flops, bms, PEAK_FP64_TFLOPS),
            "schedule": {"order": "larger N*T first" if order == S.ORDER_LONGEST_FIRST else "as given",
                         "slots_per_cu": slots, "source": os.path.relpath(src, ROOT) if src else "default"},
            "graph": True, "ms": bms, "bvps_per_s": converged / (bms / 1e3),
            "unbatched": {"launches": ngroups, "ms": ubms, "bvps_per_s": converged / (ubms / 1e3)},
            "speedup_vs_unbatched": ubms / bms}


def precision_leg(dev, prob, grid, x0, lam64, u064, it64, surplus, eval_flops_q: float, reps: int) -> dict:
    """FP32 variants beside the FP64 path on the same MI355X: the FP32 inexact
    Newton solve of the full workload with its plan, against the FP64 solve
    with its plan (errors against the FP64 GPU solve, which matches the oracle
    to ~1e-13) and FP32 feedback evaluation at 1e7 uniform
    states (errors against the FP64 GPU evaluation of the same interpolant)."""
    import dataclasses
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import autotune as A
    from paper_1507_04769_amd import workloads as W
    p32 = dataclasses.replace(prob, precision=S.FP32)
    M = x0.shape[0]
    lam = torch.empty_like(lam64)
    u0 = torch.empty_like(u064)
    V = torch.empty((M,), dtype=torch.float64, device=dev)
    st = torch.empty((M,), dtype=torch.int32, device=dev)
    it = torch.empty((M,), dtype=torch.int32, device=dev)
    ws = torch.empty((S.sgcm_solve_bvps_workspace(p32, M) // 8 + 32,), dtype=torch.float64, device=dev)
    p64 = dataclasses.replace(prob, precision=S.FP64)
    ws64 = torch.empty((S.sgcm_solve_bvps_workspace(p64, M) // 8 + 32,), dtype=torch.float64, device=dev)
    lam2, u02, V2 = torch.empty_like(lam), torch.empty_like(u0), torch.empty_like(V)
    st2, it2 = torch.empty_like(st), torch.empty_like(it)
    plan32, plan64 = S.Plan(p32), S.Plan(p64)  # as in the timed step: first steps from the plans
    ms32 = A.time_ms(lambda: S.sgcm_solve_bvps_plan(plan32, x0, lam, u0, V, None, st, it, ws), reps)
    ms64 = A.time_ms(lambda: S.sgcm_solve_bvps_plan(plan64, x0, lam2, u02, V2, None, st2, it2, ws64), reps)
    conv = int((st == S.CONVERGED).sum().item())
    el = ((lam - lam64).abs().amax(dim=1) / lam64.abs().amax(dim=1).clamp_min(1e-8)).cpu().numpy()
    eu = ((u0 - u064).abs().amax(dim=1) / u064.abs().amax(dim=1).clamp_min(1e-8)).cpu().numpy()
    i32, i64 = it.cpu().numpy(), it64
    # the same algorithmic flops as the FP64 solve; the linear solve (95 % of
    # them) runs in FP32, so the fraction is given against both peaks
    f32 = newton_flops_plan(prob.N, i32)
    rf = alu_roofline("k_newton<float>", f32, float(np.median(ms32)), PEAK_FP32_TFLOPS)
    rf["frac_of_fp64_peak"] = rf["achieved"] / PEAK_FP64_TFLOPS
    solve = {"ms": float(np.median(ms32)), "fp64_ms": float(np.median(ms64)), "roofline": rf,
             "bvps_per_s": conv / (float(np.median(ms32)) / 1e3), "converged": conv,
             "mean_iters": float(i32.mean()), "fp64_mean_iters": float(i64.mean()),
             "lambda0_rel_err": {"max": float(el.max()), "rms": float(np.sqrt(np.mean(el ** 2)))},
             "u0_rel_err": {"max": float(eu.max()), "rms": float(np.sqrt(np.mean(eu ** 2)))}}
    nq = 10_000_000
    xq = torch.tensor(W.uniform_in_box(nq, seed=3), device=dev)
    xq32 = xq.float()
    w32 = surplus.float()
    uq = torch.empty((nq, surplus.shape[1]), dtype=torch.float64, device=dev)
    uq32 = torch.empty((nq, surplus.shape[1]), dtype=torch.float32, device=dev)
    e64 = A.time_ms(lambda: S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64), reps)
    e32 = A.time_ms(lambda: S.sgcm_eval_feedback_f32(grid, w32, xq32, uq32), reps)
    err = (uq32.double() - uq).abs()
    scale = float(uq.abs().max().item())
    ev = {"queries": nq, "ms": float(np.median(e32)), "fp64_ms": float(np.median(e64)),
          "evals_per_s": nq / (float(np.median(e32)) / 1e3), "fp64_evals_per_s": nq / (float(np.median(e64)) / 1e3),
          "abs_err": {"max": float(err.max().item()), "rms": float(err.pow(2).mean().sqrt().item())},
          "max_abs_u": scale,
          "roofline": alu_roofline("k_eval_fast<6, %d, 3, float>" % grid.level, eval_flops_q * nq,
                                   float(np.median(e32)), PEAK_FP32_TFLOPS),
          "fp64_roofline": alu_roofline("k_eval_fast<6, %d, 3, double>" % grid.level, eval_flops_q * nq,
                                        float(np.median(e64)), PEAK_FP64_TFLOPS)}
    return {"fp32_newton": solve, "fp32_eval": ev,
            "note": "errors against the FP64 GPU results, which match the FP64 oracle to ~1e-13"}


def validation_leg(dev, prob, grid, u0, V, surplus, n_nodes_intervals: int, reps: int) -> dict:
    """Monte Carlo total-error estimate of the interpolant (Sec. 4.3): 1280
    uniform states, reference from 2x and 4x the nodes' intervals (Richardson
    extrapolation), for the feedback u(0, x) (the step's interpolant) and the
    value V(0, x) (an interpolant of the node values of V)."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import autotune as A
    from paper_1507_04769_amd import validation as VA
    from paper_1507_04769_amd import workloads as W
    w_V = S.build_interpolant(grid, V.view(-1, 1).contiguous())
    xs = torch.tensor(W.uniform_in_box(VA.N_SAMPLES, seed=VA.SAMPLE_SEED), device=dev)
    n_ref = 2 * n_nodes_intervals
    est = VA.Estimator(prob, n_ref)
    r = est(grid, surplus, xs, w_V)
    ms = A.time_ms(lambda: est(grid, surplus, xs, w_V), reps)
    su, sV = r.stats_u.cpu().numpy(), r.stats_V.cpu().numpy()
    st = r.status.cpu().numpy()
    return {"samples": VA.N_SAMPLES, "seed": VA.SAMPLE_SEED, "node_intervals": n_nodes_intervals,
            "reference_intervals": [n_ref, 2 * n_ref],
            "reference_converged": [int(np.sum(st[0] == S.CONVERGED)), int(np.sum(st[1] == S.CONVERGED))],
            "u_error": {"max": float(su[0]), "rms": float(su[1]), "reference_correction_max": float(su[2])},
            "V_error": {"max": float(sV[0]), "rms": float(sV[1]), "reference_correction_max": float(sV[2])},
            "ms": float(np.median(ms)), "samples_per_s": VA.N_SAMPLES / (float(np.median(ms)) / 1e3)}


def serving_leg(n_requests: int, rate: float) -> dict:
    """The serving loop on a seeded Poisson stream of mixed requests: solves of
    1..512 states (meshes 64..512, three- or two-wheel model) and queries of
    1..1e5 states against resident level-3/4/5 interpolants (FP64 or FP32).
    Reported: p50/p99 latency (arrival to results on the host) and throughput
    at the given rate with continuous batching on four streams; the same stream
    served one request per launch on one stream; and the capacity with every
    request present at once."""
    from paper_1507_04769_amd import serving as SV
    interps = {lv: SV.build_interpolant(lv, N=256) for lv in (3, 4, 5)}
    warm = SV.request_stream(40, rate, seed=700, levels=(3, 4, 5))
    SV.Server(interps).run(warm, realtime=False)
    reqs = SV.request_stream(n_requests, rate, seed=701, levels=(3, 4, 5))
    # the solve plans of the stream's solve keys, made before it is served
    plans = {k: SV.solve_plan(k) for k in sorted({r.key() for r in reqs if r.key()[0] == "solve"})}
    out = {"requests": n_requests, "rate_per_s": rate, "seed": 701, "interpolant_levels": [3, 4, 5],
           "streams": 4, "hbm_budget_bytes": 8 << 30}
    out["continuous"] = SV.Server(interps, n_streams=4, hbm_budget=8 << 30, plans=plans).run(reqs, realtime=True)
    out["one_per_launch"] = SV.Server(interps, n_streams=1, merge=False, plans=plans).run(reqs, realtime=True)
    out["capacity_all_at_once"] = SV.Server(interps, n_streams=4, hbm_budget=8 << 30, plans=plans).run(reqs, realtime=False)["throughput"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["full", "small"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=20000)
    ap.add_argument("--no-batched", action="store_true", help="skip the mixed-batch leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32 leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-validation", action="store_true", help="skip the total-error estimate leg")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--no-plan-compare", action="store_true",
                    help="skip timing the solve without the plan (profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the per-node BVPs shard with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import workloads as W

    wl = W.FULL if args.workload == "full" else W.SMALL
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    prob = S.Problem(m=wl.m, J=W.J_DIAG, B=W.input_matrix(wl.m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W,
                     T=wl.horizon, N=wl.n_intervals, tol=W.TOL, max_iter=W.MAX_ITER)
    grid = S.Grid(6, wl.level, W.BOX_LO, W.BOX_HI)
    nodes = grid.nodes()
    M = len(grid)
    xq_host = W.query_points(wl)
    x0 = torch.tensor(nodes, device=dev)
    xq = torch.tensor(xq_host, device=dev)
    lam = torch.empty((M, 6), dtype=torch.float64, device=dev)
    u0 = torch.empty((M, wl.m), dtype=torch.float64, device=dev)
    V = torch.empty((M,), dtype=torch.float64, device=dev)
    traj = torch.empty((M, wl.n_intervals + 1, 12), dtype=torch.float64, device=dev)
    st = torch.empty((M,), dtype=torch.int32, device=dev)
    it = torch.empty((M,), dtype=torch.int32, device=dev)
    ws = torch.empty((S.sgcm_solve_bvps_workspace(prob, M) // 8 + 32,), dtype=torch.float64, device=dev)
    surplus = torch.empty((M, wl.m), dtype=torch.float64, device=dev)
    uq = torch.empty((len(xq_host), wl.m), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    # the problem's solve plan (first Newton steps of the six unit initial
    # states), made once like the grid, before the timed steps
    torch.cuda.synchronize()
    t_plan = time.perf_counter()
    plan = S.Plan(prob, stream)
    plan_ms = (time.perf_counter() - t_plan) * 1e3

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        S.sgcm_solve_bvps_plan(plan, x0, lam, u0, V, traj, st, it, ws, stream)
        if ev is not None:
            ev[1].record(stream)
        S.sgcm_build_interpolant(grid, u0, surplus, stream)
        if ev is not None:
            ev[2].record(stream)
        S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64, stream)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([e[0].elapsed_time(e[3]) for e in events])
    solve_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    build_ms = np.array([e[1].elapsed_time(e[2]) for e in events])
    eval_ms = np.array([e[2].elapsed_time(e[3]) for e in events])

    status = st.cpu().numpy()
    iters = it.cpu().numpy()
    converged = int(np.sum(status == S.CONVERGED))
    total_s = float(np.sum(step_ms)) / 1e3
    value = converged * args.steps / total_s
    flops = newton_flops_plan(wl.n_intervals, iters)
    achieved = flops / (float(np.mean(solve_ms)) / 1e3) / 1e12
    # the same solve without the plan (each BVP solving its first step), for
    # comparison, on outputs of its own
    from paper_1507_04769_amd import autotune as A
    compare = {}
    if not args.no_plan_compare:
        lam_n, u0_n, V_n, traj_n = (torch.empty_like(lam), torch.empty_like(u0), torch.empty_like(V),
                                    torch.empty_like(traj))
        st_n, it_n = torch.empty_like(st), torch.empty_like(it)
        noplan_ms = A.time_ms(lambda: S.sgcm_solve_bvps(prob, x0, lam_n, u0_n, V_n, traj_n, st_n, it_n, ws), 5)
        compare = {"solve_without_plan_ms": float(np.median(noplan_ms)),
                   "same_status_and_iters_without_plan": bool(torch.equal(st, st_n) and torch.equal(it, it_n)),
                   "lambda0_max_rel_diff_without_plan":
                       float(((lam - lam_n).abs().amax(dim=1) / lam_n.abs().amax(dim=1).clamp_min(1e-8)).max().item())}
        del lam_n, u0_n, V_n, traj_n, st_n, it_n
    eval_flops_q = eval_flops_per_query(grid.keys(), wl.level, wl.m)

    batched = None if args.no_batched or args.workload != "full" else batched_leg(dev, 5)
    precision = None
    if not args.no_precision and args.workload == "full":
        precision = precision_leg(dev, prob, grid, x0, lam, u0, iters, surplus, eval_flops_q, 5)
    validation = None
    if not args.no_validation and args.workload == "full":
        validation = validation_leg(dev, prob, grid, u0, V, surplus, wl.n_intervals, 3)
    serving = None
    if not args.no_serving and args.workload == "full":
        serving = serving_leg(args.serving_requests, args.serving_rate)

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "BVPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid_level": wl.level, "grid_nodes": M, "state_dim": 6,
                   "controls": wl.m, "intervals": wl.n_intervals, "horizon": wl.horizon, "tol": W.TOL,
                   "queries": len(xq_host), "query_seed": wl.query_seed},
        "feedback_evals_per_s": len(xq_host) / (float(np.mean(eval_ms)) / 1e3),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": {"solve_bvps": float(np.mean(solve_ms)), "build_interpolant": float(np.mean(build_ms)),
                      "eval_feedback": float(np.mean(eval_ms))},
        "solve_plan": dict({"create_ms": plan_ms,
                            "note": "first Newton step of each BVP formed from the problem's plan (made once, "
                                    "outside the timed steps, like the grid)"}, **compare),
        "converged": converged,
        "newton_iters_hist": np.bincount(iters).tolist(),
        "wall_s_timed": wall,
        "roofline": {"kernel": "k_newton (sgcm_solve_bvps_plan)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic() if wl.name == W.FULL.name else None,
                     "algorithmic_flops_per_launch": flops},
        "eval_roofline": alu_roofline("k_eval_fast<6, %d, %d, double>" % (wl.level, wl.m),
                                      eval_flops_q * len(xq_host), float(np.mean(eval_ms)), PEAK_FP64_TFLOPS),
    }
    if batched is not None:
        out["batched"] = batched
    if precision is not None:
        out["precision"] = precision
    if validation is not None:
        out["validation"] = validation
    if serving is not None:
        out["serving"] = serving
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, nodes, xq_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
