#!/usr/bin/env python3
"""Benchmark of the sparse grid characteristics method's hot path on one GPU.

One step = the whole hot path on one batch of synthetic input: solve the
characteristic BVP at every node of the level-4 Smolyak CGL grid of the 6-D
rigid-body attitude problem (1457 nodes, 256 trapezoidal intervals, Newton
from the linearised guess to max|F| <= 1e-10), build the hierarchical-surplus
interpolant of u(0), and evaluate the feedback at 1e6 seeded uniform states.
The headline step is one-shot (each BVP solves its own first Newton step);
the same step with a per-problem solve plan made once is reported beside it.
Inputs are resident in HBM before the timed region; W untimed warm-up steps,
then exactly K timed steps bracketed by synchronisation.  Prints one JSON
line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload full|small]
"""
from __future__ import annotations

import argparse
import dataclasses
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

# Algorithmic FP64 work of the Newton solve, the count the roofline uses:
# 6.5 kflop per mesh interval and Newton linear solve (the residual and
# Jacobian blocks of the interval, the structured elimination of its 12 x 12
# blocks and the back-substitution).  A BVP that takes iters counted
# iterations does iters + 1 linear solves (the first one from Y = 0), or iters
# with a solve plan (newton_flops).
FLOPS_PER_INTERVAL_STEP = 6500.0


def newton_flops(N, iters: np.ndarray, plan: bool = False) -> float:
    """6.5 kflop x N x the linear solves of every BVP of a launch."""
    it = iters.astype(np.float64) + (0.0 if plan else 1.0)
    N = np.asarray(N, dtype=np.float64) + 0 * it
    return float(FLOPS_PER_INTERVAL_STEP * np.sum(N * it))


# The library's own finer count, kept as a secondary figure:
#   per interval and linear solve: assembly of the 12 x 12 system and its
#   7 right-hand sides (S P_k, A_k^T P_k, S c_k, A_k^T c_k and the block sums:
#   1098), the solve itself counted as LU plus substitution (2/3 n^3 + 2 n^2 k
#   = 1152 + 2016 for n = 12, k = 7) and the forward pass with the update (156);
#   per mesh point and evaluation: Phi, A = df/dx and W (172) and the interval
#   residual (48).  Transcendentals (two sincos per point) are not counted.
#   With a solve plan a BVP that takes iters Newton iterations does iters
#   linear solves and iters + 1 evaluations (newton_flops_plan).
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
    """Algorithmic flops of one feedback evaluation, the count the roofline
    uses: one multiply-add per node and output (2 m M), one product per
    non-trivial dimension of each node beyond the first (sum over nodes of
    max(#{k: i_k > 1} - 1, 0)), and the 1-D basis tables, 5 flops per point of
    each X^i, i = 2..level + 1, in every dimension (12,242 at level 4, m = 3)."""
    M, d = grid_keys.shape
    nontrivial = np.count_nonzero(grid_keys, axis=1)
    basis = sum(5 * (2 ** (i - 1) + 1) for i in range(2, level + 2))
    return float(2 * m * M + np.sum(np.maximum(nontrivial - 1, 0)) + d * basis)


def eval_flops_per_query_walk(grid_keys: np.ndarray, level: int, m: int) -> float:
    """The evaluation kernel's own count (secondary): one FMA per node and
    output (2 m M), the partial products of the node trie, 2 m per inner trie
    node, and the 1-D basis tables (prefix/suffix products, 3 flops per point
    of each X^i, plus one scale per new point) in every dimension."""
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


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, nodes: np.ndarray, xq: np.ndarray) -> dict:
    """The FP64 CPU oracle as it stands, on a bounded sample of the same
    workload: on all host threads (median of 3 runs: every BVP of the grid,
    and a slice of the queries) and on one thread (median of 3 runs on a
    seeded sample of BVPs and queries)."""
    from oracle import oracle as O
    from paper_1507_04769_amd import workloads as W
    wl = W.FULL if args.workload == "full" else W.SMALL
    threads = O.default_threads()
    op = O.Problem(N=wl.n_intervals, T=wl.horizon, max_halvings=W.MAX_HALVINGS)

    def timed(fn):
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            r = fn()
            t.append(time.perf_counter() - t0)
        return float(np.median(t)), r

    t_solve, r = timed(lambda: O.solve_bvps(op, nodes, nthreads=threads))
    conv = int(np.sum(r.status == O.CONVERGED))
    nq = min(len(xq), args.cpu_queries)
    w = O.build_surplus(6, wl.level, r.u0, nthreads=threads)
    t_eval, _ = timed(lambda: O.eval_hier(6, wl.level, w, xq[:nq], W.BOX_LO, W.BOX_HI, nthreads=threads))
    pick = W.sample_indices(len(nodes), min(len(nodes), 100), seed=31)
    t1_solve, r1 = timed(lambda: O.solve_bvps(op, nodes[pick], nthreads=1))
    nq1 = min(nq, 2000)
    t1_eval, _ = timed(lambda: O.eval_hier(6, wl.level, w, xq[:nq1], W.BOX_LO, W.BOX_HI, nthreads=1))
    return {"value": conv / t_solve, "unit": "BVPs/s", "cores": threads, "kind": "oracle",
            "sample": "all %d BVPs of the grid (N=%d) and %d of the %d queries, median of 3 runs" % (
                len(nodes), wl.n_intervals, nq, len(xq)),
            "cpu_model": cpu_model(), "feedback_evals_per_s": nq / t_eval, "solve_s": t_solve, "eval_s": t_eval,
            "one_core": {"bvps_per_s": int(np.sum(r1.status == O.CONVERGED)) / t1_solve,
                         "feedback_evals_per_s": nq1 / t1_eval, "cores": 1,
                         "sample": "%d seeded BVPs of the grid and %d queries, median of 3 runs" % (len(pick), nq1)}}


def small_leg(dev, steps: int, warmup: int, with_cpu: bool) -> dict:
    """The small workload (level-2 grid, 85 BVPs, N = 64, 1e3 queries): the
    same one-shot step on the GPU, and the oracle on all of it (all host
    threads and one thread, median of 3 runs)."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import workloads as W
    wl = W.SMALL
    prob = S.Problem(m=wl.m, J=W.J_DIAG, B=W.input_matrix(wl.m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W,
                     T=wl.horizon, N=wl.n_intervals, tol=W.TOL, max_iter=W.MAX_ITER, max_halvings=W.MAX_HALVINGS)
    grid = S.Grid(6, wl.level, W.BOX_LO, W.BOX_HI)
    nodes = grid.nodes()
    M = len(grid)
    xq_host = W.query_points(wl)
    x0, xq = torch.tensor(nodes, device=dev), torch.tensor(xq_host, device=dev)
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
    grid.upload(stream)

    def step(ev):
        if ev is not None:
            ev[0].record(stream)
        S.sgcm_solve_bvps(prob, x0, lam, u0, V, traj, st, it, ws, stream)
        S.sgcm_build_interpolant(grid, u0, surplus, stream)
        S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64, stream)
        if ev is not None:
            ev[1].record(stream)

    events, _ = timed_steps(step, steps, warmup, stream, 2)
    ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    conv = int((st == S.CONVERGED).sum().item())
    out = {"workload": wl.name, "grid_nodes": M, "intervals": wl.n_intervals, "queries": len(xq_host),
           "value": conv * steps / (float(np.sum(ms)) / 1e3), "unit": "BVPs/s", "ms_per_step": float(np.mean(ms)),
           "converged": conv}
    if with_cpu:
        from oracle import oracle as O
        op = O.Problem(N=wl.n_intervals, T=wl.horizon, max_halvings=W.MAX_HALVINGS)
        cpu = {}
        for name, threads in (("all_threads", O.default_threads()), ("one_core", 1)):
            t = []
            for _ in range(3):
                t0 = time.perf_counter()
                r = O.solve_bvps(op, nodes, nthreads=threads)
                w = O.build_surplus(6, wl.level, r.u0, nthreads=threads)
                O.eval_hier(6, wl.level, w, xq_host, W.BOX_LO, W.BOX_HI, nthreads=threads)
                t.append(time.perf_counter() - t0)
            cpu[name] = {"cores": threads, "ms_per_step": float(np.median(t)) * 1e3,
                         "bvps_per_s": int(np.sum(r.status == O.CONVERGED)) / float(np.median(t))}
        out["cpu_oracle"] = cpu
    return out


def time_dimension_leg(dev, steps: int, warmup: int, with_cpu: bool) -> dict:
    """Example III with the time variable as a grid dimension (Sec. 5.3):
    the level-5 grid in (t, x) over [0, 5] x [-2, 2]^3, one step = the BVPs of
    every node over [t0, T] (sgcm_solve_bvps_tx), the interpolants of V and
    u* on that grid, and their evaluation at the paper's 1200 validation
    points; errors against the closed form there (the paper reports the MAE
    of V on its level-8 grid)."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import workloads as W
    prob = S.Problem(model=S.MODEL_EXAMPLE3, n=3, m=1, T=W.EX3_T, N=W.EX3_N, tol=W.TOL, max_iter=W.MAX_ITER,
                     max_halvings=W.MAX_HALVINGS, continuation=W.EX3_CONTINUATION)
    grid = S.Grid(4, W.EX3_LEVEL, W.EX3_LO, W.EX3_HI)
    nodes = grid.nodes()
    M = len(grid)
    q_host = W.ex3_samples()
    tx, q = torch.tensor(nodes, device=dev), torch.tensor(q_host, device=dev)
    lam = torch.empty((M, 3), dtype=torch.float64, device=dev)
    V = torch.empty((M,), dtype=torch.float64, device=dev)
    u0 = torch.empty((M, 1), dtype=torch.float64, device=dev)
    st = torch.empty((M,), dtype=torch.int32, device=dev)
    it = torch.empty((M,), dtype=torch.int32, device=dev)
    ws = torch.empty((S.sgcm_solve_bvps_workspace(prob, M) // 8 + 32,), dtype=torch.float64, device=dev)
    wV = torch.empty((M, 1), dtype=torch.float64, device=dev)
    wu = torch.empty((M, 1), dtype=torch.float64, device=dev)
    qV = torch.empty((len(q_host), 1), dtype=torch.float64, device=dev)
    qu = torch.empty((len(q_host), 1), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    grid.upload(stream)

    def step(ev):
        if ev is not None:
            ev[0].record(stream)
        S.sgcm_solve_bvps_tx(prob, tx, lam, u0, V, None, st, it, ws, stream)
        if ev is not None:
            ev[1].record(stream)
        S.sgcm_build_interpolant(grid, V.view(M, 1), wV, stream)
        S.sgcm_build_interpolant(grid, u0, wu, stream)
        S.sgcm_eval_feedback(grid, wV, q, qV, S.FP64, stream)
        S.sgcm_eval_feedback(grid, wu, q, qu, S.FP64, stream)
        if ev is not None:
            ev[2].record(stream)

    events, _ = timed_steps(step, steps, warmup, stream, 3)
    solve_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    rest_ms = np.array([e[1].elapsed_time(e[2]) for e in events])
    conv = int((st == S.CONVERGED).sum().item())
    s = 1.0 + q_host[:, 1] ** 2 + q_host[:, 2] ** 2
    y = q_host[:, 3] / s
    th = np.tanh(W.EX3_T - q_host[:, 0])
    V_ex, u_ex = 0.5 * y * y * th, -y * th
    eV, eu = qV.cpu().numpy()[:, 0] - V_ex, qu.cpu().numpy()[:, 0] - u_ex
    its = it.cpu().numpy()
    out = {"workload": "example3-tx-L%d-N%d" % (W.EX3_LEVEL, W.EX3_N), "grid": "(t, x) in [0, 5] x [-2, 2]^3, d = 4",
           "grid_nodes": M, "intervals": W.EX3_N, "T": W.EX3_T, "continuation_stages": W.EX3_CONTINUATION,
           "converged": conv, "iters_max": int(its.max()), "iters_mean": float(its.mean()),
           "solve_ms": float(np.median(solve_ms)), "bvps_per_s": conv / (float(np.median(solve_ms)) / 1e3),
           "build_and_eval_ms": float(np.median(rest_ms)), "samples": len(q_host),
           "V_error": {"mae": float(np.mean(np.abs(eV))), "max": float(np.max(np.abs(eV))), "var": float(np.var(eV))},
           "u_error": {"mae": float(np.mean(np.abs(eu))), "max": float(np.max(np.abs(eu)))}}
    if with_cpu:
        from oracle import oracle as O
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            for tv in np.unique(nodes[:, 0]):
                idx = np.where(nodes[:, 0] == tv)[0]
                op = O.Problem(model=O.EXAMPLE3, n=3, m=1, T=W.EX3_T - tv, N=W.EX3_N, tol=W.TOL,
                               max_iter=W.MAX_ITER, max_halvings=W.MAX_HALVINGS, continuation=W.EX3_CONTINUATION)
                O.solve_bvps(op, nodes[idx, 1:])
            t.append(time.perf_counter() - t0)
        out["cpu_oracle_solve"] = {"cores": O.default_threads(), "ms": float(np.median(t)) * 1e3,
                                   "bvps_per_s": M / float(np.median(t))}
    return out


def batched_leg(dev, reps: int) -> dict:
    """The mixed batch (3072 level-5 nodes + 1024 uniform states, N in
    {64..512}, T in {10, 20, 40}): one persistent launch with the autotuned
    schedule, captured in a HIP graph and replayed, against the same inputs
    solved unbatched (one launch per (N, T) group)."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import autotune as A
    order, slots, nb, fc, src = A.tuned_schedule()
    problem = A.batch_problem(nb=nb, fc=fc)
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
    flops = newton_flops(N, it.cpu().numpy(), plan=True)  # first steps from the batch's per-(N, T) steps
    return {"workload": "mixed batch: " + A.W.BATCH.name, "n_bvps": n, "converged": converged,
            "roofline": alu_roofline("k_newton_batch_grid<double>" if slots == 0 else "k_newton_batch<double>",
                                     flops, bms, PEAK_FP64_TFLOPS),
            "schedule": {"order": "larger N*T first" if order == S.ORDER_LONGEST_FIRST else "as given",
                         "slots_per_cu": slots, "tile": tile_info(nb, fc, src)},
            "graph": True, "ms": bms, "bvps_per_s": converged / (bms / 1e3),
            "unbatched": {"launches": ngroups, "ms": ubms, "bvps_per_s": converged / (ubms / 1e3)},
            "speedup_vs_unbatched": ubms / bms}


def swept_steps_roofline(N: int, iters: np.ndarray, n_bvps: int, ms: float) -> dict:
    """The one-shot solve counted by the interval steps it sweeps: with 64 or
    more BVPs the call computes the first steps of the six unit initial
    states by doubling (no sweep) and every BVP combines them, so it sweeps
    N x (sum of iterations) steps; below 64 every BVP sweeps its own first
    step too."""
    steps = float(N * np.sum(iters)) if n_bvps >= 64 else float(np.sum(N * (iters + 1.0)))
    flops = FLOPS_PER_INTERVAL_STEP * steps
    achieved = flops / (ms / 1e3) / 1e12
    return {"interval_steps": steps, "flops": flops, "achieved": achieved, "frac": achieved / PEAK_FP64_TFLOPS}


def tile_info(nb: int, fc: int, src) -> dict:
    """The solver tile a leg ran with (intervals per sweep batch and per
    forward-pass chunk; 0 is the library default) and where it came from."""
    return {"sweep_batch": nb or 8, "forward_chunk": fc or 12,
            "source": os.path.relpath(src, ROOT) if src else "default"}


def rel_rows(a, b):
    """Per-row relative error max|a - b| / max(max|b|, 1e-8)."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.max(np.abs(a - b), axis=1) / np.maximum(np.max(np.abs(b), axis=1), 1e-8)


def err_stats(e) -> dict:
    e = np.asarray(e)
    return {"max": float(e.max()), "rms": float(np.sqrt(np.mean(e ** 2)))} if e.size else {"max": None, "rms": None}


def oracle_sample(op, x0: np.ndarray, n: int, seed: int):
    """The oracle on a seeded sample of the initial states: (indices, result)."""
    from oracle import oracle as O
    idx = np.unique(np.concatenate([[0, len(x0) - 1], np.sort(
        np.random.default_rng(seed).choice(len(x0), size=min(n, len(x0)), replace=False))]))
    return idx, O.solve_bvps(op, x0[idx])


def precision_leg(dev, prob, grid, x0, lam64, u064, it64, surplus, eval_flops_q: float, reps: int) -> dict:
    """FP32 variants beside the FP64 path on the same MI355X: the FP32 inexact
    Newton solve of the full workload with its plan against the FP64 solve
    with its plan, and FP32 feedback evaluation at 1e7 uniform states against
    FP64; errors against the FP64 oracle on seeded samples (solve: 64 nodes,
    evaluation: 1e4 states)."""
    import dataclasses
    import torch
    import paper_1507_04769_amd as S
    from oracle import oracle as O
    from paper_1507_04769_amd import autotune as A
    from paper_1507_04769_amd import workloads as W
    nb32, fc32, src32 = A.tuned_tile("fp32", with_plan=True)
    nb64, fc64, src64 = A.tuned_tile("fp64", with_plan=True)
    p32 = dataclasses.replace(prob, precision=S.FP32, sweep_batch=nb32, forward_chunk=fc32)
    M = x0.shape[0]
    lam = torch.empty_like(lam64)
    u0 = torch.empty_like(u064)
    V = torch.empty((M,), dtype=torch.float64, device=dev)
    st = torch.empty((M,), dtype=torch.int32, device=dev)
    it = torch.empty((M,), dtype=torch.int32, device=dev)
    ws = torch.empty((S.sgcm_solve_bvps_workspace(p32, M) // 8 + 32,), dtype=torch.float64, device=dev)
    p64 = dataclasses.replace(prob, precision=S.FP64, sweep_batch=nb64, forward_chunk=fc64)
    ws64 = torch.empty((S.sgcm_solve_bvps_workspace(p64, M) // 8 + 32,), dtype=torch.float64, device=dev)
    lam2, u02, V2 = torch.empty_like(lam), torch.empty_like(u0), torch.empty_like(V)
    st2, it2 = torch.empty_like(st), torch.empty_like(it)
    plan32, plan64 = S.Plan(p32), S.Plan(p64)  # first steps from the plans (made once)
    ms32 = A.time_ms(lambda: S.sgcm_solve_bvps_plan(plan32, x0, lam, u0, V, None, st, it, ws), reps)
    ms64 = A.time_ms(lambda: S.sgcm_solve_bvps_plan(plan64, x0, lam2, u02, V2, None, st2, it2, ws64), reps)
    conv = int((st == S.CONVERGED).sum().item())
    i32, i64 = it.cpu().numpy(), it64
    op = O.Problem(N=prob.N, T=prob.T, max_iter=prob.max_iter, max_halvings=prob.max_halvings)
    idx, o = oracle_sample(op, x0.cpu().numpy(), 64, seed=44)
    el = rel_rows(lam.cpu().numpy()[idx], o.lambda0)
    eu = rel_rows(u0.cpu().numpy()[idx], o.u0)
    el64 = rel_rows(lam2.cpu().numpy()[idx], o.lambda0)
    # the algorithmic flops of the FP64 solve; the linear solve runs in FP32,
    # so the fraction is given against both peaks
    f32 = newton_flops(prob.N, i32, plan=True)
    rf = alu_roofline("k_newton<float>", f32, float(np.median(ms32)), PEAK_FP32_TFLOPS)
    rf["frac_of_fp64_peak"] = rf["achieved"] / PEAK_FP64_TFLOPS
    rf["tile"] = tile_info(nb32, fc32, src32)
    solve = {"ms": float(np.median(ms32)), "fp64_ms": float(np.median(ms64)), "roofline": rf,
             "bvps_per_s": conv / (float(np.median(ms32)) / 1e3), "converged": conv,
             "mean_iters": float(i32.mean()), "fp64_mean_iters": float(i64.mean()),
             "vs_oracle_sample": len(idx),
             "lambda0_rel_err": err_stats(el), "u0_rel_err": err_stats(eu),
             "fp64_lambda0_rel_err": err_stats(el64)}
    nq = 10_000_000
    xq = torch.tensor(W.uniform_in_box(nq, seed=3), device=dev)
    xq32 = xq.float()
    w32 = surplus.float()
    uq = torch.empty((nq, surplus.shape[1]), dtype=torch.float64, device=dev)
    uq32 = torch.empty((nq, surplus.shape[1]), dtype=torch.float32, device=dev)
    e64 = A.time_ms(lambda: S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64), reps)
    e32 = A.time_ms(lambda: S.sgcm_eval_feedback_f32(grid, w32, xq32, uq32), reps)
    qi = W.sample_indices(nq, 10_000, seed=45)
    ref = O.eval_hier(6, grid.level, surplus.cpu().numpy(), xq.cpu().numpy()[qi], W.BOX_LO, W.BOX_HI)
    err32 = np.abs(uq32.cpu().numpy()[qi].astype(np.float64) - ref)
    err64 = np.abs(uq.cpu().numpy()[qi] - ref)
    ev = {"queries": nq, "ms": float(np.median(e32)), "fp64_ms": float(np.median(e64)),
          "evals_per_s": nq / (float(np.median(e32)) / 1e3), "fp64_evals_per_s": nq / (float(np.median(e64)) / 1e3),
          "vs_oracle_sample": len(qi),
          "abs_err": err_stats(err32.max(axis=1)), "fp64_abs_err": err_stats(err64.max(axis=1)),
          "max_abs_u": float(np.abs(ref).max()),
          "roofline": alu_roofline("k_eval_fast<6, %d, 3, float>" % grid.level, eval_flops_q * nq,
                                   float(np.median(e32)), PEAK_FP32_TFLOPS),
          "fp64_roofline": alu_roofline("k_eval_fast<6, %d, 3, double>" % grid.level, eval_flops_q * nq,
                                        float(np.median(e64)), PEAK_FP64_TFLOPS)}
    return {"fp32_newton": solve, "fp32_eval": ev,
            "note": "errors against the FP64 oracle on seeded samples (interpolant of the three-wheel u(0))"}


def underactuated_leg(dev, reps: int) -> dict:
    """The underactuated precision workload: two wheels (seeded orthonormal
    3 x 2 B), level-4 grid over the full box, N = 256, T = 20, reached by the
    virtual-torque continuation (4 stages, at most 100 iterations each); the
    FP64 and the FP32 inexact Newton solves, each against the FP64 oracle on
    a seeded sample of 64 nodes."""
    import dataclasses
    import torch
    import paper_1507_04769_amd as S
    from oracle import oracle as O
    from paper_1507_04769_amd import autotune as A
    from paper_1507_04769_amd import workloads as W
    w = W.UNDERACTUATED
    grid = S.Grid(6, w.level, W.BOX_LO, W.BOX_HI)
    nodes = grid.nodes()
    x0 = torch.tensor(nodes, device=dev)
    p64 = S.Problem(m=2, J=W.J_DIAG, B=W.input_matrix(2), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=w.horizon,
                    N=w.n_intervals, tol=W.TOL, max_iter=W.UNDERACTUATED_MAX_ITER, max_halvings=W.MAX_HALVINGS,
                    continuation=W.UNDERACTUATED_CONTINUATION)
    op = O.Problem(m=2, B=W.input_matrix(2), N=w.n_intervals, T=w.horizon, max_iter=p64.max_iter,
                   max_halvings=p64.max_halvings, continuation=p64.continuation)
    idx, o = oracle_sample(op, nodes, 64, seed=46)
    ok = o.status == O.CONVERGED
    out = {"workload": w.name, "grid_nodes": len(nodes), "continuation_stages": p64.continuation,
           "max_iter_per_stage": p64.max_iter, "vs_oracle_sample": len(idx),
           "oracle_sample_converged": int(ok.sum())}
    for name, prec in (("fp64", S.FP64), ("fp32", S.FP32)):
        p = dataclasses.replace(p64, precision=prec)
        ws = torch.empty((S.sgcm_solve_bvps_workspace(p, len(nodes)) // 8 + 32,), dtype=torch.float64, device=dev)
        res = {}

        def run():
            res["sol"] = S.solve_bvps(p, x0, workspace=ws)
        ms = A.time_ms(run, reps)
        sol = res["sol"]
        st, it = sol.status.cpu().numpy(), sol.iters.cpu().numpy()
        both = ok & (st[idx] == S.CONVERGED)
        el = rel_rows(sol.lambda0.cpu().numpy()[idx][both], o.lambda0[both])
        eu = rel_rows(sol.u0.cpu().numpy()[idx][both], o.u0[both])
        out[name] = {"ms": float(np.median(ms)), "converged": int(np.sum(st == S.CONVERGED)),
                     "status_counts": np.bincount(st, minlength=4).tolist(),
                     "bvps_per_s": int(np.sum(st == S.CONVERGED)) / (float(np.median(ms)) / 1e3),
                     "mean_total_iters": float(it.mean()), "max_total_iters": int(it.max()),
                     "same_status_and_iters_as_oracle_sample": bool(np.array_equal(st[idx], o.status) and
                                                                     np.array_equal(it[idx], o.iters)),
                     "lambda0_rel_err": err_stats(el), "u0_rel_err": err_stats(eu)}
    out["note"] = ("nodes whose continuation stalls are reported by status (MAXITER); without a converged "
                   "value at every node the grid has no interpolant, so the 1e7-point FP32/FP64 evaluation is "
                   "measured on the three-wheel interpolant (precision.fp32_eval)")
    return out


def validation_leg(dev, prob, grid, u0, V, surplus, n_nodes_intervals: int, reps: int) -> dict:
    """Monte Carlo total-error estimate of the interpolant (Sec. 4.3): 1280
    uniform states, the reference from the four-point Lobatto IIIA formula
    with error control (meshes doubled from N/4 until the order-6
    extrapolation's correction is within 1e-7), for the feedback u(0, x) (the
    step's interpolant) and the value V(0, x) (an interpolant of the node
    values of V); the trapezoid with its order-2 extrapolation on 2N and 4N
    intervals beside it."""
    import torch
    import paper_1507_04769_amd as S
    from paper_1507_04769_amd import autotune as A
    from paper_1507_04769_amd import validation as VA
    from paper_1507_04769_amd import workloads as W
    w_V = S.build_interpolant(grid, V.view(-1, 1).contiguous())
    xs = torch.tensor(W.uniform_in_box(VA.N_SAMPLES, seed=VA.SAMPLE_SEED), device=dev)
    out = {"samples": VA.N_SAMPLES, "seed": VA.SAMPLE_SEED, "node_intervals": n_nodes_intervals}
    for name, scheme, n_ref in (("lobatto4", S.LOBATTO4, max(n_nodes_intervals // 4, 1)),
                                ("trapezoid", S.TRAPEZOID, 2 * n_nodes_intervals)):
        est = VA.Estimator(prob, n_ref, scheme=scheme)
        r = est(grid, surplus, xs, w_V)
        ms = A.time_ms(lambda: est(grid, surplus, xs, w_V), reps)
        su, sV = r.stats_u.cpu().numpy(), r.stats_V.cpu().numpy()
        st = r.status.cpu().numpy()
        out[name] = {"reference_intervals": [r.n_ref, 2 * r.n_ref], "reference_order": est.order,
                     "reference_converged": [int(np.sum(st[0] == S.CONVERGED)), int(np.sum(st[1] == S.CONVERGED))],
                     "reference_error_estimate": r.correction,
                     "u_error": {"max": float(su[0]), "rms": float(su[1]), "mae": float(su[3]),
                                 "relative_mae": float(su[4]), "reference_correction_max": float(su[2])},
                     "V_error": {"max": float(sV[0]), "rms": float(sV[1]), "mae": float(sV[3]),
                                 "relative_mae": float(sV[4]), "reference_correction_max": float(sV[2])},
                     "ms": float(np.median(ms)), "samples_per_s": VA.N_SAMPLES / (float(np.median(ms)) / 1e3)}
    out["lobatto4"]["tolerance"] = VA.REF_TOL
    return out


def serving_leg(n_requests: int, rate: float) -> dict:
    """The serving loop on a seeded Poisson stream of mixed requests: solves of
    1..512 states (meshes 64..512, three- or two-wheel model) and queries of
    1..1e5 states against resident level-3/4/5 interpolants (FP64 or FP32).
    Reported: p50/p99 latency (arrival to results on the host), overall and
    per class (queries, three-wheel solves, two-wheel solves), and throughput
    at the given rate with continuous batching on four streams, in two runs of
    the same stream (run-to-run spread); the same stream served one request
    per launch on one stream; and the capacity with every request present at
    once."""
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
    again = SV.request_stream(n_requests, rate, seed=701, levels=(3, 4, 5))
    rerun = SV.Server(interps, n_streams=4, hbm_budget=8 << 30, plans=plans).run(again, realtime=True)
    out["continuous_rerun_latency_ms"] = rerun["latency_ms"]
    out["one_per_launch"] = SV.Server(interps, n_streams=1, merge=False, plans=plans).run(reqs, realtime=True)
    out["capacity_all_at_once"] = SV.Server(interps, n_streams=4, hbm_budget=8 << 30, plans=plans).run(reqs, realtime=False)["throughput"]
    return out


def pipelined_leg(prob, grid, x0, xq, m: int, steps: int, warmup: int, ref_u0, ref_uq) -> dict:
    """Consecutive steps overlapped on two streams: the solves on one, the
    surplus build and the evaluation of each step on the other, after its
    solve; step k + 1's solve runs while step k builds and evaluates (two
    sets of solve outputs, so that a solve never overwrites node values that
    a build still reads).  The short evaluation launch fills the compute
    units that the solve's longest BVPs leave idle near its end, and the
    first steps' launch.  Throughput = steps / host
    wall time between two device synchronisations; every step's results are
    checked against the sequential step's."""
    import torch
    import paper_1507_04769_amd as S
    dev = x0.device
    M, N = x0.shape[0], prob.N
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    bufs = [{"lam": torch.empty((M, 6), dtype=torch.float64, device=dev),
             "u0": torch.empty((M, m), dtype=torch.float64, device=dev),
             "V": torch.empty((M,), dtype=torch.float64, device=dev),
             "traj": torch.empty((M, N + 1, 12), dtype=torch.float64, device=dev),
             "st": torch.empty((M,), dtype=torch.int32, device=dev),
             "it": torch.empty((M,), dtype=torch.int32, device=dev)} for _ in range(2)]
    ws = torch.empty((S.sgcm_solve_bvps_workspace(prob, M) // 8 + 32,), dtype=torch.float64, device=dev)
    surplus = torch.empty((M, m), dtype=torch.float64, device=dev)
    uq = torch.empty((xq.shape[0], m), dtype=torch.float64, device=dev)
    solved = [torch.cuda.Event(), torch.cuda.Event()]
    built = [None, None]
    ok = [True]

    def run(n):
        for k in range(n):
            j = k % 2
            b = bufs[j]
            if built[j] is not None:
                sa.wait_event(built[j])  # the build of step k - 2 has read these node values
            S.sgcm_solve_bvps(prob, x0, b["lam"], b["u0"], b["V"], b["traj"], b["st"], b["it"], ws, sa)
            solved[j].record(sa)
            sb.wait_event(solved[j])
            S.sgcm_build_interpolant(grid, b["u0"], surplus, sb)
            ev = torch.cuda.Event()
            ev.record(sb)
            built[j] = ev
            S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64, sb)

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    last = bufs[(steps - 1) % 2]
    same = bool(torch.equal(last["u0"], ref_u0) and torch.equal(uq, ref_uq))
    conv = int((last["st"] == S.CONVERGED).sum().item())
    return {"ms_per_step": wall / steps * 1e3, "value": conv * steps / wall, "unit": "BVPs/s",
            "steps": steps, "same_results_as_sequential_step": same,
            "note": "step k+1's solve overlaps step k's build and evaluation (two streams); "
                    "host wall time over the timed steps"}


def timed_steps(step, steps: int, warmup: int, stream, n_events: int):
    """W untimed calls of step(), then `steps` timed ones with n_events HIP
    events recorded on the launch stream inside each; returns the events and
    the host wall time of the timed region (bracketed by synchronisation)."""
    import torch
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(n_events)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    return events, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["full", "small"], default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pipelined", action="store_true", help="skip the two-stream pipelined steps")
    ap.add_argument("--no-small", action="store_true", help="skip the small-workload line")
    ap.add_argument("--no-time-dimension", action="store_true",
                    help="skip the Example III leg with the time variable as a grid dimension")
    ap.add_argument("--cpu-queries", type=int, default=20000)
    ap.add_argument("--no-batched", action="store_true", help="skip the mixed-batch leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32 and underactuated legs")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-validation", action="store_true", help="skip the total-error estimate leg")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=250.0, help="requests per second")
    ap.add_argument("--no-plan-compare", action="store_true",
                    help="skip the step with a solve plan (profiling runs)")
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
    from paper_1507_04769_amd import autotune as A
    # the solver tile chosen by the autotuner for this workload (the tile
    # changes the time only, never a result)
    nb, fc, tile_src = A.tuned_tile("fp64") if wl.name == W.FULL.name else (0, 0, None)
    prob = S.Problem(m=wl.m, J=W.J_DIAG, B=W.input_matrix(wl.m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W,
                     T=wl.horizon, N=wl.n_intervals, tol=W.TOL, max_iter=W.MAX_ITER, max_halvings=W.MAX_HALVINGS,
                     sweep_batch=nb, forward_chunk=fc)
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
    grid.upload(stream)  # the grid's device tables, made once like the grid itself

    def make_step(solve):
        def step(ev):
            if ev is not None:
                ev[0].record(stream)
            solve()
            if ev is not None:
                ev[1].record(stream)
            S.sgcm_build_interpolant(grid, u0, surplus, stream)
            if ev is not None:
                ev[2].record(stream)
            S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64, stream)
            if ev is not None:
                ev[3].record(stream)
        return step

    # the headline: one-shot steps (nothing made beforehand; from 64 BVPs the
    # call computes the six unit initial states' first steps and combines them)
    events, wall = timed_steps(make_step(lambda: S.sgcm_solve_bvps(prob, x0, lam, u0, V, traj, st, it, ws,
                                                                   stream)), args.steps, args.warmup, stream, 4)
    step_ms = np.array([e[0].elapsed_time(e[3]) for e in events])
    solve_ms = np.array([e[0].elapsed_time(e[1]) for e in events])
    build_ms = np.array([e[1].elapsed_time(e[2]) for e in events])
    eval_ms = np.array([e[2].elapsed_time(e[3]) for e in events])
    status = st.cpu().numpy()
    iters = it.cpu().numpy()
    converged = int(np.sum(status == S.CONVERGED))
    value = converged * args.steps / (float(np.sum(step_ms)) / 1e3)
    flops = newton_flops(wl.n_intervals, iters)
    achieved = flops / (float(np.mean(solve_ms)) / 1e3) / 1e12
    builder_flops = newton_flops_plan(wl.n_intervals, iters + 1) - (wl.n_intervals + 1) * FLOPS_PER_POINT_PLAN_STEP * M

    # the same step with the problem's solve plan (first Newton steps of the
    # six unit initial states), made once before the steps: the amortised form
    with_plan = None
    if not args.no_plan_compare:
        lam_p, u0_p, V_p, traj_p = torch.empty_like(lam), torch.empty_like(u0), torch.empty_like(V), torch.empty_like(traj)
        st_p, it_p = torch.empty_like(st), torch.empty_like(it)
        torch.cuda.synchronize()
        t_plan = time.perf_counter()
        pnb, pfc, psrc = A.tuned_tile("fp64", with_plan=True) if wl.name == W.FULL.name else (0, 0, None)
        pprob = dataclasses.replace(prob, sweep_batch=pnb, forward_chunk=pfc)
        plan = S.Plan(pprob, stream)
        plan_ms = (time.perf_counter() - t_plan) * 1e3
        ev_p, _ = timed_steps(make_step(lambda: S.sgcm_solve_bvps_plan(plan, x0, lam_p, u0, V_p, traj_p, st_p, it_p,
                                                                       ws, stream)), args.steps, args.warmup, stream, 4)
        pstep = np.array([e[0].elapsed_time(e[3]) for e in ev_p])
        psolve = np.array([e[0].elapsed_time(e[1]) for e in ev_p])
        pit = it_p.cpu().numpy()
        pconv = int((st_p == S.CONVERGED).sum().item())
        pflops = newton_flops(wl.n_intervals, pit, plan=True)
        with_plan = {"value": pconv * args.steps / (float(np.sum(pstep)) / 1e3), "unit": "BVPs/s",
                     "ms_per_step": float(np.mean(pstep)), "solve_ms": float(np.mean(psolve)),
                     "create_ms": plan_ms,
                     "same_status_and_iters": bool(torch.equal(st, st_p) and torch.equal(it, it_p)),
                     "lambda0_max_rel_diff": float(((lam - lam_p).abs().amax(dim=1) /
                                                    lam.abs().amax(dim=1).clamp_min(1e-8)).max().item()),
                     "roofline": {**alu_roofline("k_newton (sgcm_solve_bvps_plan)", pflops, float(np.mean(psolve)),
                                                 PEAK_FP64_TFLOPS), "tile": tile_info(pnb, pfc, psrc)},
                     "note": "the plan is made once per problem, outside the timed steps"}
        del lam_p, u0_p, V_p, traj_p
        # the headline step's outputs feed the legs below: restore them
        S.sgcm_solve_bvps(prob, x0, lam, u0, V, traj, st, it, ws, stream)
        S.sgcm_build_interpolant(grid, u0, surplus, stream)
        torch.cuda.synchronize()

    keys = grid.keys()
    eval_flops_q = eval_flops_per_query(keys, wl.level, wl.m)

    # the same steps overlapped on two streams (compared with the sequential
    # step's results, which are restored just above)
    pipelined = None
    if not args.no_pipelined:
        S.sgcm_eval_feedback(grid, surplus, xq, uq, S.FP64, stream)
        torch.cuda.synchronize()
        ref_u0, ref_uq = u0.clone(), uq.clone()
        pipelined = pipelined_leg(prob, grid, x0, xq, wl.m, args.steps, args.warmup, ref_u0, ref_uq)

    small = None
    if args.workload == "full" and not args.no_small:
        small = small_leg(dev, args.steps, args.warmup, not args.no_cpu_baseline)

    time_dim = None
    if args.workload == "full" and not args.no_time_dimension:
        time_dim = time_dimension_leg(dev, args.steps, args.warmup, not args.no_cpu_baseline)

    batched = None if args.no_batched or args.workload != "full" else batched_leg(dev, 5)
    precision = underactuated = None
    if not args.no_precision and args.workload == "full":
        precision = precision_leg(dev, prob, grid, x0, lam, u0, iters, surplus, eval_flops_q, 5)
        underactuated = underactuated_leg(dev, 3)
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

    eval_rf = alu_roofline("k_eval_fast<6, %d, %d, double>" % (wl.level, wl.m), eval_flops_q * len(xq_host),
                           float(np.mean(eval_ms)), PEAK_FP64_TFLOPS)
    walk_q = eval_flops_per_query_walk(keys, wl.level, wl.m)
    eval_rf["flops_per_query"] = eval_flops_q
    eval_rf["kernel_count"] = {"flops_per_query": walk_q,
                               "achieved": walk_q * len(xq_host) / (float(np.mean(eval_ms)) / 1e3) / 1e12}
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
                   "queries": len(xq_host), "query_seed": wl.query_seed, "first_newton_step": ("combined from the six unit-state first steps computed by doubling inside the call"
                                         if M >= 64 else "solved per BVP")},
        "feedback_evals_per_s": len(xq_host) / (float(np.mean(eval_ms)) / 1e3),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": {"solve_bvps": float(np.mean(solve_ms)), "build_interpolant": float(np.mean(build_ms)),
                      "eval_feedback": float(np.mean(eval_ms))},
        "converged": converged,
        "newton_iters_hist": np.bincount(iters).tolist(),
        "wall_s_timed": wall,
        "roofline": {"kernel": "k_newton (sgcm_solve_bvps: the first steps by doubling, k_order and the main launch)", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic() if wl.name == W.FULL.name else None,
                     "algorithmic_flops_per_launch": flops,
                     "interval_steps_per_launch": float(np.sum(wl.n_intervals * (iters + 1.0))),
                     # the steps the call actually sweeps when it forms the
                     # first steps from the six unit states (the count above,
                     # 6.5 kflop per step, charges every BVP its own first step)
                     "swept": swept_steps_roofline(wl.n_intervals, iters, M, float(np.mean(solve_ms))),
                     "tile": tile_info(nb, fc, tile_src),
                     "kernel_count": {"flops_per_launch": builder_flops,
                                      "achieved": builder_flops / (float(np.mean(solve_ms)) / 1e3) / 1e12}},
        "eval_roofline": eval_rf,
    }
    if with_plan is not None:
        out["with_plan"] = with_plan
    if pipelined is not None:
        out["pipelined"] = pipelined
    if small is not None:
        out["small_workload"] = small
    if time_dim is not None:
        out["time_dimension"] = time_dim
    if batched is not None:
        out["batched"] = batched
    if precision is not None:
        out["precision"] = precision
    if underactuated is not None:
        out["underactuated"] = underactuated
    if validation is not None:
        out["validation"] = validation
    if serving is not None:
        out["serving"] = serving
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, nodes, xq_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
