"""Autotuner of the solver's launch choices.

Batches of BVPs with mixed meshes and horizons: times every candidate
schedule of ``sgcm_solve_bvps_batch`` (processing order x persistent
workgroups per compute unit x solver tile) on one mixed batch, with HIP
events on the launch stream, and the same inputs solved unbatched (one
``sgcm_solve_bvps_plan`` launch per (N, T) group, in sequence on one stream).

Uniform solves: times every solver tile (intervals per backward-sweep batch
x intervals per forward-pass chunk) on the full workload, in FP64 and in the
FP32 inexact Newton, with and without the solve plan.

Writes the measurements and the fastest choices to JSON files that
``bench.py`` reads; results never depend on these choices (only the time
does; the GPU tests check it bit for bit).

    python -m paper_1507_04769_amd.autotune [--reps 5] [--what batch|solve|all]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

import paper_1507_04769_amd as S
from paper_1507_04769_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuned", "batch_%s.json" % W.BATCH.name)
SOLVE_OUT = os.path.join(HERE, "tuned", "solve_%s.json" % W.FULL.name)
# solver tiles: (intervals per sweep batch, intervals per forward-pass chunk)
TILES = ((8, 12), (10, 12), (12, 12), (16, 12), (8, 8), (10, 8), (12, 8), (16, 8))
CANDIDATES = [(order, slots, nb, fc) for order in (S.ORDER_GIVEN, S.ORDER_LONGEST_FIRST)
              for slots in (0, 1, 2, 3, 4, 5, 6) for nb, fc in TILES]


def batch_problem(m: int = 3, nb: int = 0, fc: int = 0) -> S.Problem:
    return S.Problem(m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, tol=W.TOL,
                     max_iter=W.MAX_ITER, sweep_batch=nb, forward_chunk=fc)


def batch_inputs(bw: W.MixedBatch = W.BATCH):
    g = S.Grid(6, bw.level, W.BOX_LO, W.BOX_HI)
    x0 = W.batch_initial_states(bw, g.nodes())
    N, T = W.mixed_assignment(bw, len(x0))
    return x0, N, T


def time_ms(fn, reps: int) -> list:
    """Durations of reps calls of fn (after one warm-up), HIP events on the
    current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return out


def unbatched_runner(problem: S.Problem, x0_dev, N, T):
    """One sgcm_solve_bvps_plan launch per (N, T) group, in sequence (each
    group with its solve plan, as the batch forms its first Newton steps);
    plans and buffers made up front so that the timed region only launches."""
    import torch
    groups = []
    for NN, TT in sorted(set(zip(N.tolist(), T.tolist()))):
        idx = np.nonzero((N == NN) & (T == TT))[0]
        p = S.Problem(**{**problem.__dict__, "N": int(NN), "T": float(TT)})
        xi = x0_dev[torch.as_tensor(idx, device=x0_dev.device)].contiguous()
        n = len(idx)
        ws = torch.empty((max(S.sgcm_solve_bvps_workspace(p, n), 256) + 255) // 256 * 32, dtype=torch.float64,
                         device=x0_dev.device)
        outs = (torch.empty((n, 6), dtype=torch.float64, device=x0_dev.device),
                torch.empty((n, p.m), dtype=torch.float64, device=x0_dev.device),
                torch.empty((n,), dtype=torch.float64, device=x0_dev.device),
                torch.empty((n,), dtype=torch.int32, device=x0_dev.device),
                torch.empty((n,), dtype=torch.int32, device=x0_dev.device))
        groups.append((S.Plan(p), xi, ws, outs))

    def run():
        for plan, xi, ws, (lam, u0, V, st, it) in groups:
            S.sgcm_solve_bvps_plan(plan, xi, lam, u0, V, None, st, it, ws)
    return run, len(groups)


def tune(reps: int = 5, out: str = DEFAULT_OUT) -> dict:
    import torch
    problem = batch_problem()
    x0, N, T = batch_inputs()
    x0_dev = torch.tensor(x0, device="cuda")
    results = []
    for order, slots, nb, fc in CANDIDATES:
        b = S.Batch(batch_problem(nb=nb, fc=fc), N, T, order=order, slots_per_cu=slots)
        ws = S.batch_workspace(b, x0_dev.device)
        n = b.n
        lam = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        u0 = torch.empty((n, b.m), dtype=torch.float64, device="cuda")
        V = torch.empty((n,), dtype=torch.float64, device="cuda")
        st = torch.empty((n,), dtype=torch.int32, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        ms = time_ms(lambda: S.sgcm_solve_bvps_batch(b, x0_dev, lam, u0, V, st, it, ws), reps)
        results.append({"order": order, "slots_per_cu": slots, "sweep_batch": nb, "forward_chunk": fc,
                        "ms_median": float(np.median(ms)), "ms": [float(v) for v in ms]})
        print("order %d slots/CU %d tile %d/%d: %.3f ms" % (order, slots, nb, fc, float(np.median(ms))), flush=True)
    run, ngroups = unbatched_runner(problem, x0_dev, N, T)
    ums = time_ms(run, reps)
    best = min(results, key=lambda r: r["ms_median"])
    doc = {"workload": W.BATCH.name, "n_bvps": int(len(x0)), "device": torch.cuda.get_device_name(0),
           "reps": reps, "candidates": results,
           "best": {"order": best["order"], "slots_per_cu": best["slots_per_cu"], "sweep_batch": best["sweep_batch"],
                    "forward_chunk": best["forward_chunk"], "ms_median": best["ms_median"]},
           "unbatched": {"launches": ngroups, "ms_median": float(np.median(ums)), "ms": [float(v) for v in ums]}}
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("best: order %d slots/CU %d tile %d/%d (%.3f ms); unbatched %d launches %.3f ms" % (
        best["order"], best["slots_per_cu"], best["sweep_batch"], best["forward_chunk"], best["ms_median"],
        ngroups, float(np.median(ums))), flush=True)
    return doc


def full_problem(precision: int, nb: int = 0, fc: int = 0) -> S.Problem:
    w = W.FULL
    return S.Problem(m=w.m, J=W.J_DIAG, B=W.input_matrix(w.m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=w.horizon,
                     N=w.n_intervals, tol=W.TOL, max_iter=W.MAX_ITER, max_halvings=W.MAX_HALVINGS,
                     precision=precision, sweep_batch=nb, forward_chunk=fc)


def tune_solve(reps: int = 5, out: str = SOLVE_OUT) -> dict:
    """Every solver tile on the full workload (all grid nodes, one launch):
    FP64 and FP32, without and with the solve plan."""
    import torch
    g = S.Grid(6, W.FULL.level, W.BOX_LO, W.BOX_HI)
    x0 = torch.tensor(g.nodes(), device="cuda")
    n = len(g)
    doc = {"workload": W.FULL.name, "n_bvps": n, "device": torch.cuda.get_device_name(0), "reps": reps}
    for name, prec in (("fp64", S.FP64), ("fp32", S.FP32)):
        cands = []
        for nb, fc in TILES:
            p = full_problem(prec, nb, fc)
            ws = torch.empty((S.sgcm_solve_bvps_workspace(p, n) // 8 + 32,), dtype=torch.float64, device="cuda")
            lam = torch.empty((n, 6), dtype=torch.float64, device="cuda")
            u0 = torch.empty((n, p.m), dtype=torch.float64, device="cuda")
            V = torch.empty((n,), dtype=torch.float64, device="cuda")
            st = torch.empty((n,), dtype=torch.int32, device="cuda")
            it = torch.empty((n,), dtype=torch.int32, device="cuda")
            plan = S.Plan(p)
            ms = time_ms(lambda: S.sgcm_solve_bvps(p, x0, lam, u0, V, None, st, it, ws), reps)
            pms = time_ms(lambda: S.sgcm_solve_bvps_plan(plan, x0, lam, u0, V, None, st, it, ws), reps)
            cands.append({"sweep_batch": nb, "forward_chunk": fc, "ms_median": float(np.median(ms)),
                          "plan_ms_median": float(np.median(pms))})
            print("%s tile %d/%d: %.3f ms, with plan %.3f ms" % (name, nb, fc, float(np.median(ms)),
                                                                 float(np.median(pms))), flush=True)
        best = min(cands, key=lambda c: c["ms_median"])
        bestp = min(cands, key=lambda c: c["plan_ms_median"])
        doc[name] = {"candidates": cands,
                     "best": {"sweep_batch": best["sweep_batch"], "forward_chunk": best["forward_chunk"],
                              "ms_median": best["ms_median"]},
                     "best_with_plan": {"sweep_batch": bestp["sweep_batch"], "forward_chunk": bestp["forward_chunk"],
                                        "ms_median": bestp["plan_ms_median"]}}
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def tuned_schedule(path: str = DEFAULT_OUT):
    """(order, slots_per_cu, sweep_batch, forward_chunk, path) chosen by the
    last tuning run, or the defaults (larger N T first, one workgroup per
    BVP, the default tile) if none was stored."""
    try:
        with open(path) as f:
            b = json.load(f)["best"]
        return int(b["order"]), int(b["slots_per_cu"]), int(b.get("sweep_batch", 0)), \
            int(b.get("forward_chunk", 0)), path
    except (OSError, KeyError, ValueError):
        return S.ORDER_LONGEST_FIRST, 0, 0, 0, None


def tuned_tile(precision: str = "fp64", with_plan: bool = False, path: str = SOLVE_OUT):
    """(sweep_batch, forward_chunk, path) of the last solve tuning run for
    "fp64" or "fp32", or the default tile (0, 0, None)."""
    try:
        with open(path) as f:
            b = json.load(f)[precision]["best_with_plan" if with_plan else "best"]
        return int(b["sweep_batch"]), int(b["forward_chunk"]), path
    except (OSError, KeyError, ValueError):
        return 0, 0, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--what", choices=["batch", "solve", "all"], default="all")
    args = ap.parse_args()
    if args.what in ("solve", "all"):
        tune_solve(args.reps)
    if args.what in ("batch", "all"):
        tune(args.reps)


if __name__ == "__main__":
    main()
