"""Schedule autotuner for batches of BVPs with mixed meshes and horizons.

Times every candidate schedule of ``sgcm_solve_bvps_batch`` (processing order
x persistent workgroups per compute unit) on one mixed batch, with HIP events
on the launch stream, and the same inputs solved unbatched (one
``sgcm_solve_bvps`` launch per (N, T) group, in sequence on one stream).
Writes the measurements and the fastest schedule to a JSON file that
``bench.py`` reads; results never depend on the schedule (only the time does).

    python -m paper_1507_04769_amd.autotune [--reps 5] [--out FILE]
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
CANDIDATES = [(order, slots) for order in (S.ORDER_GIVEN, S.ORDER_LONGEST_FIRST)
              for slots in (0, 1, 2, 3, 4, 5, 6)]


def batch_problem(m: int = 3) -> S.Problem:
    return S.Problem(m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, tol=W.TOL,
                     max_iter=W.MAX_ITER)


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
    for order, slots in CANDIDATES:
        b = S.Batch(problem, N, T, order=order, slots_per_cu=slots)
        ws = S.batch_workspace(b, x0_dev.device)
        n = b.n
        lam = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        u0 = torch.empty((n, b.m), dtype=torch.float64, device="cuda")
        V = torch.empty((n,), dtype=torch.float64, device="cuda")
        st = torch.empty((n,), dtype=torch.int32, device="cuda")
        it = torch.empty((n,), dtype=torch.int32, device="cuda")
        ms = time_ms(lambda: S.sgcm_solve_bvps_batch(b, x0_dev, lam, u0, V, st, it, ws), reps)
        results.append({"order": order, "slots_per_cu": slots, "ms_median": float(np.median(ms)),
                        "ms": [float(v) for v in ms]})
        print("order %d slots/CU %d: %.3f ms" % (order, slots, float(np.median(ms))), flush=True)
    run, ngroups = unbatched_runner(problem, x0_dev, N, T)
    ums = time_ms(run, reps)
    best = min(results, key=lambda r: r["ms_median"])
    doc = {"workload": W.BATCH.name, "n_bvps": int(len(x0)), "device": torch.cuda.get_device_name(0),
           "reps": reps, "candidates": results,
           "best": {"order": best["order"], "slots_per_cu": best["slots_per_cu"], "ms_median": best["ms_median"]},
           "unbatched": {"launches": ngroups, "ms_median": float(np.median(ums)), "ms": [float(v) for v in ums]}}
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("best: order %d slots/CU %d (%.3f ms); unbatched %d launches %.3f ms" % (
        best["order"], best["slots_per_cu"], best["ms_median"], ngroups, float(np.median(ums))), flush=True)
    return doc


def tuned_schedule(path: str = DEFAULT_OUT):
    """(order, slots_per_cu) chosen by the last tuning run, or the default
    (larger N T first, 6 persistent workgroups per CU) if none was stored."""
    try:
        with open(path) as f:
            b = json.load(f)["best"]
        return int(b["order"]), int(b["slots_per_cu"]), path
    except (OSError, KeyError, ValueError):
        return S.ORDER_LONGEST_FIRST, 6, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    tune(args.reps, args.out)


if __name__ == "__main__":
    main()
