"""Reduced-precision variants (the precision direction of the hot path).

FP32 feedback evaluation (sgcm_eval_feedback_f32): the basis values, products
and the sum over nodes in FP32.  Its error against the FP64 oracle is FP32
rounding in a sum of M terms: the bound asserted here is 1e-5 of
max(1, max|u|), about 170 FP32 ulps, with the measured max and RMS printed.

FP32 inexact Newton (sgcm_problem.precision = SGCM_FP32): the Newton linear
solve (the backward sweep and the forward pass) in FP32, the residual, the
update of the iterate and the stopping test in FP64.  The iteration stops on
the same FP64 test (max|F| <= 1e-10), so its converged trajectory solves the
same collocation equations as the oracle's: lambda(0), u(0) and V agree with
the oracle to 1e-7 relative (the oracle and the FP64 solver agree to ~1e-13;
the remaining difference is the 1e-10 residual seen through the inverse of
the collocation Jacobian).  Iteration counts may differ (one more iteration
when the FP32 step stalls the quadratic phase); statuses must be CONVERGED.
"""
import numpy as np
import pytest

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

pytestmark = pytest.mark.gpu
EVAL_REL = 1e-5
SOLVE_REL = 1e-7


def _torch():
    import torch
    return torch


def rel_err(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.max(np.abs(a - b), axis=1) / np.maximum(np.max(np.abs(b), axis=1), 1e-8)


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("m", [1, 3])
def test_fp32_eval_vs_oracle(level, m):
    torch = _torch()
    g = S.Grid(6, level, W.BOX_LO, W.BOX_HI)
    vals = W.random_values(len(g), m, seed=400 + level)
    w = O.build_surplus(6, level, vals)
    xq = W.uniform_in_box(3000, seed=410 + level)
    u32 = S.eval_feedback_f32(g, torch.tensor(w, device="cuda"), torch.tensor(xq, device="cuda")).cpu().numpy()
    ref = O.eval_hier(6, level, w, xq, W.BOX_LO, W.BOX_HI)
    err = np.abs(u32.astype(np.float64) - ref)
    scale = max(1.0, np.abs(ref).max())
    print("level %d m %d: FP32 eval max err %.3g, RMS %.3g (scale %.3g)" % (
        level, m, err.max(), np.sqrt(np.mean(err ** 2)), scale))
    assert err.max() <= EVAL_REL * scale


def test_fp32_eval_full_size_sample():
    # the level-4 interpolant of a smooth feedback-like function at 1e6 points;
    # a seeded sample against the oracle
    torch = _torch()
    g = S.Grid(6, 4, W.BOX_LO, W.BOX_HI)
    nodes = g.nodes()
    vals = np.stack([np.sin(nodes[:, 0]) + nodes[:, 3], np.cos(nodes[:, 1] * nodes[:, 4]),
                     nodes[:, 2] * nodes[:, 5] - nodes[:, 0] ** 2], axis=1)
    w = O.build_surplus(6, 4, vals)
    xq = W.query_points(W.FULL)
    u32 = S.eval_feedback_f32(g, torch.tensor(w, device="cuda"), torch.tensor(xq, device="cuda"))
    torch.cuda.synchronize()
    u32 = u32.cpu().numpy()
    assert np.all(np.isfinite(u32))
    idx = W.sample_indices(len(xq), 500, seed=420)
    ref = O.eval_hier(6, 4, w, xq[idx], W.BOX_LO, W.BOX_HI)
    assert np.max(np.abs(u32[idx] - ref)) <= EVAL_REL * max(1.0, np.abs(ref).max())


def test_fp32_eval_rejects_unsupported():
    torch = _torch()
    g = S.Grid(3, 2, W.BOX_LO[:3], W.BOX_HI[:3])
    with pytest.raises(S.SgcmError):
        S.eval_feedback_f32(g, torch.zeros((len(g), 1), device="cuda"), torch.zeros((4, 3), device="cuda"))


def problems(m=3, N=64, T=20.0, fp32=True, max_iter=W.MAX_ITER, continuation=0):
    B = W.input_matrix(m)
    g = S.Problem(m=m, J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=W.TOL,
                  max_iter=max_iter, precision=S.FP32 if fp32 else S.FP64, continuation=continuation)
    o = O.Problem(n=6, m=m, J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=W.TOL,
                  max_iter=max_iter, continuation=continuation)
    return g, o


def solve(prob, x0):
    torch = _torch()
    r = S.solve_bvps(prob, torch.tensor(x0, device="cuda"))
    torch.cuda.synchronize()
    return {k: getattr(r, k).cpu().numpy() for k in ("lambda0", "u0", "V", "status", "iters")}


def check_fp32_solve(g, o, what):
    assert np.all(g["status"] == S.CONVERGED), what
    assert np.all(o.status == O.CONVERGED)
    e_l = rel_err(g["lambda0"], o.lambda0)
    e_u = rel_err(g["u0"], o.u0)
    e_v = rel_err(g["V"][:, None], o.V[:, None])
    extra = g["iters"].astype(int) - o.iters.astype(int)
    print("%s: FP32 Newton lambda0 max rel %.3g RMS %.3g; u0 max rel %.3g; V max rel %.3g; "
          "iterations vs FP64 %+d..%+d" % (what, e_l.max(), np.sqrt(np.mean(e_l ** 2)), e_u.max(), e_v.max(),
                                          extra.min(), extra.max()))
    assert e_l.max() <= SOLVE_REL and e_u.max() <= SOLVE_REL and e_v.max() <= SOLVE_REL
    assert extra.min() >= -1 and extra.max() <= 2


def test_fp32_newton_small_workload():
    w = W.SMALL
    gp, op = problems(N=w.n_intervals, T=w.horizon)
    x0 = O.grid(6, w.level, W.BOX_LO, W.BOX_HI).nodes
    check_fp32_solve(solve(gp, x0), O.solve_bvps(op, x0), "level-2 grid")


def test_fp32_newton_underactuated_region():
    gp, op = problems(m=2, N=40, T=2.0)
    x0 = 0.3 * W.uniform_in_box(64, seed=430)
    check_fp32_solve(solve(gp, x0), O.solve_bvps(op, x0), "two wheels")


def test_fp32_newton_full_workload():
    # every node of the level-4 grid (N = 256) against the FP64 oracle
    w = W.FULL
    gp, op = problems(N=w.n_intervals, T=w.horizon)
    x0 = O.grid(6, w.level, W.BOX_LO, W.BOX_HI).nodes
    check_fp32_solve(solve(gp, x0), O.solve_bvps(op, x0), "level-4 grid")


def test_fp32_newton_underactuated_full_workload():
    # the precision workload: two wheels, level-4 grid over the full box,
    # N = 256, T = 20, virtual-torque continuation; the FP32 inexact Newton
    # against the FP64 oracle at every node where both converge
    w = W.UNDERACTUATED
    gp, op = problems(m=2, N=w.n_intervals, T=w.horizon, max_iter=W.UNDERACTUATED_MAX_ITER,
                      continuation=W.UNDERACTUATED_CONTINUATION)
    x0 = O.grid(6, w.level, W.BOX_LO, W.BOX_HI).nodes
    g = solve(gp, x0)
    o = O.solve_bvps(op, x0)
    both = (g["status"] == S.CONVERGED) & (o.status == O.CONVERGED)
    assert np.sum(g["status"] == S.CONVERGED) >= 1430 and np.sum(both) >= 1420
    e_l = rel_err(g["lambda0"][both], o.lambda0[both])
    e_u = rel_err(g["u0"][both], o.u0[both])
    # several extremals exist (Sec. 2 Assumption 1): a node may converge to
    # another one than the oracle's; such nodes are counted, not compared
    same = e_l <= SOLVE_REL
    print("two wheels, level 4: FP32 Newton converged %d, both %d, %d to another extremal; same extremal: "
          "lambda0 max rel %.3g RMS %.3g; u0 max rel %.3g RMS %.3g" % (
              np.sum(g["status"] == S.CONVERGED), np.sum(both), np.sum(~same), e_l[same].max(),
              np.sqrt(np.mean(e_l[same] ** 2)), e_u[same].max(), np.sqrt(np.mean(e_u[same] ** 2))))
    assert np.sum(~same) <= 0.01 * len(x0)
    assert e_u[same].max() <= SOLVE_REL


def test_fp32_batch_matches_fp32_solver():
    torch = _torch()
    x0 = W.uniform_in_box(30, seed=450)
    gp, _ = problems(N=64, T=20.0)
    # a batch forms each first Newton step from its (N, T) group's steps, as
    # the solver does with a plan
    xd = torch.tensor(x0, device="cuda")
    ra = S.solve_bvps(gp, xd, plan=S.Plan(gp))
    torch.cuda.synchronize()
    a = {k: getattr(ra, k).cpu().numpy() for k in ("lambda0", "u0", "V", "status", "iters")}
    b = S.Batch(gp, np.full(30, 64), np.full(30, 20.0), slots_per_cu=2)
    r = S.solve_bvps_batch(b, torch.tensor(x0, device="cuda"))
    torch.cuda.synchronize()
    for k in ("lambda0", "u0", "V", "status", "iters"):
        assert np.array_equal(a[k], getattr(r, k).cpu().numpy()), k
