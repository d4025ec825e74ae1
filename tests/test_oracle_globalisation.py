"""Pins of the oracle's globalisation of Newton's iteration (Sec. 2
Assumption 1 asks only that the characteristic BVP have a solution; the paper
fixes no solver internals).

The rule under test, written out again here from its statement and run on the
dense Jacobian of the collocation system (a different linear algebra from the
oracle's banded LU):
* each counted Newton step d is damped by backtracking: trials Y + t d for
  t = 1, 1/2, ..., 2^-H; the first with a finite residual and
  max|F(Y + t d)| <= (1 - 1e-4 t) max|F(Y)| is taken, else t = 2^-H;
* for two controls with continuation K > 0: stages k = 0..K-1 solve the
  three-control problem with B_k = [B_1 B_2 s_k b3], s_k = 1 - k/K and
  b3 = B_1 x B_2 / |B_1 x B_2|, the first from Y = 0 with the uncounted
  linearised step, each later stage and the final two-control stage from the
  previous solution; the status is the last stage's, the iterations are
  summed.
Pinned further by: the full-size three-wheel workload keeps the undamped
iteration counts (the full step always passes there); where undamped Newton
converges the damped iteration and the continuation reach the same solution;
and the continuation's two-wheel solutions equal single shooting with the
implicit trapezoid on the sympy right-hand side.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

from test_oracle_bvp import shooting

SIGMA = 1e-4


def rigid(m=3, N=16, T=2.0, **kw):
    kw.setdefault("max_iter", W.MAX_ITER)
    return O.Problem(model=O.RIGID_BODY, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m),
                     q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=W.TOL, **kw)


def damped_newton(p, x0, Y=None):
    """The damped iteration by hand on the dense Jacobian.  Returns (status,
    iterations, Y, number of steps shorter than the full step)."""
    dim = 12 * (p.N + 1)
    short = 0
    if Y is None:  # the first, uncounted step from Y = 0
        Y = np.zeros(dim)
        Y = Y + np.linalg.solve(O.jacobian_dense(p, Y), -O.residual(p, x0, Y)[0])
    Y = Y.copy()
    it = 0
    while True:
        F = O.residual(p, x0, Y)[0]
        if not np.all(np.isfinite(F)):
            return O.NONFINITE, it, Y, short
        fn = np.max(np.abs(F))
        if fn <= p.tol:
            return O.CONVERGED, it, Y, short
        if it == p.max_iter:
            return O.MAXITER, it, Y, short
        d = np.linalg.solve(O.jacobian_dense(p, Y), -F)
        t = 1.0
        for j in range(p.max_halvings + 1):
            Yt = Y + t * d
            if j == p.max_halvings:
                break
            Ft = O.residual(p, x0, Yt)[0]
            if np.all(np.isfinite(Ft)) and np.max(np.abs(Ft)) <= (1.0 - SIGMA * t) * fn:
                break
            t *= 0.5
        short += t < 1.0
        Y = Yt
        it += 1


def continuation_by_hand(p, x0):
    B = np.asarray(p.B).reshape(3, 2)
    b3 = np.cross(B[:, 0], B[:, 1])
    b3 = b3 / np.linalg.norm(b3)
    Y, total, short = None, 0, 0
    for k in range(p.continuation + 1):
        if k < p.continuation:
            s = 1.0 - k / p.continuation
            q = O.Problem(model=p.model, n=6, m=3, J=p.J, B=np.column_stack([B, s * b3]), q_w=p.q_w,
                          r_w=p.r_w, p_w=p.p_w, T=p.T, N=p.N, tol=p.tol, max_iter=p.max_iter,
                          max_halvings=p.max_halvings)
        else:
            q = O.Problem(model=p.model, n=6, m=2, J=p.J, B=B, q_w=p.q_w, r_w=p.r_w, p_w=p.p_w, T=p.T,
                          N=p.N, tol=p.tol, max_iter=p.max_iter, max_halvings=p.max_halvings)
        st, it, Y, sh = damped_newton(q, x0, Y)
        total += it
        short += sh
        if st != O.CONVERGED:
            break
    return st, total, Y, short


def test_damped_iteration_matches_rule_by_hand():
    # two wheels, T = 5, N = 8 over the full box: the full step fails the
    # decrease test on some iterations (checked), and the oracle's iterates
    # follow the rule step for step
    p = rigid(m=2, N=8, T=5.0, max_iter=40)
    x0 = W.uniform_in_box(6, seed=901)
    r = O.solve_bvps(p, x0, want_traj=True)
    shortened = 0
    for b in range(len(x0)):
        st, it, Y, short = damped_newton(p, x0[b])
        shortened += short
        assert st == r.status[b] and it == r.iters[b], (b, st, it, r.status[b], r.iters[b])
        if st == O.CONVERGED:
            assert np.max(np.abs(Y - r.traj[b].reshape(-1))) <= 1e-9 * max(1.0, np.abs(Y).max())
    assert shortened > 0


def test_cap_zero_is_plain_newton():
    # H = 0 takes every full step: the undamped iteration, whatever the decrease
    p0 = rigid(m=2, N=8, T=5.0, max_iter=12, max_halvings=0)
    x0 = W.uniform_in_box(4, seed=902)
    r = O.solve_bvps(p0, x0, want_traj=True)
    for b in range(len(x0)):
        Y = np.zeros(12 * 9)
        Y = Y + np.linalg.solve(O.jacobian_dense(p0, Y), -O.residual(p0, x0[b], Y)[0])
        it = 0
        while True:
            F = O.residual(p0, x0[b], Y)[0]
            if not np.all(np.isfinite(F)) or np.max(np.abs(F)) <= p0.tol or it == p0.max_iter:
                break
            Y = Y + np.linalg.solve(O.jacobian_dense(p0, Y), -F)
            it += 1
        assert it == r.iters[b]


def test_full_step_kept_on_the_three_wheel_workload():
    # level-4 grid, N = 256, T = 20: the damping never shortens a step, so
    # the iteration counts are those of the undamped iteration
    g = O.grid(6, W.FULL.level, W.BOX_LO, W.BOX_HI)
    r = O.solve_bvps(rigid(N=W.FULL.n_intervals, T=W.FULL.horizon), g.nodes)
    assert np.all(r.status == O.CONVERGED)
    assert np.bincount(r.iters).tolist() == [193, 0, 180, 944, 140]


def test_damping_and_continuation_keep_converging_solutions():
    # where undamped Newton converges (two wheels, 0.3 x box, T = 2) the
    # damped iteration and the continuation reach the same discrete solution
    x0 = 0.3 * W.uniform_in_box(8, seed=903)
    plain = O.solve_bvps(rigid(m=2, N=24, T=2.0, max_halvings=0), x0, want_traj=True)
    damped = O.solve_bvps(rigid(m=2, N=24, T=2.0), x0, want_traj=True)
    cont = O.solve_bvps(rigid(m=2, N=24, T=2.0, continuation=4), x0, want_traj=True)
    assert np.all(plain.status == O.CONVERGED) and np.all(cont.status == O.CONVERGED)
    assert np.array_equal(plain.iters, damped.iters)
    scale = np.abs(plain.traj).max()
    assert np.max(np.abs(damped.traj - plain.traj)) <= 1e-12 * scale
    assert np.max(np.abs(cont.traj - plain.traj)) <= 1e-9 * scale


def test_continuation_matches_rule_by_hand():
    p = rigid(m=2, N=8, T=5.0, max_iter=40, continuation=3)
    x0 = W.uniform_in_box(5, seed=904)
    r = O.solve_bvps(p, x0, want_traj=True)
    for b in range(len(x0)):
        st, it, Y, _ = continuation_by_hand(p, x0[b])
        assert st == r.status[b] and it == r.iters[b], (b, st, it, r.status[b], r.iters[b])
        if st == O.CONVERGED:
            assert np.max(np.abs(Y - r.traj[b].reshape(-1))) <= 1e-9 * max(1.0, np.abs(Y).max())


def test_continuation_solution_equals_trapezoid_shooting():
    # full box, two wheels, T = 2, N = 16: the converged continuation solves
    # the same discrete equations that single shooting solves (shooting's own
    # Newton starts 1e-2 away from the continuation's lambda(0): from 0 it
    # diverges on these states)
    p = rigid(m=2, N=16, T=2.0, max_iter=60, continuation=4)
    x0 = W.uniform_in_box(3, seed=905)
    r = O.solve_bvps(p, x0, want_traj=True)
    assert np.all(r.status == O.CONVERGED)
    for b in range(len(x0)):
        ys = shooting("rigid", 2, x0[b], 16, 2.0, l0=r.lambda0[b] + 1e-2)
        assert np.max(np.abs(ys - r.traj[b])) < 1e-10 * max(1, np.abs(ys).max())


def test_continuation_reaches_the_underactuated_full_box():
    # level-2 grid over the full box, two wheels, N = 64, T = 20: undamped
    # Newton from the linearised step converges at a handful of nodes; the
    # continuation (K = 4, at most 100 iterations per stage) at all but one
    g = O.grid(6, 2, W.BOX_LO, W.BOX_HI)
    plain = O.solve_bvps(rigid(m=2, N=64, T=20.0, max_halvings=0), g.nodes)
    cont = O.solve_bvps(rigid(m=2, N=64, T=20.0, max_iter=100, continuation=4), g.nodes)
    assert np.sum(plain.status == O.CONVERGED) <= 10
    assert np.sum(cont.status == O.CONVERGED) >= 84
    assert np.all(cont.status[cont.status != O.CONVERGED] == O.MAXITER)


def test_continuation_ignored_for_three_controls():
    x0 = W.uniform_in_box(3, seed=906)
    a = O.solve_bvps(rigid(N=16, T=2.0), x0, want_traj=True)
    b = O.solve_bvps(rigid(N=16, T=2.0, continuation=4), x0, want_traj=True)
    assert np.array_equal(a.traj, b.traj) and np.array_equal(a.iters, b.iters)
