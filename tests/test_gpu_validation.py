"""Monte Carlo total-error estimate (Sec. 4.3) on the GPU against the oracle.

* sgcm_total_error against oracle.total_error on seeded inputs: the reference
  and the per-sample errors bit for bit (the same correctly rounded
  operations), the maxima exactly, the RMS to rounding; sizes from empty to
  several passes of the 1024-thread workgroup with a ragged tail; NaN rows.
* The whole estimate (reference solves, interpolant evaluation, comparison)
  against the oracle's pipeline on the same inputs: level-2 grid, nodes on 64
  intervals, 96 random states; the trapezoidal reference on meshes 64 and
  128, and the error-controlled four-point Lobatto IIIA reference (meshes
  doubled from 16 until the correction is within 1e-7, the same doubling
  replayed on the oracle).
* The estimate at full size (level-4 grid from 256-interval node solves, 1280
  random states, the error-controlled Lobatto reference): every reference
  solve converges, the reference's estimated error is within its tolerance
  and far below the error it measures, and a sample of states is checked
  against the oracle one by one.
"""
import dataclasses

import numpy as np
import pytest
import torch

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import validation as VA
from paper_1507_04769_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("order", [2, 6])
@pytest.mark.parametrize("n,m", [(0, 3), (1, 1), (1000, 3), (1024, 1), (3001, 3), (5000, 2), (700, 64)])
def test_total_error_kernel_matches_oracle(n, m, order):
    g = np.random.default_rng(700 + n + m)
    fine = g.standard_normal((n, m))
    coarse = fine + 1e-3 * g.standard_normal((n, m))
    interp = fine + 1e-2 * g.standard_normal((n, m))
    ref, err, stats = S.total_error(gpu(interp), gpu(coarse), gpu(fine), order=order)
    o_ref, o_err, o_stats = O.total_error(interp, coarse, fine, order=order)
    assert np.array_equal(ref.cpu().numpy(), o_ref)
    assert np.array_equal(err.cpu().numpy(), o_err)
    st = stats.cpu().numpy()
    assert st[0] == o_stats[0] and st[2] == o_stats[2]
    for k in (1, 3, 4):  # sums: equal to rounding of the summation order
        assert abs(st[k] - o_stats[k]) <= 1e-14 * max(o_stats[k], 1e-300), k


def test_total_error_kernel_nan_rows():
    g = np.random.default_rng(710)
    n, m = 2500, 3
    fine = g.standard_normal((n, m))
    coarse = fine.copy()
    interp = fine + 1e-2 * g.standard_normal((n, m))
    interp[7, 1] = np.nan
    coarse[2049, 0] = np.nan
    ref, err, stats = S.total_error(gpu(interp), gpu(coarse), gpu(fine))
    o_ref, o_err, o_stats = O.total_error(interp, coarse, fine)
    e = err.cpu().numpy()
    assert np.array_equal(np.isnan(e), np.isnan(o_err)) and np.isnan(e[7]) and np.isnan(e[2049])
    assert np.array_equal(e[~np.isnan(e)], o_err[~np.isnan(o_err)])
    assert np.all(np.isnan(stats.cpu().numpy()))


def problem(N, T=20.0, m=3):
    return S.Problem(m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N,
                     tol=W.TOL, max_iter=W.MAX_ITER)


def oracle_problem(N, T=20.0, m=3, scheme=O.TRAPEZOID):
    return O.Problem(n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N,
                     tol=W.TOL, max_iter=W.MAX_ITER, scheme=scheme)


def oracle_lobatto_reference(xs, n_ref, tol=VA.REF_TOL, max_ref=VA.MAX_REF):
    """The error-controlled Lobatto reference replayed on the oracle:
    (N_r, coarse, fine)."""
    n_r = n_ref
    c = O.solve_bvps(oracle_problem(n_r, scheme=O.LOBATTO4), xs)
    while True:
        f = O.solve_bvps(oracle_problem(2 * n_r, scheme=O.LOBATTO4), xs)
        corr = max(O.total_error(np.zeros_like(c.u0), c.u0, f.u0, order=6)[2][2],
                   O.total_error(np.zeros((len(xs), 1)), c.V[:, None], f.V[:, None], order=6)[2][2])
        if corr <= tol or 4 * n_r > max_ref:
            return n_r, c, f
        n_r *= 2
        c = f


def device_interpolants(level, N):
    grid = S.Grid(6, level, W.BOX_LO, W.BOX_HI)
    nodes = grid.nodes()
    sol = S.solve_bvps(problem(N), gpu(nodes))
    w_u = S.build_interpolant(grid, sol.u0)
    w_V = S.build_interpolant(grid, sol.V.view(-1, 1).contiguous())
    return grid, nodes, sol, w_u, w_V


def test_estimate_matches_oracle_pipeline():
    level, N, n_ref = 2, 64, 64
    grid, nodes, sol, w_u, w_V = device_interpolants(level, N)
    xs = W.uniform_in_box(96, seed=711)
    est = VA.Estimator(problem(N), n_ref, scheme=S.TRAPEZOID)
    r = est(grid, w_u, gpu(xs), w_V)
    # the oracle's pipeline on the same inputs
    o_sol = O.solve_bvps(oracle_problem(N), nodes)
    o_wu = O.build_surplus(6, level, o_sol.u0)
    o_wV = O.build_surplus(6, level, o_sol.V[:, None])
    o_uint = O.eval_hier(6, level, o_wu, xs, W.BOX_LO, W.BOX_HI)
    o_Vint = O.eval_hier(6, level, o_wV, xs, W.BOX_LO, W.BOX_HI)
    oc = O.solve_bvps(oracle_problem(n_ref), xs)
    of = O.solve_bvps(oracle_problem(2 * n_ref), xs)
    assert np.array_equal(r.status.cpu().numpy(), np.stack([oc.status, of.status]))
    assert np.array_equal(r.iters.cpu().numpy(), np.stack([oc.iters, of.iters]))
    for (ref, err, stats), (intp, c, f) in (((r.ref_u, r.err_u, r.stats_u), (o_uint, oc.u0, of.u0)),
                                            ((r.ref_V, r.err_V, r.stats_V), (o_Vint, oc.V[:, None], of.V[:, None]))):
        o_ref, o_err, o_stats = O.total_error(intp, c, f)
        scale = np.abs(o_ref).max()
        assert np.max(np.abs(ref.cpu().numpy() - o_ref)) <= 1e-8 * scale
        # errors are differences of values that agree to 1e-8 of their scale
        assert np.max(np.abs(err.cpu().numpy() - o_err)) <= 2e-8 * scale
        assert np.max(np.abs(stats.cpu().numpy() - o_stats)) <= 2e-8 * scale


def test_lobatto_estimate_matches_oracle_pipeline():
    level, N = 2, 64
    grid, nodes, sol, w_u, w_V = device_interpolants(level, N)
    xs = W.uniform_in_box(96, seed=715)
    r = VA.Estimator(problem(N), 16)(grid, w_u, gpu(xs), w_V)
    o_sol = O.solve_bvps(oracle_problem(N), nodes)
    o_uint = O.eval_hier(6, level, O.build_surplus(6, level, o_sol.u0), xs, W.BOX_LO, W.BOX_HI)
    o_Vint = O.eval_hier(6, level, O.build_surplus(6, level, o_sol.V[:, None]), xs, W.BOX_LO, W.BOX_HI)
    n_r, oc, of = oracle_lobatto_reference(xs, 16)
    assert r.n_ref == n_r and n_r > 16  # the doubling went at least once
    assert np.array_equal(r.status.cpu().numpy(), np.stack([oc.status, of.status]))
    assert np.array_equal(r.iters.cpu().numpy(), np.stack([oc.iters, of.iters]))
    for (ref, err, stats), (intp, c, f) in (((r.ref_u, r.err_u, r.stats_u), (o_uint, oc.u0, of.u0)),
                                            ((r.ref_V, r.err_V, r.stats_V), (o_Vint, oc.V[:, None], of.V[:, None]))):
        o_ref, o_err, o_stats = O.total_error(intp, c, f, order=6)
        scale = np.abs(o_ref).max()
        assert np.max(np.abs(ref.cpu().numpy() - o_ref)) <= 1e-8 * scale
        assert np.max(np.abs(err.cpu().numpy() - o_err)) <= 2e-8 * scale
        assert np.max(np.abs(stats.cpu().numpy()[[0, 1, 3]] - o_stats[[0, 1, 3]])) <= 2e-8 * scale
        assert abs(stats.cpu().numpy()[4] - o_stats[4]) <= 1e-6 * o_stats[4]
    assert r.correction <= VA.REF_TOL


def test_estimate_at_full_size_with_sampled_oracle_checks():
    level, N = W.FULL.level, W.FULL.n_intervals
    grid, nodes, sol, w_u, w_V = device_interpolants(level, N)
    xs = W.uniform_in_box(VA.N_SAMPLES, seed=VA.SAMPLE_SEED)
    r = VA.Estimator(problem(N), 64)(grid, w_u, gpu(xs), w_V)
    assert np.all(r.status.cpu().numpy() == S.CONVERGED)
    su, sV = r.stats_u.cpu().numpy(), r.stats_V.cpu().numpy()
    assert np.all(np.isfinite(su)) and np.all(np.isfinite(sV))
    # the reference's estimated error is within its tolerance and orders of
    # magnitude below the error being measured (the paper: at least three)
    assert r.correction <= VA.REF_TOL
    assert su[2] < su[3] / 1000 and sV[2] < sV[3] / 1000
    # sampled states, one by one through the oracle: the reference solves on
    # the accepted meshes and the interpolant of the device surplus
    pick = W.sample_indices(VA.N_SAMPLES, 4, seed=713)
    oc = O.solve_bvps(oracle_problem(r.n_ref, scheme=O.LOBATTO4), xs[pick])
    of = O.solve_bvps(oracle_problem(2 * r.n_ref, scheme=O.LOBATTO4), xs[pick])
    o_uint = O.eval_hier(6, level, w_u.cpu().numpy(), xs[pick], W.BOX_LO, W.BOX_HI)
    o_ref, o_err, _ = O.total_error(o_uint, oc.u0, of.u0, order=6)
    scale = np.abs(o_ref).max()
    assert np.max(np.abs(r.ref_u.cpu().numpy()[pick] - o_ref)) <= 1e-8 * scale
    assert np.max(np.abs(r.err_u.cpu().numpy()[pick] - o_err)) <= 2e-8 * scale


@pytest.mark.parametrize("n", [0, 1])
def test_estimate_empty_and_single_sample(n):
    level, N = 2, 64
    grid, nodes, sol, w_u, w_V = device_interpolants(level, N)
    xs = W.uniform_in_box(max(n, 1), seed=714)[:n]
    r = VA.Estimator(problem(N), 32)(grid, w_u, gpu(xs).reshape(n, 6), w_V)
    assert r.err_u.shape == (n,) and r.ref_u.shape == (n, 3) and r.err_V.shape == (n,)
    su = r.stats_u.cpu().numpy()
    if n == 0:
        assert np.array_equal(su, np.zeros(5)) and np.array_equal(r.stats_V.cpu().numpy(), np.zeros(5))
    else:
        # one sample: the max and the RMS are its error
        e = r.err_u.cpu().numpy()[0]
        assert su[0] == e and abs(su[1] - e) <= 1e-15 * e


def test_estimator_refuses_non_converged_references():
    # a reference solve that stops at max_iter is no reference: the estimator
    # raises SGCM_ENOTCONVERGED instead of reporting statistics from it
    grid, nodes, sol, w_u, w_V = device_interpolants(2, 64)
    xs = W.uniform_in_box(32, seed=712)
    p = dataclasses.replace(problem(64), max_iter=0)
    for scheme in (S.TRAPEZOID, S.LOBATTO4):
        est = VA.Estimator(p, 32, scheme=scheme, max_ref=128)
        with pytest.raises(S.SgcmError) as e:
            est(grid, w_u, gpu(xs), w_V)
        assert e.value.code == S.SGCM_ENOTCONVERGED
