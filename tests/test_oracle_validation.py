"""Pins of the oracle's Monte Carlo total-error estimate (Sec. 4.3).

* the statistics on a hand-computed example (values derived from the
  definitions, all exactly representable);
* NaN propagation and the empty sample;
* the Richardson reference on the linearised model against the continuous
  LQR solution (Riccati closed form through the Hamiltonian matrix
  exponential): its error falls at order 4 in h, while the solutions it is
  formed from converge at order 2 (a wrong extrapolation weight leaves order 2);
* the whole estimate on the linearised model, where V is quadratic and u is
  linear in x, so a level-2 Smolyak interpolant is exact and the estimated
  total error must equal the node solutions' discretisation error, computed
  directly against the closed form.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_1507_04769_amd import workloads as W


def linear(N, T, m=3):
    return O.Problem(model=O.LINEARISED, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W,
                     p_w=W.P_W, T=T, N=N, tol=W.TOL, max_iter=W.MAX_ITER)


def lqr_P0(T, m=3):
    # y = (x, lambda) obeys y' = H y with H the Hamiltonian matrix of the
    # linearised problem; lambda(T) = p_w x(T) gives lambda(0) = P0 x(0)
    J = np.array(W.J_DIAG)
    A = np.zeros((6, 6))
    A[:3, 3:] = np.eye(3)
    Bt = np.zeros((6, m))
    Bt[3:, :] = W.input_matrix(m) / J[:, None]
    H = np.block([[A, -Bt @ Bt.T / W.R_W], [-W.Q_W * np.eye(6), -A.T]])
    D = scipy.linalg.expm(-T * H) @ np.vstack([np.eye(6), W.P_W * np.eye(6)])
    return D[6:] @ np.linalg.inv(D[:6])


def test_total_error_hand_example():
    coarse = np.array([[2.0, 1.0], [0.5, -1.0]])
    fine = np.array([[1.25, 2.5], [0.5, -1.75]])
    interp = np.array([[1.5, 2.75], [0.5, -2.125]])
    ref, err, stats = O.total_error(interp, coarse, fine)
    # (4 * 1.25 - 2) / 3 = 1, (4 * 2.5 - 1) / 3 = 3, (2 - 0.5) / 3 = 0.5, (-7 + 1) / 3 = -2
    assert np.array_equal(ref, [[1.0, 3.0], [0.5, -2.0]])
    # |interp - ref| = [[0.5, 0.25], [0, 0.125]]
    assert np.array_equal(err, [0.5, 0.125])
    # |fine - ref| = [[0.25, 0.5], [0, 0.25]]
    assert stats[0] == 0.5 and stats[2] == 0.5
    assert stats[1] == np.sqrt((0.25 + 0.015625) / 2)
    # the mean absolute error and the mean relative error (max |ref| per row: 3, 2)
    assert stats[3] == (0.5 + 0.125) / 2
    assert stats[4] == (0.5 / 3.0 + 0.125 / 2.0) / 2
    # order 6: (64 fine - coarse) / 63
    ref6, _, _ = O.total_error(interp, coarse, fine, order=6)
    assert np.array_equal(ref6, (64.0 * fine - coarse) / 63.0)


def test_total_error_nan_and_empty():
    a = np.zeros((3, 2))
    interp = a.copy()
    interp[1, 1] = np.nan
    ref, err, stats = O.total_error(interp, a, a)
    assert err[0] == 0.0 and np.isnan(err[1]) and err[2] == 0.0
    assert np.isnan(stats[0]) and np.isnan(stats[1]) and stats[2] == 0.0
    ref, err, stats = O.total_error(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)))
    assert ref.shape == (0, 3) and err.shape == (0,) and np.array_equal(stats, np.zeros(5))


def test_richardson_reference_is_fourth_order_on_linear_model():
    T = 5.0
    x = W.uniform_in_box(4, seed=31)
    P0 = lqr_P0(T)
    lam_ex = x @ P0.T
    V_ex = 0.5 * np.einsum("bi,ij,bj->b", x, P0, x)
    e_ref_lam, e_ref_V, e_fine_lam = [], [], []
    for N in (16, 32, 64):
        c = O.solve_bvps(linear(N, T), x)
        f = O.solve_bvps(linear(2 * N, T), x)
        assert np.all(c.status == O.CONVERGED) and np.all(f.status == O.CONVERGED)
        ref, _, stats = O.total_error(np.zeros_like(c.lambda0), c.lambda0, f.lambda0)
        refV, _, _ = O.total_error(np.zeros((len(x), 1)), c.V[:, None], f.V[:, None])
        e_ref_lam.append(np.abs(ref - lam_ex).max())
        e_ref_V.append(np.abs(refV[:, 0] - V_ex).max())
        e_fine_lam.append(np.abs(f.lambda0 - lam_ex).max())
        # the correction |fine - ref| is the fine solution's error, to leading order
        assert abs(stats[2] / e_fine_lam[-1] - 1.0) < 0.05
    for e in (e_ref_lam, e_ref_V):
        orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(orders - 4.0) < 0.3), orders
    orders = np.log2(np.array(e_fine_lam[:-1]) / np.array(e_fine_lam[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.1), orders
    assert e_ref_lam[1] < 1e-2 * e_fine_lam[1]


def test_lobatto_reference_on_linear_model():
    # the four-point Lobatto IIIA solutions on N and 2N intervals, extrapolated
    # at order 6: the reference is far more accurate than the fine solution,
    # whose error the correction |fine - ref| estimates (order 6 in h)
    T = 5.0
    x = W.uniform_in_box(4, seed=33)
    lam_ex = x @ lqr_P0(T).T
    e_ref, e_fine = [], []
    for N in (4, 8, 16):
        c = O.solve_bvps(O.Problem(**{**linear(N, T).__dict__, "scheme": O.LOBATTO4}), x)
        f = O.solve_bvps(O.Problem(**{**linear(2 * N, T).__dict__, "scheme": O.LOBATTO4}), x)
        ref, _, stats = O.total_error(np.zeros_like(c.lambda0), c.lambda0, f.lambda0, order=6)
        e_ref.append(np.abs(ref - lam_ex).max())
        e_fine.append(np.abs(f.lambda0 - lam_ex).max())
        assert abs(stats[2] / e_fine[-1] - 1.0) < 0.1
    orders = np.log2(np.array(e_fine[:-1]) / np.array(e_fine[1:]))
    assert np.all(np.abs(orders - 6.0) < 0.3), orders
    assert np.all(np.array(e_ref) < 0.05 * np.array(e_fine))


@pytest.mark.parametrize("level", [2, 3])
def test_estimate_equals_node_discretisation_error_on_linear_model(level):
    # nodes solved on 16 intervals (a large discretisation error), reference
    # from 64 and 128 intervals; V quadratic and u linear in x are reproduced
    # exactly by the Smolyak interpolant, so e_interp vanishes to rounding
    T, N = 5.0, 16
    g = O.grid(6, level, W.BOX_LO, W.BOX_HI)
    nodes = g.nodes
    sol = O.solve_bvps(linear(N, T), nodes)
    w_u = O.build_surplus(6, level, sol.u0)
    w_V = O.build_surplus(6, level, sol.V[:, None])
    x = W.uniform_in_box(40, seed=32)
    u_int = O.eval_hier(6, level, w_u, x, W.BOX_LO, W.BOX_HI)
    V_int = O.eval_hier(6, level, w_V, x, W.BOX_LO, W.BOX_HI)
    c = O.solve_bvps(linear(64, T), x)
    f = O.solve_bvps(linear(128, T), x)
    _, err_u, st_u = O.total_error(u_int, c.u0, f.u0)
    _, err_V, st_V = O.total_error(V_int, c.V[:, None], f.V[:, None])
    # the node solutions' own error at x, against the closed form
    at_x = O.solve_bvps(linear(N, T), x)
    P0 = lqr_P0(T)
    V_ex = 0.5 * np.einsum("bi,ij,bj->b", x, P0, x)
    e_bvp_V = np.abs(at_x.V - V_ex)
    assert np.max(np.abs(err_V - e_bvp_V)) < 1e-3 * e_bvp_V.max()
    # the fine reference mesh has 8 times the nodes' intervals, so the
    # correction (the fine solution's error) is about 1/64 of what is measured
    assert st_V[2] < st_V[0] / 32
    # the interpolated feedback equals the solve at x up to rounding: the
    # estimate is the discretisation error of u on 16 intervals
    assert np.max(np.abs(u_int - at_x.u0)) < 1e-11 * np.abs(at_x.u0).max()
    assert np.max(np.abs(err_u - np.max(np.abs(at_x.u0 - (4 * f.u0 - c.u0) / 3), axis=1))) < 1e-11
