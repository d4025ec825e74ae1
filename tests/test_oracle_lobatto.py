"""Pins of the oracle's four-point Lobatto IIIA collocation (the paper's BVP
formula, Sec. 3.1 and Sec. 5.1).

* The tableau against the properties that define it: nodes 0, (5 -+ sqrt 5)/10,
  1 (the Gauss-Lobatto points), the first row zero, the collocation
  conditions sum_j a_ij c_j^(q-1) = c_i^q / q for q = 1..4, and the last row
  equal to the Lobatto quadrature weights (1, 5, 5, 1)/12, exact for
  polynomials of degree 5.
* The whole solver on the linearised model against the continuous LQR
  solution (matrix exponential of the Hamiltonian matrix): the error of
  lambda(0) and of V falls at order 6 under N -> 2N (the formula's order at the
  mesh points); the trapezoid falls at order 2 on the same problem.
* The Example III closed form (Sec. 5.3) at high order.
* Newton's iterates against a dense LU of the full collocation Jacobian, the
  Jacobian against finite differences, and the rigid-body solution against
  the trapezoid's Richardson limit.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

from test_oracle_bvp import continuous_riccati_P0, example3_exact


def linear(N, T, scheme=O.LOBATTO4, m=3):
    return O.Problem(model=O.LINEARISED, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W,
                     p_w=W.P_W, T=T, N=N, tol=W.TOL, max_iter=W.MAX_ITER, scheme=scheme)


def rigid(N, T, scheme=O.LOBATTO4, m=3, **kw):
    return O.Problem(model=O.RIGID_BODY, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m), q_w=W.Q_W, r_w=W.R_W,
                     p_w=W.P_W, T=T, N=N, tol=W.TOL, max_iter=W.MAX_ITER, scheme=scheme, **kw)


def test_tableau():
    c, A = O.lobatto_tableau()
    r5 = np.sqrt(5.0)
    assert np.allclose(c, [0.0, (5 - r5) / 10, (5 + r5) / 10, 1.0], rtol=0, atol=1e-15)
    assert np.all(A[0] == 0.0)
    for q in range(1, 5):
        assert np.allclose(A @ c ** (q - 1), c ** q / q, rtol=0, atol=1e-15), q
    assert np.allclose(A[3], np.array([1, 5, 5, 1]) / 12.0, rtol=0, atol=1e-15)
    for q in range(0, 6):
        assert abs(A[3] @ c ** q - 1.0 / (q + 1)) < 1e-15, q
    assert abs(A[3] @ c ** 6 - 1.0 / 7) > 1e-4  # and not of degree 6


def _order(errs):
    return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))


def test_linear_model_converges_at_order_six():
    T = 5.0
    x0 = W.uniform_in_box(4, seed=22)
    P0 = continuous_riccati_P0(T)
    lam_ref = x0 @ P0.T
    V_ref = 0.5 * np.einsum("bi,ij,bj->b", x0, P0, x0)
    e_l, e_v, e_t = [], [], []
    for N in (8, 16, 32):
        r = O.solve_bvps(linear(N, T), x0)
        assert np.all(r.status == O.CONVERGED) and np.all(r.iters == 0)
        e_l.append(np.max(np.abs(r.lambda0 - lam_ref)))
        e_v.append(np.max(np.abs(r.V - V_ref)))
        t = O.solve_bvps(linear(N, T, scheme=O.TRAPEZOID), x0)
        e_t.append(np.max(np.abs(t.lambda0 - lam_ref)))
    for e in (e_l, e_v):
        assert np.all(np.abs(_order(e) - 6.0) < 0.3), (e, _order(e))
    assert np.all(np.abs(_order(e_t) - 2.0) < 0.2), _order(e_t)
    assert e_l[-1] < 1e-7 * np.abs(lam_ref).max()


def test_linear_model_two_controls_order_six():
    # the underactuated linearisation (not stabilisable) is still a linear BVP
    T = 2.0
    x0 = W.uniform_in_box(3, seed=24)
    P0 = continuous_riccati_P0(T, m=2)
    lam_ref = x0 @ P0.T
    errs = [np.max(np.abs(O.solve_bvps(linear(N, T, m=2), x0).lambda0 - lam_ref)) for N in (4, 8, 16)]
    assert np.all(np.abs(_order(errs) - 6.0) < 0.4), (errs, _order(errs))


@pytest.mark.parametrize("T", [1.0, 5.0])
def test_example3_closed_form_high_order(T):
    x0 = np.random.default_rng(31).uniform(-2.0, 2.0, (6, 3))
    V_ref, u_ref, g_ref = example3_exact(x0, T)
    e_l, e_u, e_v = [], [], []
    for N in (16, 32, 64):
        p = O.Problem(model=O.EXAMPLE3, n=3, m=1, T=T, N=N, tol=1e-12, max_iter=30, scheme=O.LOBATTO4)
        r = O.solve_bvps(p, x0)
        assert np.all(r.status == O.CONVERGED)
        e_l.append(np.max(np.abs(r.lambda0 - g_ref)))
        e_u.append(np.max(np.abs(r.u0[:, 0] - u_ref)))
        e_v.append(np.max(np.abs(r.V - V_ref)))
    for e in (e_l, e_u, e_v):
        assert np.all(_order(e) > 5.0), (e, _order(e))
    assert e_l[-1] < 1e-7 and e_u[-1] < 1e-7


def test_newton_iterates_match_dense_lu():
    p = rigid(4, 2.0)
    x0 = W.uniform_in_box(3, seed=52)
    r = O.solve_bvps(p, x0, want_unknowns=True)
    dim = O.collocation_dim(p)
    assert dim == 12 * (3 * 4 + 1)
    for b in range(3):
        Y = np.zeros(dim)
        its = -1
        while True:
            F = O.residual(p, x0[b], Y)[0]
            if its >= 0 and np.max(np.abs(F)) <= p.tol:
                break
            Y = Y + np.linalg.solve(O.jacobian_dense(p, Y), -F)
            its += 1
        assert its == r.iters[b]
        assert np.max(np.abs(Y - r.unknowns[b])) < 1e-12 * np.abs(Y).max()


def test_jacobian_matches_finite_differences():
    p = rigid(3, 1.0)
    dim = O.collocation_dim(p)
    Y = np.random.default_rng(62).uniform(-0.5, 0.5, dim)
    x0 = np.zeros(6)
    Jd = O.jacobian_dense(p, Y)
    eps = 1e-6
    for j in range(0, dim, 5):
        e = np.zeros_like(Y)
        e[j] = eps
        col = (O.residual(p, x0, Y + e)[0] - O.residual(p, x0, Y - e)[0]) / (2 * eps)
        assert np.max(np.abs(col - Jd[:, j])) < 1e-7


def test_rigid_body_agrees_with_the_trapezoid_limit():
    # T = 20, three wheels: Lobatto on 64 intervals against the Richardson
    # extrapolation (4 y_2N - y_N) / 3 of the trapezoid on 512 and 1024
    # intervals (error O(h^4) ~ 1e-7); the trapezoid on 64 intervals alone is
    # off by ~1e-2
    x0 = W.uniform_in_box(3, seed=53)
    lob = O.solve_bvps(rigid(64, 20.0), x0)
    t1 = O.solve_bvps(rigid(512, 20.0, scheme=O.TRAPEZOID), x0)
    t2 = O.solve_bvps(rigid(1024, 20.0, scheme=O.TRAPEZOID), x0)
    t64 = O.solve_bvps(rigid(64, 20.0, scheme=O.TRAPEZOID), x0)
    ref = (4 * t2.lambda0 - t1.lambda0) / 3
    assert np.all(lob.status == O.CONVERGED)
    assert np.max(np.abs(lob.lambda0 - ref)) < 1e-5 * np.abs(ref).max()
    assert np.max(np.abs(t64.lambda0 - ref)) > 1e-4 * np.abs(ref).max()
    Vref = (4 * t2.V - t1.V) / 3
    assert np.max(np.abs(lob.V - Vref)) < 1e-5 * np.abs(Vref).max()


def test_status_rules_and_mesh_output():
    p = rigid(16, 2.0)
    x0 = np.vstack([np.zeros(6), W.uniform_in_box(3, seed=82)])
    r = O.solve_bvps(p, x0, want_traj=True, want_unknowns=True)
    assert r.status[0] == O.CONVERGED and r.iters[0] == 0
    assert np.all(r.status == O.CONVERGED)
    # the trajectory is the mesh values: every third point of the unknowns
    U = r.unknowns.reshape(4, 3 * 16 + 1, 12)
    assert np.array_equal(r.traj, U[:, ::3])
    xn = x0[1:2].copy()
    xn[0, 1] = np.nan
    rn = O.solve_bvps(p, xn)
    assert rn.status[0] == O.NONFINITE and rn.iters[0] == 0
