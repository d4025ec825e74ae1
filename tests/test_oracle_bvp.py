"""Pins of the oracle's characteristic BVP solver (Sec. 2 and 3.1).

What each test pins, and against what:
* the rigid-body kinematics E(v) against the definition of body angular
  velocity for (3,2,1) Euler angles (R = Rz(psi) Ry(theta) Rx(phi),
  R' = R [w]x) and the gyroscopic term against conservation of kinetic energy
  and angular-momentum magnitude;
* u* = argmin H and the characteristic right-hand side Phi with its Jacobian
  against sympy derivations written from the definitions (partials of H at
  fixed u, then u* substituted, then differentiated);
* the whole solver on the linearised model against the exact discrete Riccati
  recursion of the trapezoidal rule and, at O(h^2), against the continuous
  LQR solution (matrix exponential of the Hamiltonian matrix);
* the nonlinear solver against the closed-form solution of Example III
  (Sec. 5.3) at O(h^2);
* the nonlinear solver against single shooting with the implicit trapezoid
  on the sympy right-hand side (a different algorithm reaching the same
  discrete solution), and against Newton with a dense LU of the full Jacobian;
* the status rules (non-finite input, iteration cap, zero tolerance).
"""
import functools

import numpy as np
import pytest
import scipy.linalg
import sympy as sp

from oracle import oracle as O
from paper_1507_04769_amd import workloads as W


def rigid(m=3, N=16, T=2.0, **kw):
    return O.Problem(model=O.RIGID_BODY, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m),
                     q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=W.TOL,
                     max_iter=W.MAX_ITER, **kw)


def linear(m=3, N=64, T=20.0):
    return O.Problem(model=O.LINEARISED, n=6, m=m, J=W.J_DIAG, B=W.input_matrix(m),
                     q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=W.TOL, max_iter=W.MAX_ITER)


def example3(N=64, T=1.0):
    return O.Problem(model=O.EXAMPLE3, n=3, m=1, T=T, N=N, tol=1e-12, max_iter=30)


# ---------------------------------------------------------------------------
# sympy derivations, written from the definitions in Sec. 2 / 3.1
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def sympy_model(kind, m):
    if kind == "example3":
        n, m = 3, 1
    else:
        n = 6
    x = sp.symbols("x0:%d" % n, real=True)
    lam = sp.symbols("l0:%d" % n, real=True)
    u = sp.symbols("u0:%d" % m, real=True)
    if kind == "example3":
        s = 1 + x[0] ** 2 + x[1] ** 2
        f = [-x[0] + x[1], -x[1] + x[2] / s,
             (-2 * x[0] ** 2 + 2 * x[0] * x[1] - 2 * x[1] ** 2 + 2 * x[1] * x[2] / s) * x[2] / s
             + s * u[0]]
        L = sp.Rational(1, 2) * (x[2] ** 2 / s ** 2 + u[0] ** 2)
    else:
        J = [sp.nsimplify(j) for j in W.J_DIAG]
        B = sp.Matrix(W.input_matrix(m))
        Bu = B * sp.Matrix(u)
        w = sp.Matrix(x[3:6])
        Jw = sp.Matrix([J[0] * w[0], J[1] * w[1], J[2] * w[2]])
        gyro = w.cross(Jw)
        phi, th = x[0], x[1]
        if kind == "rigid":
            E = sp.Matrix([[1, sp.sin(phi) * sp.tan(th), sp.cos(phi) * sp.tan(th)],
                           [0, sp.cos(phi), -sp.sin(phi)],
                           [0, sp.sin(phi) / sp.cos(th), sp.cos(phi) / sp.cos(th)]])
            vdot = E * w
            wdot = [(Bu[i] - gyro[i]) / J[i] for i in range(3)]
        else:  # linearised about the origin
            vdot = w
            wdot = [Bu[i] / J[i] for i in range(3)]
        f = list(vdot) + list(wdot)
        L = sp.Rational(1, 2) * (sp.nsimplify(W.Q_W) * sum(xi ** 2 for xi in x)
                                 + sp.nsimplify(W.R_W) * sum(ui ** 2 for ui in u))
    H = L + sum(lam[i] * f[i] for i in range(n))
    sol = sp.solve([sp.diff(H, ui) for ui in u], u, dict=True)[0]
    ustar = [sol[ui] for ui in u]
    # partials at fixed u, then u = u*(x, lambda)
    Phi = [sp.diff(H, lam[i]) for i in range(n)] + [-sp.diff(H, x[i]) for i in range(n)]
    Phi = [sp.simplify(e.subs(sol)) if kind == "example3" else e.subs(sol) for e in Phi]
    y = list(x) + list(lam)
    dPhi = sp.Matrix(Phi).jacobian(y)
    fPhi = sp.lambdify([y], Phi, "numpy")
    fdPhi = sp.lambdify([y], dPhi, "numpy")
    fu = sp.lambdify([y], ustar, "numpy")
    fL = sp.lambdify([y], L.subs(sol), "numpy")
    return n, m, fPhi, fdPhi, fu, fL


def sym_phi(kind, m, y):
    n, m, fPhi, fdPhi, fu, fL = sympy_model(kind, m)
    return (np.array(fPhi(list(y)), dtype=float),
            np.array(fdPhi(list(y)), dtype=float).reshape(2 * n, 2 * n))


# ---------------------------------------------------------------------------
# model pins
# ---------------------------------------------------------------------------

def _rot(v):
    phi, th, psi = v
    Rx = np.array([[1, 0, 0], [0, np.cos(phi), -np.sin(phi)], [0, np.sin(phi), np.cos(phi)]])
    Ry = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    Rz = np.array([[np.cos(psi), -np.sin(psi), 0], [np.sin(psi), np.cos(psi), 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def test_euler_kinematics_is_body_rate_of_321_rotation():
    rng = np.random.default_rng(1)
    p = rigid()
    for _ in range(5):
        v = rng.uniform(-1.0, 1.0, 3)
        w = rng.uniform(-1.0, 1.0, 3)
        y = np.concatenate([v, w, np.zeros(6)])  # lambda = 0 -> u* = 0
        vdot = O.phi(p, y, jacobian=False)[0, :3]
        eps = 1e-6
        Rdot = (_rot(v + eps * vdot) - _rot(v - eps * vdot)) / (2 * eps)
        wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        assert np.max(np.abs(Rdot - _rot(v) @ wx)) < 1e-8


def test_free_rigid_body_invariants():
    rng = np.random.default_rng(2)
    p = rigid()
    J = np.array(W.J_DIAG)
    for _ in range(5):
        y = np.concatenate([rng.uniform(-1, 1, 6), np.zeros(6)])
        wdot = O.phi(p, y, jacobian=False)[0, 3:6]
        w = y[3:6]
        assert abs(w @ (J * wdot)) < 1e-14          # kinetic energy
        assert abs((J * w) @ (J * wdot)) < 1e-14    # |J w|^2


@pytest.mark.parametrize("kind,m", [("rigid", 3), ("rigid", 2), ("linear", 3), ("example3", 1)])
def test_phi_and_jacobian_match_sympy(kind, m):
    rng = np.random.default_rng(3)
    if kind == "rigid":
        p = rigid(m)
    elif kind == "linear":
        p = linear(m)
    else:
        p = example3()
    n = p.n
    for _ in range(6):
        y = np.concatenate([rng.uniform(-0.8, 0.8, n), rng.uniform(-3, 3, n)])
        P, D = O.phi(p, y)
        Ps, Ds = sym_phi(kind, m, y)
        assert np.max(np.abs(P[0] - Ps)) < 1e-13 * max(1, np.abs(Ps).max())
        assert np.max(np.abs(D[0] - Ds)) < 1e-13 * max(1, np.abs(Ds).max())
        us = np.array(sympy_model(kind, m)[4](list(y)), dtype=float)
        assert np.max(np.abs(O.ustar(p, y)[0] - us)) < 1e-13 * max(1, np.abs(us).max())


def test_ustar_closed_form_rigid_body():
    # u* = -(1/r_w) B^T J^{-1} lambda_w
    rng = np.random.default_rng(4)
    for m in (3, 2):
        p = rigid(m)
        y = rng.standard_normal((7, 12))
        B = W.input_matrix(m)
        expect = -(1 / W.R_W) * (y[:, 9:12] / np.array(W.J_DIAG)) @ B
        assert np.allclose(O.ustar(p, y), expect, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# linearised model: exact discrete Riccati and continuous LQR
# ---------------------------------------------------------------------------

def hamiltonian_matrix(m=3):
    J = np.array(W.J_DIAG)
    A = np.zeros((6, 6))
    A[:3, 3:] = np.eye(3)
    Bt = np.zeros((6, m))
    Bt[3:, :] = W.input_matrix(m) / J[:, None]
    S = Bt @ Bt.T / W.R_W
    Q = W.Q_W * np.eye(6)
    return np.block([[A, -S], [-Q, -A.T]])


def discrete_riccati(N, T, m=3):
    M = hamiltonian_matrix(m)
    h = T / N
    C = np.linalg.solve(np.eye(12) + 0.5 * h * M, np.eye(12) - 0.5 * h * M)
    P = W.P_W * np.eye(6)
    Ps = [P]
    for _ in range(N):
        D = C @ np.vstack([np.eye(6), P])
        P = D[6:] @ np.linalg.inv(D[:6])
        Ps.append(P)
    return Ps[::-1]  # P_0 .. P_N


def continuous_riccati_P0(T, m=3):
    M = hamiltonian_matrix(m)
    E = scipy.linalg.expm(-T * M)  # maps y(T) back to y(0)
    D = E @ np.vstack([np.eye(6), W.P_W * np.eye(6)])
    return D[6:] @ np.linalg.inv(D[:6])


@pytest.mark.parametrize("m", [3, 2])
def test_linear_model_matches_discrete_riccati(m):
    p = linear(m, N=64, T=20.0)
    x0 = W.uniform_in_box(12, seed=21)
    r = O.solve_bvps(p, x0, want_traj=True)
    assert np.all(r.status == O.CONVERGED) and np.all(r.iters == 0)
    Ps = discrete_riccati(64, 20.0, m)
    lam_ref = x0 @ Ps[0].T
    assert np.max(np.abs(r.lambda0 - lam_ref)) < 1e-12 * np.abs(lam_ref).max()
    # lambda_k = P_k x_k along the whole trajectory
    for k in (0, 17, 40, 64):
        xk, lk = r.traj[:, k, :6], r.traj[:, k, 6:]
        assert np.max(np.abs(lk - xk @ Ps[k].T)) < 1e-11 * np.abs(lam_ref).max()


def test_linear_model_converges_to_continuous_lqr_at_order_two():
    T = 5.0
    x0 = W.uniform_in_box(4, seed=22)
    P0 = continuous_riccati_P0(T)
    lam_ref = x0 @ P0.T
    V_ref = 0.5 * np.einsum("bi,ij,bj->b", x0, P0, x0)
    errs, verrs = [], []
    for N in (32, 64, 128):
        r = O.solve_bvps(linear(N=N, T=T), x0)
        errs.append(np.max(np.abs(r.lambda0 - lam_ref)))
        verrs.append(np.max(np.abs(r.V - V_ref)))
    for e in (errs, verrs):
        orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(orders - 2.0) < 0.15), orders


def test_linear_model_long_horizon_matches_are():
    # T = 20: P(0) is the stabilising ARE solution up to O(exp(-2 mu T)).
    M = hamiltonian_matrix()
    A, S = M[:6, :6], -M[:6, 6:]
    J = np.array(W.J_DIAG)
    Bt = np.zeros((6, 3))
    Bt[3:] = np.eye(3) / J[:, None]
    Pare = scipy.linalg.solve_continuous_are(A, Bt, W.Q_W * np.eye(6), W.R_W * np.eye(3))
    x0 = W.uniform_in_box(3, seed=23)
    r = O.solve_bvps(linear(N=256, T=20.0), x0)
    lam_ref = x0 @ Pare.T
    assert np.max(np.abs(r.lambda0 - lam_ref)) < 2e-3 * np.abs(lam_ref).max()


# ---------------------------------------------------------------------------
# Example III closed form (Sec. 5.3)
# ---------------------------------------------------------------------------

def example3_exact(x0, T):
    s = 1 + x0[:, 0] ** 2 + x0[:, 1] ** 2
    y = x0[:, 2] / s
    th = np.tanh(T)
    V = 0.5 * y ** 2 * th
    u = -y * th
    # gradient of V = 0.5 tanh(T) x3^2 / s^2
    gV = np.stack([-2 * th * x0[:, 2] ** 2 * x0[:, 0] / s ** 3,
                   -2 * th * x0[:, 2] ** 2 * x0[:, 1] / s ** 3,
                   th * x0[:, 2] / s ** 2], axis=1)
    return V, u, gV


@pytest.mark.parametrize("T", [1.0, 5.0])
def test_example3_closed_form_second_order(T):
    x0 = np.random.default_rng(31).uniform(-2.0, 2.0, (6, 3))
    V_ref, u_ref, g_ref = example3_exact(x0, T)
    e_l, e_u, e_v = [], [], []
    for N in (64, 128, 256):
        r = O.solve_bvps(example3(N=N, T=T), x0)
        assert np.all(r.status == O.CONVERGED)
        e_l.append(np.max(np.abs(r.lambda0 - g_ref)))
        e_u.append(np.max(np.abs(r.u0[:, 0] - u_ref)))
        e_v.append(np.max(np.abs(r.V - V_ref)))
    for e in (e_l, e_u, e_v):
        orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(orders - 2.0) < 0.2), (e, orders)
    assert e_l[-1] < 3e-3 and e_u[-1] < 3e-3


def test_example3_state_continuation():
    # Newton from the linearised first step stalls at corners of the box for
    # some horizons (here T = 2.5); the continuation in the initial state
    # (stages (k / K) x0, each from the one before) converges there, to the
    # same discrete solution wherever the plain iteration converges too, and
    # to the closed form at second order
    corners = np.array([[-2.0, -2.0, -2.0], [-2.0, -2.0, 2.0], [-2.0, 2.0, 2.0], [2.0, 2.0, 2.0]])
    import dataclasses
    plain = O.solve_bvps(example3(N=64, T=2.5), corners)
    assert np.all(plain.status == O.MAXITER)
    V_ref, u_ref, g_ref = example3_exact(corners, 2.5)
    e_v, e_l = [], []
    for N in (64, 128, 256):
        r = O.solve_bvps(dataclasses.replace(example3(N=N, T=2.5), continuation=2), corners)
        assert np.all(r.status == O.CONVERGED)
        e_v.append(np.max(np.abs(r.V - V_ref)))
        e_l.append(np.max(np.abs(r.lambda0 - g_ref)))
    for e in (e_v, e_l):
        orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(orders - 2.0) < 0.25), (e, orders)
    x0 = np.random.default_rng(33).uniform(-2.0, 2.0, (8, 3))
    a = O.solve_bvps(example3(N=64, T=1.0), x0, want_traj=True)
    b = O.solve_bvps(dataclasses.replace(example3(N=64, T=1.0), continuation=3), x0, want_traj=True)
    assert np.all(a.status == O.CONVERGED) and np.all(b.status == O.CONVERGED)
    assert np.max(np.abs(a.traj - b.traj)) <= 1e-11 * np.max(np.abs(a.traj))
    assert np.all(b.iters >= 3)  # each of the three stages takes at least one step


# ---------------------------------------------------------------------------
# nonlinear rigid body: same discrete solution by other algorithms
# ---------------------------------------------------------------------------

def shooting(kind, m, x0, N, T, l0=None):
    """Single shooting: unknown lambda(0) (from l0, default 0); each mesh step
    solves the implicit trapezoid equation with Newton on the sympy
    right-hand side; a dense Newton (finite-difference Jacobian) drives
    lambda_N - p_w x_N to zero."""
    n = 6
    h = T / N

    def march(l0):
        y = np.concatenate([x0, l0])
        ys = [y]
        for _ in range(N):
            P0, _ = sym_phi(kind, m, y)
            z = y + h * P0
            for _ in range(50):
                P1, D1 = sym_phi(kind, m, z)
                g = z - y - 0.5 * h * (P0 + P1)
                dz = np.linalg.solve(np.eye(2 * n) - 0.5 * h * D1, -g)
                z = z + dz
                if np.max(np.abs(dz)) < 1e-15 * max(1, np.abs(z).max()):
                    break
            y = z
            ys.append(y)
        return np.array(ys)

    def mismatch(l0):
        ys = march(l0)
        return ys[-1, n:] - W.P_W * ys[-1, :n]

    l0 = np.zeros(n) if l0 is None else np.array(l0, dtype=np.float64)
    for _ in range(30):
        r = mismatch(l0)
        if np.max(np.abs(r)) < 1e-13:
            break
        Jm = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1e-7
            Jm[:, j] = (mismatch(l0 + e) - mismatch(l0 - e)) / 2e-7
        l0 = l0 - np.linalg.solve(Jm, r)
    return march(l0)


@pytest.mark.parametrize("m,N,T", [(3, 4, 0.5), (3, 8, 1.0), (2, 16, 2.0)])
def test_collocation_equals_trapezoid_shooting(m, N, T):
    x0 = W.uniform_in_box(2, seed=41 + N)
    p = rigid(m, N=N, T=T)
    r = O.solve_bvps(p, x0, want_traj=True)
    assert np.all(r.status == O.CONVERGED)
    for b in range(2):
        ys = shooting("rigid", m, x0[b], N, T)
        assert np.max(np.abs(ys - r.traj[b])) < 1e-10 * max(1, np.abs(ys).max())


def test_newton_iterates_match_dense_lu():
    p = rigid(N=8, T=2.0)
    x0 = W.uniform_in_box(3, seed=51)
    r = O.solve_bvps(p, x0, want_traj=True)
    for b in range(3):
        Y = np.zeros(12 * 9)
        its = -1
        while True:
            F = O.residual(p, x0[b], Y)[0]
            if its >= 0 and np.max(np.abs(F)) <= p.tol:
                break
            Jd = O.jacobian_dense(p, Y)
            Y = Y + np.linalg.solve(Jd, -F)
            its += 1
        assert its == r.iters[b]
        assert np.max(np.abs(Y - r.traj[b].reshape(-1))) < 1e-12 * np.abs(Y).max()


def test_jacobian_matches_finite_differences():
    p = rigid(N=4, T=1.0)
    Y = np.random.default_rng(61).uniform(-0.5, 0.5, 12 * 5)
    x0 = np.zeros(6)
    Jd = O.jacobian_dense(p, Y)
    eps = 1e-6
    for j in range(0, Y.size, 7):
        e = np.zeros_like(Y)
        e[j] = eps
        col = (O.residual(p, x0, Y + e)[0] - O.residual(p, x0, Y - e)[0]) / (2 * eps)
        assert np.max(np.abs(col - Jd[:, j])) < 1e-7


# ---------------------------------------------------------------------------
# outputs and status rules
# ---------------------------------------------------------------------------

def test_outputs_consistent_with_trajectory():
    p = rigid(N=32, T=4.0)
    x0 = W.uniform_in_box(4, seed=71)
    r = O.solve_bvps(p, x0, want_traj=True)
    assert np.array_equal(r.lambda0, r.traj[:, 0, 6:])
    B = W.input_matrix(3)
    u_ref = -(1 / W.R_W) * (r.lambda0[:, 3:] / np.array(W.J_DIAG)) @ B
    assert np.allclose(r.u0, u_ref, rtol=1e-14, atol=1e-14)
    # V = trapezoid of L along the trajectory + 0.5 p_w |x_N|^2
    h = p.T / p.N
    u = O.ustar(p, r.traj.reshape(-1, 12)).reshape(4, p.N + 1, 3)
    Lk = 0.5 * (W.Q_W * np.sum(r.traj[:, :, :6] ** 2, axis=2) + W.R_W * np.sum(u ** 2, axis=2))
    V = h * (0.5 * Lk[:, 0] + Lk[:, 1:-1].sum(axis=1) + 0.5 * Lk[:, -1])
    V += 0.5 * W.P_W * np.sum(r.traj[:, -1, :6] ** 2, axis=1)
    assert np.allclose(r.V, V, rtol=1e-13)


def test_status_rules():
    p = rigid(N=16, T=2.0)
    x0 = np.vstack([np.zeros(6), W.uniform_in_box(3, seed=81)])
    # zero initial state: the linearised step is exact, 0 iterations
    r = O.solve_bvps(p, x0)
    assert r.status[0] == O.CONVERGED and r.iters[0] == 0
    assert np.all(r.status == O.CONVERGED) and np.all(r.iters[1:] >= 1)
    # max_iter = 0: MAXITER everywhere except the zero state
    p0 = rigid(N=16, T=2.0, )
    p0.max_iter = 0
    r0 = O.solve_bvps(p0, x0)
    assert r0.status[0] == O.CONVERGED and np.all(r0.status[1:] == O.MAXITER)
    assert np.all(r0.iters == 0)
    # tol = 0 cannot be met: MAXITER after max_iter iterations
    pt = rigid(N=16, T=2.0)
    pt.tol, pt.max_iter = 0.0, 3
    rt = O.solve_bvps(pt, x0[1:])
    assert np.all(rt.status == O.MAXITER) and np.all(rt.iters == 3)
    # a NaN in the initial state: NONFINITE at the first test
    xn = x0[1:2].copy()
    xn[0, 4] = np.nan
    rn = O.solve_bvps(p, xn)
    assert rn.status[0] == O.NONFINITE and rn.iters[0] == 0
