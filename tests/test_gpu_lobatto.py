"""GPU parity of the four-point Lobatto IIIA solver (the paper's BVP formula,
Sec. 3.1, Sec. 5.1) against the oracle's Lobatto IIIA collocation.

Bar: as for the trapezoidal solver, Newton status and iteration count
bit-exact; lambda(0), u(0), V and the mesh trajectory within 1e-8 relative per
BVP.  The two eliminate the Newton system differently (the oracle: a banded LU
of the whole system with its stages; the GPU: condensation of the interior
stages, then a Riccati sweep), so values agree to rounding.
"""
import numpy as np
import pytest

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

pytestmark = pytest.mark.gpu
REL = 1e-8


def rel_err(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.max(np.abs(a - b), axis=1) / np.maximum(np.max(np.abs(b), axis=1), 1e-8)


def problems(model=S.MODEL_RIGID_BODY, m=3, N=16, T=20.0, tol=W.TOL, max_iter=W.MAX_ITER, continuation=0):
    B = W.input_matrix(m)
    g = S.Problem(model=model, m=m, J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=tol,
                  max_iter=max_iter, continuation=continuation, scheme=S.LOBATTO4)
    o = O.Problem(model={S.MODEL_RIGID_BODY: O.RIGID_BODY, S.MODEL_LINEARISED: O.LINEARISED}[model], n=6, m=m,
                  J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=T, N=N, tol=tol, max_iter=max_iter,
                  continuation=continuation, scheme=O.LOBATTO4)
    return g, o


def gpu_solve(prob, x0, want_traj=True):
    import torch
    r = S.solve_bvps(prob, torch.tensor(np.asarray(x0, dtype=np.float64), device="cuda"), want_traj=want_traj)
    torch.cuda.synchronize()
    return {k: (getattr(r, k).cpu().numpy() if getattr(r, k) is not None else None)
            for k in ("lambda0", "u0", "V", "traj", "status", "iters")}


def assert_parity(g, o):
    assert np.array_equal(g["status"], o.status), (g["status"], o.status)
    assert np.array_equal(g["iters"], o.iters), (g["iters"], o.iters)
    ok = o.status == O.CONVERGED
    assert np.all(rel_err(g["lambda0"][ok], o.lambda0[ok]) <= REL)
    assert np.all(rel_err(g["u0"][ok], o.u0[ok]) <= REL)
    assert np.all(rel_err(g["V"][ok, None], o.V[ok, None]) <= REL)
    if g["traj"] is not None and o.traj is not None:
        assert np.all(rel_err(g["traj"][ok], o.traj[ok]) <= REL)


def test_small_grid_parity():
    # level-2 grid (85 nodes), three wheels, N = 16, T = 20
    gp, op = problems(N=16, T=20.0)
    x0 = O.grid(6, 2, W.BOX_LO, W.BOX_HI).nodes
    g = gpu_solve(gp, x0)
    o = O.solve_bvps(op, x0, want_traj=True)
    assert np.all(o.status == O.CONVERGED)
    assert_parity(g, o)


def test_linear_model_is_one_step():
    gp, op = problems(S.MODEL_LINEARISED, N=24, T=5.0)
    x0 = W.uniform_in_box(30, seed=960)
    g = gpu_solve(gp, x0)
    assert np.all(g["status"] == S.CONVERGED) and np.all(g["iters"] == 0)
    assert_parity(g, O.solve_bvps(op, x0, want_traj=True))


@pytest.mark.parametrize("n_bvps,N,T", [(1, 1, 0.5), (3, 2, 1.0), (65, 7, 2.0), (4, 100, 20.0)])
def test_ragged_and_extreme_meshes(n_bvps, N, T):
    gp, op = problems(N=N, T=T)
    x0 = W.uniform_in_box(n_bvps, seed=961 + N)
    assert_parity(gpu_solve(gp, x0), O.solve_bvps(op, x0, want_traj=True))


def test_status_rules():
    gp, op = problems(N=12, T=4.0)
    x0 = np.vstack([np.zeros(6), W.uniform_in_box(5, seed=965)])
    x0[3, 4] = np.nan
    g = gpu_solve(gp, x0)
    o = O.solve_bvps(op, x0, want_traj=True)
    assert g["status"][0] == S.CONVERGED and g["iters"][0] == 0
    assert g["status"][3] == S.NONFINITE
    assert_parity(g, o)
    for tol, max_iter in [(W.TOL, 0), (0.0, 2)]:
        gp2, op2 = problems(N=12, T=4.0, tol=tol, max_iter=max_iter)
        g2 = gpu_solve(gp2, x0)
        o2 = O.solve_bvps(op2, x0)
        assert np.array_equal(g2["status"], o2.status) and np.array_equal(g2["iters"], o2.iters)


def test_two_wheels_damped_and_continued():
    # damped steps (two wheels, T = 5) and the virtual-torque continuation
    # (T = 20) with the Lobatto formula
    gp, op = problems(m=2, N=8, T=5.0, max_iter=40)
    x0 = W.uniform_in_box(24, seed=966)
    assert_parity(gpu_solve(gp, x0), O.solve_bvps(op, x0, want_traj=True))
    gp, op = problems(m=2, N=16, T=20.0, max_iter=W.UNDERACTUATED_MAX_ITER, continuation=W.UNDERACTUATED_CONTINUATION)
    x0 = 0.5 * W.uniform_in_box(12, seed=967)
    o = O.solve_bvps(op, x0, want_traj=True)
    assert np.sum(o.status == O.CONVERGED) >= 10
    assert_parity(gpu_solve(gp, x0), o)


def test_validation_sample_size():
    # the total-error estimate's reference solves: 1280 uniform states of the
    # three-wheel problem, T = 20, on 64 intervals (every state against the
    # oracle, status and iterations bit-exact)
    from paper_1507_04769_amd import validation as VA
    gp, op = problems(N=64, T=20.0)
    x0 = W.uniform_in_box(VA.N_SAMPLES, seed=VA.SAMPLE_SEED)
    g = gpu_solve(gp, x0, want_traj=False)
    o = O.solve_bvps(op, x0)
    assert np.all(o.status == O.CONVERGED)
    assert_parity(g, o)


def test_unsupported_combinations():
    import torch
    gp, _ = problems(N=8, T=1.0)
    with pytest.raises(S.SgcmError) as e:
        S.Plan(gp)
    assert e.value.code == S.SGCM_EUNSUPPORTED
    gp.precision = S.FP32
    with pytest.raises(S.SgcmError) as e:
        S.solve_bvps(gp, torch.zeros((2, 6), dtype=torch.float64, device="cuda"))
    assert e.value.code == S.SGCM_EUNSUPPORTED
