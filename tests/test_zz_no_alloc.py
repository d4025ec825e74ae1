"""The allocation-free solve (sgcm_solve_bvps_static) against the solve with
a caller workspace (sgcm_solve_bvps), through the C ABI.

Both run the same kernels on the same inputs, so every output must be
bitwise the same (each BVP's result does not depend on the workspace or the
launch order); two calls in a row, the second with fewer BVPs, the third on
another problem (two wheels with continuation), share the library's scratch.
A request beyond the scratch is refused before any device work.
"""
import ctypes

import numpy as np
import pytest

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

pytestmark = pytest.mark.gpu
KEYS = ("lambda0", "u0", "V", "traj", "status", "iters")


def outputs(problem, n):
    import torch
    return {"lambda0": torch.empty((n, 6), dtype=torch.float64, device="cuda"),
            "u0": torch.empty((n, problem.m), dtype=torch.float64, device="cuda"),
            "V": torch.empty((n,), dtype=torch.float64, device="cuda"),
            "traj": torch.empty((n, problem.N + 1, 12), dtype=torch.float64, device="cuda"),
            "status": torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            "iters": torch.full((n,), -7, dtype=torch.int32, device="cuda")}


def static_solve(problem, x0):
    """sgcm_solve_bvps_static called through the C ABI."""
    import torch
    n = x0.shape[0]
    o = outputs(problem, n)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = S.lib().sgcm_solve_bvps_static(ctypes.byref(problem.c()), n, vp(x0), vp(o["lambda0"]), vp(o["u0"]),
                                        vp(o["V"]), vp(o["traj"]), vp(o["status"]), vp(o["iters"]),
                                        S._stream(None))
    assert rc == S.SGCM_OK, S.strerror(rc)
    return o


def workspace_solve(problem, x0):
    import torch
    n = x0.shape[0]
    o = outputs(problem, n)
    ws = torch.empty((S.sgcm_solve_bvps_workspace(problem, n) // 8 + 32,), dtype=torch.float64, device="cuda")
    S.sgcm_solve_bvps(problem, x0, o["lambda0"], o["u0"], o["V"], o["traj"], o["status"], o["iters"], ws)
    return o


def host(o):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_static_solve_equals_workspace_solve_on_calls_in_a_row():
    import torch
    three = S.Problem(N=256, T=20.0)
    nodes = O.grid(6, 4, W.BOX_LO, W.BOX_HI).nodes
    first = torch.tensor(nodes[:160], device="cuda")     # 160 BVPs: about 63 MB of the 64 MiB
    second = torch.tensor(nodes[700:723], device="cuda")  # then a smaller call
    a1 = host(static_solve(three, first))
    a2 = host(static_solve(three, second))
    b1, b2 = host(workspace_solve(three, first)), host(workspace_solve(three, second))
    for a, b in ((a1, b1), (a2, b2)):
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k
    assert np.all(a1["status"] == S.CONVERGED) and np.all(a2["status"] == S.CONVERGED)
    # against the oracle (status and iterations bit-exact, lambda(0) to 1e-8)
    o = O.solve_bvps(O.Problem(N=256, T=20.0), nodes[700:723])
    assert np.array_equal(a2["status"], o.status) and np.array_equal(a2["iters"], o.iters)
    rel = np.abs(a2["lambda0"] - o.lambda0).max(axis=1) / np.maximum(np.abs(o.lambda0).max(axis=1), 1e-8)
    assert rel.max() <= 1e-8
    # a third call on another problem: two wheels, continuation in four stages
    two = S.Problem(m=2, B=W.input_matrix(2), N=64, T=20.0, max_iter=W.UNDERACTUATED_MAX_ITER,
                    continuation=W.UNDERACTUATED_CONTINUATION)
    x2 = torch.tensor(W.uniform_in_box(12, seed=950), device="cuda")
    a3, b3 = host(static_solve(two, x2)), host(workspace_solve(two, x2))
    for k in KEYS:
        assert np.array_equal(a3[k], b3[k]), k


def test_static_solve_refuses_more_than_its_scratch():
    import torch
    p = S.Problem(N=256, T=20.0)
    need = S.sgcm_solve_bvps_workspace(p, 200)
    assert need > S.STATIC_SCRATCH_BYTES
    x0 = torch.zeros((200, 6), dtype=torch.float64, device="cuda")
    o = outputs(p, 200)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = S.lib().sgcm_solve_bvps_static(ctypes.byref(p.c()), 200, vp(x0), vp(o["lambda0"]), vp(o["u0"]),
                                        vp(o["V"]), vp(o["traj"]), vp(o["status"]), vp(o["iters"]),
                                        S._stream(None))
    assert rc == S.SGCM_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(o["status"] == -7)  # nothing ran
    assert S.lib().sgcm_solve_bvps_static(ctypes.byref(p.c()), 0, None, None, None, None, None, None, None,
                                          None) == S.SGCM_OK
