"""Batches of characteristic BVPs with per-BVP mesh size and horizon in one
launch (plain or persistent schedule, optionally captured in a HIP graph),
against the oracle (Sec. 3.1, eq. hamchar; the oracle solves each (N, T)
group separately).  Bar as for the uniform solver: status and iterations
bit-exact, lambda(0), u(0), V within 1e-8 relative; the schedule must not
change any result (bitwise).
"""
import numpy as np
import pytest

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

pytestmark = pytest.mark.gpu
REL = 1e-8


def _torch():
    import torch
    return torch


def rel_err(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.max(np.abs(a - b), axis=1) / np.maximum(np.max(np.abs(b), axis=1), 1e-8)


def problem(m=3):
    B = W.input_matrix(m)
    return S.Problem(m=m, J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=1.0, N=1, tol=W.TOL,
                     max_iter=W.MAX_ITER)


def oracle_groups(x0, N, T, m=3, idx=None):
    """Oracle solution of every BVP in idx (default all), one call per (N, T) group."""
    idx = np.arange(len(x0)) if idx is None else np.asarray(idx)
    out = {k: {} for k in ("lambda0", "u0", "V", "status", "iters")}
    B = W.input_matrix(m)
    for NN, TT in sorted(set(zip(N[idx].tolist(), T[idx].tolist()))):
        sel = idx[(N[idx] == NN) & (T[idx] == TT)]
        p = O.Problem(n=6, m=m, J=W.J_DIAG, B=B, q_w=W.Q_W, r_w=W.R_W, p_w=W.P_W, T=TT, N=NN, tol=W.TOL,
                      max_iter=W.MAX_ITER)
        r = O.solve_bvps(p, x0[sel])
        for j, i in enumerate(sel):
            out["lambda0"][i] = r.lambda0[j]
            out["u0"][i] = r.u0[j]
            out["V"][i] = r.V[j]
            out["status"][i] = r.status[j]
            out["iters"][i] = r.iters[j]
    return {k: np.array([v[i] for i in idx]) for k, v in out.items()}


def gpu_batch(batch, x0):
    torch = _torch()
    r = S.solve_bvps_batch(batch, torch.tensor(x0, device="cuda"))
    torch.cuda.synchronize()
    return {k: getattr(r, k).cpu().numpy() for k in ("lambda0", "u0", "V", "status", "iters")}


def assert_parity(g, o):
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["iters"], o["iters"])
    ok = o["status"] == O.CONVERGED
    assert np.all(rel_err(g["lambda0"][ok], o["lambda0"][ok]) <= REL)
    assert np.all(rel_err(g["u0"][ok], o["u0"][ok]) <= REL)
    assert np.all(rel_err(g["V"][ok, None], o["V"][ok, None]) <= REL)


def small_mixed(n=41, seed=120):
    g = np.random.default_rng(seed)
    N = g.choice(np.array([1, 3, 8, 17, 40]), size=n).astype(np.int32)
    T = g.choice(np.array([0.5, 2.0, 6.0]), size=n)
    x0 = W.uniform_in_box(n, seed=seed + 1)
    return x0, N, T


@pytest.mark.parametrize("order,slots", [(S.ORDER_LONGEST_FIRST, 0), (S.ORDER_GIVEN, 0),
                                         (S.ORDER_LONGEST_FIRST, 1), (S.ORDER_GIVEN, 3)])
def test_small_mixed_batch_parity(order, slots):
    x0, N, T = small_mixed()
    b = S.Batch(problem(), N, T, order=order, slots_per_cu=slots)
    g = gpu_batch(b, x0)
    o = oracle_groups(x0, N, T)
    assert_parity(g, o)


def test_schedule_does_not_change_results():
    x0, N, T = small_mixed(n=77, seed=130)
    ref = None
    for order, slots in [(0, 0), (1, 0), (0, 1), (1, 2), (1, 6)]:
        g = gpu_batch(S.Batch(problem(), N, T, order=order, slots_per_cu=slots), x0)
        if ref is None:
            ref = g
        for k in ref:
            assert np.array_equal(g[k], ref[k]), (order, slots, k)


def test_batch_equals_uniform_solver():
    # every BVP with N = 64, T = 20: the batch path and sgcm_solve_bvps_plan
    # run the same per-BVP code (each first Newton step formed from the steps
    # of the unit initial states of its (N, T)), so the results agree bitwise
    torch = _torch()
    x0 = W.uniform_in_box(50, seed=140)
    n = len(x0)
    p = problem()
    p.N, p.T = 64, 20.0
    r = S.solve_bvps(p, torch.tensor(x0, device="cuda"), plan=S.Plan(p))
    torch.cuda.synchronize()
    for slots in (0, 2):
        g = gpu_batch(S.Batch(problem(), np.full(n, 64), np.full(n, 20.0), slots_per_cu=slots), x0)
        for k in ("lambda0", "u0", "V", "status", "iters"):
            assert np.array_equal(g[k], getattr(r, k).cpu().numpy()), (slots, k)


def test_underactuated_mixed_batch():
    # two wheels: the general (non-invertible S_w) form of the 3 x 3 step
    g0 = np.random.default_rng(150)
    n = 30
    N = g0.choice(np.array([8, 20, 40]), size=n).astype(np.int32)
    T = g0.choice(np.array([1.0, 2.0]), size=n)
    x0 = 0.3 * W.uniform_in_box(n, seed=151)
    b = S.Batch(problem(m=2), N, T, slots_per_cu=1)
    g = gpu_batch(b, x0)
    o = oracle_groups(x0, N, T, m=2)
    assert np.all(o["status"] == O.CONVERGED)
    assert_parity(g, o)


def test_graph_capture_replays():
    # the persistent batch launch (counter reset by a kernel, no memset) in a
    # HIP graph: every replay, with eager work and synchronisation between
    # replays, equals the eager result bitwise
    torch = _torch()
    x0h, N, T = small_mixed(n=64, seed=160)
    b = S.Batch(problem(), N, T, slots_per_cu=2)
    x0 = torch.tensor(x0h, device="cuda")
    eager = S.solve_bvps_batch(b, x0)
    torch.cuda.synchronize()
    ws = S.batch_workspace(b, x0.device)
    n, m = b.n, b.m
    lam = torch.zeros((n, 6), dtype=torch.float64, device="cuda")
    u0 = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    V = torch.zeros((n,), dtype=torch.float64, device="cuda")
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        S.sgcm_solve_bvps_batch(b, x0, lam, u0, V, st, it, ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        S.sgcm_solve_bvps_batch(b, x0, lam, u0, V, st, it, ws)
    for rep in range(3):
        for t in (lam, u0, V):
            t.fill_(float("nan"))
        st.fill_(-1)
        it.fill_(-1)
        other = S.solve_bvps_batch(b, x0)  # eager work on the same plan between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, t in (("lambda0", lam), ("u0", u0), ("V", V), ("status", st), ("iters", it)):
            assert torch.equal(t, getattr(eager, k)), (rep, k)
            assert torch.equal(getattr(other, k), getattr(eager, k)), (rep, k)


def test_full_mixed_batch():
    # 3072 level-5 nodes + 1024 uniform states, N in {64..512}, T in {10, 20, 40}
    bw = W.BATCH
    g = S.Grid(6, bw.level, W.BOX_LO, W.BOX_HI)
    x0 = W.batch_initial_states(bw, g.nodes())
    N, T = W.mixed_assignment(bw, len(x0))
    b = S.Batch(problem(), N, T, slots_per_cu=6)
    r = gpu_batch(b, x0)
    assert np.all(r["status"] == S.CONVERGED)
    # every BVP against the oracle (one oracle call per (N, T) group)
    assert_parity(r, oracle_groups(x0, N, T))


def test_batch_with_and_without_group_first_steps():
    # (N, T) groups of at least 8 BVPs take their first Newton steps from the
    # group's unit-state steps, smaller groups solve their own: against the
    # oracle, and bitwise against the solver with and without a plan
    torch = _torch()
    sizes = {(16, 2.0): 20, (8, 0.5): 5, (24, 6.0): 10, (4, 1.0): 3}
    N = np.concatenate([np.full(c, k[0]) for k, c in sizes.items()]).astype(np.int32)
    T = np.concatenate([np.full(c, k[1]) for k, c in sizes.items()])
    perm = np.random.default_rng(150).permutation(len(N))
    N, T = N[perm], T[perm]
    x0 = W.uniform_in_box(len(N), seed=151)
    g = gpu_batch(S.Batch(problem(), N, T), x0)
    assert_parity(g, oracle_groups(x0, N, T))
    for (NN, TT), c in sizes.items():
        sel = np.nonzero((N == NN) & (T == TT))[0]
        p = problem()
        p.N, p.T = int(NN), float(TT)
        r = S.solve_bvps(p, torch.tensor(x0[sel], device="cuda"), plan=S.Plan(p) if c >= 8 else None)
        torch.cuda.synchronize()
        for k in ("lambda0", "u0", "V", "status", "iters"):
            assert np.array_equal(g[k][sel], getattr(r, k).cpu().numpy()), ((NN, TT), k)
