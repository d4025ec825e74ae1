"""Host-side checks of the C ABI (no GPU needed).

* libsgcm.so loads and exports every function include/sgcm.h declares;
* the host grid layer (Sec. 3.2) gives the oracle's grid: identical keys and
  canonical order, coordinates equal to rounding;
* argument validation returns SGCM_EINVAL / SGCM_EUNSUPPORTED before any
  device work, and the documented no-op sizes return SGCM_OK.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1507_04769_amd as S
from oracle import oracle as O
from paper_1507_04769_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgcm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgcm_[a-z_0-9]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(S.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in _declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sgcm_\w+)", out))
    assert set(_declared()) <= exported
    assert S.sgcm_version() >= 100
    assert S.strerror(S.SGCM_EINVAL) == "invalid argument"


@pytest.mark.parametrize("d,level", [(1, 0), (1, 5), (2, 3), (3, 4), (6, 2), (6, 4), (6, 5), (8, 2)])
def test_host_grid_matches_oracle(d, level):
    lo = -np.arange(1, d + 1) * 0.3
    hi = np.arange(1, d + 1) * 0.5
    g = S.Grid(d, level, lo, hi)
    og = O.grid(d, level, lo, hi)
    assert len(g) == og.nodes.shape[0] == O.grid_size(d, level)
    assert np.array_equal(g.keys(), og.keys)
    assert np.max(np.abs(g.nodes() - og.nodes)) < 4e-16 * np.max(np.abs(hi - lo)) * 4


def test_workload_grid_sizes():
    for level, size in [(2, 85), (3, 389), (4, 1457), (5, 4865)]:
        assert len(S.Grid(6, level, W.BOX_LO, W.BOX_HI)) == size


def test_grid_argument_validation():
    with pytest.raises(S.SgcmError) as e:
        S.Grid(0, 2, [], [])
    assert e.value.code == S.SGCM_EINVAL
    with pytest.raises(S.SgcmError) as e:
        S.Grid(2, 6, [0, 0], [1, 1])
    assert e.value.code == S.SGCM_EUNSUPPORTED
    with pytest.raises(S.SgcmError) as e:
        S.Grid(2, 2, [0, 1], [1, 1])  # empty interval
    assert e.value.code == S.SGCM_EINVAL
    assert S.lib().sgcm_grid_size(None) == -1
    S.lib().sgcm_grid_destroy(None)


def _ws(problem, n):
    out = ctypes.c_size_t(0)
    rc = S.lib().sgcm_solve_bvps_workspace(ctypes.byref(problem.c()), n, ctypes.byref(out))
    return rc, out.value


def test_problem_validation():
    good = S.Problem(N=64)
    rc, nbytes = _ws(good, 10)
    assert rc == S.SGCM_OK and nbytes > 0 and nbytes % 256 == 0
    assert _ws(good, 0) == (S.SGCM_OK, 0)
    bad = [dict(n=5), dict(m=0), dict(m=4), dict(N=0), dict(N=70000), dict(r_w=0.0), dict(T=-1.0),
           dict(J=(1.0, 0.0, 1.0)), dict(max_iter=-1), dict(tol=float("nan")), dict(model=7),
           dict(q_w=-1.0), dict(max_halvings=-1), dict(max_halvings=61), dict(continuation=-1),
           dict(continuation=65)]
    for kw in bad:
        p = S.Problem(**kw)
        assert _ws(p, 1)[0] == S.SGCM_EINVAL, kw
    assert _ws(S.Problem(precision=S.FP32), 1)[0] == S.SGCM_OK  # FP32 inexact Newton
    assert _ws(S.Problem(precision=7), 1)[0] == S.SGCM_EINVAL
    for kw in (dict(max_halvings=0), dict(max_halvings=60), dict(continuation=64),
               dict(m=2, B=W.input_matrix(2), continuation=4)):
        assert _ws(S.Problem(**kw), 1)[0] == S.SGCM_OK, kw
    # a continuation keeps the workspace of the problem itself
    assert _ws(S.Problem(m=2, B=W.input_matrix(2), continuation=4), 3) == _ws(S.Problem(), 3)


def test_entry_points_validate_before_device_work():
    L = S.lib()
    p = S.Problem()
    vp = ctypes.c_void_p
    # n_bvps == 0 is a no-op, negative is invalid, NULL outputs are invalid
    assert L.sgcm_solve_bvps(ctypes.byref(p.c()), 0, None, None, None, None, None, None, None, None, 0,
                             None) == S.SGCM_OK
    assert L.sgcm_solve_bvps(ctypes.byref(p.c()), -1, None, None, None, None, None, None, None, None, 0,
                             None) == S.SGCM_EINVAL
    assert L.sgcm_solve_bvps(ctypes.byref(p.c()), 4, None, None, None, None, None, None, None, None, 0,
                             None) == S.SGCM_EINVAL
    fake = vp(4096)
    # misaligned workspace and too-small workspace
    assert L.sgcm_solve_bvps(ctypes.byref(p.c()), 1, fake, fake, fake, None, None, fake, fake, vp(4100),
                             1 << 30, None) == S.SGCM_EINVAL
    assert L.sgcm_solve_bvps(ctypes.byref(p.c()), 1, fake, fake, fake, None, None, fake, fake, fake, 8,
                             None) == S.SGCM_EINVAL
    assert L.sgcm_characteristic_rhs(ctypes.byref(p.c()), 0, None, None, None, None) == S.SGCM_OK
    assert L.sgcm_characteristic_rhs(ctypes.byref(p.c()), 3, None, None, None, None) == S.SGCM_EINVAL
    g = S.Grid(6, 2, W.BOX_LO, W.BOX_HI)
    assert L.sgcm_eval_feedback(g.handle, 3, None, 0, None, None, S.FP64, None) == S.SGCM_OK
    assert L.sgcm_eval_feedback(g.handle, 3, fake, 10, fake, fake, S.FP32, None) == S.SGCM_EUNSUPPORTED
    assert L.sgcm_eval_feedback(g.handle, 0, fake, 10, fake, fake, S.FP64, None) == S.SGCM_EINVAL
    assert L.sgcm_eval_feedback(g.handle, 3, fake, -1, fake, fake, S.FP64, None) == S.SGCM_EINVAL
    assert L.sgcm_eval_feedback(None, 3, fake, 10, fake, fake, S.FP64, None) == S.SGCM_EINVAL
    assert L.sgcm_build_interpolant(g.handle, 3, fake, fake, None) == S.SGCM_EINVAL  # aliasing
    assert L.sgcm_build_interpolant(g.handle, 0, fake, vp(8192), None) == S.SGCM_EINVAL


def test_plan_entry_points_validate_before_device_work():
    L = S.lib()
    vp = ctypes.c_void_p
    out = vp(1234)
    assert L.sgcm_plan_create(ctypes.byref(S.Problem(N=0).c()), None, ctypes.byref(out)) == S.SGCM_EINVAL
    assert out.value is None  # cleared on failure
    assert L.sgcm_plan_create(ctypes.byref(S.Problem(model=7).c()), None, ctypes.byref(out)) == S.SGCM_EINVAL
    assert L.sgcm_plan_create(ctypes.byref(S.Problem().c()), None, None) == S.SGCM_EINVAL
    assert L.sgcm_plan_create(None, None, ctypes.byref(out)) == S.SGCM_EINVAL
    assert L.sgcm_solve_bvps_plan(None, 1, None, None, None, None, None, None, None, None, 0,
                                  None) == S.SGCM_EINVAL
    L.sgcm_plan_destroy(None)


def test_batch_create_validates_before_device_work():
    # every rejected argument is caught on the host, before any HIP call
    L = S.lib()
    p = S.Problem()
    vp = ctypes.c_void_p
    out = vp()

    def create(N, T, sched=(1, 0), n=None, prob=p):
        N = np.ascontiguousarray(N, dtype=np.int32)
        T = np.ascontiguousarray(T, dtype=np.float64)
        sc = S._CSchedule(*sched)
        return L.sgcm_batch_create(ctypes.byref(prob.c()), len(N) if n is None else n,
                                   N.ctypes.data_as(vp), T.ctypes.data_as(vp), ctypes.byref(sc),
                                   ctypes.byref(out))

    assert create([64, 0], [1.0, 1.0]) == S.SGCM_EINVAL          # N < 1
    assert create([64, 70000], [1.0, 1.0]) == S.SGCM_EINVAL      # N > 65536
    assert create([64, 64], [1.0, 0.0]) == S.SGCM_EINVAL         # T <= 0
    assert create([64, 64], [1.0, float("inf")]) == S.SGCM_EINVAL
    assert create([64], [1.0], n=0) == S.SGCM_EINVAL             # empty batch
    assert create([64], [1.0], sched=(2, 0)) == S.SGCM_EINVAL    # unknown order
    assert create([64], [1.0], sched=(0, 9)) == S.SGCM_EINVAL    # too many slots
    assert create([64], [1.0], prob=S.Problem(m=4)) == S.SGCM_EINVAL
    # continuation stages are launches of their own: not in a batch
    assert create([64], [1.0], prob=S.Problem(m=2, B=W.input_matrix(2), continuation=2)) == S.SGCM_EUNSUPPORTED
    assert out.value is None
    # the problem's own N and T are ignored by a batch: valid arguments get past
    # validation (without a GPU the device query then fails)
    rc = create([64], [1.0], prob=S.Problem(N=0, T=-1.0))
    assert rc in (S.SGCM_OK, S.SGCM_EDEVICE)
    if rc == S.SGCM_OK:
        L.sgcm_batch_destroy(out)
    nb = ctypes.c_size_t(0)
    assert L.sgcm_batch_workspace(None, ctypes.byref(nb)) == S.SGCM_EINVAL
    assert L.sgcm_solve_bvps_batch(None, None, None, None, None, None, None, None, 0, None) == S.SGCM_EINVAL
    L.sgcm_batch_destroy(None)


def test_total_error_argument_validation():
    # every rejection happens before any device work; fake non-null pointers
    # are never dereferenced on these paths
    L = S.lib()
    p = ctypes.c_void_p(256)
    assert L.sgcm_total_error(-1, 3, 2, p, p, p, p, p, p, None) == S.SGCM_EINVAL   # n < 0
    assert L.sgcm_total_error(10, 0, 2, p, p, p, p, p, p, None) == S.SGCM_EINVAL   # m < 1
    assert L.sgcm_total_error(10, 65, 2, p, p, p, p, p, p, None) == S.SGCM_EINVAL  # m > 64
    assert L.sgcm_total_error(10, 3, 0, p, p, p, p, p, p, None) == S.SGCM_EINVAL   # order < 1
    assert L.sgcm_total_error(10, 3, 17, p, p, p, p, p, p, None) == S.SGCM_EINVAL  # order > 16
    assert L.sgcm_total_error(10, 3, 2, p, p, p, p, p, None, None) == S.SGCM_EINVAL  # no stats
    assert L.sgcm_total_error(10, 3, 2, None, p, p, p, p, p, None) == S.SGCM_EINVAL  # no interp
    assert L.sgcm_total_error(10, 3, 2, p, p, p, p, None, p, None) == S.SGCM_EINVAL  # no err
    assert L.sgcm_total_error(2**62, 3, 2, p, p, p, p, p, p, None) == S.SGCM_EINVAL  # n * m overflows


def test_scheme_validation():
    # the four-point Lobatto IIIA formula: FP64 only, no plans or batches
    assert _ws(S.Problem(scheme=S.LOBATTO4), 2)[0] == S.SGCM_OK
    assert _ws(S.Problem(scheme=7), 1)[0] == S.SGCM_EINVAL
    assert _ws(S.Problem(scheme=S.LOBATTO4, precision=S.FP32), 1)[0] == S.SGCM_EUNSUPPORTED
    # its workspace per BVP (stages, their Jacobians and the condensation) is
    # larger than the trapezoid's
    assert _ws(S.Problem(scheme=S.LOBATTO4, N=64), 1)[1] > _ws(S.Problem(N=64), 1)[1]
    L = S.lib()
    out = ctypes.c_void_p()
    assert L.sgcm_plan_create(ctypes.byref(S.Problem(scheme=S.LOBATTO4).c()), None, ctypes.byref(out)) == \
        S.SGCM_EUNSUPPORTED
    N = np.ascontiguousarray([8], dtype=np.int32)
    T = np.ascontiguousarray([1.0])
    sc = S._CSchedule(1, 0)
    assert L.sgcm_batch_create(ctypes.byref(S.Problem(scheme=S.LOBATTO4).c()), 1, N.ctypes.data_as(ctypes.c_void_p),
                               T.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sc), ctypes.byref(out)) == \
        S.SGCM_EUNSUPPORTED


def test_tile_validation():
    # the tiles of the trapezoidal solve: sweep batch 8, 10, 12 or 16, forward chunk 8
    # or 12 (0: the defaults); they do not change the workspace
    for nb in (0, 8, 10, 12, 16):
        for fc in (0, 8, 12):
            assert _ws(S.Problem(sweep_batch=nb, forward_chunk=fc), 5) == _ws(S.Problem(), 5), (nb, fc)
    for kw in (dict(sweep_batch=-1), dict(forward_chunk=-8)):
        assert _ws(S.Problem(**kw), 1)[0] == S.SGCM_EINVAL, kw
    for kw in (dict(sweep_batch=9), dict(sweep_batch=14), dict(sweep_batch=20), dict(forward_chunk=10),
               dict(forward_chunk=16)):
        assert _ws(S.Problem(**kw), 1)[0] == S.SGCM_EUNSUPPORTED, kw


def _ex3(**kw):
    base = dict(model=S.MODEL_EXAMPLE3, n=3, m=1, T=5.0, N=64, tol=1e-10, max_iter=20)
    base.update(kw)
    return S.Problem(**base)


def test_example3_validation():
    # Example III (Sec. 5.3): its own workspace (Y, trial point, step and
    # residual, Phi and its Jacobian per mesh point, and per interval a slot
    # of 42 doubles for its 6 x 7 element, then its sweep values; rounded up
    # to 32 doubles), validated before device work
    NP = 65
    per = (NP * 6 * 4 + NP * 6 + NP * 36 + 64 * 42 + 31) // 32 * 32
    # plus the launch order (int32 per BVP, rounded up to 256 bytes)
    assert _ws(_ex3(), 7) == (S.SGCM_OK, 7 * per * 8 + 256)
    assert _ws(_ex3(continuation=2), 1) == (S.SGCM_OK, per * 8 + 256)
    assert _ws(_ex3(), 8193) == (S.SGCM_OK, 8193 * per * 8)  # above 8192 BVPs: no order
    for kw in (dict(n=6), dict(m=3), dict(T=0.0), dict(N=0), dict(max_iter=-1), dict(continuation=65)):
        assert _ws(_ex3(**kw), 1)[0] == S.SGCM_EINVAL, kw
    for kw in (dict(precision=S.FP32), dict(scheme=S.LOBATTO4)):
        assert _ws(_ex3(**kw), 1)[0] == S.SGCM_EUNSUPPORTED, kw
    L = S.lib()
    p = _ex3()
    args = (None,) * 8 + (0, None)
    assert L.sgcm_solve_bvps_tx(ctypes.byref(p.c()), 0, *args) == S.SGCM_OK
    assert L.sgcm_solve_bvps_tx(ctypes.byref(p.c()), 3, *args) == S.SGCM_EINVAL
    # the (t, x) solve covers Example III only; plans and batches none of it
    assert L.sgcm_solve_bvps_tx(ctypes.byref(S.Problem().c()), 3, *args) == S.SGCM_EUNSUPPORTED
    h = ctypes.c_void_p()
    assert L.sgcm_plan_create(ctypes.byref(p.c()), None, ctypes.byref(h)) == S.SGCM_EUNSUPPORTED
