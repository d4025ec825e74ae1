"""Python binding of libsgcm, the MI355X (gfx950) sparse grid characteristics
method (Kang & Wilcox): per-node characteristic BVPs (Sec. 3.1), the
hierarchical sparse-grid interpolant (Sec. 3.2-3.3) and on-line feedback
evaluation.

This module only marshals arguments: every step runs in the HIP kernels of
``libsgcm.so`` behind the C ABI of ``include/sgcm.h``.  The functions named
``sgcm_*`` mirror the C entry points one to one; the few helpers below them
allocate the outputs with PyTorch (device memory and streams only) and call
those entry points.  Importing works without the library; the first call
raises if ``libsgcm.so`` has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgcm.so")

SGCM_OK, SGCM_EINVAL, SGCM_ENOMEM, SGCM_EDEVICE, SGCM_EUNSUPPORTED, SGCM_ENOTCONVERGED = 0, -1, -2, -3, -4, -5
CONVERGED, MAXITER, SINGULAR, NONFINITE = 0, 1, 2, 3
MODEL_RIGID_BODY, MODEL_LINEARISED, MODEL_EXAMPLE3 = 0, 1, 2
FP64, FP32 = 0, 1
TRAPEZOID, LOBATTO4 = 0, 1  # collocation formulas (sgcm_scheme)

# every extern "C" symbol declared in include/sgcm.h
EXPORTS = ("sgcm_strerror", "sgcm_version", "sgcm_solve_bvps_workspace", "sgcm_solve_bvps", "sgcm_solve_bvps_static",
           "sgcm_solve_bvps_tx",
           "sgcm_characteristic_rhs", "sgcm_plan_create", "sgcm_solve_bvps_plan", "sgcm_plan_destroy",
           "sgcm_batch_create", "sgcm_batch_workspace", "sgcm_solve_bvps_batch",
           "sgcm_batch_destroy", "sgcm_grid_create", "sgcm_grid_upload", "sgcm_grid_size", "sgcm_grid_nodes",
           "sgcm_grid_keys", "sgcm_grid_destroy", "sgcm_build_interpolant", "sgcm_eval_feedback",
           "sgcm_eval_feedback_f32", "sgcm_total_error")


class SgcmError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what or "sgcm", strerror(code), code))


class _CProblem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("J", ctypes.c_double * 3), ("B", ctypes.c_double * 9),
                ("q_w", ctypes.c_double), ("r_w", ctypes.c_double), ("p_w", ctypes.c_double),
                ("T", ctypes.c_double), ("N", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("continuation", ctypes.c_int32),
                ("scheme", ctypes.c_int32), ("sweep_batch", ctypes.c_int32),
                ("forward_chunk", ctypes.c_int32)]


@dataclass
class Problem:
    """sgcm_problem: the optimal-control problem of Sec. 2 and its mesh."""
    model: int = MODEL_RIGID_BODY
    m: int = 3
    J: tuple = (2.0, 3.0, 4.0)
    B: np.ndarray = field(default_factory=lambda: np.eye(3))  # 3 x m
    q_w: float = 1.0
    r_w: float = 0.1
    p_w: float = 10.0
    T: float = 20.0
    N: int = 64
    tol: float = 1e-10
    max_iter: int = 20
    precision: int = FP64
    n: int = 6
    max_halvings: int = 10  # backtracking cap of each counted Newton step (0: full steps)
    continuation: int = 0   # two controls: stages of the virtual-torque continuation
    scheme: int = TRAPEZOID  # collocation formula
    sweep_batch: int = 0     # tile: intervals per sweep batch (8, 10, 12 or 16; 0: 8)
    forward_chunk: int = 0   # tile: intervals per forward-pass chunk (8 or 12; 0: 12)

    def c(self) -> _CProblem:
        p = _CProblem()
        p.model, p.n, p.m = int(self.model), int(self.n), int(self.m)
        for i in range(3):
            p.J[i] = float(self.J[i])
        Bm = np.asarray(self.B, dtype=np.float64).reshape(3, -1)
        flat = np.zeros(9)
        flat[: Bm.size] = Bm.T.reshape(-1)  # column-major B[i + 3 j]
        for i in range(9):
            p.B[i] = float(flat[i])
        p.q_w, p.r_w, p.p_w, p.T = float(self.q_w), float(self.r_w), float(self.p_w), float(self.T)
        p.N, p.tol, p.max_iter = int(self.N), float(self.tol), int(self.max_iter)
        p.precision = int(self.precision)
        p.max_halvings, p.continuation = int(self.max_halvings), int(self.continuation)
        p.scheme = int(self.scheme)
        p.sweep_batch, p.forward_chunk = int(self.sweep_batch), int(self.forward_chunk)
        return p


_lib = None


class _CSchedule(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("slots_per_cu", ctypes.c_int32)]


def lib() -> ctypes.CDLL:
    """The loaded libsgcm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsgcm.so is not built (expected at %s); run "
                           "`python -m paper_1507_04769_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER(_CProblem)
    sig = {
        "sgcm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sgcm_version": (ctypes.c_int, []),
        "sgcm_solve_bvps_workspace": (ctypes.c_int, [P, i64, ctypes.POINTER(ctypes.c_size_t)]),
        "sgcm_solve_bvps": (ctypes.c_int, [P, i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "sgcm_solve_bvps_static": (ctypes.c_int, [P, i64, vp, vp, vp, vp, vp, vp, vp, vp]),
        "sgcm_solve_bvps_tx": (ctypes.c_int, [P, i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "sgcm_characteristic_rhs": (ctypes.c_int, [P, i64, vp, vp, vp, vp]),
        "sgcm_plan_create": (ctypes.c_int, [P, vp, ctypes.POINTER(vp)]),
        "sgcm_solve_bvps_plan": (ctypes.c_int, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "sgcm_plan_destroy": (None, [vp]),
        "sgcm_batch_create": (ctypes.c_int, [P, i64, vp, vp, ctypes.POINTER(_CSchedule), ctypes.POINTER(vp)]),
        "sgcm_batch_workspace": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "sgcm_solve_bvps_batch": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "sgcm_batch_destroy": (None, [vp]),
        "sgcm_grid_create": (ctypes.c_int, [i32, i32, vp, vp, ctypes.POINTER(vp)]),
        "sgcm_grid_upload": (ctypes.c_int, [vp, vp]),
        "sgcm_grid_size": (i64, [vp]),
        "sgcm_grid_nodes": (ctypes.c_int, [vp, vp]),
        "sgcm_grid_keys": (ctypes.c_int, [vp, vp]),
        "sgcm_grid_destroy": (None, [vp]),
        "sgcm_build_interpolant": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "sgcm_eval_feedback": (ctypes.c_int, [vp, i32, vp, i64, vp, vp, i32, vp]),
        "sgcm_eval_feedback_f32": (ctypes.c_int, [vp, i32, vp, i64, vp, vp, vp]),
        "sgcm_total_error": (ctypes.c_int, [i64, i32, i32, vp, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().sgcm_strerror(code).decode()
    except RuntimeError:
        return "status %d" % code


def _check(rc: int, what: str):
    if rc != SGCM_OK:
        raise SgcmError(rc, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t, dtype=None, name="tensor", numel=None):
    """Device pointer of a contiguous CUDA tensor (or None); with numel, the
    tensor must hold at least that many elements (checked on the host so an
    undersized buffer never reaches a kernel)."""
    if t is None:
        return None
    import torch
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# C entry points
# ---------------------------------------------------------------------------

def sgcm_version() -> int:
    return lib().sgcm_version()


def sgcm_solve_bvps_workspace(problem: Problem, n_bvps: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().sgcm_solve_bvps_workspace(ctypes.byref(problem.c()), int(n_bvps), ctypes.byref(out)),
           "sgcm_solve_bvps_workspace")
    return int(out.value)


def _solve_args(problem: Problem, x0, lambda0, u0, V, traj, status, iters, workspace, stream, cols=None):
    import torch
    f64, i32 = torch.float64, torch.int32
    ns = int(problem.n)
    cols = ns if cols is None else cols
    n = x0.shape[0] if x0 is not None else 0
    if x0 is not None and (x0.dim() != 2 or x0.shape[1] != cols):
        raise ValueError("the initial points must be n x %d" % cols)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    m, NP = int(problem.m), int(problem.N) + 1
    return (int(n), _ptr(x0, f64, "x0"), _ptr(lambda0, f64, "lambda0", ns * n), _ptr(u0, f64, "u0", m * n),
            _ptr(V, f64, "V", n), _ptr(traj, f64, "traj", 2 * ns * NP * n), _ptr(status, i32, "status", n),
            _ptr(iters, i32, "iters", n), _ptr(workspace, None, "workspace"), ctypes.c_size_t(ws_bytes),
            _stream(stream))


def sgcm_solve_bvps(problem: Problem, x0, lambda0, u0, V, traj, status, iters, workspace, stream=None):
    args = _solve_args(problem, x0, lambda0, u0, V, traj, status, iters, workspace, stream)
    _check(lib().sgcm_solve_bvps(ctypes.byref(problem.c()), *args), "sgcm_solve_bvps")


STATIC_SCRATCH_BYTES = 64 << 20  # SGCM_STATIC_SCRATCH_BYTES


def sgcm_solve_bvps_tx(problem: Problem, tx, lambda0, u0, V, traj, status, iters, workspace, stream=None):
    """The BVPs from the (t0, x0) rows of tx (n x (1 + problem.n)), each over [t0, T]."""
    args = _solve_args(problem, tx, lambda0, u0, V, traj, status, iters, workspace, stream, cols=1 + int(problem.n))
    _check(lib().sgcm_solve_bvps_tx(ctypes.byref(problem.c()), *args), "sgcm_solve_bvps_tx")


def sgcm_solve_bvps_static(problem: Problem, x0, lambda0, u0, V, traj, status, iters, stream=None):
    """The solve without a workspace argument and without allocation (the
    library's per-device scratch); calls on one device must not overlap."""
    args = _solve_args(problem, x0, lambda0, u0, V, traj, status, iters, None, stream)
    n, ptrs, strm = args[0], args[1:8], args[10]
    _check(lib().sgcm_solve_bvps_static(ctypes.byref(problem.c()), n, *ptrs, strm), "sgcm_solve_bvps_static")


class Plan:
    """sgcm_plan: a problem with the first Newton steps of the six unit
    initial states (the step is linear in the initial state), owned by
    libsgcm; creating it runs one small solve and synchronizes the stream."""

    def __init__(self, problem: Problem, stream=None):
        self.problem = problem
        h = ctypes.c_void_p()
        _check(lib().sgcm_plan_create(ctypes.byref(problem.c()), _stream(stream), ctypes.byref(h)),
               "sgcm_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.sgcm_plan_destroy(h)
            self._h = None


def sgcm_solve_bvps_plan(plan: Plan, x0, lambda0, u0, V, traj, status, iters, workspace, stream=None):
    args = _solve_args(plan.problem, x0, lambda0, u0, V, traj, status, iters, workspace, stream)
    _check(lib().sgcm_solve_bvps_plan(plan.handle, *args), "sgcm_solve_bvps_plan")


def sgcm_characteristic_rhs(problem: Problem, y, phi, dphi=None, stream=None):
    import torch
    ny = 2 * int(problem.n)
    if y.dim() != 2 or y.shape[1] != ny:
        raise ValueError("y must be n x %d" % ny)
    n = y.shape[0]
    rc = lib().sgcm_characteristic_rhs(ctypes.byref(problem.c()), int(n), _ptr(y, torch.float64, "y"),
                                       _ptr(phi, torch.float64, "phi", ny * n),
                                       _ptr(dphi, torch.float64, "dphi", ny * ny * n), _stream(stream))
    _check(rc, "sgcm_characteristic_rhs")


ORDER_GIVEN, ORDER_LONGEST_FIRST = 0, 1


class Batch:
    """sgcm_batch: a plan for BVPs of one problem with per-BVP mesh size N and
    horizon T (the problem's own N and T are ignored), owned by libsgcm."""

    def __init__(self, problem: Problem, N, T, order: int = ORDER_LONGEST_FIRST, slots_per_cu: int = 0):
        N = np.ascontiguousarray(N, dtype=np.int32).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        if N.shape != T.shape:
            raise ValueError("N and T must have the same length")
        self.n, self.N, self.T = int(N.size), N, T
        self.m = int(problem.m)
        self.schedule = (int(order), int(slots_per_cu))
        h = ctypes.c_void_p()
        sc = _CSchedule(int(order), int(slots_per_cu))
        _check(lib().sgcm_batch_create(ctypes.byref(problem.c()), self.n, N.ctypes.data_as(ctypes.c_void_p),
                                       T.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sc), ctypes.byref(h)),
               "sgcm_batch_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self) -> int:
        out = ctypes.c_size_t(0)
        _check(lib().sgcm_batch_workspace(self._h, ctypes.byref(out)), "sgcm_batch_workspace")
        return int(out.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.sgcm_batch_destroy(h)
            self._h = None


def sgcm_solve_bvps_batch(batch: Batch, x0, lambda0, u0, V, status, iters, workspace, stream=None):
    import torch
    f64, i32 = torch.float64, torch.int32
    n, m = batch.n, batch.m
    if x0.dim() != 2 or x0.shape[1] != 6 or x0.shape[0] != n:
        raise ValueError("x0 must be n x 6 with n = %d" % n)
    ws_bytes = workspace.numel() * workspace.element_size()
    rc = lib().sgcm_solve_bvps_batch(batch.handle, _ptr(x0, f64, "x0"), _ptr(lambda0, f64, "lambda0", 6 * n),
                                     _ptr(u0, f64, "u0", m * n), _ptr(V, f64, "V", n),
                                     _ptr(status, i32, "status", n), _ptr(iters, i32, "iters", n),
                                     _ptr(workspace, None, "workspace"), ctypes.c_size_t(ws_bytes),
                                     _stream(stream))
    _check(rc, "sgcm_solve_bvps_batch")


class Grid:
    """sgcm_grid: the Smolyak CGL sparse grid (Sec. 3.2) owned by libsgcm."""

    def __init__(self, d: int, level: int, lo, hi):
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        if lo.size != d or hi.size != d:
            raise ValueError("lo and hi need d entries")
        h = ctypes.c_void_p()
        _check(lib().sgcm_grid_create(int(d), int(level), lo.ctypes.data_as(ctypes.c_void_p),
                                      hi.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
               "sgcm_grid_create")
        self._h = h
        self._uploaded = set()  # devices that hold the grid's tables
        self.d, self.level = int(d), int(level)
        self.lo, self.hi = lo.copy(), hi.copy()

    @property
    def handle(self):
        return self._h

    def upload(self, stream=None):
        """sgcm_grid_upload: the grid's device tables on the current device
        (allocated, then copied on the stream); a no-op once done there."""
        import torch
        dev = torch.cuda.current_device()
        if dev not in self._uploaded:
            _check(lib().sgcm_grid_upload(self._h, _stream(stream)), "sgcm_grid_upload")
            self._uploaded.add(dev)

    def __len__(self):
        return int(lib().sgcm_grid_size(self._h))

    @property
    def size(self) -> int:
        return len(self)

    def nodes(self) -> np.ndarray:
        out = np.zeros((len(self), self.d))
        _check(lib().sgcm_grid_nodes(self._h, out.ctypes.data_as(ctypes.c_void_p)), "sgcm_grid_nodes")
        return out

    def keys(self) -> np.ndarray:
        out = np.zeros((len(self), self.d), dtype=np.int32)
        _check(lib().sgcm_grid_keys(self._h, out.ctypes.data_as(ctypes.c_void_p)), "sgcm_grid_keys")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sgcm_grid_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sgcm_build_interpolant(grid: Grid, values, surplus, stream=None):
    import torch
    if values.dim() != 2 or values.shape[0] != len(grid):
        raise ValueError("values must be M x m with M = %d" % len(grid))
    m = values.shape[1]
    grid.upload(stream)
    rc = lib().sgcm_build_interpolant(grid.handle, int(m), _ptr(values, torch.float64, "values"),
                                      _ptr(surplus, torch.float64, "surplus", len(grid) * m),
                                      _stream(stream))
    _check(rc, "sgcm_build_interpolant")


def sgcm_eval_feedback(grid: Grid, surplus, xq, uq, precision: int = FP64, stream=None):
    import torch
    if surplus.dim() != 2 or surplus.shape[0] != len(grid):
        raise ValueError("surplus must be M x m with M = %d" % len(grid))
    if xq.dim() != 2 or xq.shape[1] != grid.d:
        raise ValueError("xq must be n_q x %d" % grid.d)
    m, nq = surplus.shape[1], xq.shape[0]
    grid.upload(stream)
    rc = lib().sgcm_eval_feedback(grid.handle, int(m), _ptr(surplus, torch.float64, "surplus"),
                                  int(nq), _ptr(xq, torch.float64, "xq"),
                                  _ptr(uq, torch.float64, "uq", nq * m), int(precision), _stream(stream))
    _check(rc, "sgcm_eval_feedback")


def sgcm_total_error(interp, coarse, fine, ref, err, stats, stream=None, order: int = 2):
    import torch
    if interp.dim() != 2:
        raise ValueError("interp must be n x m")
    n, m = interp.shape
    for name, t in (("coarse", coarse), ("fine", fine)):
        if tuple(t.shape) != (n, m):
            raise ValueError("%s must be %d x %d" % (name, n, m))
    f64 = torch.float64
    rc = lib().sgcm_total_error(int(n), int(m), int(order), _ptr(interp, f64, "interp"),
                                _ptr(coarse, f64, "coarse"), _ptr(fine, f64, "fine"), _ptr(ref, f64, "ref", n * m),
                                _ptr(err, f64, "err", n), _ptr(stats, f64, "stats", 5), _stream(stream))
    _check(rc, "sgcm_total_error")


# ---------------------------------------------------------------------------
# allocation helpers (outputs allocated with torch; compute in libsgcm)
# ---------------------------------------------------------------------------

@dataclass
class BVPSolution:
    lambda0: "object"
    u0: "object"
    V: "object"
    traj: "object"
    status: "object"
    iters: "object"


def solve_bvps(problem: Problem, x0, want_traj: bool = False, want_V: bool = True, workspace=None,
               stream=None, plan: "Plan | None" = None) -> BVPSolution:
    """Solve the BVPs from the initial states x0 (n x 6, device); with a plan
    (whose problem is then the one solved) each first Newton step is formed
    from the plan."""
    import torch
    if plan is not None:
        problem = plan.problem
    dev = x0.device
    n, ns = x0.shape[0], int(problem.n)
    lam = torch.empty((n, ns), dtype=torch.float64, device=dev)
    u0 = torch.empty((n, problem.m), dtype=torch.float64, device=dev)
    V = torch.empty((n,), dtype=torch.float64, device=dev) if want_V else None
    traj = torch.empty((n, problem.N + 1, 2 * ns), dtype=torch.float64, device=dev) if want_traj else None
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    it = torch.empty((n,), dtype=torch.int32, device=dev)
    if workspace is None:
        nbytes = sgcm_solve_bvps_workspace(problem, n)
        workspace = torch.empty((max(nbytes, 256) + 255) // 256 * 32, dtype=torch.float64, device=dev)
    if plan is not None:
        sgcm_solve_bvps_plan(plan, x0, lam, u0, V, traj, st, it, workspace, stream)
    else:
        sgcm_solve_bvps(problem, x0, lam, u0, V, traj, st, it, workspace, stream)
    return BVPSolution(lam, u0, V, traj, st, it)


def solve_bvps_tx(problem: Problem, tx, want_traj: bool = False, want_V: bool = True, workspace=None,
                  stream=None) -> BVPSolution:
    """The BVPs from the points (t0, x0) of a grid in (t, x) (rows of tx,
    n x (1 + problem.n), device), each over [t0, problem.T]: the time
    variable as a grid dimension (Sec. 5.3)."""
    import torch
    dev = tx.device
    n, ns = tx.shape[0], int(problem.n)
    lam = torch.empty((n, ns), dtype=torch.float64, device=dev)
    u0 = torch.empty((n, problem.m), dtype=torch.float64, device=dev)
    V = torch.empty((n,), dtype=torch.float64, device=dev) if want_V else None
    traj = torch.empty((n, problem.N + 1, 2 * ns), dtype=torch.float64, device=dev) if want_traj else None
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    it = torch.empty((n,), dtype=torch.int32, device=dev)
    if workspace is None:
        nbytes = sgcm_solve_bvps_workspace(problem, n)
        workspace = torch.empty((max(nbytes, 256) + 255) // 256 * 32, dtype=torch.float64, device=dev)
    sgcm_solve_bvps_tx(problem, tx, lam, u0, V, traj, st, it, workspace, stream)
    return BVPSolution(lam, u0, V, traj, st, it)


def batch_workspace(batch: Batch, device):
    import torch
    nbytes = batch.workspace_bytes()
    return torch.empty((max(nbytes, 256) + 255) // 256 * 32, dtype=torch.float64, device=device)


def solve_bvps_batch(batch: Batch, x0, want_V: bool = True, workspace=None, stream=None) -> BVPSolution:
    import torch
    dev = x0.device
    n = batch.n
    lam = torch.empty((n, 6), dtype=torch.float64, device=dev)
    u0 = torch.empty((n, batch.m), dtype=torch.float64, device=dev)
    V = torch.empty((n,), dtype=torch.float64, device=dev) if want_V else None
    st = torch.empty((n,), dtype=torch.int32, device=dev)
    it = torch.empty((n,), dtype=torch.int32, device=dev)
    if workspace is None:
        workspace = batch_workspace(batch, dev)
    sgcm_solve_bvps_batch(batch, x0, lam, u0, V, st, it, workspace, stream)
    return BVPSolution(lam, u0, V, None, st, it)


def characteristic_rhs(problem: Problem, y, jacobian: bool = True, stream=None):
    import torch
    ny = 2 * int(problem.n)
    phi = torch.empty_like(y)
    dphi = torch.empty((y.shape[0], ny, ny), dtype=torch.float64, device=y.device) if jacobian else None
    sgcm_characteristic_rhs(problem, y, phi, dphi, stream)
    return phi, dphi


def require_converged(status):
    """Raise SgcmError(SGCM_ENOTCONVERGED) unless every status is CONVERGED
    (the node values of a BVP that did not converge are its last iterate and
    are not interpolated).  Reads the statuses on the host."""
    bad = int((status != CONVERGED).sum().item())
    if bad:
        raise SgcmError(SGCM_ENOTCONVERGED, "%d of %d BVPs did not converge" % (bad, status.numel()))


def build_interpolant(grid: Grid, values, stream=None, status=None):
    """Surpluses of the node values (M x m, device).  With `status` (the
    statuses of the solve that produced the values) the build is refused
    unless every BVP converged."""
    import torch
    if status is not None:
        require_converged(status)
    surplus = torch.empty_like(values)
    sgcm_build_interpolant(grid, values, surplus, stream)
    return surplus


def build_feedback_interpolant(grid: Grid, solution: "BVPSolution", stream=None):
    """The interpolant of the feedback u(0, x) from a solve at the grid's
    nodes; raises SgcmError(SGCM_ENOTCONVERGED) if any node's BVP did not
    converge."""
    return build_interpolant(grid, solution.u0, stream, status=solution.status)


def sgcm_eval_feedback_f32(grid: Grid, surplus, xq, uq, stream=None):
    import torch
    f32 = torch.float32
    m = surplus.shape[1]
    if xq.dim() != 2 or xq.shape[1] != grid.d:
        raise ValueError("xq must be n x %d" % grid.d)
    n = xq.shape[0]
    grid.upload(stream)
    rc = lib().sgcm_eval_feedback_f32(grid.handle, int(m), _ptr(surplus, f32, "surplus", len(grid) * m), int(n),
                                      _ptr(xq, f32, "xq"), _ptr(uq, f32, "uq", n * m), _stream(stream))
    _check(rc, "sgcm_eval_feedback_f32")


def eval_feedback_f32(grid: Grid, surplus, xq, stream=None):
    """FP32 evaluation: surplus and xq are rounded to FP32 if they are not
    already; returns FP32 results."""
    import torch
    surplus = surplus.to(torch.float32).contiguous()
    xq = xq.to(torch.float32).contiguous()
    uq = torch.empty((xq.shape[0], surplus.shape[1]), dtype=torch.float32, device=xq.device)
    sgcm_eval_feedback_f32(grid, surplus, xq, uq, stream)
    return uq


def eval_feedback(grid: Grid, surplus, xq, precision: int = FP64, stream=None):
    import torch
    uq = torch.empty((xq.shape[0], surplus.shape[1]), dtype=torch.float64, device=xq.device)
    sgcm_eval_feedback(grid, surplus, xq, uq, precision, stream)
    return uq


def total_error(interp, coarse, fine, stream=None, order: int = 2):
    """The total-error estimate of the interpolant at sample states: returns
    (ref, err, stats) with ref = (2^p fine - coarse) / (2^p - 1) (n x m), err
    the per-sample max error (n) and stats = [max err, RMS err,
    max |fine - ref|, mean err, mean relative err] (device tensors)."""
    import torch
    n, m = interp.shape
    ref = torch.empty((n, m), dtype=torch.float64, device=interp.device)
    err = torch.empty((n,), dtype=torch.float64, device=interp.device)
    stats = torch.empty((5,), dtype=torch.float64, device=interp.device)
    sgcm_total_error(interp, coarse, fine, ref, err, stats, stream, order)
    return ref, err, stats
