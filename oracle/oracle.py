"""ctypes binding of the FP64 CPU oracle (``sgcm_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference the GPU
library is checked against; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import this module.  It shares nothing with
the GPU library except the seeded input generators.

Every function follows a passage of Kang & Wilcox (see ``sgcm_oracle.cpp``):
the CGL sparse grid (Sec. 3.2, eq. CGL), hierarchical surpluses (Sec. 3.3,
eq. interpo), the combination formula (eq. interpolation2), and the
characteristic BVP (Sec. 3.1, eq. hamchar / optuv) by trapezoidal collocation
and Newton's method; the Monte Carlo total-error estimate (Sec. 4.3) is plain
numpy here (``total_error``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgcm_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

RIGID_BODY, LINEARISED, EXAMPLE3 = 0, 1, 2
TRAPEZOID, LOBATTO4 = 0, 1  # collocation formulas (two- and four-point Lobatto IIIA)
CONVERGED, MAXITER, SINGULAR, NONFINITE = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, OpenMP) next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("J", ctypes.c_double * 3), ("B", ctypes.c_double * 9),
                ("q_w", ctypes.c_double), ("r_w", ctypes.c_double), ("p_w", ctypes.c_double),
                ("T", ctypes.c_double), ("N", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_halvings", ctypes.c_int32),
                ("continuation", ctypes.c_int32), ("scheme", ctypes.c_int32)]


@dataclass
class Problem:
    """Optimal-control problem of Sec. 2 for one of the oracle's models."""
    model: int = RIGID_BODY
    n: int = 6
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
    max_halvings: int = 10   # backtracking cap of each Newton step (0: full steps)
    continuation: int = 0    # two controls: stages of the virtual-torque continuation
    scheme: int = TRAPEZOID  # collocation formula

    def c(self) -> _Problem:
        p = _Problem()
        p.model, p.n, p.m = self.model, self.n, self.m
        for i in range(3):
            p.J[i] = float(self.J[i])
        B = np.zeros(9)
        if self.model != EXAMPLE3:
            Bm = np.asarray(self.B, dtype=np.float64).reshape(3, self.m)
            B[: 3 * self.m] = Bm.T.reshape(-1)  # column-major
        for i in range(9):
            p.B[i] = B[i]
        p.q_w, p.r_w, p.p_w = self.q_w, self.r_w, self.p_w
        p.T, p.N, p.tol, p.max_iter = self.T, self.N, self.tol, self.max_iter
        p.max_halvings, p.continuation = self.max_halvings, self.continuation
        p.scheme = self.scheme
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        # SGCM_ORACLE_LIB: another build of the same source (the host
        # sanitizer test loads an AddressSanitizer build this way)
        _lib = ctypes.CDLL(os.environ.get("SGCM_ORACLE_LIB") or build())
        P = ctypes.POINTER(_Problem)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        i64, ci = ctypes.c_int64, ctypes.c_int
        sig = {
            "oracle_phi": (None, [P, i64, d, d, d]),
            "oracle_ustar": (None, [P, i64, d, d]),
            "oracle_residual": (None, [P, i64, d, d, d, ci]),
            "oracle_jacobian_dense": (None, [P, d, d]),
            "oracle_solve_bvps": (None, [P, i64, d, d, d, d, d, i32, i32, d, ci]),
            "oracle_solve_bvps_full": (None, [P, i64, d, d, d, d, d, i32, i32, d, d, ci]),
            "oracle_collocation_dim": (i64, [P]),
            "oracle_lobatto_tableau": (None, [d, d]),
            "oracle_grid_size": (i64, [ci, ci]),
            "oracle_grid": (i64, [ci, ci, d, d, d, d, i32, i32]),
            "oracle_lagrange": (None, [ci, ci, i64, d, d]),
            "oracle_cgl_points": (None, [ci, d]),
            "oracle_build_surplus": (None, [ci, ci, ci, d, d, ci]),
            "oracle_eval_hier": (None, [ci, ci, ci, d, d, d, i64, d, d, ci]),
            "oracle_eval_comb": (None, [ci, ci, ci, d, d, d, i64, d, d, ci]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype, f.argtypes = res, args
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# --- characteristic equations ---------------------------------------------

def phi(prob: Problem, y, jacobian: bool = True):
    """Phi(y) = [dH/dlambda; -dH/dx] at u* (eq. hamchar) and dPhi/dy."""
    ny = 2 * prob.n
    y = _f64(y).reshape(-1, ny)
    P = np.zeros_like(y)
    D = np.zeros((y.shape[0], ny, ny)) if jacobian else None
    lib().oracle_phi(ctypes.byref(prob.c()), y.shape[0], _dp(y), _dp(P), _dp(D))
    return (P, D) if jacobian else P


def ustar(prob: Problem, y):
    y = _f64(y).reshape(-1, 2 * prob.n)
    u = np.zeros((y.shape[0], prob.m))
    lib().oracle_ustar(ctypes.byref(prob.c()), y.shape[0], _dp(y), _dp(u))
    return u


def lobatto_tableau():
    """(c, A) of the four-point Lobatto IIIA formula (4 and 4 x 4)."""
    c, a = np.zeros(4), np.zeros(16)
    lib().oracle_lobatto_tableau(_dp(c), _dp(a))
    return c, a.reshape(4, 4)


def collocation_dim(prob: Problem) -> int:
    """Unknowns of the collocation system: 2n (N + 1) for the trapezoid,
    2n (3N + 1) for the four-point Lobatto IIIA formula (with its stages)."""
    return int(lib().oracle_collocation_dim(ctypes.byref(prob.c())))


def residual(prob: Problem, x0, traj, nthreads: int | None = None):
    """Collocation residual F(Y) of given unknown vectors (nb x dim; for the
    trapezoid the trajectories nb x (N+1) x 2n)."""
    x0 = _f64(x0).reshape(-1, prob.n)
    nb = x0.shape[0]
    Y = _f64(traj).reshape(nb, -1)
    F = np.zeros_like(Y)
    lib().oracle_residual(ctypes.byref(prob.c()), nb, _dp(x0), _dp(Y), _dp(F),
                          nthreads or default_threads())
    return F


def jacobian_dense(prob: Problem, Y):
    dim = collocation_dim(prob)
    Y = _f64(Y).reshape(dim)
    Jd = np.zeros((dim, dim))
    lib().oracle_jacobian_dense(ctypes.byref(prob.c()), _dp(Y), _dp(Jd))
    return Jd


@dataclass
class BVPResult:
    lambda0: np.ndarray
    u0: np.ndarray
    V: np.ndarray
    traj: np.ndarray | None
    status: np.ndarray
    iters: np.ndarray
    fnorm: np.ndarray
    unknowns: np.ndarray | None = None


def solve_bvps(prob: Problem, x0, want_traj: bool = False, nthreads: int | None = None,
               want_unknowns: bool = False):
    """Solve the characteristic BVP (eq. hamchar) from every row of x0; traj
    holds the mesh values, unknowns the whole unknown vector."""
    n, m, N = prob.n, prob.m, prob.N
    x0 = _f64(x0).reshape(-1, n)
    nb = x0.shape[0]
    lam = np.zeros((nb, n))
    u0 = np.zeros((nb, m))
    V = np.zeros(nb)
    traj = np.zeros((nb, N + 1, 2 * n)) if want_traj else None
    unk = np.zeros((nb, collocation_dim(prob))) if want_unknowns else None
    st = np.zeros(nb, dtype=np.int32)
    it = np.zeros(nb, dtype=np.int32)
    fn = np.zeros(nb)
    lib().oracle_solve_bvps_full(ctypes.byref(prob.c()), nb, _dp(x0), _dp(lam), _dp(u0), _dp(V),
                                 _dp(traj), _ip(st), _ip(it), _dp(fn), _dp(unk), nthreads or default_threads())
    return BVPResult(lam, u0, V, traj, st, it, fn, unk)


# --- sparse grid and interpolation -----------------------------------------

def grid_size(d: int, level: int) -> int:
    return int(lib().oracle_grid_size(d, level))


@dataclass
class Grid:
    nodes: np.ndarray   # M x d, box coordinates, canonical order
    xi: np.ndarray      # M x d, [0,1] coordinates
    keys: np.ndarray    # M x d point ids
    levels: np.ndarray  # M x d multi-indices


def grid(d: int, level: int, lo=None, hi=None) -> Grid:
    lo = _f64(np.zeros(d) if lo is None else lo)
    hi = _f64(np.ones(d) if hi is None else hi)
    M = grid_size(d, level)
    nodes = np.zeros((M, d))
    xi = np.zeros((M, d))
    keys = np.zeros((M, d), dtype=np.int32)
    levels = np.zeros((M, d), dtype=np.int32)
    lib().oracle_grid(d, level, _dp(lo), _dp(hi), _dp(nodes), _dp(xi), _ip(keys), _ip(levels))
    return Grid(nodes, xi, keys, levels)


def cgl_points(i: int):
    n = 1 if i == 1 else 2 ** (i - 1) + 1
    out = np.zeros(n)
    lib().oracle_cgl_points(i, _dp(out))
    return out


def lagrange(i: int, k: int, x):
    """u^i_k(x): Lagrange basis on X^i for its k-th point (1-based)."""
    x = _f64(x).reshape(-1)
    out = np.zeros_like(x)
    lib().oracle_lagrange(i, k, x.size, _dp(x), _dp(out))
    return out


def build_surplus(d: int, level: int, values, nthreads: int | None = None):
    values = _f64(values)
    M, m = values.shape
    out = np.zeros_like(values)
    lib().oracle_build_surplus(d, level, m, _dp(values), _dp(out), nthreads or default_threads())
    return out


def eval_hier(d: int, level: int, surplus, xq, lo=None, hi=None, nthreads: int | None = None):
    surplus = _f64(surplus)
    m = surplus.shape[1]
    xq = _f64(xq).reshape(-1, d)
    lo = _f64(np.zeros(d) if lo is None else lo)
    hi = _f64(np.ones(d) if hi is None else hi)
    out = np.zeros((xq.shape[0], m))
    lib().oracle_eval_hier(d, level, m, _dp(lo), _dp(hi), _dp(surplus), xq.shape[0], _dp(xq),
                           _dp(out), nthreads or default_threads())
    return out


def eval_comb(d: int, level: int, values, xq, lo=None, hi=None, nthreads: int | None = None):
    values = _f64(values)
    m = values.shape[1]
    xq = _f64(xq).reshape(-1, d)
    lo = _f64(np.zeros(d) if lo is None else lo)
    hi = _f64(np.ones(d) if hi is None else hi)
    out = np.zeros((xq.shape[0], m))
    lib().oracle_eval_comb(d, level, m, _dp(lo), _dp(hi), _dp(values), xq.shape[0], _dp(xq),
                           _dp(out), nthreads or default_threads())
    return out


def total_error(interp, coarse, fine, order: int = 2):
    """Monte Carlo estimate of e_interp + e_bvp (Sec. 4.3): the interpolant's
    values at sample states (``interp``, n x m) against a reference solution
    that is more accurate than the solutions at the grid nodes.  The paper takes
    the reference from an error-controlled solver; here it is the Richardson
    extrapolation of the solutions of a formula of order p on N (``coarse``)
    and 2N (``fine``) intervals of the same horizon, whose global errors are
    c h^p + higher order: ref = (2^p fine - coarse) / (2^p - 1) (p = 2: the
    trapezoid; p = 6: the four-point Lobatto IIIA formula).

    Returns (ref, err, stats): err[i] = max_c |interp[i, c] - ref[i, c]|
    (NaN if any term is NaN) and stats = [max err, RMS err, max |fine - ref|,
    mean err (the MAE of Sec. 5.1), mean of err / max(max_c |ref|, 1e-8) (the
    relative MAE)], with zeros for an empty sample."""
    interp, coarse, fine = (np.asarray(a, dtype=np.float64) for a in (interp, coarse, fine))
    s = 2.0 ** order
    ref = (s * fine - coarse) / (s - 1.0)
    n = interp.shape[0]
    if n == 0:
        return ref, np.zeros(0), np.zeros(5)
    err = np.max(np.abs(interp - ref), axis=1)
    corr = np.max(np.abs(fine - ref))
    rel = err / np.maximum(np.max(np.abs(ref), axis=1), 1e-8)
    stats = np.array([np.max(err), np.sqrt(np.mean(err * err)), corr, np.mean(err), np.mean(rel)])
    return ref, err, stats
