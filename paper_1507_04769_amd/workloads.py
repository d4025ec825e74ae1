"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

This module is shared by the oracle-side tests and the GPU-side tests, bench
and smoke check.  It holds the problem parameters of the rigid-body attitude
workloads, the box in which the sparse grid and the query points live, and
seeded uniform generators (numpy PCG64).  It never computes a grid, a BVP or
an interpolant.

The rigid-body model is the gyroscopic simplification of the paper's
momentum-wheel model (Sec. 5, eq. sat_model): Euler angles in (3,2,1) order,
J w' = -w x (J w) + B u, running cost 0.5 (q_w x^T x + r_w u^T u) and final
cost 0.5 p_w x^T x.  The paper samples validation points uniformly at random
in a box (Sec. 4.3 and 5.1); the query sets here follow that recipe.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

D = 6  # state dimension of the rigid body
ANGLE_HALF_WIDTH = math.pi / 4
RATE_HALF_WIDTH = 0.5
BOX_LO = np.array([-ANGLE_HALF_WIDTH] * 3 + [-RATE_HALF_WIDTH] * 3)
BOX_HI = -BOX_LO


@dataclass(frozen=True)
class Workload:
    name: str
    level: int          # sparse-grid level (q = level + d)
    n_intervals: int    # trapezoidal collocation intervals
    horizon: float
    n_queries: int
    query_seed: int
    m: int = 3          # number of wheel torques


# Plain FP64 path, smallest case: level-2 grid (85 nodes), 64 intervals, 1e3 queries.
SMALL = Workload("rigid-body-6d-L2-N64-q1e3", level=2, n_intervals=64, horizon=20.0,
                 n_queries=1000, query_seed=0)
# Plain FP64 path at scale: level-4 grid (1457 nodes), 256 intervals, 1e6 queries.
FULL = Workload("rigid-body-6d-L4-N256-q1e6", level=4, n_intervals=256, horizon=20.0,
                n_queries=1_000_000, query_seed=1)



@dataclass(frozen=True)
class MixedBatch:
    """BVPs with per-BVP mesh size and horizon: the first n_nodes nodes (canonical
    order) of a level-`level` grid plus n_random uniform states, each BVP's N and
    T drawn from `meshes` and `horizons` by PCG64(assign_seed)."""
    name: str
    level: int
    n_nodes: int
    n_random: int
    random_seed: int
    meshes: tuple
    horizons: tuple
    assign_seed: int
    m: int = 3


# Batching: 3072 level-5 nodes + 1024 uniform states, N in {64, 128, 256, 512},
# T in {10, 20, 40}.
BATCH = MixedBatch("rigid-body-6d-L5n3072+u1024-mixedNT", level=5, n_nodes=3072, n_random=1024,
                   random_seed=102, meshes=(64, 128, 256, 512), horizons=(10.0, 20.0, 40.0), assign_seed=202)


def mixed_assignment(b: MixedBatch, n: int):
    """Per-BVP (N, T) of a mixed batch of n BVPs (int32, float64)."""
    g = np.random.default_rng(b.assign_seed)
    N = g.choice(np.asarray(b.meshes), size=n).astype(np.int32)
    T = g.choice(np.asarray(b.horizons, dtype=np.float64), size=n)
    return N, T


def batch_initial_states(b: MixedBatch, grid_nodes: np.ndarray) -> np.ndarray:
    """Initial states of a mixed batch: the first n_nodes rows of the given grid
    node table (canonical order, level b.level) and n_random uniform states."""
    return np.vstack([np.asarray(grid_nodes)[:b.n_nodes], uniform_in_box(b.n_random, b.random_seed)])


J_DIAG = (2.0, 3.0, 4.0)
Q_W, R_W, P_W = 1.0, 0.1, 10.0
TOL = 1e-10
MAX_ITER = 20
MAX_HALVINGS = 10  # backtracking cap of each counted Newton step

# Underactuated (two-wheel) precision workload: the level-4 grid over the full
# box, 256 intervals, T = 20, reached by the virtual-torque continuation in
# four stages, at most 100 Newton iterations per stage.
UNDERACTUATED = Workload("rigid-body-6d-2wheel-L4-N256", level=4, n_intervals=256, horizon=20.0,
                         n_queries=10_000_000, query_seed=3, m=2)
UNDERACTUATED_CONTINUATION = 4
UNDERACTUATED_MAX_ITER = 100


def input_matrix(m: int = 3) -> np.ndarray:
    """3 x m wheel-torque input matrix: identity for three wheels; for two
    wheels, seeded orthonormal columns (QR of a PCG64(103) normal draw with
    the signs fixed so that diag(R) > 0)."""
    if m == 3:
        return np.eye(3)
    if m != 2:
        raise ValueError("m must be 2 or 3")
    g = np.random.default_rng(103).standard_normal((3, 2))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def uniform_in_box(n: int, seed: int, lo=BOX_LO, hi=BOX_HI) -> np.ndarray:
    """n points uniform in the box [lo, hi] (n x d), PCG64(seed)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    u = np.random.default_rng(seed).random((n, lo.size))
    return lo + (hi - lo) * u


def query_points(w: Workload) -> np.ndarray:
    return uniform_in_box(w.n_queries, w.query_seed)


def random_values(n: int, m: int, seed: int) -> np.ndarray:
    """Seeded standard-normal node values for interpolation tests."""
    return np.random.default_rng(seed).standard_normal((n, m))


def sample_indices(total: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices of range(total), sorted, PCG64(seed)."""
    k = min(k, total)
    return np.sort(np.random.default_rng(seed).choice(total, size=k, replace=False))


# Example III of Sec. 5.3 with the time variable as a grid dimension: the
# sparse grid in (t, x) over [0, 5] x [-2, 2]^3 (the paper's region D), the
# final time T = 5 (the paper does not state T; the closed form holds for any
# T >= 5), N = 64 intervals on every [t0, T], continuation in the initial
# state in two stages, and the paper's 1200 uniform validation points in D.
EX3_LO = np.array([0.0, -2.0, -2.0, -2.0])
EX3_HI = np.array([5.0, 2.0, 2.0, 2.0])
EX3_T = 5.0
EX3_N = 64
EX3_CONTINUATION = 2
EX3_LEVEL = 5
EX3_SAMPLES = 1200
EX3_SAMPLE_SEED = 53


def ex3_samples(n: int = EX3_SAMPLES, seed: int = EX3_SAMPLE_SEED) -> np.ndarray:
    """n points (t, x) uniform in the region D of Example III."""
    return uniform_in_box(n, seed, EX3_LO, EX3_HI)

