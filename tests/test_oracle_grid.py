"""Pins of the oracle's sparse grid (Sec. 3.2) and 1-D CGL basis (Sec. 3.3).

The grid is checked against every number the paper prints about it: the
complete 2-D CGL point sets of Fig. 3 (q = 6 and q = 8), the grid sizes of
Sec. 3.2, Example I and Example III, and the points-per-dimension counts.
"""
import math
import os

import numpy as np
import pytest
from scipy.interpolate import BarycentricInterpolator

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _printed(q):
    return np.loadtxt(os.path.join(GOLDEN, "paper_cgl_2d_q%d.txt" % q))


@pytest.mark.parametrize("q", [6, 8])
def test_printed_2d_cgl_grids(q):
    # Fig. 3 prints the CGL grids on [-1,1]^2 (the caption says [0,1]^2).
    pts = _printed(q)
    g = O.grid(2, q - 2, lo=[-1.0, -1.0], hi=[1.0, 1.0])
    assert g.nodes.shape[0] == pts.shape[0] == {6: 65, 8: 321}[q]
    # set equality with tolerance: each printed point has exactly one match
    dist = np.max(np.abs(pts[:, None, :] - g.nodes[None, :, :]), axis=2)
    assert np.all(np.min(dist, axis=1) < 1e-12)
    assert np.all(np.min(dist, axis=0) < 1e-12)
    assert np.all(np.sum(dist < 1e-12, axis=1) == 1)


@pytest.mark.parametrize("d,q,size,per_dim", [
    (2, 8, 321, None),        # Sec. 3.2 (modified and CGL grids, q = 8)
    (6, 13, 44689, 129),      # Example I (Sec. 5.1); Table 1 prints 44,698, a typo
    (4, 12, 18945, 257),      # Example III (Sec. 5.3)
])
def test_printed_grid_sizes(d, q, size, per_dim):
    level = q - d
    assert O.grid_size(d, level) == size
    if per_dim is not None:
        g = O.grid(d, level)
        assert np.unique(g.xi[:, 0]).size == per_dim == 2 ** (q - d) + 1


@pytest.mark.parametrize("level,size", [(2, 85), (3, 389), (4, 1457), (5, 4865)])
def test_workload_grid_sizes(level, size):
    assert O.grid_size(6, level) == size


def test_nested_cgl_sets():
    # X^{i-1} is a subset of X^i (the telescope structure of Sec. 3.2)
    assert np.array_equal(O.cgl_points(1), [0.5])
    assert np.allclose(O.cgl_points(2), [0.0, 0.5, 1.0], atol=1e-16, rtol=0)
    for i in range(3, 8):
        fine, coarse = O.cgl_points(i), O.cgl_points(i - 1)
        assert np.max(np.abs(fine[::2] - coarse)) < 1e-15
        # points are the Chebyshev extrema mapped to [0,1]
        n = 2 ** (i - 1)
        cheb = np.cos(np.pi * np.arange(n + 1) / n)
        assert np.max(np.abs(fine - 0.5 * (1 - cheb))) < 1e-15


def test_grid_keys_order_and_symmetry():
    g = O.grid(3, 4)
    keys = [tuple(k) for k in g.keys]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    # the sparse grid is symmetric under xi -> 1 - xi in each coordinate
    for j in range(3):
        mirrored = g.xi.copy()
        mirrored[:, j] = 1.0 - mirrored[:, j]
        dist = np.max(np.abs(mirrored[:, None, :] - g.xi[None, :, :]), axis=2)
        assert np.all(np.min(dist, axis=1) < 1e-14)
    # |i| <= q with i >= 1 (the Smolyak index set)
    assert g.levels.min() >= 1 and g.levels.sum(axis=1).max() <= 4 + 3


def test_kronecker_property():
    for i in range(2, 7):
        X = O.cgl_points(i)
        for k in range(1, X.size + 1):
            vals = O.lagrange(i, k, X)
            expect = np.zeros(X.size)
            expect[k - 1] = 1.0
            assert np.array_equal(vals, expect)


def test_lagrange_matches_barycentric_library():
    rng = np.random.default_rng(11)
    x = rng.random(200)
    for i in range(2, 7):
        X = O.cgl_points(i)
        f = rng.standard_normal(X.size)
        ours = sum(f[k] * O.lagrange(i, k + 1, x) for k in range(X.size))
        ref = BarycentricInterpolator(X, f)(x)
        assert np.max(np.abs(ours - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_lebesgue_constants():
    # Lambda_i = max_x sum_k |u^i_k(x)| (Sec. 4.1).  For the three points
    # {0, 1/2, 1} the textbook value is 5/4 (at x = 1/4 and 3/4).  For every
    # level the paper's bound eq. lebesgue with n = 2^{i-1} holds.
    x = np.linspace(0.0, 1.0, 20001)
    gamma = 0.5772156649015329
    lam = []
    for i in range(1, 8):
        X = O.cgl_points(i)
        s = sum(np.abs(O.lagrange(i, k + 1, x)) for k in range(X.size))
        lam.append(float(np.max(s)))
    assert lam[0] == 1.0
    assert abs(lam[1] - 1.25) < 1e-12
    for i in range(2, 8):
        n = 2 ** (i - 1)
        bound = 2 / math.pi * (math.log(n) + gamma + math.log(8 / math.pi))
        assert lam[i - 1] <= bound
    assert all(b > a for a, b in zip(lam, lam[1:]))
