"""Pins of the oracle's sparse-grid interpolant (Sec. 3.3).

* d = 1 reduces to Lagrange interpolation on X^{level+1}: checked against
  scipy's barycentric interpolator (a library routine the oracle never uses).
* Interpolation: the interpolant reproduces the node values.
* Exactness: the Smolyak interpolant reproduces exactly the monomials
  xi^alpha with sum_k lev(alpha_k) <= q, lev(a) = min{i : N_i >= a + 1}, and
  no others (the polynomial space of the nested Smolyak construction).
* Route A (hierarchical surpluses, eq. interpo) equals route B (combination
  formula, eq. interpolation2), two different formulas of the paper.
* The e_bvp bound of Theorem 1 with the Lebesgue bound eq. lebesgue reproduces
  the printed 3.66e4 for q = 13, d = 6 (checks the multi-index enumeration).
"""
import itertools
import math

import numpy as np
import pytest
from scipy.interpolate import BarycentricInterpolator

from oracle import oracle as O


def lev(a):
    i = 1
    while (1 if i == 1 else 2 ** (i - 1) + 1) < a + 1:
        i += 1
    return i


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_one_dimension_is_lagrange_interpolation(level):
    g = O.grid(1, level)
    rng = np.random.default_rng(level)
    f = rng.standard_normal((g.xi.shape[0], 1))
    w = O.build_surplus(1, level, f)
    x = rng.random((300, 1))
    ours = O.eval_hier(1, level, w, x)[:, 0]
    order = np.argsort(g.xi[:, 0])
    ref = BarycentricInterpolator(g.xi[order, 0], f[order, 0])(x[:, 0])
    assert np.max(np.abs(ours - ref)) < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("d,level", [(2, 4), (3, 3), (6, 2)])
def test_node_reproduction(d, level):
    g = O.grid(d, level)
    vals = np.random.default_rng(5).standard_normal((g.xi.shape[0], 2))
    w = O.build_surplus(d, level, vals)
    back = O.eval_hier(d, level, w, g.xi)
    assert np.max(np.abs(back - vals)) < 1e-12 * np.abs(vals).max()


@pytest.mark.parametrize("d,level", [(2, 3), (3, 2), (6, 2)])
def test_polynomial_exactness(d, level):
    q = level + d
    g = O.grid(d, level)
    xq = np.random.default_rng(7).random((64, d))
    max_deg = 2 ** level + 2
    checked_in = checked_out = 0
    for alpha in itertools.product(range(max_deg + 1), repeat=min(d, 3)):
        alpha = tuple(alpha) + (0,) * (d - len(alpha))
        if sum(alpha) > max_deg:
            continue
        vals = np.prod(g.xi ** np.array(alpha), axis=1)[:, None]
        w = O.build_surplus(d, level, vals)
        approx = O.eval_hier(d, level, w, xq)[:, 0]
        exact = np.prod(xq ** np.array(alpha), axis=1)
        err = np.max(np.abs(approx - exact))
        if sum(lev(a) for a in alpha) <= q:
            assert err < 1e-12, (alpha, err)
            checked_in += 1
        else:
            assert err > 1e-8, (alpha, err)
            checked_out += 1
    assert checked_in > 3 and checked_out > 3


@pytest.mark.parametrize("d,level", [(2, 5), (3, 3), (6, 2), (6, 3)])
def test_hierarchical_equals_combination_formula(d, level):
    g = O.grid(d, level)
    rng = np.random.default_rng(d * 10 + level)
    vals = rng.standard_normal((g.xi.shape[0], 3))
    lo, hi = -np.ones(d), 2 * np.ones(d)
    xq = lo + (hi - lo) * rng.random((50, d))
    w = O.build_surplus(d, level, vals)
    a = O.eval_hier(d, level, w, xq, lo, hi)
    b = O.eval_comb(d, level, vals, xq, lo, hi)
    assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.abs(b).max())


def test_combination_formula_reproduces_constants():
    d, level = 6, 3
    g = O.grid(d, level)
    xq = np.random.default_rng(3).random((20, d))
    out = O.eval_comb(d, level, np.ones((g.xi.shape[0], 1)), xq)
    assert np.max(np.abs(out - 1.0)) < 1e-12


def test_out_of_box_is_the_same_polynomial():
    # outside [0,1]^d the interpolant is the same polynomial (no clamping):
    # a reproduced monomial stays exact outside the box.
    d, level = 2, 3
    g = O.grid(d, level)
    vals = (g.xi[:, 0] ** 2 * g.xi[:, 1])[:, None]
    w = O.build_surplus(d, level, vals)
    xq = np.array([[1.5, -0.25], [-0.7, 1.3]])
    out = O.eval_hier(d, level, w, xq)[:, 0]
    # outside the box the Lebesgue function grows, so rounding is amplified
    assert np.allclose(out, xq[:, 0] ** 2 * xq[:, 1], rtol=0, atol=1e-10)


def test_ebvp_bound_printed_value():
    # Theorem 1 (i) with Lambda_i from eq. lebesgue, n = 2^{i-1} (the degree)
    # and Lambda_1 = 1, for the CGL grid q = 13, d = 6: at most 3.66e4.
    d, q = 6, 13
    gamma = 0.5772156649015329

    def Lam(i):
        if i == 1:
            return 1.0
        n = 2 ** (i - 1)
        return 2 / math.pi * (math.log(n) + gamma + math.log(8 / math.pi))

    def S(l):
        tot = 0.0
        for mi in itertools.product(range(1, l - d + 2), repeat=d):
            if sum(mi) == l:
                tot += math.prod(Lam(i) for i in mi)
        return tot

    bound = sum(math.comb(d - 1, q - l) * S(l) for l in range(q - d + 1, q + 1))
    assert 3.64e4 < bound <= 3.66e4
