"""Pins of the reduction-intrinsic oracle (CPU only): exact rational
arithmetic, closed-form sums, and cancellation that a naive left-to-right sum
gets wrong."""
from fractions import Fraction

import numpy as np

from oracle import reduce as R


def test_sum_matches_exact_rational_sum():
    rng = np.random.default_rng(11)
    for n in (1, 2, 7, 100, 1001):
        x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-8, 9, n)
        exact = sum(Fraction(float(v)) for v in x)
        assert R.sum_exact(x) == float(exact)  # float(Fraction) rounds to nearest


def test_dot_rounds_products_then_sums_exactly():
    rng = np.random.default_rng(12)
    x, y = rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 300)
    exact = sum(Fraction(float(a * b)) for a, b in zip(x, y))  # FP64-rounded products
    assert R.dot_exact(x, y) == float(exact)
    # and not the exact sum of the unrounded products (the products are rounded first)
    unrounded = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y))
    assert abs(float(unrounded) - R.dot_exact(x, y)) < 1e-14


def test_closed_forms():
    n = 1 << 20
    i = np.arange(1, n + 1, dtype=np.float64)
    assert R.sum_exact(i) == n * (n + 1) / 2
    assert R.dot_exact(i, i) == n * (n + 1) * (2 * n + 1) / 6  # < 2^53, exact
    # telescoping: sum of (1/k - 1/(k+1)) = 1 - 1/(n+1), each term rounded first
    k = np.arange(1, 1001, dtype=np.float64)
    t = 1.0 / k - 1.0 / (k + 1.0)
    assert abs(R.sum_exact(t) - (1.0 - 1.0 / 1001.0)) < 1e-15


def test_cancellation_and_empty():
    assert R.sum_exact(np.array([1e16, 1.0, -1e16])) == 1.0
    assert (1e16 + 1.0) - 1e16 == 0.0  # a left-to-right sum loses the 1
    assert R.sum_exact(np.zeros(0)) == 0.0
    assert R.dot_exact(np.zeros(0), np.zeros(0)) == 0.0
    assert R.abs_sum(np.array([-1.0, 2.0, -3.0])) == 6.0
    assert R.abs_sum(np.array([-1.0, 2.0]), np.array([3.0, -4.0])) == 11.0


def test_order_bound_covers_a_left_to_right_sum():
    rng = np.random.default_rng(13)
    x = rng.uniform(-1, 1, 5000)
    s = 0.0
    for v in x:  # recursive summation, depth n - 1
        s += float(v)
    assert abs(s - R.sum_exact(x)) <= R.order_bound(len(x) - 1, R.abs_sum(x))
