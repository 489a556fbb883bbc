"""Oracle for the Fortran ``sum`` and ``dot_product`` intrinsics over FP64
vectors.  TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper lowers both intrinsics to a reduction initialised at zero that adds
every element (for ``dot_product``: every elementwise product) into the
accumulator (Sec. "Handling of other constructs"); its intrinsics table
measures them on a 32768 x 32768 FP64 array and on FP64 vectors of 134
million elements.  Any order of the additions is a valid evaluation of the
intrinsic, so the oracle returns the one order-free answer: the exact sum of
the addends, correctly rounded to FP64 (``math.fsum``, Shewchuk's exact
summation).  Products are rounded to FP64 first, exactly as an unfused
multiply then add computes them.  A GPU result is checked against this value
within the error bound of its own summation order.
"""
from __future__ import annotations

import math

import numpy as np


def sum_exact(x: np.ndarray) -> float:
    """Correctly rounded sum of the FP64 elements of x (any shape)."""
    return math.fsum(np.asarray(x, dtype=np.float64).ravel().tolist())


def dot_exact(x: np.ndarray, y: np.ndarray) -> float:
    """Correctly rounded sum of the FP64-rounded products x_i * y_i."""
    p = np.asarray(x, dtype=np.float64).ravel() * np.asarray(y, dtype=np.float64).ravel()
    return math.fsum(p.tolist())


def abs_sum(x: np.ndarray, y: np.ndarray | None = None) -> float:
    """Sum of |addend|, the scale of the summation error bound."""
    p = np.asarray(x, dtype=np.float64).ravel()
    if y is not None:
        p = p * np.asarray(y, dtype=np.float64).ravel()
    return math.fsum(np.abs(p).tolist())


def order_bound(depth: int, scale: float) -> float:
    """Error bound of recursive FP64 summation whose longest chain of
    dependent additions is `depth`: gamma_depth * sum|addends| (Higham,
    Accuracy and Stability of Numerical Algorithms, Sec. 4.2)."""
    u = 2.0 ** -53
    return depth * u / (1.0 - depth * u) * scale
