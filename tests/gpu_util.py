"""Helpers shared by the GPU tests (parity against the CPU oracle)."""
import sys

import numpy as np
import pytest
import torch

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")

# Per-point FP64 sweep tolerance (relative, with a scale term for cancellation):
# |g - o| <= 1e-13 * max(|o|, (sum|neighbours| + h^2 |f|) / 6).
SWEEP_RTOL = 1e-13
# Residual norm tolerance (relative).
RESID_RTOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sweep_scale(u, f, h):
    """(sum of |neighbours| + h^2 |f|) / 6 over the interior, shape (nz, ny, nx)."""
    a = np.abs(u)
    s = (a[1:-1, 1:-1, :-2] + a[1:-1, 1:-1, 2:] + a[1:-1, :-2, 1:-1] + a[1:-1, 2:, 1:-1]
         + a[:-2, 1:-1, 1:-1] + a[2:, 1:-1, 1:-1])
    return (s + h * h * np.abs(f[1:-1, 1:-1, 1:-1])) / 6.0


def assert_sweep_close(got, want, u, f, h, rtol=SWEEP_RTOL):
    gi = got[1:-1, 1:-1, 1:-1]
    wi = want[1:-1, 1:-1, 1:-1]
    bound = rtol * np.maximum(np.abs(wi), sweep_scale(u, f, h))
    err = np.abs(gi - wi)
    bad = err > bound
    assert not bad.any(), "%d points off; worst %g (bound %g)" % (bad.sum(), err.max(), bound.flat[np.argmax(err)])
    return int(np.count_nonzero(gi != wi))


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
