"""GPU parity of the sum and dot_product intrinsics against the exact oracle.

The device adds in a fixed tree; the oracle returns the correctly rounded
exact sum.  The bound is the recursive-summation bound of the device's tree:
its longest chain of dependent additions is the per-thread run (chunk/256
addends), the wavefront butterfly (6), the four wavefronts of a block (3),
then the final reduce's per-thread run over the block partials, its
butterfly (6) and its 16 wavefronts (15).
"""
import math

import numpy as np
import pytest
import torch

import synth
from gpu_util import needs_gpu, say
from oracle import reduce as R

pytestmark = [pytest.mark.gpu, needs_gpu]

from paper_2409_18824_amd import j3d  # noqa: E402

STEP = 256 * 8
MAXB = 65536


def depth(n):
    per = max(1, -(-n // (MAXB * STEP)))
    chunk = STEP * per
    nb = -(-n // chunk) if n else 0
    return chunk // 256 + 6 + 3 + -(-nb // 1024) + 6 + 15


def vec(n, seed, stream):
    return synth.uniform(seed, stream, np.arange(n, dtype=np.uint64), -1.0, 1.0)


@pytest.mark.parametrize("n", [0, 1, 2, 255, 256, 257, 2047, 2048, 2049, 4097, 100003, (1 << 20) + 7])
def test_sum_and_dot_within_order_bound(n):
    say("sum/dot", n)
    x, y = vec(n, 21, 1), vec(n, 21, 2)
    dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    s, d = j3d.j3d_sum(dx), j3d.j3d_dot(dx, dy)
    assert abs(s - R.sum_exact(x)) <= R.order_bound(depth(n), R.abs_sum(x))
    assert abs(d - R.dot_exact(x, y)) <= R.order_bound(depth(n), R.abs_sum(x, y))
    # reproducible bit for bit, and the asynchronous form agrees
    out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    j3d.j3d_sum(dx, out=out[0:1])
    j3d.j3d_dot(dx, dy, out=out[1:2])
    torch.cuda.synchronize()
    assert out[0].item() == s and out[1].item() == d
    assert j3d.j3d_sum(dx) == s and j3d.j3d_dot(dx, dy) == d


def test_dot_of_a_vector_with_itself_and_cancellation():
    n = 50000
    x = vec(n, 22, 1)
    dx = torch.from_numpy(x).cuda()
    assert abs(j3d.j3d_dot(dx, dx) - R.dot_exact(x, x)) <= R.order_bound(depth(n), R.abs_sum(x, x))
    # x followed by -x: every block that holds a pair cancels exactly only if
    # the tree pairs them; the bound still holds and the exact answer is 0
    z = np.concatenate([x, -x])
    dz = torch.from_numpy(z).cuda()
    assert abs(j3d.j3d_sum(dz)) <= R.order_bound(depth(2 * n), R.abs_sum(z))


@pytest.mark.parametrize("which", ["sum", "dot"])
def test_full_size_integer_data_is_exact(which):
    """The paper's sizes: sum over a 32768 x 32768 FP64 array, dot_product of
    two 134M-element (2^27) FP64 vectors.  Integer-valued addends keep every
    partial sum an integer below 2^53, so any order is exact and the device
    result must equal the integer sum bit for bit."""
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    if which == "sum":
        n = 32768 * 32768
        say("full-size sum", n)
        xi = torch.randint(-1000, 1001, (n,), device="cuda", generator=g, dtype=torch.int64)
        want = int(xi.sum().item())
        x = xi.to(torch.float64)
        del xi
        got = j3d.j3d_sum(x)
    else:
        n = 1 << 27
        say("full-size dot", n)
        xi = torch.randint(-1000, 1001, (n,), device="cuda", generator=g, dtype=torch.int64)
        yi = torch.randint(-1000, 1001, (n,), device="cuda", generator=g, dtype=torch.int64)
        want = int((xi * yi).sum().item())
        x, y = xi.to(torch.float64), yi.to(torch.float64)
        del xi, yi
        got = j3d.j3d_dot(x, y)
    assert abs(want) < 2 ** 53
    assert got == float(want)


def test_rejects_bad_tensors():
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        j3d.j3d_sum(x[::2])
    with pytest.raises(TypeError):
        j3d.j3d_sum(x.float())
    with pytest.raises(ValueError):
        j3d.j3d_dot(x, x[:5])
    assert j3d.j3d_sum(x[:0]) == 0.0
