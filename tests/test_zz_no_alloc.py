"""The allocation-free three-sweep entry point against jacobi3d_sweep3.

jacobi3d_sweep3_noalloc runs the same kernels with the tile partials in the
library's static device array; its output and fused residual must equal
those of jacobi3d_sweep3 (which allocates its scratch) on the same inputs,
over two calls in a row, the second on a smaller grid (the array keeps the
first call's partials, which must not leak into the second result), and
with the residual fused at each stage of the pass.  Each result is also
checked against three oracle sweeps.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import RESID_RTOL, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

# (nx, ny, nz): several tiles in every direction with ragged tails, then a
# smaller grid of a single tile column
SHAPES = [(150, 70, 90), (37, 20, 29)]


def _inputs(nx, ny, nz, seed):
    u = synth.uniform_field(nx, ny, nz, seed, synth.STREAM_U0, 0.0, 1.0)
    f = synth.uniform_field(nx, ny, nz, seed, synth.STREAM_F, -1.0, 1.0)
    return u, f


@pytest.mark.parametrize("after", [0, 1, 2])
def test_noalloc_equals_sweep3_twice(after):
    from paper_2409_18824_amd import j3d

    torch.cuda.set_device(0)
    for call, (nx, ny, nz) in enumerate(SHAPES):
        say("noalloc: call %d, shape %s, residual after %d sweeps" % (call, (nx, ny, nz), after))
        h = 1.0 / (max(nx, ny, nz) + 1)
        u, f = _inputs(nx, ny, nz, 11 + call)
        du, df = j3d.FArray.from_numpy(u), j3d.FArray.from_numpy(f)
        ref, got = j3d.FArray.from_numpy(u), j3d.FArray.from_numpy(u)
        r_ref = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        r_got = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
        j3d.jacobi3d_sweep3(du, ref, df, h, resid_out=r_ref, resid_after=after)
        j3d.jacobi3d_sweep3_noalloc(du, got, df, h, r_got, resid_after=after)
        torch.cuda.synchronize()
        g, w = got.to_numpy(), ref.to_numpy()
        assert np.array_equal(g, w), "u_out differs from jacobi3d_sweep3 at %s" % ((nx, ny, nz),)
        assert rel(r_got.item(), r_ref.item()) <= RESID_RTOL, (r_got.item(), r_ref.item())
        # and both against the oracle
        it = [u]
        for _ in range(3):
            it.append(oracle.sweep(it[-1], f, h))
        assert np.array_equal(g, it[3]), "u_out differs from three oracle sweeps"
        ro = oracle.residual_l2(it[after], f, h)
        assert rel(r_got.item(), ro) <= RESID_RTOL, (r_got.item(), ro)


def test_noalloc_rejects_host_result_and_f32():
    from paper_2409_18824_amd import j3d

    torch.cuda.set_device(0)
    nx, ny, nz = 20, 12, 9
    u, f = _inputs(nx, ny, nz, 3)
    du, dv, df = j3d.FArray.from_numpy(u), j3d.FArray.from_numpy(u), j3d.FArray.from_numpy(f)
    r = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(j3d.J3DError) as e:
        j3d.jacobi3d_sweep3_noalloc(du, dv, df, 0.1, r, flags=j3d.HOST_RESULT)
    assert e.value.code == j3d.EINVAL
    with pytest.raises(j3d.J3DError) as e:
        j3d.jacobi3d_sweep3_noalloc(du, dv, df, 0.1, None)
    assert e.value.code == j3d.EINVAL
    a32 = [j3d.FArray.from_numpy(x.astype(np.float32)) for x in (u, u, f)]
    with pytest.raises(j3d.J3DError) as e:
        j3d.jacobi3d_sweep3_noalloc(*a32, 0.1, r)
    assert e.value.code == j3d.EDTYPE
