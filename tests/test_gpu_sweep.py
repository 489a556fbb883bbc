"""GPU parity of the sweep, the fused and standalone residual, and fills.

Every case runs the HIP path through the C ABI and compares it with the CPU
oracle on the same seeded inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import RESID_RTOL, assert_sweep_close, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

from paper_2409_18824_amd import j3d  # noqa: E402

SHAPES = [(1, 1, 1), (4, 4, 4), (3, 4, 5), (17, 9, 33), (64, 64, 64), (130, 67, 45), (65, 3, 70)]
# (rows, planes, variant bits: 1 LDS, 2/16 rows per thread, 4 nontemporal; persistent; order[; cols])
TUNES = [(1, 16, 20, 0, 1, 2), (2, 8, 4, 1, 0, 4), (4, 32, 6, 0, 2, 2), (1, 4, 20, 0, 0, 4), (8, 16, 4, 0, 1, 2),
         (4, 2, 20, 1, 2, 4), (1, 8, 0, 0, 0), (2, 16, 1, 0, 0), (4, 32, 2, 0, 0), (4, 32, 3, 1, 0), (8, 64, 4, 1, 0), (8, 128, 7, 0, 0),
         (1, 16, 6, 0, 0), (2, 8, 5, 1, 0), (1, 1, 4, 0, 1), (2, 4, 1, 1, 1), (8, 2, 7, 0, 1),
         (1, 8, 22, 0, 1), (4, 32, 22, 0, 0), (2, 2, 23, 1, 1), (8, 16, 19, 0, 0), (1, 4, 20, 0, 1),
         (1, 8, 20, 0, 2), (4, 16, 6, 1, 2), (2, 4, 21, 0, 2), (1, 1, 18, 1, 2)]


def make_inputs(nx, ny, nz, seed=1):
    h = 1.0 / (max(nx, ny, nz) + 1)
    u = synth.uniform_field(nx, ny, nz, seed, synth.STREAM_U0, 0.0, 1.0)
    f = synth.uniform_field(nx, ny, nz, seed, synth.STREAM_F, -1.0, 1.0)
    # non-zero Dirichlet data in the halo exercises boundary reads
    halo = synth.uniform(seed, 9, np.arange(u.size, dtype=np.uint64), -0.5, 0.5).reshape(u.shape)
    mask = np.ones(u.shape, dtype=bool)
    mask[1:-1, 1:-1, 1:-1] = False
    u[mask] = halo[mask]
    return u, f, h


def test_fill_uniform_matches_generator():
    for (nx, ny, nz) in [(17, 9, 33), (64, 64, 64), (1, 1, 1)]:
        say("fill", nx, ny, nz)
        a = j3d.FArray.empty(nx, ny, nz, lbound=(1, -2, 3))
        j3d.j3d_fill_uniform(a, 1234, synth.STREAM_F, -1.0, 1.0, halo=0.25)
        torch.cuda.synchronize()
        want = synth.uniform_field(nx, ny, nz, 1234, synth.STREAM_F, -1.0, 1.0, halo=0.25)
        assert np.array_equal(a.to_numpy(), want)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tune", TUNES)
def test_sweep_fp64_parity(shape, tune):
    nx, ny, nz = shape
    say("sweep fp64", shape, tune)
    u, f, h = make_inputs(nx, ny, nz)
    j3d.j3d_tune_set_single(j3d.F64, nx, ny, nz, tune)
    du = j3d.FArray.from_numpy(u)
    dv = j3d.FArray.from_numpy(np.zeros_like(u))
    dv.copy_from(u)  # same halo in both ping-pong arrays
    dv.view()[1:-1, 1:-1, 1:-1] = -7.0  # interior must be overwritten
    df = j3d.FArray.from_numpy(f)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    got = dv.to_numpy()
    want = oracle.sweep(u, f, h)
    ndiff = assert_sweep_close(got, want, u, f, h)
    assert ndiff == 0, "expected bitwise equality (same order, no contraction)"
    # halo untouched
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[:, :, -1], u[:, :, -1])
    # fused residual of the input iterate
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL
    # standalone residual with the same tile shape: identical reduction order
    assert j3d.residual_l2(du, df, h) == float(r.item())


TUNES2 = [(1, 32, 20, 0, 1, 1), (4, 16, 4, 0, 2, 1), (2, 16, 20, 0, 1, 1), (8, 8, 6, 1, 0, 1), (4, 8, 0, 0, 0), (8, 32, 4, 0, 1), (4, 16, 4, 0, 2), (4, 1, 0, 1, 1), (8, 3, 0, 1, 2),
          (2, 128, 2, 0, 0), (1, 16, 20, 0, 1), (4, 8, 16, 1, 2), (8, 16, 6, 0, 0), (2, 32, 20, 0, 2)]
SHAPES2 = [(1, 1, 1), (3, 4, 5), (60, 6, 9), (61, 7, 10), (62, 6, 9), (121, 30, 17), (17, 45, 64), (200, 14, 3),
           (64, 5, 7), (65, 9, 4), (129, 33, 18)]


@pytest.mark.parametrize("shape", SHAPES2)
@pytest.mark.parametrize("tune", TUNES2)
def test_sweep2_equals_two_sweeps(shape, tune):
    nx, ny, nz = shape
    say("sweep2", shape, tune)
    u, f, h = make_inputs(nx, ny, nz, seed=4)
    j3d.j3d_tune_set_single(j3d.KIND_F64X2, nx, ny, nz, tune)
    du = j3d.FArray.from_numpy(u)
    dv = j3d.FArray.from_numpy(u)
    dv.view()[1:-1, 1:-1, 1:-1] = -7.0
    df = j3d.FArray.from_numpy(f, ld_extra=3)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep2(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    want = oracle.sweep(oracle.sweep(u, f, h), f, h)
    got = dv.to_numpy()
    assert np.array_equal(got, want), "max diff %g" % np.max(np.abs(got - want))
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL
    assert np.array_equal(du.to_numpy(), u)  # input untouched


TUNES3 = [(4, 32, 20, 0, 1, 1), (2, 16, 20, 0, 0, 1), (8, 8, 6, 0, 2, 1), (4, 7, 6, 0, 1, 1), (8, 64, 20, 0, 0, 1),
          (2, 3, 20, 0, 2, 1), (4, 48, 20, 0, 1, 1), (4, 24, 20, 0, 2, 1), (16, 24, 6, 0, 1, 1),
          (16, 144, 6, 0, 1, 1), (16, 5, 6, 0, 2, 1)]
SHAPES3 = [(1, 1, 1), (3, 4, 5), (58, 6, 9), (59, 12, 10), (57, 13, 8), (117, 30, 17), (17, 45, 64), (200, 28, 3)]


@pytest.mark.parametrize("shape", SHAPES3)
@pytest.mark.parametrize("tune", TUNES3)
def test_sweep3_equals_three_sweeps(shape, tune):
    nx, ny, nz = shape
    say("sweep3", shape, tune)
    u, f, h = make_inputs(nx, ny, nz, seed=7)
    j3d.j3d_tune_set_single(j3d.KIND_F64X3, nx, ny, nz, tune)
    du = j3d.FArray.from_numpy(u)
    dv = j3d.FArray.from_numpy(u)
    dv.view()[1:-1, 1:-1, 1:-1] = -7.0
    df = j3d.FArray.from_numpy(f, ld_extra=3)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep3(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    want = oracle.sweep(oracle.sweep(oracle.sweep(u, f, h), f, h), f, h)
    got = dv.to_numpy()
    assert np.array_equal(got, want), "max diff %g" % np.max(np.abs(got - want))
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL
    assert np.array_equal(du.to_numpy(), u)  # input untouched


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 4, 5), (59, 12, 10), (117, 30, 17), (17, 45, 64), (200, 28, 3)])
@pytest.mark.parametrize("tune", [(4, 32, 20, 0, 1, 1), (2, 16, 20, 0, 0, 1), (8, 8, 6, 0, 2, 1), (2, 3, 20, 0, 2, 1),
                                  (16, 24, 6, 0, 0, 1)])
@pytest.mark.parametrize("after", [1, 2])
def test_sweep3_residual_of_intermediate_iterates(shape, tune, after):
    """The residual fused at stage 2 or 3 of the pass is that of J(u) or
    J(J(u)); the output is still three sweeps."""
    nx, ny, nz = shape
    say("sweep3 resid after", after, shape, tune)
    u, f, h = make_inputs(nx, ny, nz, seed=11)
    j3d.j3d_tune_set_single(j3d.KIND_F64X3, nx, ny, nz, tune)
    du = j3d.FArray.from_numpy(u)
    dv = j3d.FArray.from_numpy(u)
    dv.view()[1:-1, 1:-1, 1:-1] = -7.0
    df = j3d.FArray.from_numpy(f, ld_extra=3)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep3(du, dv, df, h, resid_out=r, resid_after=after)
    hr = j3d.jacobi3d_sweep3(du, dv, df, h, host_result=True, resid_after=after)
    torch.cuda.synchronize()
    u1 = oracle.sweep(u, f, h)
    u2 = oracle.sweep(u1, f, h)
    assert np.array_equal(dv.to_numpy(), oracle.sweep(u2, f, h))
    want = oracle.residual_l2(u1 if after == 1 else u2, f, h)
    assert rel(float(r.item()), want) <= RESID_RTOL
    assert float(r.item()) == hr  # same kernel, same partials, same reduction


@pytest.mark.parametrize("shape", [(70, 13, 21), (1, 1, 1), (130, 40, 9), (58, 14, 33)])
@pytest.mark.parametrize("tune", [(8, 32, 20, 0, 1, 1), (4, 16, 6, 0, 0, 1), (2, 8, 20, 0, 2, 1), (8, 48, 6, 0, 2, 1),
                                  (16, 7, 6, 0, 1, 1)])
def test_sweep3_fp32_equals_three_fp32_sweeps(shape, tune):
    nx, ny, nz = shape
    say("sweep3 fp32", shape, tune)
    e = synth.uniform_field(nx, ny, nz, 8, 1, -1, 1).astype(np.float32)
    r32 = synth.uniform_field(nx, ny, nz, 8, 2, -1, 1).astype(np.float32)
    h = 1.0 / (max(shape) + 1)
    h2 = np.float32(h * h)
    j3d.j3d_tune_set_single(j3d.KIND_F32X3, nx, ny, nz, tune)
    de = j3d.FArray.from_numpy(e, dtype=j3d.F32)
    do = j3d.FArray.from_numpy(e, dtype=j3d.F32)
    dr = j3d.FArray.from_numpy(r32, dtype=j3d.F32)
    j3d.jacobi3d_sweep3(de, do, dr, h)
    torch.cuda.synchronize()
    want = oracle.sweep_f32(oracle.sweep_f32(oracle.sweep_f32(e, r32, h2), r32, h2), r32, h2)
    assert np.array_equal(do.to_numpy(), want)


def test_sweep3_full_size_512():
    n = 512
    say("512^3 sweep3")
    h = 1.0 / (n + 1)
    f = synth.manufactured_f(n, n, n, h)
    du = j3d.FArray.empty(n, n, n)
    j3d.j3d_fill_uniform(du, 2, synth.STREAM_U0, 0.0, 1.0)
    dv = j3d.FArray.empty(n, n, n)
    df = j3d.FArray.from_numpy(f)
    say("tile", j3d.j3d_tune_query_single(j3d.KIND_F64X3, n, n, n))
    r = torch.zeros(3, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep3(du, dv, df, h, resid_out=r[0:1])
    j3d.jacobi3d_sweep3(du, dv, df, h, resid_out=r[1:2], resid_after=1)
    j3d.jacobi3d_sweep3(du, dv, df, h, resid_out=r[2:3], resid_after=2)
    torch.cuda.synchronize()
    u = du.to_numpy()
    u1 = oracle.sweep(u, f, h)
    u2 = oracle.sweep(u1, f, h)
    want = oracle.sweep(u2, f, h)
    assert np.array_equal(dv.to_numpy()[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1])
    for q, it in enumerate((u, u1, u2)):
        assert rel(float(r[q].item()), oracle.residual_l2(it, f, h)) <= RESID_RTOL


def test_sweep2_shapes_with_wide_tiles_rejected():
    for kind in (j3d.KIND_F64X2, j3d.KIND_F32X2):
        for t in [(4, 32, 20, 0, 1, 2), (2, 16, 20, 0, 1, 4), (4, 32, 1, 0, 1, 1), (1, 8, 0, 0, 1, 1)]:
            with pytest.raises(j3d.J3DError) as ei:
                j3d.j3d_tune_set_single(kind, 64, 64, 64, t)
            assert ei.value.code == j3d.EINVAL
    with pytest.raises(j3d.J3DError):
        j3d.j3d_tune_set_single(j3d.KIND_F32X2, 64, 64, 64, (4, 32, 16, 0, 1, 1))  # FP32: nontemporal only


def test_sweep2_full_size_512():
    n = 512
    say("512^3 sweep2")
    h = 1.0 / (n + 1)
    f = synth.manufactured_f(n, n, n, h)
    du = j3d.FArray.empty(n, n, n)
    j3d.j3d_fill_uniform(du, 2, synth.STREAM_U0, 0.0, 1.0)
    dv = j3d.FArray.empty(n, n, n)
    df = j3d.FArray.from_numpy(f)
    # the benchmark's launch configuration: the library's default shape
    say("tile", j3d.j3d_tune_query_single(j3d.KIND_F64X2, n, n, n))
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep2(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    u = du.to_numpy()
    want = oracle.sweep(oracle.sweep(u, f, h), f, h)
    assert np.array_equal(dv.to_numpy()[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1])
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL


@pytest.mark.parametrize("tune", [(2, 16, 20, 0, 1, 2), (1, 8, 6, 1, 0, 4), (1, 8, 0, 0, 0), (4, 32, 1, 0, 0), (8, 16, 0, 1, 0), (2, 16, 6, 0, 2), (4, 64, 7, 1, 0),
                                  (1, 8, 22, 0, 1), (2, 4, 23, 1, 0)])
def test_sweep_fp32_parity(tune):
    nx, ny, nz = 70, 13, 21
    say("sweep fp32", tune)
    e = synth.uniform_field(nx, ny, nz, 5, 1, -1, 1).astype(np.float32)
    r32 = synth.uniform_field(nx, ny, nz, 5, 2, -1, 1).astype(np.float32)
    h2 = np.float32((1.0 / 71) ** 2)
    j3d.j3d_tune_set_single(j3d.F32, nx, ny, nz, tune)
    de = j3d.FArray.from_numpy(e, dtype=j3d.F32)
    do = j3d.FArray.from_numpy(e, dtype=j3d.F32)
    dr = j3d.FArray.from_numpy(r32, dtype=j3d.F32)
    j3d.jacobi3d_sweep(de, do, dr, 1.0 / 71)
    torch.cuda.synchronize()
    got = do.to_numpy()
    want = oracle.sweep_f32(e, r32, h2)
    assert got.dtype == np.float32
    # same order, correctly rounded FP32 division, no contraction: bitwise
    assert np.array_equal(got, want)


TUNES2_F32 = [(4, 32, 20, 0, 1, 1), (1, 16, 20, 0, 2, 1), (2, 8, 6, 1, 0, 1), (4, 16, 4, 0, 1, 1), (2, 4, 20, 0, 0, 1),
              (8, 64, 6, 0, 2, 1), (1, 8, 20, 1, 1, 1)]


@pytest.mark.parametrize("shape", [(70, 13, 21), (1, 1, 1), (130, 40, 9), (62, 14, 33), (64, 7, 5), (129, 10, 6)])
@pytest.mark.parametrize("tune", TUNES2_F32)
def test_sweep2_fp32_equals_two_fp32_sweeps(shape, tune):
    nx, ny, nz = shape
    say("sweep2 fp32", shape, tune)
    e = synth.uniform_field(nx, ny, nz, 6, 1, -1, 1).astype(np.float32)
    r32 = synth.uniform_field(nx, ny, nz, 6, 2, -1, 1).astype(np.float32)
    h = 1.0 / (max(shape) + 1)
    h2 = np.float32(h * h)
    j3d.j3d_tune_set_single(j3d.KIND_F32X2, nx, ny, nz, tune)
    de = j3d.FArray.from_numpy(e, dtype=j3d.F32)
    stale = e.copy()
    stale[1:-1, 1:-1, 1:-1] = -3.0  # same halo, stale interior
    do = j3d.FArray.from_numpy(stale, dtype=j3d.F32)
    dr = j3d.FArray.from_numpy(r32, dtype=j3d.F32)
    j3d.jacobi3d_sweep2(de, do, dr, h)
    torch.cuda.synchronize()
    got = do.to_numpy()
    want = oracle.sweep_f32(oracle.sweep_f32(e, r32, h2), r32, h2)
    assert got.dtype == np.float32
    assert np.array_equal(got, want)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(j3d.J3DError) as ei:
        j3d.jacobi3d_sweep2(de, do, dr, h, resid_out=r)
    assert ei.value.code == j3d.EDTYPE


def test_fp32_fused_residual_rejected():
    a = j3d.FArray.empty(4, 4, 4, dtype=j3d.F32)
    b = j3d.FArray.empty(4, 4, 4, dtype=j3d.F32)
    c = j3d.FArray.empty(4, 4, 4, dtype=j3d.F32)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(j3d.J3DError) as ei:
        j3d.jacobi3d_sweep(a, b, c, 0.1, resid_out=r)
    assert ei.value.code == j3d.EDTYPE


def test_strided_views_and_lbounds():
    nx, ny, nz = 33, 18, 12
    say("strided views")
    u, f, h = make_inputs(nx, ny, nz, seed=3)
    want = oracle.sweep(u, f, h)
    j3d.j3d_tune_set_single(j3d.F64, nx, ny, nz, (4, 8, 1, 0, 0))
    du = j3d.FArray.from_numpy(u, lbound=(-3, 5, 2), ld_extra=7, plane_extra=5)
    dv = j3d.FArray.from_numpy(u, lbound=(1, 1, 1), align_bytes=8)
    df = j3d.FArray.from_numpy(f, lbound=(0, 0, 0), ld_extra=1, plane_extra=123)
    assert du.stride[1] != dv.stride[1] != df.stride[1]
    j3d.jacobi3d_sweep(du, dv, df, h)
    torch.cuda.synchronize()
    assert np.array_equal(dv.to_numpy(), want)
    # element addressing through the descriptor (lbound subtraction)
    assert j3d.j3d_element_offset(du, -3, 5, 2) == 0
    assert j3d.j3d_element_offset(du, -2, 6, 3) == 1 + du.stride[1] + du.stride[2]


def test_full_size_sweep_512():
    """The bench's grid (512^3, FP64) in the bench's launch configuration."""
    n = 512
    say("512^3 sweep + fused residual")
    h = 1.0 / (n + 1)
    f = synth.manufactured_f(n, n, n, h)
    du = j3d.FArray.empty(n, n, n)
    j3d.j3d_fill_uniform(du, 2, synth.STREAM_U0, 0.0, 1.0)
    dv = j3d.FArray.empty(n, n, n)
    df = j3d.FArray.from_numpy(f)
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    u = du.to_numpy()
    assert np.array_equal(u, synth.uniform_field(n, n, n, 2, synth.STREAM_U0, 0.0, 1.0)[:, :, :])
    want = oracle.sweep(u, f, h)
    got = dv.to_numpy()
    assert np.array_equal(got[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1])
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL


@pytest.mark.parametrize("tune", [(1, 2, 20, 0, 1, 1), (2, 4, 6, 0, 2, 2)])
def test_sweep_output_plane_of_2gib(tune):
    """An output array whose rows are padded so that one plane spans more
    than 2^31 bytes (9.5 GB in all): the pass must take its pointer-addressed
    path, give the oracle's bits and leave every element outside the interior
    (halo and padding) unchanged."""
    nx, ny, nz = 70, 9, 2
    ld = (1 << 28) // (ny + 1) + 64
    say("sweep with an output plane over 2 GiB", tune, "row stride", ld)
    u, f, h = make_inputs(nx, ny, nz)
    j3d.j3d_tune_set_single(j3d.F64, nx, ny, nz, tune)
    du = j3d.FArray.from_numpy(u)
    df = j3d.FArray.from_numpy(f)
    dv = j3d.FArray.empty(nx, ny, nz, ld_extra=ld - 80)
    assert dv.stride[1] * (ny + 1) * 8 >= 1 << 31
    dv.storage.fill_(0.375)
    dv.copy_from(u)
    before = dv.storage.clone()
    r = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep(du, dv, df, h, resid_out=r)
    torch.cuda.synchronize()
    want = oracle.sweep(u, f, h)
    assert np.array_equal(dv.to_numpy(), want)
    assert rel(float(r.item()), oracle.residual_l2(u, f, h)) <= RESID_RTOL
    # outside the interior nothing changed
    dv.view()[1:-1, 1:-1, 1:-1] = 0.0
    after = dv.storage
    bv = torch.as_strided(before, dv.view().shape, dv.view().stride(), dv.offset)
    bv[1:-1, 1:-1, 1:-1] = 0.0
    assert torch.equal(before, after)


def test_bandwidth_probe_sane():
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = j3d.j3d_bandwidth_probe(a, b, reps=5)
    say("copy GB/s", g)
    assert torch.equal(a, b)
    assert 500.0 < g < 8000.0 * 1.05
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    g3 = j3d.j3d_bandwidth_probe_triad(a, c, b, reps=3)
    say("two reads + one write GB/s", g3)
    assert torch.equal(b, torch.full_like(b, 3.0))
    assert 500.0 < g3 < 8000.0 * 1.05
