"""Parity of the multi-field stencils (pw_advection, tracer_advection) with
the CPU oracle, bit for bit: ragged shapes spanning several tiles for every
tile shape, padded layouts, and sampled points at the full sizes of the
paper's pw-advection (2048 x 1024 x 1024, more than 2^31 elements per field)
and tra-adv (1024 x 512 x 512, 20 steps) in the benchmark's launch
configuration.  Sampled references are computed from the CPU input
generator's values of a small box around each point."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import needs_gpu, say
from paper_2409_18824_amd import j3d

pytestmark = [pytest.mark.gpu, needs_gpu]

# rows per thread, z-planes per wavefront, nontemporal stores[, loads one plane ahead]
TILES = ["2,7,0", "2,128,1", "4,5,1", "4,128,0", "8,3,0", "8,64,1", "2,7,0,1", "2,128,1,1", "4,5,1,1", "4,128,0,1",
         "8,3,0,1"]
# x tiles are 64 wide, y tiles 4 x rows-per-thread, z chunks `planes` deep
SHAPES = [(1, 1, 1), (64, 4, 3), (65, 8, 2), (63, 17, 9), (130, 37, 19), (125, 9, 131)]


def rand_padded(nx, ny, nz, seed, stream, lo=-1.0, hi=1.0):
    """A padded field whose every element, halo included, is random."""
    big = synth.uniform_field(nx + 2, ny + 2, nz + 2, seed, stream, lo, hi)
    return np.ascontiguousarray(big[1:-1, 1:-1, 1:-1])


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tile", TILES)
def test_pw_advection_parity(tile, shape, monkeypatch):
    monkeypatch.setenv("J3D_ADVECT_TILE", tile)
    nx, ny, nz = shape
    say("pw_advection", tile, shape)
    u, v, w = (rand_padded(nx, ny, nz, 21, s) for s in (6, 7, 8))
    d = (0.3, 0.11, 1.7)
    want = oracle.pw_advection(u, v, w, *d)
    ins = [j3d.FArray.from_numpy(a, ld_extra=2, plane_extra=1) for a in (u, v, w)]
    outs = [j3d.FArray.empty(nx, ny, nz, ld_extra=3, plane_extra=5) for _ in range(3)]
    for o in outs:
        j3d.j3d_fill_const(o, 7.5)
    j3d.pw_advection(*ins, *outs, *d)
    torch.cuda.synchronize()
    for o, wt in zip(outs, want):
        g = o.to_numpy()
        assert np.array_equal(g[1:-1, 1:-1, 1:-1], wt[1:-1, 1:-1, 1:-1])
        g[1:-1, 1:-1, 1:-1] = 7.5
        assert np.all(g == 7.5)  # the halo is not written


def test_pw_advection_uniform_flow_is_zero():
    nx, ny, nz = 70, 9, 6
    ins = [j3d.FArray.empty(nx, ny, nz) for _ in range(3)]
    for a, c in zip(ins, (0.3, -1.7, 2.9)):
        j3d.j3d_fill_const(a, c)
    outs = [j3d.FArray.empty(nx, ny, nz) for _ in range(3)]
    for o in outs:
        j3d.j3d_fill_const(o, 1.0)
    j3d.pw_advection(*ins, *outs, 0.1, 0.2, 0.3)
    torch.cuda.synchronize()
    for o in outs:
        assert np.all(o.to_numpy()[1:-1, 1:-1, 1:-1] == 0.0)


# two-step tracer passes: rows per thread 2, 4 or 6 (x tiles 60 wide,
# workgroups of 4 x rows-per-thread rows, the outer two a ring)
TILES2 = ["2,7,0", "4,64,1", "6,64,1", "4,5,0", "6,3,0", "2,64,1"]


@pytest.mark.parametrize("shape", SHAPES + [(60, 8, 4), (61, 9, 70), (121, 3, 2), (64, 22, 5), (65, 23, 4),
                                            (60, 45, 3), (17, 14, 9)])
@pytest.mark.parametrize("tile,tile2,steps", [(t, TILES2[n % len(TILES2)], 1 + n % 2) for n, t in enumerate(TILES)]
                         + [(TILES[1], t2, 2) for t2 in TILES2])
def test_tracer_advection_parity(tile, tile2, steps, shape, monkeypatch):
    monkeypatch.setenv("J3D_ADVECT_TILE", tile)
    monkeypatch.setenv("J3D_TRACER2_TILE", tile2)
    monkeypatch.setenv("J3D_TRACER_STEPS_PER_PASS", str(steps))
    nx, ny, nz = shape
    say("tracer_advection", tile, tile2, steps, shape)
    t = rand_padded(nx, ny, nz, 22, synth.STREAM_TRACER, 0.0, 1.0)
    u, v, w = (rand_padded(nx, ny, nz, 22, s, -0.1, 0.1) for s in (6, 7, 8))
    u[::3, ::2, ::5] = 0.0  # zero transports take neither branch
    v[1::4, ::3, ::2] = -0.0
    r = rand_padded(nx, ny, nz, 22, synth.STREAM_RVOL, 0.5, 1.5)
    fields = [j3d.FArray.from_numpy(a) for a in (u, v, w, r)]
    for niter in (0, 1, 2, 3, 4, 5):
        want = oracle.tracer_advection(t, u, v, w, r, niter)
        da, db = j3d.FArray.from_numpy(t), j3d.FArray.from_numpy(t)
        j3d.tracer_advection(da, db, *fields, niter)
        torch.cuda.synchronize()
        got = (da if niter % 2 == 0 else db).to_numpy()
        assert np.array_equal(got, want), niter


def sample_points(shape, count, seams, seed):
    """count random interior points plus every combination of the seam
    coordinates (tile edges, domain corners) per axis."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    pts = [tuple(int(rng.integers(1, n + 1)) for n in (nx, ny, nz)) for _ in range(count)]
    sx, sy, sz = seams
    pts += [(i, j, k) for i in sx for j in sy for k in sz]
    return pts


def gather(a: j3d.FArray, pts):
    """Values of a device array at the (i, j, k) points."""
    idx = torch.tensor(pts, dtype=torch.long, device="cuda")
    return a.view()[idx[:, 2], idx[:, 1], idx[:, 0]].cpu().numpy()


def test_pw_advection_full_size_sampled():
    nx, ny, nz = synth.PW_SHAPE
    recipe, d = synth.pw_recipe()
    say("pw_advection full size", synth.PW_SHAPE)
    ins = []
    for fr in recipe:
        a = j3d.FArray.empty(nx, ny, nz)
        j3d.j3d_fill_uniform(a, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo)
        ins.append(a)
    outs = [j3d.FArray.empty(nx, ny, nz) for _ in range(3)]
    j3d.pw_advection(*ins, *outs, *d)  # the library's default tile shape
    torch.cuda.synchronize()
    seams = ((1, 2, 63, 64, 65, 128, 129, 2047, 2048), (1, 4, 5, 16, 17, 1023, 1024), (1, 128, 129, 1024))
    pts = sample_points((nx, ny, nz), 1500, seams, 31)
    got = [gather(o, pts) for o in outs]
    # the inputs on the device are the generator's (checked on a few boxes)
    for (i, j, k) in pts[:20]:
        for a, fr in zip(ins, recipe):
            box = synth.uniform_box(nx, ny, nz, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo,
                                    i - 1, i + 2, j - 1, j + 2, k - 1, k + 2)
            assert np.array_equal(a.view()[k - 1:k + 2, j - 1:j + 2, i - 1:i + 2].cpu().numpy(), box)
    bad = 0
    for n, (i, j, k) in enumerate(pts):
        boxes = [np.ascontiguousarray(synth.uniform_box(nx, ny, nz, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo,
                                                        i - 1, i + 2, j - 1, j + 2, k - 1, k + 2))
                 for fr in recipe]
        want = oracle.pw_advection(*boxes, *d)
        for c in range(3):
            bad += int(got[c][n] != want[c][1, 1, 1])
    assert bad == 0
    del ins, outs
    torch.cuda.empty_cache()


def test_tracer_advection_full_size_sampled():
    nx, ny, nz = synth.TRA_SHAPE
    niter = synth.TRA_ITERS
    rt, rvel, rr = synth.tracer_recipe()
    say("tracer_advection full size", synth.TRA_SHAPE, niter)
    recipe = [rt, rt] + rvel + [rr]
    arrs = []
    for fr in recipe:
        a = j3d.FArray.empty(nx, ny, nz)
        j3d.j3d_fill_uniform(a, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo)
        arrs.append(a)
    j3d.tracer_advection(*arrs, niter)
    torch.cuda.synchronize()
    res = arrs[0] if niter % 2 == 0 else arrs[1]
    seams = ((1, 60, 61, 64, 65, 1020, 1021, 1024), (1, 16, 17, 512), (1, 64, 65, 512))
    pts = sample_points((nx, ny, nz), 20, seams, 32)
    got = gather(res, pts)
    R = niter + 1  # the result at a point depends on cells within niter steps
    bad = 0
    for n, (i, j, k) in enumerate(pts):
        lo = [max(c - R, 0) for c in (i, j, k)]
        hi = [min(c + R, m + 1) + 1 for c, m in zip((i, j, k), (nx, ny, nz))]
        boxes = [np.ascontiguousarray(synth.uniform_box(nx, ny, nz, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo,
                                                        lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]))
                 for fr in [rt] + rvel + [rr]]
        # the box's outer layer stays fixed: real halo, or cells farther than niter steps
        want = oracle.tracer_advection(*boxes, niter)
        bad += int(got[n] != want[k - lo[2], j - lo[1], i - lo[0]])
    assert bad == 0
    del arrs, res
    torch.cuda.empty_cache()


def test_non_finite_inputs_follow_the_oracle(monkeypatch):
    """NaN and infinity propagate (or not) exactly as the definitions give:
    an upwind flux with a NaN transport takes neither branch and is zero, a
    NaN tracer or velocity value spreads to the stencil's points."""
    nx, ny, nz = 70, 9, 6
    u, v, w = (rand_padded(nx, ny, nz, 23, s) for s in (6, 7, 8))
    u[3, 4, 5] = np.nan
    v[2, 2, 60] = np.inf
    w[4, 7, 1] = -np.inf
    want = oracle.pw_advection(u, v, w, 0.5, 0.25, 0.125)
    ins = [j3d.FArray.from_numpy(a) for a in (u, v, w)]
    outs = [j3d.FArray.empty(nx, ny, nz) for _ in range(3)]
    j3d.pw_advection(*ins, *outs, 0.5, 0.25, 0.125)
    torch.cuda.synchronize()
    for o, wt in zip(outs, want):
        g = o.to_numpy()[1:-1, 1:-1, 1:-1]
        assert np.array_equal(g, wt[1:-1, 1:-1, 1:-1], equal_nan=True)
        assert not np.isfinite(g).all()
    t = rand_padded(nx, ny, nz, 24, synth.STREAM_TRACER, 0.0, 1.0)
    t[3, 3, 30] = np.nan
    q = [0.1 * a for a in (u, v, w)]
    q[0][2, 5, 10] = np.nan  # a NaN transport gives a zero flux
    r = rand_padded(nx, ny, nz, 24, synth.STREAM_RVOL, 0.5, 1.5)
    want = oracle.tracer_advection(t, *q, r, 4)
    for steps in ("1", "2"):
        monkeypatch.setenv("J3D_TRACER_STEPS_PER_PASS", steps)
        da, db = j3d.FArray.from_numpy(t), j3d.FArray.from_numpy(t)
        j3d.tracer_advection(da, db, *[j3d.FArray.from_numpy(a) for a in q + [r]], 4)
        torch.cuda.synchronize()
        assert np.array_equal(da.to_numpy(), want, equal_nan=True), steps
