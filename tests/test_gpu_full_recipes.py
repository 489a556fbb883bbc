"""The batched and served workloads at their full recipes, sampled against the oracle.

Batch: the 256 grids of the batch benchmark (each axis uniform in
{32..256}, f ~ U[-1,1) drawn on the device, u0 = 0), 200 sweeps with the
residual every 10 sweeps, in one jacobi3d_sweep_batch call on the autotuned
path.  Eight grids (the smallest, the largest, the first and last of the tile
list, four seeded others) are compared with the oracle: iterates bit for bit,
residual rows within the residual tolerance; every grid's residual row must
be finite and decreasing.

Serve: the first 30 requests with n <= 128 of the served request stream
(f ~ U[-1,1) from each request's seed, tolerance 1e-6 or 1e-8, cap 5000
sweeps), all submitted at once to a server with 8 slots, so they run in
mixes that change as requests retire and waiting ones are admitted; each
result is compared with the oracle's mixed-precision solve of the same
request alone, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import RESID_RTOL, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

from paper_2409_18824_amd import j3d  # noqa: E402


def test_batch_full_recipe_sampled():
    shapes = synth.batch_shapes(256, 4)
    nsw, every = 200, 10
    say("batch full recipe: %d grids, %.3g points" % (len(shapes), sum(g.nx * g.ny * g.nz for g in shapes)))
    grids = []
    for g in shapes:
        ua, ub, f = j3d.FArray.empty(g.nx, g.ny, g.nz), j3d.FArray.empty(g.nx, g.ny, g.nz), \
            j3d.FArray.empty(g.nx, g.ny, g.nz)
        j3d.j3d_fill_const(ua, 0.0)
        j3d.j3d_fill_const(ub, 0.0)
        j3d.j3d_fill_uniform(f, g.seed, synth.STREAM_F, -1.0, 1.0)
        grids.append((ua, ub, f, g.h))
    out = torch.full((len(grids), nsw // every + 1), -1.0, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep_batch(grids, nsw, every, out)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    assert np.all(np.isfinite(r)) and np.all(np.diff(r, axis=1) < 0), "residual rows must decrease"
    pts = [g.nx * g.ny * g.nz for g in shapes]
    pick = {int(np.argmin(pts)), int(np.argmax(pts)), 0, len(shapes) - 1}
    rng = np.random.default_rng(7)
    while len(pick) < 8:
        pick.add(int(rng.integers(0, len(shapes))))
    for gi in sorted(pick):
        g = shapes[gi]
        say("batch full recipe: grid %d %s" % (gi, (g.nx, g.ny, g.nz)))
        f = synth.batch_rhs(g)
        assert np.array_equal(grids[gi][2].to_numpy(), f), "the device-drawn f differs from synth's"
        uo, ro = oracle.solve_plain(np.zeros_like(f), f, g.h, rtol=0.0, check_every=every, max_sweeps=nsw)
        assert ro.sweeps == nsw and len(ro.history) == nsw // every + 1
        assert np.array_equal(grids[gi][0].to_numpy(), uo), "grid %d differs from the oracle" % gi
        for q in range(nsw // every + 1):
            assert rel(r[gi, q], ro.history[q]) <= RESID_RTOL, (gi, q, r[gi, q], ro.history[q])


def test_serve_full_recipe_first_requests():
    reqs = [x for x in synth.serve_requests(1000) if x.n <= 128][:30]
    say("serve full recipe: %d requests, n = %s" % (len(reqs), [x.n for x in reqs]))
    outs, tick = {}, {}
    with j3d.Server(hbm_budget_bytes=200 * 10 ** 9, max_slots=8, cycle_sweeps=50) as s:
        for x in reqs:
            u = np.zeros((x.n + 2,) * 3)
            t = s.submit(x.n, x.h, x.rtol, x.max_sweeps, seed=x.seed, u_out=u)
            tick[t] = x
            outs[x.rid] = u
        # the oracle runs while the server works
        want = {}
        for x in reqs:
            f = synth.uniform_field(x.n, x.n, x.n, x.seed, synth.STREAM_F, -1.0, 1.0)
            want[x.rid] = oracle.solve_mixed(np.zeros_like(f), f, x.h, rtol=x.rtol, inner=50,
                                             max_sweeps=x.max_sweeps)
        s.drain(timeout_s=300)
        got = {tick[r["ticket"]].rid: r for r in s.poll(4096)}
    assert len(got) == len(reqs)
    for x in reqs:
        uo, ro = want[x.rid]
        g = got[x.rid]
        assert g["status"] == j3d.OK
        assert g["converged"] == ro.converged and g["sweeps"] == ro.sweeps, (x, g, ro.sweeps)
        assert rel(g["resid"], ro.resid) <= RESID_RTOL, (x.rid, g["resid"], ro.resid)
        assert np.array_equal(outs[x.rid], uo), "request %d differs from the oracle" % x.rid
