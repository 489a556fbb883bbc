"""GPU parity of the batched, graph-captured sweep over uneven grids."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import RESID_RTOL, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

from paper_2409_18824_amd import j3d  # noqa: E402


def make_batch(shapes, seed=4):
    grids, host = [], []
    for g, (nx, ny, nz) in enumerate(shapes):
        h = 1.0 / (max(nx, ny, nz) + 1)
        f = synth.uniform_field(nx, ny, nz, seed * 65536 + g, synth.STREAM_F, -1, 1)
        u0 = np.zeros_like(f)
        ua, ub, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
        grids.append((ua, ub, df, h))
        host.append((u0, f, h))
    return grids, host


SHAPES = [(33, 40, 35), (64, 17, 90), (5, 70, 3), (128, 32, 33), (1, 1, 1), (70, 70, 70)]


@pytest.mark.parametrize("tune", [(2, 16, 20, 0, 1, 2), (1, 8, 4, 1, 2, 4), (4, 32, 0, 0, 0), (2, 16, 1, 1, 0), (8, 8, 6, 1, 0), (1, 16, 7, 0, 0),
                                  (1, 8, 20, 0, 2), (2, 4, 22, 1, 1), (1, 16, 28 - 8, 0, 2)])
@pytest.mark.parametrize("nsweeps,every", [(20, 5), (7, 3)])
def test_batch_matches_oracle(tune, nsweeps, every):
    check_batch_against_oracle(tune, nsweeps, every)


@pytest.mark.parametrize("nsweeps,every", [(20, 4), (9, 2), (6, 2), (2, 2), (8, 8), (3, 2), (1, 2), (0, 2)])
@pytest.mark.parametrize("tune", [(1, 16, 20, 0, 1, 1), (4, 8, 6, 1, 2, 2)])
def test_batch_two_sweep_passes_match_oracle(monkeypatch, tune, nsweeps, every):
    """Sweeps two per pass (forced): the schedule keeps u_a/u_b placement and the residual cadence."""
    monkeypatch.setenv("J3D_BATCH_PAIRS", "1")
    check_batch_against_oracle(tune, nsweeps, every)


@pytest.mark.parametrize("nsweeps,every", [(20, 4), (9, 2), (6, 2), (2, 2), (8, 8), (3, 2), (1, 2), (0, 2), (20, 10),
                                            (13, 5), (7, 3), (11, 1), (10, 3), (17, 7), (4, 3), (5, 5)])
@pytest.mark.parametrize("tune", [(4, 16, 20, 0, 1, 1), (8, 8, 6, 0, 2, 1), (1, 16, 20, 0, 1, 2)])
def test_batch_three_sweep_passes_match_oracle(monkeypatch, tune, nsweeps, every):
    """Passes of up to three sweeps (forced), residuals fused at the stage that
    forms their iterate: iterates bit-exact, u_a/u_b placement by the parity
    of nsweeps, every residual of the cadence."""
    monkeypatch.setenv("J3D_BATCH_TRIPLES", "1")
    check_batch_against_oracle(tune, nsweeps, every)


@pytest.mark.parametrize("nsweeps,every", [(20, 4), (13, 5), (7, 3), (11, 1)])
@pytest.mark.parametrize("tile3", ["16,24,6,3", "8,16,20,3", "2,8,20,3", "4,64,6,3", "16,96,6,3"])
def test_batch_three_sweep_slot_order_matches_oracle(monkeypatch, tile3, nsweeps, every):
    """Three-sweep passes launched from the balanced slot list (tiles cut into
    eight runs of equal work, each longest tile first): every tile runs once,
    iterates bit-exact, every residual of the cadence."""
    monkeypatch.setenv("J3D_BATCH_TRIPLES", "1")
    monkeypatch.setenv("J3D_BATCH_TILE3", tile3)
    check_batch_against_oracle(None, nsweeps, every)
    rows, planes, var, order = (int(x) for x in tile3.split(","))
    assert j3d.j3d_batch_last_plan() == (3, (rows, planes, var, 0, order, 1))


@pytest.mark.parametrize("shapes,tile3", [([(70, 70, 70)], "16,24,6,3"), ([(1, 1, 1)], "2,8,20,3"),
                                          ([(3, 300, 2), (120, 1, 9)], "16,5,6,3")])
def test_batch_slot_order_few_tiles(monkeypatch, shapes, tile3):
    """Slot lists with fewer tiles than XCDs, or one grid only: runs left
    empty hold no tile, every tile still runs once."""
    monkeypatch.setenv("J3D_BATCH_TRIPLES", "1")
    monkeypatch.setenv("J3D_BATCH_TILE3", tile3)
    say("batch slots few", shapes, tile3)
    grids, host = make_batch(shapes)
    out = torch.zeros((len(grids), 4), dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep_batch(grids, 9, 3, out)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for g, ((ua, ub, _, _), (u0, f, h)) in enumerate(zip(grids, host)):
        u = u0.copy()
        want = []
        for s in range(10):
            if s % 3 == 0:
                want.append(oracle.residual_l2(u, f, h))
            if s < 9:
                u = oracle.sweep(u, f, h)
        assert np.array_equal(ub.to_numpy(), u), "grid %d" % g  # 9 sweeps: odd, result in u_b
        assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res[g], want)), (g, res[g], want)


@pytest.mark.parametrize("shape", ["16,24,6", "8,16,20"])
def test_batch_slot_order_equals_blocked_order_bitwise(monkeypatch, shape):
    """The slot order changes only which workgroup runs a tile: iterates and
    residuals (same per-tile partials, same reduction) are bitwise those of
    the XCD-blocked order."""
    monkeypatch.setenv("J3D_BATCH_TRIPLES", "1")
    results = []
    for order in ("0", "3"):
        monkeypatch.setenv("J3D_BATCH_TILE3", shape + "," + order)
        say("batch slots", shape, order)
        grids, _ = make_batch(SHAPES)
        out = torch.zeros((len(grids), 5), dtype=torch.float64, device="cuda")
        j3d.jacobi3d_sweep_batch(grids, 20, 5, out)
        torch.cuda.synchronize()
        results.append(([ua.to_numpy() for ua, _, _, _ in grids], out.cpu().numpy()))
    (u0, r0), (u3, r3) = results
    assert all(np.array_equal(a, b) for a, b in zip(u0, u3))
    assert np.array_equal(r0, r3)


def test_batch_tile3_override_rejects_bad_shapes(monkeypatch):
    grids, _ = make_batch(SHAPES[:2])
    for bad in ("3,24,6,0", "16,24,6,4", "16,24", "8,0,20,3"):
        monkeypatch.setenv("J3D_BATCH_TILE3", bad)
        with pytest.raises(RuntimeError, match="J3D_BATCH_TILE3"):
            j3d.jacobi3d_sweep_batch(grids, 6, 3, None)


def check_batch_against_oracle(tune, nsweeps, every):
    say("batch", tune, nsweeps, every)
    grids, host = make_batch(SHAPES)
    nres = nsweeps // every + 1
    out = torch.full((len(grids), nres), -1.0, dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep_batch(grids, nsweeps, every, out, tune=tune)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    for g, ((ua, ub, _, _), (u0, f, h)) in enumerate(zip(grids, host)):
        u = u0.copy()
        want = []
        for s in range(nsweeps + 1):
            if s % every == 0:
                want.append(oracle.residual_l2(u, f, h))
            if s < nsweeps:
                u = oracle.sweep(u, f, h)
        result = (ua if nsweeps % 2 == 0 else ub).to_numpy()
        assert np.array_equal(result, u), "grid %d" % g
        assert len(want) == nres
        assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res[g], want)), (g, res[g], want)


@pytest.mark.parametrize("pairs,triples", [("0", "0"), ("1", "0"), ("0", "1"), ("1", "1")])
def test_batch_equals_solo_bitwise_and_replays(monkeypatch, pairs, triples):
    monkeypatch.setenv("J3D_BATCH_PAIRS", pairs)
    monkeypatch.setenv("J3D_BATCH_TRIPLES", triples)
    tune = (4, 16, 0, 1, 0) if triples == "0" else (4, 16, 20, 0, 1, 1)
    say("batch vs solo", pairs, triples)
    grids, host = make_batch(SHAPES, seed=7)
    nres = 10 // 2 + 1
    out = torch.zeros((len(grids), nres), dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep_batch(grids, 10, 2, out, tune=tune)
    torch.cuda.synchronize()
    batch_u = [g[0].to_numpy() for g in grids]
    batch_r = out.cpu().numpy().copy()
    for g, (grid, (u0, f, h)) in enumerate(zip(grids, host)):
        ua, ub, df, _ = grid
        ua.copy_from(u0)
        o1 = torch.zeros((1, nres), dtype=torch.float64, device="cuda")
        j3d.jacobi3d_sweep_batch([grid], 10, 2, o1, tune=tune)
        torch.cuda.synchronize()
        assert np.array_equal(ua.to_numpy(), batch_u[g])
        assert np.array_equal(o1.cpu().numpy()[0], batch_r[g])
    # replaying the cached graph after resetting the inputs gives the same numbers
    for grid, (u0, _, _) in zip(grids, host):
        grid[0].copy_from(u0)
    out2 = torch.zeros_like(out)
    for rep in range(3):
        for grid, (u0, _, _) in zip(grids, host):
            grid[0].copy_from(u0)
        torch.cuda.synchronize()
        out.zero_()
        j3d.jacobi3d_sweep_batch(grids, 10, 2, out, tune=tune)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), batch_r), "replay %d" % rep
    del out2


def test_batch_autotune_choice_is_valid_and_used():
    say("batch autotune")
    grids, host = make_batch([(40, 50, 60), (100, 30, 20), (64, 64, 64)], seed=9)
    best = j3d.j3d_autotune(grids)
    assert best in j3d.tune_list()
    out = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    j3d.jacobi3d_sweep_batch(grids, 4, 4, out)  # tune=None: the cached choice
    torch.cuda.synchronize()
    for g, ((ua, _, _, _), (u0, f, h)) in enumerate(zip(grids, host)):
        u = u0
        for _ in range(4):
            u = oracle.sweep(u, f, h)
        assert np.array_equal(ua.to_numpy(), u)
        assert rel(out[g, 1].item(), oracle.residual_l2(u, f, h)) <= RESID_RTOL
