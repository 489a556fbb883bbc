"""GPU parity of poisson_solve (plain FP64 and mixed precision) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import RESID_RTOL, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

# pass lengths forced on the small test grids ("" lets the solver choose:
# two-sweep and single passes there, three-sweep passes on large grids)
STEPS = ["", "1", "3"]

from paper_2409_18824_amd import j3d  # noqa: E402


def test_small_plain_100_sweeps_residual_every_sweep():
    """64^3 FP64, u0 ~ U[0,1), f ~ U[-1,1), h = 1/65: 100 sweeps, residual after each."""
    say("64^3 x 100 sweeps")
    u0, f, h = synth.small_plain(64, seed=1)
    du = j3d.FArray.from_numpy(u0)
    df = j3d.FArray.from_numpy(f)
    res = j3d.poisson_solve(du, df, h, mode=j3d.MODE_FP64, rtol=0.0, max_sweeps=100, check_every=1)
    uo, ro = oracle.solve_plain(u0, f, h, rtol=0.0, check_every=1, max_sweeps=100)
    assert res.sweeps == ro.sweeps == 100 and not res.converged
    assert len(res.history) == len(ro.history) == 101
    worst = max(rel(a, b) for a, b in zip(res.history, ro.history))
    say("worst residual rel err", worst)
    assert worst <= RESID_RTOL
    assert rel(res.norm_f, ro.norm_f) <= RESID_RTOL
    assert np.array_equal(du.to_numpy(), uo)


@pytest.mark.parametrize("max_sweeps,check_every", [(0, 1), (7, 3), (10, 5), (1, 1), (10, 2), (9, 4), (1, 2),
                                                   (3, 2), (0, 2), (23, 10), (8, 3), (5, 9), (17, 8)])
@pytest.mark.parametrize("step", STEPS)
def test_plain_cadence_edges(max_sweeps, check_every, step, monkeypatch):
    monkeypatch.setenv("J3D_SOLVE_SWEEPS_PER_PASS", step)
    n = (9, 11, 6)
    say("cadence", max_sweeps, check_every)
    u0 = synth.uniform_field(*n, 4, 1, 0, 1)
    f = synth.uniform_field(*n, 4, 2, -1, 1)
    h = 0.1
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    res = j3d.poisson_solve(du, df, h, rtol=0.0, max_sweeps=max_sweeps, check_every=check_every)
    uo, ro = oracle.solve_plain(u0, f, h, rtol=0.0, check_every=check_every, max_sweeps=max_sweeps)
    assert res.sweeps == ro.sweeps
    assert len(res.history) == len(ro.history)
    assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
    assert rel(res.resid, ro.resid) <= RESID_RTOL
    assert np.array_equal(du.to_numpy(), uo)


def test_plain_early_exit_matches_oracle():
    n = 20
    say("plain early exit")
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 2, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h)
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    res = j3d.poisson_solve(du, df, h, rtol=1e-6, max_sweeps=100000, check_every=10)
    uo, ro = oracle.solve_plain(u0, f, h, rtol=1e-6, check_every=10, max_sweeps=100000)
    assert ro.converged and res.converged
    assert res.sweeps == ro.sweeps
    assert rel(res.resid, ro.resid) <= RESID_RTOL and res.resid <= 1e-6 * res.norm_f
    assert np.array_equal(du.to_numpy(), uo)


@pytest.mark.parametrize("n,rtol", [(12, 1e-3), (16, 2e-5), (9, 1e-12)])
def test_plain_early_exit_every_sweep_matches_oracle(n, rtol):
    """A check after every sweep (each check reduced by a workgroup of the
    next pass, which runs before the verdict is known): the solve stops at
    the oracle's sweep with the oracle's iterate, including exits inside a
    replayed chunk."""
    say("plain early exit, check every sweep", n, rtol)
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 5, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h)
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    res = j3d.poisson_solve(du, df, h, rtol=rtol, max_sweeps=100000, check_every=1)
    uo, ro = oracle.solve_plain(u0, f, h, rtol=rtol, check_every=1, max_sweeps=100000)
    assert ro.converged and res.converged
    assert res.sweeps == ro.sweeps
    assert len(res.history) == len(ro.history)
    assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
    assert np.array_equal(du.to_numpy(), uo)


@pytest.mark.parametrize("n,S,rtol,tune", [(64, 100, 0.0, None), (9, 1, 0.0, None), (9, 0, 0.0, None),
                                           (11, 1001, 0.0, None), (12, 100000, 1e-3, None), (10, 7, 0.0, None),
                                           (13, 13, 0.0, None),
                                           # one to sixteen wavefronts per workgroup (the reducing workgroup
                                           # stands in for 1024 / T threads), persistent grids, LDS variants
                                           (40, 50, 0.0, (1, 4, 20, 1, 2, 1)), (40, 50, 0.0, (8, 2, 6, 0, 1, 2)),
                                           (40, 50, 0.0, (2, 2, 21, 0, 1, 1)), (40, 50, 0.0, (4, 8, 20, 1, 0, 4)),
                                           (33, 40, 0.0, (1, 16, 4, 0, 2, 1))])
def test_fused_checks_equal_reduction_kernels(n, S, rtol, tune, monkeypatch):
    """The checks reduced inside the next pass give the same bits as the
    schedule with a reduction kernel per check: history, sweeps, iterate."""
    say("fused checks", n, S, rtol, tune)
    if tune is not None:
        j3d.j3d_tune_set_single(j3d.F64, n, n, n, tune)
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 7, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h) if rtol > 0 else synth.uniform_field(n, n, n, 7, 2, -1, 1)
    df = j3d.FArray.from_numpy(f)
    out = []
    for fused in ("1", "0"):
        monkeypatch.setenv("J3D_SOLVE_FUSED_CHECKS", fused)
        du = j3d.FArray.from_numpy(u0)
        r = j3d.poisson_solve(du, df, h, rtol=rtol, max_sweeps=S, check_every=1)
        out.append((r.sweeps, r.converged, list(r.history), r.resid, du.to_numpy()))
    a, b = out
    assert a[0] == b[0] and a[1] == b[1] and a[3] == b[3]
    assert a[2] == b[2], "residual histories differ"
    assert np.array_equal(a[4], b[4])


@pytest.mark.parametrize("n,inner,rtol,cap", [(24, 50, 1e-8, 100000), (13, 7, 1e-10, 100000),
                                              (16, 50, 1e-14, 120), (10, 1, 1e-3, 1000), (11, 2, 1e-9, 100000),
                                              (12, 3, 1e-9, 100000), (9, 4, 1e-9, 100000), (14, 6, 1e-12, 53),
                                              (70, 50, 1e-7, 100000), (15, 5, 1e-9, 100000),
                                              (17, 9, 1e-10, 100000), (19, 10, 1e-9, 100000)])
@pytest.mark.parametrize("step", STEPS)
def test_mixed_matches_oracle(n, inner, rtol, cap, step, monkeypatch):
    monkeypatch.setenv("J3D_SOLVE_SWEEPS_PER_PASS", step)
    say("mixed", n, inner, rtol, cap, step)
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 2, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h)
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    res = j3d.poisson_solve(du, df, h, mode=j3d.MODE_MIXED, rtol=rtol, max_sweeps=cap, inner_sweeps=inner)
    uo, ro = oracle.solve_mixed(u0, f, h, rtol=rtol, inner=inner, max_sweeps=cap)
    assert res.converged == ro.converged
    assert res.sweeps == ro.sweeps
    assert len(res.history) == len(ro.history)
    assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
    # FP32 sweeps, FP64 defects, same order on both sides: the fields agree bitwise
    assert np.array_equal(du.to_numpy(), uo)


def test_mixed_and_plain_reach_tolerance_at_same_sweep_count():
    n = 24
    say("mixed vs plain sweep count")
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 2, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h)
    a, b = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(u0)
    df = j3d.FArray.from_numpy(f)
    rp = j3d.poisson_solve(a, df, h, mode=j3d.MODE_FP64, rtol=1e-8, max_sweeps=10 ** 6, check_every=50)
    rm = j3d.poisson_solve(b, df, h, mode=j3d.MODE_MIXED, rtol=1e-8, max_sweeps=10 ** 6, inner_sweeps=50)
    assert rp.converged and rm.converged and rp.sweeps == rm.sweeps
    # the converged fields agree to the tolerance's order
    ua, ub = a.to_numpy(), b.to_numpy()
    assert np.max(np.abs(ua - ub)) <= 1e-7 * np.max(np.abs(ua))
    # both residuals verified on the CPU
    assert oracle.residual_l2(ub, f, h) <= 1e-8 * rm.norm_f * (1 + 1e-9)


def test_nonfinite_reported():
    n = 8
    u0 = np.zeros((n + 2,) * 3)
    f = synth.uniform_field(n, n, n, 3, 2, -1, 1)
    f[4, 4, 4] = np.nan
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    with pytest.raises(j3d.J3DError) as ei:
        j3d.poisson_solve(du, df, 0.1, rtol=1e-8, max_sweeps=50, check_every=5)
    assert ei.value.code == j3d.ENONFINITE
    r = j3d.poisson_solve(du, df, 0.1, mode=j3d.MODE_MIXED, rtol=1e-8, max_sweeps=50, raise_nonfinite=False)
    assert r.status == j3d.ENONFINITE and not r.converged


def test_warm_start_resume():
    """Solving in two halves from the returned iterate equals one solve."""
    n = 12
    h = 1.0 / 13
    u0 = synth.uniform_field(n, n, n, 6, 1, 0, 1)
    f = synth.uniform_field(n, n, n, 6, 2, -1, 1)
    a, b = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(u0)
    df = j3d.FArray.from_numpy(f)
    j3d.poisson_solve(a, df, h, rtol=0.0, max_sweeps=60, check_every=10)
    j3d.poisson_solve(b, df, h, rtol=0.0, max_sweeps=30, check_every=10)
    j3d.poisson_solve(b, df, h, rtol=0.0, max_sweeps=30, check_every=10)
    assert np.array_equal(a.to_numpy(), b.to_numpy())


@pytest.mark.parametrize("S,every", [(1234, 2), (1001, 1), (1200, 3), (999, 4), (1100, 7), (997, 6), (1000, 10)])
@pytest.mark.parametrize("step", STEPS)
def test_plain_graph_replay_and_tail(S, every, step, monkeypatch):
    """Long solves replay a captured chunk graph, then finish directly: same
    iterate and history as the oracle, and again on a second call (cached
    graph)."""
    monkeypatch.setenv("J3D_SOLVE_SWEEPS_PER_PASS", step)
    n = 24
    say("graph replay", S, every, step)
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 8, 1, 0, 1)
    f = synth.uniform_field(n, n, n, 8, 2, -1, 1)
    uo, ro = oracle.solve_plain(u0, f, h, rtol=0.0, check_every=every, max_sweeps=S)
    df = j3d.FArray.from_numpy(f)
    for rep in range(2):
        du = j3d.FArray.from_numpy(u0)
        res = j3d.poisson_solve(du, df, h, rtol=0.0, max_sweeps=S, check_every=every)
        assert res.sweeps == S and len(res.history) == len(ro.history)
        assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
        assert np.array_equal(du.to_numpy(), uo), "call %d" % rep


@pytest.mark.parametrize("step", STEPS)
def test_mixed_graph_replay_matches_oracle(step, monkeypatch):
    monkeypatch.setenv("J3D_SOLVE_SWEEPS_PER_PASS", step)
    n = 24
    say("mixed graph replay", step)
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 9, 1, 0, 1)
    f = synth.uniform_field(n, n, n, 9, 2, -1, 1)
    uo, ro = oracle.solve_mixed(u0, f, h, rtol=0.0, inner=50, max_sweeps=5030)
    df = j3d.FArray.from_numpy(f)
    for rep in range(2):
        du = j3d.FArray.from_numpy(u0)
        res = j3d.poisson_solve(du, df, h, mode=j3d.MODE_MIXED, rtol=0.0, max_sweeps=5030, inner_sweeps=50)
        assert res.sweeps == ro.sweeps == 5030 and len(res.history) == len(ro.history)
        assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
        assert np.array_equal(du.to_numpy(), uo), "call %d" % rep


@pytest.mark.parametrize("mode,shape,every", [(j3d.MODE_FP64, (320, 300, 230), 5), (j3d.MODE_MIXED, (360, 350, 340), 7)])
def test_large_grids_choose_three_sweep_passes(mode, shape, every, monkeypatch):
    """Grids whose pass arrays overflow the cache (over 512 MB: FP64 u, w, f;
    FP32 r, e0, e1) run three-sweep passes by themselves: same iterate and
    history as the oracle."""
    monkeypatch.delenv("J3D_SOLVE_SWEEPS_PER_PASS", raising=False)
    nx, ny, nz = shape
    say("large solve", mode, shape, every)
    h = 1.0 / (max(shape) + 1)
    u0 = synth.uniform_field(nx, ny, nz, 10, 1, 0, 1)
    f = synth.uniform_field(nx, ny, nz, 10, 2, -1, 1)
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    if mode == j3d.MODE_FP64:
        assert 24 * nx * ny * nz > 512e6
        res = j3d.poisson_solve(du, df, h, rtol=0.0, max_sweeps=13, check_every=every)
        uo, ro = oracle.solve_plain(u0, f, h, rtol=0.0, check_every=every, max_sweeps=13)
    else:
        assert 12 * nx * ny * nz > 512e6
        res = j3d.poisson_solve(du, df, h, mode=j3d.MODE_MIXED, rtol=0.0, max_sweeps=2 * every,
                                inner_sweeps=every)
        uo, ro = oracle.solve_mixed(u0, f, h, rtol=0.0, inner=every, max_sweeps=2 * every)
    assert res.sweeps == ro.sweeps and len(res.history) == len(ro.history)
    assert all(rel(a, b) <= RESID_RTOL for a, b in zip(res.history, ro.history))
    assert np.array_equal(du.to_numpy(), uo)
