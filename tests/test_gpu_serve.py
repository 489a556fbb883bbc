"""GPU tests of the continuous-batching server."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import RESID_RTOL, needs_gpu, rel, say

pytestmark = [pytest.mark.gpu, needs_gpu]

from paper_2409_18824_amd import j3d  # noqa: E402


def rhs(n, seed):
    return synth.uniform_field(n, n, n, seed, synth.STREAM_F, -1.0, 1.0)


def run(server, reqs, gaps=None):
    outs, tickets = {}, {}
    for k, (n, rtol, cap, seed, use_host_f) in enumerate(reqs):
        u = np.zeros((n + 2,) * 3)
        f = rhs(n, seed) if use_host_f else None
        t = server.submit(n, 1.0 / (n + 1), rtol, cap, seed=seed, f_host=f, u_out=u)
        tickets[t] = k
        outs[k] = u
        if gaps:
            time.sleep(gaps)
    server.drain(timeout_s=120)
    results = {tickets[r["ticket"]]: r for r in server.poll(4096)}
    assert len(results) == len(reqs)
    return results, outs


@pytest.mark.parametrize("cycle", [1, 2, 3, 4, 5, 6, 7, 9])
@pytest.mark.parametrize("triples", ["0", "1"])
def test_served_cycle_lengths_match_oracle(cycle, triples, monkeypatch):
    """Cycle lengths that take each branch of the correction-sweep schedule,
    with two-sweep and with three-sweep passes."""
    monkeypatch.setenv("J3D_SERVE_TRIPLES", triples)
    reqs = [(10, 1e-8, 400, 21, True), (13, 1e-6, 400, 22, False)]
    say("serve cycle", cycle, triples)
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=4, cycle_sweeps=cycle) as s:
        got, got_u = run(s, reqs)
    for k, (n, rtol, cap, seed, _) in enumerate(reqs):
        f = rhs(n, seed)
        cap_c = -(-cap // cycle) * cycle  # whole cycles
        uo, ro = oracle.solve_mixed(np.zeros((n + 2,) * 3), f, 1.0 / (n + 1), rtol=rtol, inner=cycle,
                                    max_sweeps=cap_c)
        assert got[k]["converged"] == ro.converged and got[k]["sweeps"] == ro.sweeps
        assert rel(got[k]["resid"], ro.resid) <= RESID_RTOL
        assert np.array_equal(got_u[k], uo)


@pytest.mark.parametrize("triples", ["0", "1"])
def test_served_equals_oracle_and_solo(triples, monkeypatch):
    monkeypatch.setenv("J3D_SERVE_TRIPLES", triples)
    reqs = [(12, 1e-8, 5000, 11, True), (16, 1e-6, 5000, 12, False), (20, 1e-8, 300, 13, True),
            (9, 1e-10, 5000, 14, False), (24, 1e-6, 200, 15, True)]
    say("serve mix", triples)
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=8, cycle_sweeps=50) as s:
        mix, mix_u = run(s, reqs)
    for k, (n, rtol, cap, seed, _) in enumerate(reqs):
        say("serve solo", k)
        with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=1, cycle_sweeps=50) as s:
            solo, solo_u = run(s, [reqs[k]])
        a, b = mix[k], solo[0]
        # bitwise: the same kernels, tile shapes and reduction order alone and in the mix
        assert np.array_equal(mix_u[k], solo_u[0])
        assert (a["sweeps"], a["converged"], a["resid"]) == (b["sweeps"], b["converged"], b["resid"])
        # against the oracle's mixed solve with the same cycle length
        f = rhs(n, seed)
        h = 1.0 / (n + 1)
        uo, ro = oracle.solve_mixed(np.zeros((n + 2,) * 3), f, h, rtol=rtol, inner=50, max_sweeps=cap)
        assert a["converged"] == ro.converged and a["sweeps"] == ro.sweeps
        assert rel(a["resid"], ro.resid) <= RESID_RTOL
        assert rel(a["norm_f"], ro.norm_f) <= RESID_RTOL
        assert np.array_equal(mix_u[k], uo)
        assert a["t_submit"] <= a["t_admit"] <= a["t_done"]


def test_budget_admission_and_rejection():
    per = j3d.j3d_request_bytes(20, 20, 20)
    say("budget", per)
    with j3d.Server(hbm_budget_bytes=2 * per + 10, max_slots=8, cycle_sweeps=10) as s:
        big = j3d.j3d_request_bytes(40, 40, 40)
        assert big > 2 * per + 10
        with pytest.raises(j3d.J3DError) as ei:
            s.submit(40, 1 / 41, 1e-8, 100, seed=1)
        assert ei.value.code == j3d.EBUDGET
        reqs = [(20, 1e-12, 40, 30 + k, False) for k in range(5)]
        res, _ = run(s, reqs)
        # at most two fit at once: admissions happen as earlier ones retire
        order = sorted(res.values(), key=lambda r: r["t_admit"])
        for k in range(2, 5):
            earlier_done = sorted(r["t_done"] for r in order[:k])
            assert order[k]["t_admit"] >= earlier_done[k - 2] - 1e-3
        assert all(r["sweeps"] == 40 and not r["converged"] for r in res.values())


def test_continuous_batching_late_arrivals_join():
    """Requests arriving while others run are admitted at cycle boundaries."""
    reqs = [(160, 1e-14, 20000, 40, False)] + [(12, 1e-8, 5000, 41 + k, False) for k in range(4)]
    say("late arrivals")
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=8, cycle_sweeps=50) as s:
        res, _ = run(s, reqs, gaps=0.005)
    long = res[0]
    for k in range(1, 5):
        # each short request was admitted and finished while the long one was still running
        assert res[k]["t_admit"] < long["t_done"]
        assert res[k]["t_done"] < long["t_done"]


def test_active_points_target_limits_concurrency():
    pts = 20 ** 3
    say("active points target")
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=8, cycle_sweeps=10, max_active_points=2 * pts) as s:
        reqs = [(20, 1e-12, 40, 60 + k, False) for k in range(5)]
        res, _ = run(s, reqs)
    order = sorted(res.values(), key=lambda r: r["t_admit"])
    for k in range(2, 5):
        earlier_done = sorted(r["t_done"] for r in order[:k])
        assert order[k]["t_admit"] >= earlier_done[k - 2] - 1e-3
    # FIFO: admitted in submission order
    assert [r["ticket"] for r in order] == sorted(r["ticket"] for r in order)


@pytest.mark.parametrize("cycle", [1, 2, 3, 4, 5, 7, 50])
@pytest.mark.parametrize("triples", ["0", "1"])
def test_fp64_served_cycles_match_oracle(cycle, triples, monkeypatch):
    """FP64 precision: every result equals the oracle's plain solve with a
    check every cycle sweeps (cycle lengths with an odd and an even number of
    passes, so the iterate ends cycles in either array), alone and in a mix."""
    monkeypatch.setenv("J3D_SERVE_TRIPLES", triples)
    reqs = [(10, 1e-8, 300, 71, True), (13, 1e-6, 300, 72, False), (7, 1e-3, 300, 73, False),
            (17, 1e-12, 120, 74, True)]
    say("serve fp64", cycle, triples)
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=8, cycle_sweeps=cycle, precision=j3d.SERVE_FP64) as s:
        got, got_u = run(s, reqs)
    for k, (n, rtol, cap, seed, _) in enumerate(reqs):
        f = rhs(n, seed)
        cap_c = -(-cap // cycle) * cycle  # whole cycles
        uo, ro = oracle.solve_plain(np.zeros((n + 2,) * 3), f, 1.0 / (n + 1), rtol=rtol, check_every=cycle,
                                    max_sweeps=cap_c)
        assert got[k]["converged"] == ro.converged and got[k]["sweeps"] == ro.sweeps, (k, got[k], ro.sweeps)
        assert rel(got[k]["resid"], ro.resid) <= RESID_RTOL
        assert rel(got[k]["norm_f"], ro.norm_f) <= RESID_RTOL
        assert np.array_equal(got_u[k], uo)
    # the first request alone gives the same bits
    with j3d.Server(hbm_budget_bytes=1 << 30, max_slots=1, cycle_sweeps=cycle, precision=j3d.SERVE_FP64) as s:
        solo, solo_u = run(s, [reqs[0]])
    assert np.array_equal(solo_u[0], got_u[0])
    assert (solo[0]["sweeps"], solo[0]["resid"]) == (got[0]["sweeps"], got[0]["resid"])


def test_fp64_serving_budget_uses_fp64_state():
    per = j3d.j3d_request_state_bytes(j3d.SERVE_FP64, 20, 20, 20)
    assert per < j3d.j3d_request_bytes(20, 20, 20)
    with j3d.Server(hbm_budget_bytes=per + 10, max_slots=4, cycle_sweeps=10, precision=j3d.SERVE_FP64) as s:
        res, _ = run(s, [(20, 1e-12, 20, 80 + k, False) for k in range(3)])
    order = sorted(res.values(), key=lambda r: r["t_admit"])
    # one at a time
    for k in range(1, 3):
        assert order[k]["t_admit"] >= order[k - 1]["t_done"] - 1e-3
