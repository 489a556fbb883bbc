"""bench.py command-line contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_graft_entry_has_build_and_smoke():
    sys.path.insert(0, ROOT)
    import __graft_entry__ as ge

    assert callable(ge.build) and callable(ge.smoke)


def test_pass_plan_covers_every_sweep_and_residual_once():
    """The benchmark's pass schedule: every sweep in exactly one pass, every
    residual point gE < S fused exactly once at a stage its pass has, and the
    default workload's shape (166 three-sweep passes and one two-sweep pass,
    residuals fused at stages 0, 1, 2 in turn)."""
    sys.path.insert(0, ROOT)
    import bench

    for S in range(0, 40):
        for E in range(1, 13):
            for P in (1, 2, 3):
                plan = bench.pass_plan(S, E, P)
                assert [s for s, _, _ in plan] == [sum(m for _, m, _ in plan[:i]) for i in range(len(plan))]
                assert sum(m for _, m, _ in plan) == S
                assert all(1 <= m <= P for _, m, _ in plan)
                assert all(st is None or st == 0 or (m == 3 and st in (1, 2)) for _, m, st in plan)
                assert [s + st for s, _, st in plan if st is not None] == list(range(0, S, E))
    plan = bench.pass_plan(500, 10, 3)
    assert sum(1 for _, m, _ in plan if m == 3) == 166 and [m for _, m, _ in plan][-1] == 2
    assert [sum(1 for _, _, st in plan if st == k) for k in range(3)] == [17, 17, 16]
    assert bench.pass_plan(500, 10, 2) == [(s, 2, 0 if s % 10 == 0 else None) for s in range(0, 500, 2)]
