"""Benchmark of the 3D 7-point Jacobi hot path on one MI355X.

Default workload: 512^3 interior + halo, FP64, two ping-pong arrays plus f,
u0 ~ U[0,1) (seed 2), f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z), h = 1/513;
one step = 500 sweeps with the L2 residual fused into every 10th sweep
(r_0, r_10, ..., r_490 fused, r_500 by a standalone pass).  The sweeps run
as 166 three-sweep passes and a final two-sweep pass (jacobi3d_sweep3: the
intermediate iterates stay on chip); the pass through which iterate 10g
passes fuses its residual at the stage that forms it (the pass's input, or
the iterate after its first or second sweep).  --passes 2 runs 250
two-sweep passes instead, --passes 1 500 single sweeps.  Throughput is grid-point updates per second (GLUP/s) over the timed
steps.

The JSON line also carries
  roofline:     the dominant kernel (the multi-sweep pass without a fused
                residual: 116 of the 167 passes of a step), its average
                duration from HIP events on the stream it
                runs on, and its algorithmic bandwidth against the MI355X HBM
                peak.  Algorithmic bytes per launch: 24 per interior point
                (read u, read f, write the result) for every pass; a
                three-sweep pass does three updates per point for them (8
                bytes per update), a two-sweep pass two (12), a single sweep
                one (24);
  cpu_baseline: the CPU oracle timed on a bounded sample of the same
                workload (a few of the 500 sweeps, on all host threads).

Other workloads (their own JSON line; not the default):
  --workload mixed   FP32-sweep / FP64-defect-correction solve against the
                     plain FP64 solve of the same manufactured problem, both
                     to a relative residual of 1e-8 (time to solution);
  --workload batch   256 independent grids, each axis uniform in {32..256},
                     200 sweeps with residuals every 10, one graph launch;
                     the line names the pass kind and tile shape the call ran
                     and, for three-sweep passes, carries that kernel's
                     roofline (graphs of ten passes without residuals);
  --workload serve   a Poisson request stream (200/s, n log-uniform in
                     [32, 384], tolerance 1e-6 or 1e-8, 5000-sweep cap) through
                     the continuous-batching server: solves/s, p50/p99 latency;
  --workload reduce  the sum and dot_product intrinsics at the paper's sizes
                     (32768 x 32768 and 2^27 FP64 elements): GB/s streamed;
  --workload small   64^3, 100 sweeps, residual after every sweep, one solve
                     call (launch-latency bound): microseconds per sweep;
  --workload jacobi2d  the paper's own jacobi benchmark: Laplace on 1024^2,
                     100000 iterations (the paper's CPU times quoted as context).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--workload plain|mixed|batch|serve|reduce|small|jacobi2d]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLUP/s + % HBM roofline; served solves/s and p50/p99 latency at 1e-8 resid"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP_F64 = 24.0


# device sources of the FP64 pass of each length
KERNEL_SOURCES = {1: ("sweep.h", "kernels_f64.hip", "j3d_internal.h"),
                  2: ("sweep.h", "sweep2.h", "kernels_sweep2.hip", "j3d_internal.h"),
                  3: ("sweep.h", "sweep3.h", "kernels_sweep3.hip", "j3d_internal.h")}


def kernel_source_hash(passes: int = 3) -> str:
    """Hash of the device sources of the pass of that length; counter
    summaries name the hash they were taken on."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[passes]:
        with open(os.path.join(ROOT, "paper_2409_18824_amd", "csrc", name), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def pass_plan(S: int, E: int, P: int):
    """The passes of one step, in sweep order: (first sweep, sweeps in the
    pass, residual stage).  Passes of P sweeps run straight through the S
    sweeps; a pass through which iterate gE passes (g = 0, 1, ...) carries
    its residual at the stage where that iterate is formed: 0 for the pass's
    input, 1 or 2 for the iterate after its first or second sweep (three-sweep
    passes only).  A shorter pass ends at the second residual point it would
    hold, and a two-sweep pass whose second iterate is a residual point stops
    before it; the last residual (iterate S, when E divides S) is left to a
    standalone pass."""
    plan = []
    s = 0
    while s < S:
        m = min(P, S - s)
        offs = [q * E - s for q in range(s // E, (s + m) // E + 1) if 0 <= q * E - s < m]
        if len(offs) > 1:
            m = offs[1]
            offs = offs[:1]
        if offs and offs[0] > 0 and m < 3:
            m = offs[0]
            offs = []
        plan.append((s, m, offs[0] if offs else None))
        s += m
    return plan


def measured_traffic(kernel_hash: str, passes: int, tile):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source with this tile
    shape."""
    path = os.path.join(ROOT, "profiles", "sweep%s_fp64_512_counters.json" % {1: "", 2: "2", 3: "3"}[passes])
    try:
        with open(path) as fp:
            d = json.load(fp)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sources_sha256_16") != kernel_hash:
        return None
    if d.get("tile") != list(tile):
        return None
    return d.get("bytes_per_launch")


def host_cpu():
    """CPU model and the number of host threads this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count()
    return model, nproc


def cpu_baseline(n: int, h: float, budget_s: float = 10.0):
    """Time the oracle on a bounded sample: sweeps of the same 512^3 grid with
    the same residual cadence (a residual pass before sweep 0 and every 10th),
    in groups of 10 sweeps; value is the rate over the whole sample, median
    the median rate of its groups."""
    import numpy as np

    import oracle
    import synth

    u0, f = synth.uniform_field(n, n, n, 2, synth.STREAM_U0, 0.0, 1.0), synth.manufactured_f(n, n, n, h)
    a, b = u0, u0.copy()
    t0 = time.perf_counter()
    sweeps = 0
    groups = []
    tg = t0
    while True:
        if sweeps % 10 == 0:
            oracle.residual_l2(a, f, h)
        oracle.sweep(a, f, h, out=b)
        a, b = b, a
        sweeps += 1
        now = time.perf_counter()
        if sweeps % 10 == 0:
            groups.append(10 * n ** 3 / (now - tg) / 1e9)
            tg = now
        el = now - t0
        if el >= budget_s or sweeps >= 500:
            break
    glups = sweeps * n ** 3 / el / 1e9
    del u0, f, a, b
    model, nproc = host_cpu()
    return {"value": glups, "unit": "GLUP/s", "cores": oracle.threads(), "kind": "oracle",
            "median": float(np.median(groups)) if groups else glups, "cpu_model": model, "host_threads": nproc,
            "sample": "%d of the 500 FP64 sweeps of the %d^3 grid (%d residual passes), %.1f s; median over "
                      "groups of 10 sweeps" % (sweeps, n, (sweeps + 9) // 10, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=500)
    ap.add_argument("--resid-every", type=int, default=10)
    ap.add_argument("--passes", type=int, default=3, choices=[1, 2, 3],
                    help="sweeps per pass over memory (2, 3: temporally blocked passes, run straight through "
                         "the step; residuals fused at the stage that forms their iterate)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time the tile shapes first and use the fastest (default: the library's default "
                         "shape, the one the committed counter profiles were taken with)")
    ap.add_argument("--workload", default="plain", choices=["plain", "mixed", "batch", "serve", "reduce", "small", "jacobi2d",
                             "pw-advection", "tra-adv"])
    ap.add_argument("--requests", type=int, default=200, help="serve: number of requests")
    ap.add_argument("--active-points", type=float, default=2e8,
                    help="serve: admission target for active interior points (0: no limit)")
    ap.add_argument("--rtol", type=float, default=1e-8, help="mixed: target relative residual")
    ap.add_argument("--max-sweeps", type=int, default=0,
                    help="mixed: stop each solve after this many sweeps (0: run to the tolerance; for profiling)")
    ap.add_argument("--chunk-sweeps", type=int, default=100000,
                    help="mixed: sweeps per solve call between progress lines (whole 50-sweep cycles)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: request arrival rate per second")
    ap.add_argument("--sweeps2d", type=int, default=100000, help="jacobi2d: iterations")
    ap.add_argument("--tile", default=None,
                    help="pin the tile shape as rows,planes,variant,persistent,order[,cols] instead of autotuning")
    ap.add_argument("--probe", action="store_true",
                    help="advection workloads: also time the copy kernels on 2 x 1 GiB (achievable-bandwidth "
                         "ceiling; the default workload always does)")
    ap.add_argument("--no-probe", action="store_true",
                    help="default workload: skip the copy-ceiling probe")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2409_18824_amd import j3d

    torch.cuda.set_device(0)
    if args.workload != "plain":
        out = {"mixed": run_mixed, "batch": run_batch, "serve": run_serve, "reduce": run_reduce,
               "small": run_small, "jacobi2d": run_jacobi2d, "pw-advection": run_pw_advection,
               "tra-adv": run_tra_adv}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    n, S, E = args.n, args.sweeps, args.resid_every
    h = 1.0 / (n + 1)
    print("[bench] allocating %d^3 FP64 (u_a, u_b, f)" % n, file=sys.stderr, flush=True)
    ua = j3d.FArray.empty(n, n, n)
    ub = j3d.FArray.empty(n, n, n)
    j3d.j3d_fill_uniform(ua, 2, synth.STREAM_U0, 0.0, 1.0)
    j3d.j3d_fill_const(ub, 0.0)
    df = j3d.FArray.from_numpy(synth.manufactured_f(n, n, n, h))
    torch.cuda.synchronize()
    P = args.passes
    kind = {1: j3d.F64, 2: j3d.KIND_F64X2, 3: j3d.KIND_F64X3}[P]
    plan = pass_plan(S, E, P)
    lengths = sorted({m for _, m, _ in plan})
    if args.tile:
        j3d.j3d_tune_set_single(kind, n, n, n, tuple(int(x) for x in args.tile.split(",")))
    elif args.autotune:
        j3d.j3d_autotune_single(kind, n, n, n)
        for m in lengths:  # the other pass lengths of the plan, and the standalone residual pass
            if m != P:
                j3d.j3d_autotune_single({1: j3d.F64, 2: j3d.KIND_F64X2}[m], n, n, n)
        if 1 not in lengths:
            j3d.j3d_autotune_single(j3d.F64, n, n, n)
    tune = j3d.j3d_tune_query_single(kind, n, n, n)  # the shape the timed passes use
    print("[bench] tile shape (rows, planes, variant, persistent, order, cols) = %s" % (tune,), file=sys.stderr, flush=True)

    nres = S // E + 1
    resid = torch.zeros(nres, dtype=torch.float64, device="cuda")
    sweeps_of = {1: j3d.jacobi3d_sweep, 2: j3d.jacobi3d_sweep2, 3: j3d.jacobi3d_sweep3}
    n_plain = sum(1 for _, m, st in plan if st is None and m == P)
    events = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(n_plain)] for _ in range(args.steps)]

    state = {"cur": ua, "nxt": ub}

    def step(ev):
        cur, nxt = state["cur"], state["nxt"]
        timed = ev is not None
        q = 0
        for s, m, stage in plan:
            sweep = sweeps_of[m]
            if stage is not None:
                g = (s + stage) // E
                if stage == 0:
                    sweep(cur, nxt, df, h, resid_out=resid[g:g + 1])
                else:
                    sweep(cur, nxt, df, h, resid_out=resid[g:g + 1], resid_after=stage)
            elif timed and m == P:
                ev[q][0].record()
                sweep(cur, nxt, df, h)
                ev[q][1].record()
                q += 1
            else:
                sweep(cur, nxt, df, h)
            cur, nxt = nxt, cur
        if S % E == 0:
            j3d.residual_l2(cur, df, h, out=resid[S // E:S // E + 1])
        state["cur"], state["nxt"] = cur, nxt

    for w in range(args.warmup):
        step(None)
        torch.cuda.synchronize()
        print("[bench] warmup %d done" % w, file=sys.stderr, flush=True)

    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(args.steps):
        step(events[k])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for ev in events:
        kernel_ms.extend(a.elapsed_time(b) for a, b in ev)
    print("[bench] %d timed steps done" % args.steps, file=sys.stderr, flush=True)
    gpu_s = e0.elapsed_time(e1) / 1e3
    elapsed = max(wall, gpu_s)
    lups = float(n) ** 3 * S * args.steps
    glups = lups / elapsed / 1e9
    r = resid.cpu().numpy()
    assert np.all(np.isfinite(r)) and r[-1] < r[0], "residual did not decrease"

    avg_ms = float(np.mean(kernel_ms))
    med_ms = float(np.median(kernel_ms))
    bytes_launch = BYTES_PER_LUP_F64 * n ** 3  # read u, read f, write the result
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    khash = kernel_source_hash(P)
    kname = {1: "k_pass_one<double, F_WRITE> (FP64 sweep)",
             2: "k_sweep2_one<F_WRITE> (two FP64 sweeps per pass)",
             3: "k_sweep3_one<F_WRITE> (three FP64 sweeps per pass)"}[P]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(khash, P, tune),
            "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 2), "median_launch_us": round(med_ms * 1e3, 2),
            "launches": len(kernel_ms), "bytes_per_launch_algorithmic": int(bytes_launch),
            "updates_per_point_per_launch": P}

    if not args.no_probe:
        # the achievable streaming rate of this machine: the best of the library's
        # copy kernels over 1 GiB (read + write bytes per second)
        nprobe = 1 << 27  # 1 GiB of doubles per buffer
        src = torch.ones(nprobe, dtype=torch.float64, device="cuda")
        dst = torch.zeros(nprobe, dtype=torch.float64, device="cuda")
        copy_gbps = j3d.j3d_bandwidth_probe(src, dst, reps=5)
        roof["copy_ceiling_gbps"] = round(copy_gbps, 1)
        roof["frac_of_copy_ceiling"] = round(achieved / copy_gbps, 4)
        # the pass's own mix (two streams read, one written: dst = a + b)
        src2 = torch.ones(nprobe, dtype=torch.float64, device="cuda")
        triad_gbps = j3d.j3d_bandwidth_probe_triad(src, src2, dst, reps=5)
        roof["triad_ceiling_gbps"] = round(triad_gbps, 1)
        roof["frac_of_triad_ceiling"] = round(achieved / triad_gbps, 4)
        del src, src2, dst

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(n, h)

    out = {
        "metric": METRIC, "value": round(glups, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "jacobi3d-7pt-fp64-%dcubed-%dsweeps-resid%d" % (n, S, E),
                   "grid": [n, n, n], "halo": 1, "layout": "fortran-column-major",
                   "sweeps_per_step": S, "resid_every": E, "sweeps_per_pass": P,
                   "passes_by_length": {str(m): sum(1 for _, x, _ in plan if x == m) for m in lengths},
                   "residuals_fused_at_stage": [sum(1 for _, _, st in plan if st == k) for k in range(3)],
                   "tile": tune,
                   "single_sweep_equivalent_gbs": round(glups * BYTES_PER_LUP_F64, 1)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _base(args, metric, value, unit, ms, dtype, workload, higher=True, extra=None):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
         "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": {"workload": workload}}
    if extra:
        d["config"].update(extra)
    return d


def run_mixed(args):
    """Time to a 1e-8 relative residual: plain FP64 Jacobi vs FP32 sweeps with
    FP64 defect correction every 50 sweeps, same problem, same GPU."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2409_18824_amd import j3d

    n = args.n
    h = 1.0 / (n + 1)
    f = synth.manufactured_f(n, n, n, h)
    df = j3d.FArray.from_numpy(f)
    u = j3d.FArray.empty(n, n, n)
    if args.autotune:
        for kind in (j3d.F64, j3d.F32, j3d.KIND_F64X2, j3d.KIND_F32X2, j3d.KIND_F64X3, j3d.KIND_F32X3):
            j3d.j3d_autotune_single(kind, n, n, n)
    res = {}
    chunk = max(50, args.chunk_sweeps // 50 * 50)
    for mode, name in ((j3d.MODE_MIXED, "mixed"), (j3d.MODE_FP64, "fp64")):
        j3d.j3d_fill_uniform(u, 2, synth.STREAM_U0, 0.0, 1.0)
        torch.cuda.synchronize()
        print("[bench] %s solve to %g on %d^3" % (name, args.rtol, n), file=sys.stderr, flush=True)
        # The solve runs in chunks of whole 50-sweep cycles, each resuming from
        # the iterate the previous one returned (the same sequence of
        # operations as one call), so progress can be reported between chunks.
        t0 = time.perf_counter()
        sweeps = 0
        cap = args.max_sweeps if args.max_sweeps > 0 else 10 ** 8
        while True:
            r = j3d.poisson_solve(u, df, h, mode=mode, rtol=args.rtol, max_sweeps=min(chunk, cap - sweeps),
                                  check_every=50, inner_sweeps=50, history_cap=0)
            sweeps += r.sweeps
            if r.converged or r.sweeps < chunk or sweeps >= cap:
                break
            print("[bench] %s: %d sweeps, relative residual %.3e, %.1f s" % (
                name, sweeps, r.resid / r.norm_f, time.perf_counter() - t0), file=sys.stderr, flush=True)
        el = time.perf_counter() - t0
        # the oracle's one-pass FP64 residual of the returned solution
        uo = u.to_numpy()
        rr = oracle.residual_l2(uo, f, h)
        res[name] = {"seconds": round(el, 3), "sweeps": sweeps, "converged": r.converged,
                     "rel_resid_gpu": r.resid / r.norm_f, "rel_resid_oracle": rr / oracle.norm2(f),
                     "glups": round(float(n) ** 3 * sweeps / el / 1e9, 2)}
        print("[bench] %s: %s" % (name, res[name]), file=sys.stderr, flush=True)
        del uo
    speedup = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    return _base(args, "time to 1e-8 relative residual (mixed vs FP64)", round(speedup, 3), "x speedup",
                 res["mixed"]["seconds"] * 1e3, "f32+f64", "poisson-manufactured-%dcubed-mixed-vs-fp64" % n,
                 extra={"grid": [n, n, n], "rtol": args.rtol, "inner_sweeps": 50, "check_every": 50,
                        "results": res})


def run_batch(args):
    """256 uneven grids, 200 sweeps each with residuals every 10, one graph."""
    import numpy as np
    import torch

    import synth
    from paper_2409_18824_amd import j3d

    shapes = synth.batch_shapes(256, 4)
    grids = []
    for g in shapes:
        ua = j3d.FArray.empty(g.nx, g.ny, g.nz)
        ub = j3d.FArray.empty(g.nx, g.ny, g.nz)
        f = j3d.FArray.empty(g.nx, g.ny, g.nz)
        j3d.j3d_fill_uniform(f, g.seed, synth.STREAM_F, -1.0, 1.0)
        grids.append((ua, ub, f, g.h))
    torch.cuda.synchronize()
    pts = sum(g.nx * g.ny * g.nz for g in shapes)
    nsw, every = 200, 10
    out = torch.zeros((len(grids), nsw // every + 1), dtype=torch.float64, device="cuda")
    print("[bench] batch of %d grids, %.3g points; autotuning" % (len(grids), pts), file=sys.stderr, flush=True)
    tune = j3d.j3d_autotune(grids)
    for _ in range(args.warmup):
        j3d.jacobi3d_sweep_batch(grids, nsw, every, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        j3d.jacobi3d_sweep_batch(grids, nsw, every, out)
    e1.record()
    torch.cuda.synchronize()
    el = max(time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3)
    glups = pts * nsw * args.steps / el / 1e9
    r = out.cpu().numpy()
    assert np.all(np.isfinite(r)) and np.all(r[:, -1] < r[:, 0])
    # the pass kind and shape the timed calls ran; with three-sweep passes,
    # their kernel alone: a call of 30 sweeps without residuals is ten
    # three-sweep batched passes back to back in one graph (timed with events
    # on the stream the graph runs on; per pass: the call's time / 10)
    kind, shape = j3d.j3d_batch_last_plan()
    roof = None
    if kind == 3:
        j3d.jacobi3d_sweep_batch(grids, 30, every, None)
        torch.cuda.synchronize()
        assert j3d.j3d_batch_last_plan() == (kind, shape)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(6)]
        for a0, a1 in evs:
            a0.record()
            j3d.jacobi3d_sweep_batch(grids, 30, every, None)
            a1.record()
        torch.cuda.synchronize()
        us = sorted(a0.elapsed_time(a1) * 1e3 / 10 for a0, a1 in evs)
        avg = sum(us) / len(us)
        alg = BYTES_PER_LUP_F64 * pts
        gbs = alg / avg / 1e3
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_sweep3_batch<F_WRITE> (three FP64 sweeps per pass over all grids)",
                "avg_launch_us": round(avg, 1), "median_launch_us": round(us[len(us) // 2], 1),
                "launches": 10 * len(us), "bytes_per_launch_algorithmic": int(alg),
                "timing": "6 graphs of 10 passes; median over the graphs"}
    # one more call from u0 = 0, sampled against the oracle: the smallest and
    # the largest grid, the first and last of the tile list, four seeded others
    import oracle

    for ua, ub, _, _ in grids:
        j3d.j3d_fill_const(ua, 0.0)
        j3d.j3d_fill_const(ub, 0.0)
    j3d.jacobi3d_sweep_batch(grids, nsw, every, out)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    sizes = [g.nx * g.ny * g.nz for g in shapes]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes)), 0, len(shapes) - 1}
    rng = np.random.default_rng(7)
    while len(pick) < 8:
        pick.add(int(rng.integers(0, len(shapes))))
    err_u, err_r, t_or, lups_or = 0.0, 0.0, 0.0, 0.0
    for gi in sorted(pick):
        g = shapes[gi]
        f = synth.batch_rhs(g)
        t0 = time.perf_counter()
        uo, ro = oracle.solve_plain(np.zeros_like(f), f, g.h, rtol=0.0, check_every=every, max_sweeps=nsw)
        t_or += time.perf_counter() - t0
        lups_or += float(sizes[gi]) * nsw
        got = grids[gi][0].to_numpy()
        err_u = max(err_u, float(np.max(np.abs(got - uo))) / max(float(np.max(np.abs(uo))), 1e-300))
        err_r = max(err_r, float(np.max(np.abs(r[gi] - ro.history) / ro.history)))
    print("[bench] batch oracle check: %d grids, max rel diff u %.3g, residuals %.3g" % (len(pick), err_u, err_r),
          file=sys.stderr, flush=True)
    out_d = _base(args, "GLUP/s (batched uneven grids)", round(glups, 3), "GLUP/s", round(el / args.steps * 1e3, 3),
                  "f64", "batch-256-grids-32to256-200sweeps-resid10",
                  extra={"grids": len(grids), "points": pts, "tile": tune,
                         "sweeps_per_pass": kind, "pass_tile": list(shape),
                         "single_sweep_equivalent_gbs": round(glups * 24.0, 1)})
    if roof is not None:
        out_d["roofline"] = roof
    out_d["oracle_error"] = {"grids_checked": sorted(pick), "max_rel_diff_u": err_u, "max_rel_diff_resid": err_r,
                             "reference": "oracle.solve_plain of each sampled grid alone, 200 sweeps, residual every 10"}
    model, nproc = host_cpu()
    out_d["cpu_baseline"] = {"value": round(lups_or / t_or / 1e9, 3), "unit": "GLUP/s", "cores": oracle.threads(),
                             "kind": "oracle", "cpu_model": model, "host_threads": nproc,
                             "sample": "the %d sampled grids, 200 sweeps each with residuals every 10, %.1f s" % (
                                 len(pick), t_or)}
    return out_d


def run_small(args):
    """64^3 FP64, 100 sweeps with the residual after every sweep, as one
    poisson_solve call (the launch-latency-bound configuration)."""
    import numpy as np
    import torch

    import synth
    from paper_2409_18824_amd import j3d

    n = 64
    u0, f, h = synth.small_plain(n, seed=1)
    du, df = j3d.FArray.from_numpy(u0), j3d.FArray.from_numpy(f)
    hist = None
    for _ in range(max(1, args.warmup)):
        du.copy_from(u0)
        j3d.poisson_solve(du, df, h, rtol=0.0, max_sweeps=100, check_every=1)
    times = []
    for _ in range(args.steps):
        du.copy_from(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = j3d.poisson_solve(du, df, h, rtol=0.0, max_sweeps=100, check_every=1)
        times.append(time.perf_counter() - t0)
        hist = r.history
    med = float(np.median(times))
    assert len(hist) == 101 and hist[-1] < hist[0]
    return _base(args, "GLUP/s (64^3, 100 sweeps, residual after every sweep)", round(n ** 3 * 100 / med / 1e9, 3),
                 "GLUP/s", round(med * 1e3, 3), "f64", "small-64cubed-100sweeps-resid1",
                 extra={"us_per_sweep": round(med / 100 * 1e6, 2), "best_ms": round(min(times) * 1e3, 3)})


def run_jacobi2d(args):
    """The paper's jacobi benchmark: Laplace's equation on a 1024 x 1024 grid,
    100000 Jacobi iterations (zero interior, top edge 1, other edges 0)."""
    import numpy as np
    import torch

    from paper_2409_18824_amd import j3d

    n, S = 1024, args.sweeps2d
    u0 = np.zeros((n + 2, n + 2))
    u0[-1, :] = 1.0
    ua, ub = j3d.FArray.from_numpy2d(u0), j3d.FArray.from_numpy2d(u0)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    j3d.jacobi2d_sweeps(ua, ub, 1024, 1.0 / (n + 1))  # warm-up (captures the graph)
    times = []
    for _ in range(max(1, args.steps)):
        ua.copy_from(u0[None]), ub.copy_from(u0[None])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        j3d.jacobi2d_sweeps(ua, ub, S, 1.0 / (n + 1), resid_out=out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print("[bench] jacobi2d %d sweeps: %.3f s" % (S, times[-1]), file=sys.stderr, flush=True)
    med = float(np.median(times))
    return _base(args, "GLUP/s (2D Laplace jacobi, 1024^2, %d iterations)" % S, round(n * n * S / med / 1e9, 2),
                 "GLUP/s", round(med * 1e3, 2), "f64", "jacobi2d-1024sq-%dsweeps" % S,
                 extra={"seconds": round(med, 4), "resid_l2": out.item(),
                        "paper_cpu_seconds_context": {"this work's lowering, serial": 249.08, "Flang": 277.67}})


def run_reduce(args):
    """The paper's reduction intrinsics at its sizes: sum over a 32768 x 32768
    FP64 array and dot_product of two FP64 vectors of 2^27 (134 million)
    elements; bytes streamed per second against the HBM peak."""
    import torch

    from paper_2409_18824_amd import j3d

    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    out = {}
    for name, n in (("sum", 32768 * 32768), ("dot", 1 << 27)):
        x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
        y = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) if name == "dot" else None
        res = torch.zeros(1, dtype=torch.float64, device="cuda")
        call = (lambda: j3d.j3d_sum(x, out=res)) if name == "sum" else (lambda: j3d.j3d_dot(x, y, out=res))
        for _ in range(max(1, args.warmup)):
            call()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for a, b in ev:
            a.record()
            call()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        nbytes = 8 * n * (2 if name == "dot" else 1)
        med = ms[len(ms) // 2]
        out[name] = {"elements": n, "bytes": nbytes, "median_ms": round(med, 4), "best_ms": round(ms[0], 4),
                     "gbps": round(nbytes / (med * 1e-3) / 1e9, 1),
                     "frac_of_hbm_peak": round(nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        print("[bench] %s: %s" % (name, out[name]), file=sys.stderr, flush=True)
        del x, y
    tot_bytes = sum(v["bytes"] for v in out.values())
    tot_ms = sum(v["median_ms"] for v in out.values())
    return _base(args, "GB/s streamed by the sum / dot_product intrinsics", round(tot_bytes / (tot_ms * 1e-3) / 1e9, 1),
                 "GB/s", tot_ms, "f64", "reduce-sum32768sq-dot2p27", extra={"results": out})


ADVECT_SOURCES = ("advect.h", "advect.cpp", "kernels_advect.hip", "sweep.h")


def advect_source_hash() -> str:
    h = hashlib.sha256()
    for name in ADVECT_SOURCES:
        with open(os.path.join(ROOT, "paper_2409_18824_amd", "csrc", name), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def advect_tile() -> str:
    return "%s/%s/%s" % (os.environ.get("J3D_ADVECT_TILE", "default"), os.environ.get("J3D_TRACER2_TILE", "default"),
                         os.environ.get("J3D_TRACER_STEPS_PER_PASS", "default"))


def advect_traffic(name: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current advection kernel source with the same tile."""
    try:
        with open(os.path.join(ROOT, "profiles", "%s_counters.json" % name)) as fp:
            d = json.load(fp)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sources_sha256_16") != advect_source_hash() or d.get("tile") != advect_tile():
        return None
    return d.get("bytes_per_launch")


def _event_times(call, steps):
    import torch

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        call()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) * 1e-3 for a, b in ev]


def _advect_roofline(alg_bytes, launch_s, traffic, launches, args):
    gbs = alg_bytes / launch_s / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_us": round(launch_s * 1e6, 1), "launches": launches}
    if args.probe:
        import torch

        from paper_2409_18824_amd import j3d

        nprobe = 1 << 27  # 1 GiB of doubles per buffer
        src = torch.ones(nprobe, dtype=torch.float64, device="cuda")
        dst = torch.zeros(nprobe, dtype=torch.float64, device="cuda")
        roof["copy_ceiling_gbps"] = round(j3d.j3d_bandwidth_probe(src, dst, reps=5), 1)
        roof["frac_of_copy_ceiling"] = round(gbs / roof["copy_ceiling_gbps"], 4)
        del src, dst
    return roof


def run_pw_advection(args):
    """Momentum advection standing in for the paper's pw-advection: three
    velocity fields in, three tendencies out, on 2048 x 1024 x 1024 FP64."""
    import numpy as np

    import synth
    from paper_2409_18824_amd import j3d

    nx, ny, nz = synth.PW_SHAPE
    recipe, d = synth.pw_recipe()
    print("[bench] allocating 6 x %dx%dx%d FP64" % (nx, ny, nz), file=sys.stderr, flush=True)
    ins = []
    for fr in recipe:
        a = j3d.FArray.empty(nx, ny, nz)
        j3d.j3d_fill_uniform(a, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo)
        ins.append(a)
    outs = [j3d.FArray.empty(nx, ny, nz) for _ in range(3)]
    call = lambda: j3d.pw_advection(*ins, *outs, *d)
    for _ in range(max(1, args.warmup)):
        call()
    times = _event_times(call, args.steps)
    med = float(np.median(times))
    pts = nx * ny * nz
    alg = 48 * pts  # read u, v, w and write su, sv, sw once per point
    out = _base(args, "grid points per second (momentum advection, 3 fields in / 3 out, %dx%dx%d)" % (nx, ny, nz),
                round(pts / med / 1e9, 2), "Gpoints/s", round(med * 1e3, 3), "f64",
                "pw-advection-%dx%dx%d" % (nx, ny, nz),
                extra={"tile": advect_tile(), "algorithmic_bytes_per_launch": alg, "launches_per_step": 1})
    del ins, outs
    out["roofline"] = _advect_roofline(alg, med, advect_traffic("pw_advection"), len(times), args)
    if not args.no_cpu_baseline:
        import oracle

        kz = 6
        fields = [synth.uniform_field(nx, ny, kz, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo) for fr in recipe]
        t0, calls = time.perf_counter(), 0
        while True:
            oracle.pw_advection(*fields, *d)
            calls += 1
            el = time.perf_counter() - t0
            if el >= 10.0 or calls >= 200:
                break
        out["cpu_baseline"] = {"value": round(calls * nx * ny * kz / el / 1e9, 4), "unit": "Gpoints/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": "%d calls on the first %d z-planes (%dx%dx%d), %.1f s" % (
                                   calls, kz, nx, ny, kz, el)}
    return out


def run_tra_adv(args):
    """Tracer advection standing in for the paper's tra-adv: six fields on
    1024 x 512 x 512 FP64, 20 donor-cell steps per call."""
    import numpy as np

    import synth
    from paper_2409_18824_amd import j3d

    nx, ny, nz = synth.TRA_SHAPE
    S = synth.TRA_ITERS
    rt, rvel, rr = synth.tracer_recipe()
    recipe = [rt, rt] + rvel + [rr]
    arrs = []
    for fr in recipe:
        a = j3d.FArray.empty(nx, ny, nz)
        j3d.j3d_fill_uniform(a, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo)
        arrs.append(a)
    call = lambda: j3d.tracer_advection(*arrs, S)
    for _ in range(max(1, args.warmup)):
        call()
    times = _event_times(call, args.steps)
    med = float(np.median(times))
    pts = nx * ny * nz
    # the library's schedule: two steps per launch (one pass over memory),
    # unless J3D_TRACER_STEPS_PER_PASS=1; S = 20 needs no single-step launch
    per_launch = 1 if os.environ.get("J3D_TRACER_STEPS_PER_PASS") == "1" else 2
    launches = S // per_launch
    alg = 48 * pts  # per launch: read t, u, v, w, r and write t once per point
    out = _base(args, "point updates per second (tracer advection, 6 fields, %dx%dx%d, %d steps)" % (nx, ny, nz, S),
                round(pts * S / med / 1e9, 2), "GLUP/s", round(med * 1e3, 3), "f64",
                "tra-adv-%dx%dx%d-%dsteps" % (nx, ny, nz, S),
                extra={"tile": advect_tile(), "steps_per_launch": per_launch, "algorithmic_bytes_per_launch": alg,
                       "launches_per_step": launches,
                       "single_step_equivalent_gbs": round(48 * pts * S / med / 1e9, 1)})
    del arrs
    out["roofline"] = _advect_roofline(alg, med / launches, advect_traffic("tracer_advection"),
                                       len(times) * launches, args)
    if not args.no_cpu_baseline:
        import oracle

        kz = 8
        fields = [synth.uniform_field(nx, ny, kz, fr.seed, fr.stream, fr.lo, fr.hi, fr.halo)
                  for fr in [rt] + rvel + [rr]]
        t0, calls = time.perf_counter(), 0
        while True:
            oracle.tracer_advection(*fields, S)
            calls += 1
            el = time.perf_counter() - t0
            if el >= 10.0 or calls >= 100:
                break
        out["cpu_baseline"] = {"value": round(calls * nx * ny * kz * S / el / 1e9, 4), "unit": "GLUP/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": "%d calls of %d steps on the first %d z-planes (%dx%dx%d), %.1f s" % (
                                   calls, S, kz, nx, ny, kz, el)}
    return out


def _serve_stream(reqs, precision, args, sample):
    """Push the request stream through a server of the given precision, at
    the stream's arrival times.  Returns the results (by request id), the
    host copies of the sampled requests' solutions and the run's span."""
    import numpy as np

    from paper_2409_18824_amd import j3d

    budget = 200 * 10 ** 9
    results, outs, tick = {}, {}, {}
    with j3d.Server(hbm_budget_bytes=budget, max_slots=2048, cycle_sweeps=50,
                    max_active_points=int(args.active_points), precision=precision) as s:
        t_start = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t_start
            if r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            u = None
            if r.rid in sample:
                u = outs[r.rid] = np.zeros((r.n + 2,) * 3)
            tick[s.submit(r.n, r.h, r.rtol, r.max_sweeps, seed=r.seed, u_out=u)] = r
            for x in s.poll():
                results[tick[x["ticket"]].rid] = x
        last = time.perf_counter()
        while len(results) < len(reqs):
            for x in s.poll():
                results[tick[x["ticket"]].rid] = x
            if time.perf_counter() - last > 5:
                st = s.stats()
                print("[bench] serve: %d done, %d active, %d queued" % (len(results), st["active"], st["queued"]),
                      file=sys.stderr, flush=True)
                last = time.perf_counter()
            time.sleep(0.01)
        s.drain(600)
    return results, outs


def _serve_stats(reqs, results):
    import numpy as np

    by = {r.rid: r for r in reqs}
    ids = sorted(results)
    lat = np.array([results[i]["t_done"] - results[i]["t_submit"] for i in ids])
    t0 = min(results[i]["t_submit"] for i in ids)
    t1 = max(results[i]["t_done"] for i in ids)
    conv = np.array([results[i]["converged"] for i in ids])
    tol8 = np.array([by[i].rtol == 1e-8 for i in ids])
    relres = np.array([results[i]["resid"] / results[i]["norm_f"] for i in ids])
    sweeps = np.array([results[i]["sweeps"] for i in ids], dtype=np.float64)
    ns = np.array([by[i].n for i in ids], dtype=np.float64)

    def pct(mask):
        if not mask.any():
            return None
        return {"count": int(mask.sum()), "p50_s": round(float(np.percentile(lat[mask], 50)), 3),
                "p99_s": round(float(np.percentile(lat[mask], 99)), 3),
                "rel_resid_median": float(np.median(relres[mask])), "rel_resid_max": float(np.max(relres[mask]))}

    return {
        "solves_per_s": round(len(ids) / (t1 - t0), 3), "span_s": round(t1 - t0, 3),
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "tol1e-8": {"all": pct(tol8), "converged": pct(tol8 & conv), "capped": pct(tol8 & ~conv)},
        "tol1e-6": {"all": pct(~tol8), "converged": pct(~tol8 & conv), "capped": pct(~tol8 & ~conv)},
        "converged_fraction": round(float(conv.mean()), 3),
        "lups": float(np.sum(ns ** 3 * sweeps)), "sweeps": sweeps, "ns": ns, "checks": np.ceil(sweeps / 50.0) + 1,
    }


def run_serve(args):
    """The served request stream (Poisson arrivals, cubic n log-uniform in
    [32, 384], tolerance 1e-6 or 1e-8, cap 5000 sweeps) through the
    continuous-batching server, once in mixed precision (the served form)
    and once in plain FP64 (the form it is measured against), same stream,
    same GPU.  Every 10th request with n <= 128 is also solved by the oracle
    alone and its result compared with the served one."""
    import numpy as np

    import oracle
    import synth
    from paper_2409_18824_amd import j3d

    reqs = synth.serve_requests(args.requests, rate=args.rate, seed=5)
    sample = {r.rid for r in reqs if r.rid % 10 == 0 and r.n <= 128}
    for prec in (j3d.SERVE_MIXED, j3d.SERVE_FP64):  # warm the kernels with one small solve
        with j3d.Server(hbm_budget_bytes=8 << 30, max_slots=4, cycle_sweeps=50, precision=prec) as s:
            s.submit(32, 1 / 33, 1e-6, 100, seed=1)
            s.drain(60)
            s.poll()
    runs = {}
    for prec, name in ((j3d.SERVE_MIXED, "mixed"), (j3d.SERVE_FP64, "fp64")):
        print("[bench] serving %d requests at %g/s, %s" % (len(reqs), args.rate, name), file=sys.stderr, flush=True)
        results, outs = _serve_stream(reqs, prec, args, sample)
        st = _serve_stats(reqs, results)
        # the oracle alone on the sampled requests
        t_or, lups_or, err_u, err_r = 0.0, 0.0, 0.0, 0.0
        for r in reqs:
            if r.rid not in sample:
                continue
            f = synth.uniform_field(r.n, r.n, r.n, r.seed, synth.STREAM_F, -1.0, 1.0)
            t0 = time.perf_counter()
            if prec == j3d.SERVE_MIXED:
                uo, ro = oracle.solve_mixed(np.zeros_like(f), f, r.h, rtol=r.rtol, inner=50, max_sweeps=r.max_sweeps)
            else:
                uo, ro = oracle.solve_plain(np.zeros_like(f), f, r.h, rtol=r.rtol, check_every=50,
                                            max_sweeps=r.max_sweeps)
            t_or += time.perf_counter() - t0
            lups_or += float(r.n) ** 3 * ro.sweeps
            g = results[r.rid]
            assert g["sweeps"] == ro.sweeps and g["converged"] == ro.converged, (r, g, ro.sweeps)
            err_u = max(err_u, float(np.max(np.abs(outs[r.rid] - uo))) / max(float(np.max(np.abs(uo))), 1e-300))
            err_r = max(err_r, abs(g["resid"] - ro.resid) / ro.resid)
        st["oracle_error"] = {"requests_checked": len(sample), "max_rel_diff_u": err_u,
                              "max_rel_diff_resid": err_r,
                              "reference": "oracle.solve_%s of each sampled request alone" % (
                                  "mixed" if prec == j3d.SERVE_MIXED else "plain")}
        st["oracle_glups"] = round(lups_or / t_or / 1e9, 3) if t_or > 0 else None
        st["oracle_seconds"] = round(t_or, 2)
        print("[bench] %s: %.3f solves/s, p50 %.3f s, p99 %.3f s, oracle error %s" % (
            name, st["solves_per_s"], st["latency_s"]["p50"], st["latency_s"]["p99"], st["oracle_error"]),
            file=sys.stderr, flush=True)
        runs[name] = st
    mx, fp = runs["mixed"], runs["fp64"]
    # algorithmic bytes of the mixed run, per pass as the loaded server runs
    # its 50-sweep cycles: the defect step 20 per point (read u, f; write
    # r32), a two-sweep pass from zero 8 (read r32, write e), fifteen
    # three-sweep passes 12 each (read e, r32; write e) and the last pass 24
    # (read e, r32; read and write u): 232 bytes per point per cycle, plus a
    # final defect step per request
    cycles = mx["sweeps"] / 50.0
    bytes_mx = float(np.sum(mx["ns"] ** 3 * (232.0 * cycles + 20.0)))
    gbs = bytes_mx / mx["span_s"] / 1e9
    for st in runs.values():
        st["glups_served"] = round(st["lups"] / st["span_s"] / 1e9, 2)
        for k in ("lups", "sweeps", "ns", "checks"):
            st.pop(k)
    out = _base(args, "served solves/s (mixed precision, continuous batching)", mx["solves_per_s"],
                "solves/s", round(mx["span_s"] * 1e3, 1), "f32+f64",
                "serve-poisson-%grps-n32to384-tol1e-6or1e-8-cap5000" % args.rate,
                extra={"requests": len(reqs), "offered_rate_per_s": args.rate, "hbm_budget_bytes": 200 * 10 ** 9,
                       "max_active_points": int(args.active_points), "cycle_sweeps": 50})
    out["latency_s"] = mx["latency_s"]
    out["mixed"] = mx
    out["fp64"] = fp
    out["speedup_mixed_vs_fp64_solves_per_s"] = round(mx["solves_per_s"] / fp["solves_per_s"], 3)
    out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "basis": "algorithmic bytes of the mixed run's passes (232 per point per 50-sweep cycle "
                                "with three-sweep FP32 passes) over its span"}
    model, nproc = host_cpu()
    out["cpu_baseline"] = {"value": mx["oracle_glups"], "unit": "GLUP/s", "cores": oracle.threads(),
                           "kind": "oracle", "cpu_model": model, "host_threads": nproc,
                           "sample": "the %d sampled requests (every 10th with n <= 128) solved one by one by "
                                     "oracle.solve_mixed, %.1f s" % (len(sample), mx["oracle_seconds"])}
    return out


if __name__ == "__main__":
    main()
