"""C-ABI checks that need no GPU: symbols, descriptors, validation codes.

Every call here fails validation (or is host-only) before the library
touches a device, so it runs on a machine without a GPU.
"""
import ctypes
import json
import os
import re

import pytest

from paper_2409_18824_amd import j3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "j3d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("jacobi3d_sweep", "residual_l2", "poisson_solve", "jacobi3d_sweep_batch",
                 "poisson_serve_create", "poisson_serve_submit", "poisson_serve_poll",
                 "poisson_serve_drain", "poisson_serve_destroy"):
        assert must in names


# Intent of every pointer argument of the boundary (stream and server
# handles aside): "in" if the call only reads what it points to, "out" if it
# writes it, "inout" if it reads and then writes it.  An array descriptor
# counts by the array it describes (the paper types Fortran dummies by their
# intent, Sec. "Handling of control structures").
INTENT = {
    "j3d_element_offset": {"a": "in", "offset": "out"},
    "j3d_check_array": {"a": "in"},
    "jacobi3d_sweep": {"u_in": "in", "u_out": "out", "f": "in", "resid_out": "out"},
    "jacobi3d_sweep2": {"u_in": "in", "u_out": "out", "f": "in", "resid_out": "out"},
    "jacobi3d_sweep3": {"u_in": "in", "u_out": "out", "f": "in", "resid_out": "out"},
    "jacobi3d_sweep3_noalloc": {"u_in": "in", "u_out": "out", "f": "in", "resid_out": "out"},
    "residual_l2": {"u": "in", "f": "in", "out": "out"},
    "j3d_sum": {"x": "in", "out": "out"},
    "j3d_dot": {"x": "in", "y": "in", "out": "out"},
    "jacobi2d_sweeps": {"u_a": "inout", "u_b": "inout", "resid_out": "out"},
    "pw_advection": {"u": "in", "v": "in", "w": "in", "su": "out", "sv": "out", "sw": "out"},
    "tracer_advection": {"t_a": "inout", "t_b": "inout", "u": "in", "v": "in", "w": "in", "r": "in"},
    "poisson_solve": {"u": "inout", "f": "in", "opts": "in", "result": "out"},
    "j3d_tune_get": {"out": "out"},
    "jacobi3d_sweep_batch": {"grids": "inout", "resid_out": "out", "tune": "in"},
    "j3d_autotune": {"grids": "inout", "best": "out"},
    "j3d_autotune_single": {"best": "out"},
    "j3d_tune_set_single": {"t": "in"},
    "j3d_tune_query_single": {"out": "out"},
    "j3d_batch_last_plan": {"sweeps_per_pass": "out", "shape": "out"},
    "poisson_serve_create": {"opts": "in", "out": "out"},
    "poisson_serve_submit": {"req": "in", "ticket": "out"},
    "poisson_serve_poll": {"out": "out", "n": "out"},
    "poisson_serve_stats": {"now": "out", "active": "out", "queued": "out", "finished": "out"},
    "j3d_fill_uniform": {"a": "out"},
    "j3d_fill_const": {"a": "out"},
    "j3d_bandwidth_probe": {"src": "in", "dst": "out", "gbps": "out"},
    "j3d_bandwidth_probe_triad": {"a": "in", "b": "in", "dst": "out", "gbps": "out"},
}


def header_prototypes():
    src = open(os.path.join(ROOT, "include", "j3d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    protos = {}
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(([^)]*)\)\s*;",
                         src, flags=re.M):
        params = [" ".join(p.split()) for p in m.group(2).split(",")]
        protos[m.group(1)] = [p for p in params if p and p != "void"]
    return protos


def test_exactly_the_intent_in_pointers_are_const():
    protos = header_prototypes()
    seen = set()
    for fn, params in protos.items():
        for p in params:
            if "*" not in p:
                continue
            name = p.split("*")[-1].strip()
            if name == "stream" or re.match(r"^j3d_server\* \w+$", p):
                continue  # opaque handles
            assert fn in INTENT and name in INTENT[fn], "no intent recorded for %s(%s)" % (fn, p)
            want_const = INTENT[fn][name] == "in"
            assert p.startswith("const ") == want_const, "%s: %s should %sbe const" % (
                fn, p, "" if want_const else "not ")
            seen.add((fn, name))
    recorded = {(fn, n) for fn, d in INTENT.items() for n in d}
    assert recorded == seen, recorded ^ seen


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(j3d.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every one of them under the same name
    assert set(header_functions()) == set(j3d.EXPORTED)


def test_abi_version():
    assert j3d.abi_version() == 2


def fake_desc(nx, ny, nz, dtype=j3d.F64, base=0x10000, lb=(0, 0, 0), ld=None, plane=None):
    d = j3d.J3DArray()
    d.base = base
    d.dtype = dtype
    d.reserved = 0
    ex, ey, ez = nx + 2, ny + 2, nz + 2
    ld = ex if ld is None else ld
    plane = ld * ey if plane is None else plane
    for k, (l, e) in enumerate(zip(lb, (ex, ey, ez))):
        d.lbound[k] = l
        d.ubound[k] = l + e - 1
    d.stride[0], d.stride[1], d.stride[2] = 1, ld, plane
    return d


def test_element_offset_matches_paper_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "fortran_index.json")))
    lib = ctypes.CDLL(j3d.LIB_PATH)
    lib.j3d_element_offset.argtypes = [ctypes.POINTER(j3d.J3DArray), ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    # The paper's 1-D example as a 10 x 1 x 1 array with lbound 1 (extents
    # padded to 3 on the unused axes, which lbound subtraction ignores).
    ex = g["paper_example"]
    d = j3d.J3DArray()
    d.base, d.dtype, d.reserved = 0x10000, j3d.F64, 0
    for k, (l, e) in enumerate(((ex["lbound"], ex["extent"]), (1, 3), (1, 3))):
        d.lbound[k], d.ubound[k] = l, l + e - 1
    d.stride[0], d.stride[1], d.stride[2] = 1, ex["extent"], 3 * ex["extent"]
    out = ctypes.c_int64()
    assert lib.j3d_element_offset(ctypes.byref(d), ex["index"], 1, 1, ctypes.byref(out)) == 0
    assert out.value == ex["offset"]
    for c in g["cases_3d"]:
        d = j3d.J3DArray()
        d.base, d.dtype, d.reserved = 0x10000, j3d.F64, 0
        for k in range(3):
            d.lbound[k] = c["lbound"][k]
            d.ubound[k] = c["lbound"][k] + 5
            d.stride[k] = c["stride"][k]
        d.stride[1] = max(d.stride[1], 6)
        d.stride[2] = max(d.stride[2], 6 * d.stride[1])
        want = sum((c["index"][k] - c["lbound"][k]) * d.stride[k] for k in range(3))
        if d.stride[1] == c["stride"][1] and d.stride[2] == c["stride"][2]:
            assert want == c["offset"]
        assert lib.j3d_element_offset(ctypes.byref(d), *c["index"], ctypes.byref(out)) == 0
        assert out.value == want
    # outside the bounds
    assert lib.j3d_element_offset(ctypes.byref(d), 1000, 0, 0, ctypes.byref(out)) == j3d.EINVAL


@pytest.mark.parametrize("mutate,code", [
    (lambda d: setattr(d, "base", None), j3d.EINVAL),
    (lambda d: setattr(d, "reserved", 1), j3d.EINVAL),
    (lambda d: setattr(d, "dtype", 7), j3d.EDTYPE),
    (lambda d: d.stride.__setitem__(0, 2), j3d.EINVAL),
    (lambda d: d.stride.__setitem__(1, 3), j3d.EINVAL),
    (lambda d: d.stride.__setitem__(2, 5), j3d.EINVAL),
    (lambda d: d.ubound.__setitem__(2, d.lbound[2] + 1), j3d.EINVAL),  # no interior on z
    (lambda d: setattr(d, "base", 0x10003), j3d.EINVAL),              # misaligned
])
def test_check_array_rejects(mutate, code):
    d = fake_desc(4, 5, 6)
    assert j3d.j3d_check_array(d, j3d.F64) == 0
    mutate(d)
    assert j3d.j3d_check_array(d, -1) == code


def test_check_array_dtype_and_views():
    d = fake_desc(4, 5, 6, dtype=j3d.F32)
    assert j3d.j3d_check_array(d, j3d.F64) == j3d.EDTYPE
    assert j3d.j3d_check_array(d, j3d.F32) == 0
    # strided subview: padded leading dimension and plane stride are fine
    d = fake_desc(4, 5, 6, ld=64, plane=64 * 7 + 3, lb=(-3, 5, 2))
    assert j3d.j3d_check_array(d, j3d.F64) == 0
    # offsets beyond 2^31 are rejected
    d = fake_desc(2000, 2000, 2000)
    assert j3d.j3d_check_array(d, j3d.F64) == j3d.EINVAL


def _call_sweep(a, b, c, h=0.1, flags=0):
    lib = j3d._lib
    return lib.jacobi3d_sweep(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), h, flags, None, None)


def test_sweep_validation_codes():
    n = 4
    span = (n + 2) ** 3 * 8
    a = fake_desc(n, n, n, base=0x100000)
    b = fake_desc(n, n, n, base=0x100000 + span)
    c = fake_desc(n, n, n, base=0x100000 + 2 * span)
    # overlapping input and output
    b_alias = fake_desc(n, n, n, base=0x100000 + 8)
    assert _call_sweep(a, b_alias, c) == j3d.EALIAS
    assert "overlap" in j3d.last_error()
    # output overlapping f
    assert _call_sweep(a, b, fake_desc(n, n, n, base=0x100000 + span + 64)) == j3d.EALIAS
    # mismatched interiors
    assert _call_sweep(a, b, fake_desc(n, n, n + 1, base=0x100000 + 2 * span)) == j3d.EINVAL
    # mixed dtypes
    assert _call_sweep(a, fake_desc(n, n, n, dtype=j3d.F32, base=0x100000 + span), c) == j3d.EDTYPE
    # bad h
    assert _call_sweep(a, b, c, h=0.0) == j3d.EINVAL
    assert _call_sweep(a, b, c, h=float("nan")) == j3d.EINVAL
    # unknown flag bits
    assert _call_sweep(a, b, c, flags=0x80) == j3d.EINVAL


def test_solve_and_batch_validation_codes():
    lib = j3d._lib
    n = 4
    span = (n + 2) ** 3 * 8
    u = fake_desc(n, n, n, base=0x200000)
    f = fake_desc(n, n, n, base=0x200000 + span)
    o = j3d.SolveOpts(5, 10, 50, 0, 100, 1e-8, None, 0)
    r = j3d.SolveResult()
    assert lib.poisson_solve(ctypes.byref(u), ctypes.byref(f), 0.1, ctypes.byref(o), ctypes.byref(r), None) == j3d.EINVAL
    o = j3d.SolveOpts(0, 0, 50, 0, 100, 1e-8, None, 0)
    assert lib.poisson_solve(ctypes.byref(u), ctypes.byref(f), 0.1, ctypes.byref(o), ctypes.byref(r), None) == j3d.EINVAL
    o = j3d.SolveOpts(0, 10, 50, 0, -1, 1e-8, None, 0)
    assert lib.poisson_solve(ctypes.byref(u), ctypes.byref(f), 0.1, ctypes.byref(o), ctypes.byref(r), None) == j3d.EINVAL
    # batch: grid 1's u_b overlaps grid 0's f
    g = (j3d.Grid * 2)()
    g[0].u_a, g[0].u_b, g[0].f, g[0].h = fake_desc(n, n, n, base=0x300000), fake_desc(n, n, n, base=0x300000 + span), \
        fake_desc(n, n, n, base=0x300000 + 2 * span), 0.1
    g[1].u_a, g[1].u_b, g[1].f, g[1].h = fake_desc(n, n, n, base=0x300000 + 3 * span), \
        fake_desc(n, n, n, base=0x300000 + 2 * span + 16), fake_desc(n, n, n, base=0x300000 + 5 * span), 0.1
    assert lib.jacobi3d_sweep_batch(2, g, 10, 1, None, None, None) == j3d.EALIAS
    # two grids may share one read-only f
    g[1].u_b = fake_desc(n, n, n, base=0x300000 + 4 * span)
    g[1].f = g[0].f
    t = j3d.Tune(3, 32, 0, 0, 0)  # unsupported rows -> rejected before any device work
    assert lib.jacobi3d_sweep_batch(2, g, 10, 1, None, ctypes.byref(t), None) == j3d.EINVAL
    assert lib.jacobi3d_sweep_batch(0, g, 10, 1, None, None, None) == j3d.EINVAL


def test_tune_list_and_request_bytes():
    tl = j3d.tune_list()
    assert len(set(tl)) == len(tl)
    assert all(r in (1, 2, 4, 8) and 0 <= v <= 23 and not v & 8 and p in (0, 1) and o in (0, 1, 2)
               and c in (1, 2, 4) for r, _, v, p, o, c in tl)
    # one wavefront along x: every rows x planes x variant x persistent x order
    assert sum(1 for t in tl if t[5] == 1) == 4 * 8 * 16 * 2 * 3
    # several along x: the nontemporal no-LDS variants, at most 16 wavefronts
    wide = [t for t in tl if t[5] > 1]
    assert {t[2] for t in wide} == {4, 6, 20}
    assert all(t[0] * t[5] <= 16 for t in wide)
    assert len(wide) == (4 + 3) * 8 * 3 * 2 * 3
    # 28 bytes per padded point (u, f FP64; r32, e0, e1 FP32) plus row padding
    b = j3d.j3d_request_bytes(384, 384, 384)
    assert 28 * 386 ** 3 <= b <= 1.1 * 28 * 386 ** 3
    assert j3d.j3d_request_bytes(0, 4, 4) == 0
    assert j3d.j3d_request_state_bytes(j3d.SERVE_MIXED, 384, 384, 384) == b
    # FP64 serving: 24 bytes per padded point (u, f, w FP64) plus row padding
    b64 = j3d.j3d_request_state_bytes(j3d.SERVE_FP64, 384, 384, 384)
    assert 24 * 386 ** 3 <= b64 <= 1.1 * 24 * 386 ** 3
    assert j3d.j3d_request_state_bytes(2, 8, 8, 8) == 0
    assert j3d.j3d_request_state_bytes(j3d.SERVE_FP64, 8, 0, 8) == 0


def test_sum_dot_validation_before_device_work():
    lib = j3d._lib
    out = ctypes.c_double()
    po = ctypes.cast(ctypes.byref(out), ctypes.c_void_p)
    x = ctypes.c_void_p(0x100000)
    assert lib.j3d_sum(x, 10, j3d.HOST_RESULT, None, None) == j3d.EINVAL  # no out
    assert lib.j3d_sum(x, -1, j3d.HOST_RESULT, po, None) == j3d.EINVAL  # n < 0
    assert lib.j3d_sum(None, 5, j3d.HOST_RESULT, po, None) == j3d.EINVAL  # null x
    assert lib.j3d_sum(x, 5, 0x80, po, None) == j3d.EINVAL  # unknown flag
    assert lib.j3d_sum(ctypes.c_void_p(0x100004), 5, j3d.HOST_RESULT, po, None) == j3d.EINVAL  # misaligned
    assert lib.j3d_dot(x, None, 5, j3d.HOST_RESULT, po, None) == j3d.EINVAL  # null y
    # a device result inside an input
    assert lib.j3d_dot(x, ctypes.c_void_p(0x200000), 100, 0, ctypes.c_void_p(0x200000 + 80), None) == j3d.EALIAS
    assert "overlaps" in j3d.last_error()


def test_bandwidth_probes_validate_before_device_work():
    lib = j3d._lib
    g = ctypes.c_double()
    pg = ctypes.byref(g)
    a, b, d = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert lib.j3d_bandwidth_probe_triad(a, b, None, 64, 1, pg, None) == j3d.EINVAL  # null dst
    assert lib.j3d_bandwidth_probe_triad(a, b, d, 1, 1, pg, None) == j3d.EINVAL  # n < 2
    assert lib.j3d_bandwidth_probe_triad(a, b, d, 64, 0, pg, None) == j3d.EINVAL  # reps < 1
    assert lib.j3d_bandwidth_probe_triad(a, b, ctypes.c_void_p(0x300008), 64, 1, pg, None) == j3d.EINVAL  # misaligned
    assert lib.j3d_bandwidth_probe_triad(a, b, ctypes.c_void_p(0x200000 + 256), 64, 1, pg, None) == j3d.EALIAS
    assert lib.j3d_bandwidth_probe(a, ctypes.c_void_p(0x100000 + 256), 64, 1, pg, None) == j3d.EALIAS
    assert lib.j3d_bandwidth_probe(a, None, 64, 1, pg, None) == j3d.EINVAL


def test_tune_query_default_set_and_bad_kind():
    # defaults (no cache entry for this odd shape)
    assert j3d.j3d_tune_query_single(j3d.F64, 97, 5, 3) == (4, 2, 6, 0, 0, 1)  # at most 64^3 points
    assert j3d.j3d_tune_query_single(j3d.F64, 65, 64, 64) == (1, 16, 20, 0, 2, 1)
    assert j3d.j3d_tune_query_single(j3d.F32, 97, 5, 3) == (1, 16, 20, 0, 2, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F64X2, 97, 5, 3) == (4, 16, 20, 0, 1, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F32X2, 97, 5, 3) == (8, 8, 20, 0, 0, 1)
    # a pinned shape is what later calls of that kind and shape use
    j3d.j3d_tune_set_single(j3d.F32, 97, 5, 3, (2, 8, 6, 1, 2, 1))
    assert j3d.j3d_tune_query_single(j3d.F32, 97, 5, 3) == (2, 8, 6, 1, 2, 1)
    assert j3d.j3d_tune_query_single(j3d.F64, 97, 5, 3) == (4, 2, 6, 0, 0, 1)
    with pytest.raises(j3d.J3DError) as ei:
        j3d.j3d_tune_query_single(7, 97, 5, 3)
    assert ei.value.code == j3d.EDTYPE
    with pytest.raises(j3d.J3DError):
        j3d.j3d_tune_query_single(j3d.F64, 0, 5, 3)


def test_batch_last_plan_before_any_batch_call():
    """Host-only query: no batch call on this thread yet -> ESTATE; null pointers -> EINVAL."""
    with pytest.raises(j3d.J3DError) as ei:
        j3d.j3d_batch_last_plan()
    assert ei.value.code == j3d.ESTATE
    k = ctypes.c_int32()
    assert j3d._lib.j3d_batch_last_plan(None, ctypes.byref(j3d.Tune())) == j3d.EINVAL
    assert j3d._lib.j3d_batch_last_plan(ctypes.byref(k), None) == j3d.EINVAL


def test_jacobi2d_validation_before_device_work():
    lib = j3d._lib
    a = fake_desc(10, 8, 1)
    a.lbound[2] = a.ubound[2] = 0  # rank 2
    b = fake_desc(10, 8, 1, base=0x900000)
    b.lbound[2] = b.ubound[2] = 0
    assert lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(b), -1, 0.1, 0, None, None) == j3d.EINVAL
    c = fake_desc(10, 8, 3, base=0x900000)  # rank 3
    assert lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(c), 4, 0.1, 0, None, None) == j3d.EINVAL
    assert "rank-2" in j3d.last_error()
    d = fake_desc(11, 8, 1, base=0x900000)
    d.lbound[2] = d.ubound[2] = 0
    assert lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(d), 4, 0.1, 0, None, None) == j3d.EINVAL
    e = fake_desc(10, 8, 1, base=0x10000 + 64)  # overlaps a
    e.lbound[2] = e.ubound[2] = 0
    assert lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(e), 4, 0.1, 0, None, None) == j3d.EALIAS
    out = ctypes.c_double()
    assert lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(b), 4, -1.0, j3d.HOST_RESULT,
                               ctypes.cast(ctypes.byref(out), ctypes.c_void_p), None) == j3d.EINVAL


def _descs(n, nx=10, ny=8, nz=6, gap=0x1000000):
    return [fake_desc(nx, ny, nz, base=0x10000 + q * gap) for q in range(n)]


def _call_pw(d, dx=0.1, dy=0.1, dz=0.1):
    return j3d._lib.pw_advection(*[ctypes.byref(x) for x in d], dx, dy, dz, None)


def _call_tracer(d, niter=2):
    return j3d._lib.tracer_advection(*[ctypes.byref(x) for x in d], niter, None)


def test_pw_advection_validation_before_device_work():
    d = _descs(6)
    d[1] = fake_desc(11, 8, 6, base=d[1].base)  # v extent differs
    assert _call_pw(d) == j3d.EINVAL
    d = _descs(6)
    d[2] = fake_desc(10, 8, 6, base=d[2].base, ld=16)  # w stride differs from u
    assert _call_pw(d) == j3d.EINVAL and "strides" in j3d.last_error()
    d = _descs(6)
    d[4] = fake_desc(10, 8, 6, base=d[4].base, ld=16)  # sv stride differs from su
    assert _call_pw(d) == j3d.EINVAL
    d = _descs(6)
    d[3] = fake_desc(10, 8, 7, base=d[3].base)  # su interior differs
    assert _call_pw(d) == j3d.EINVAL
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        assert _call_pw(_descs(6), dz=bad) == j3d.EINVAL
    d = _descs(6)
    d[5] = fake_desc(10, 8, 6, base=d[0].base + 8)  # sw overlaps u
    assert _call_pw(d) == j3d.EALIAS
    d = _descs(6)
    d[4] = fake_desc(10, 8, 6, base=d[3].base + 64)  # sv overlaps su
    assert _call_pw(d) == j3d.EALIAS
    d = _descs(6)
    d[0].dtype = j3d.F32
    assert _call_pw(d) == j3d.EDTYPE
    # a plane whose own offsets exceed 2^31 is rejected
    big = [fake_desc(10, 8, 6, base=0x10000 + q * (1 << 40), ld=1 << 28) for q in range(6)]
    assert _call_pw(big) == j3d.EINVAL and "plane" in j3d.last_error()


def test_tracer_advection_validation_before_device_work():
    assert _call_tracer(_descs(6), niter=-1) == j3d.EINVAL
    d = _descs(6)
    d[3] = fake_desc(10, 8, 6, base=d[3].base, plane=11 * 12 * 10)  # v plane stride differs
    assert _call_tracer(d) == j3d.EINVAL
    d = _descs(6)
    d[1] = fake_desc(10, 8, 6, base=d[0].base + 8)  # t_b overlaps t_a
    assert _call_tracer(d) == j3d.EALIAS
    d = _descs(6)
    d[0] = fake_desc(10, 8, 6, base=d[5].base)  # t_a overlaps r
    assert _call_tracer(d) == j3d.EALIAS


def test_wide_arrays_only_where_planes_are_addressed_in_64_bit():
    """An array of more than 2^31 elements (small planes, many of them) passes
    the advection checks' size rule but not the Jacobi sweep's."""
    nx, ny, nz = 30, 30, 3000000  # 32*32*3000002 > 2^31 elements
    u = fake_desc(nx, ny, nz)
    o = fake_desc(nx, ny, nz, base=0x10000 + (1 << 40))
    f = fake_desc(nx, ny, nz, base=0x10000 + (2 << 40))
    assert j3d._lib.jacobi3d_sweep(ctypes.byref(u), ctypes.byref(o), ctypes.byref(f), 0.1, 0, None,
                                   None) == j3d.EINVAL
    assert "2^31" in j3d.last_error()
    d = [fake_desc(nx, ny, nz, base=0x10000 + q * (1 << 40)) for q in range(6)]
    d[5].dtype = j3d.F32  # fails on the dtype, after the size rule accepted the others
    assert _call_pw(d) == j3d.EDTYPE


def test_three_sweep_kind_defaults_and_validation():
    assert j3d.j3d_tune_query_single(j3d.KIND_F64X3, 97, 5, 3) == (4, 16, 6, 0, 0, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F32X3, 97, 5, 3) == (4, 16, 6, 0, 0, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F64X3, 256, 256, 256) == (4, 16, 20, 0, 2, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F32X3, 384, 384, 384) == (8, 32, 6, 0, 2, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F64X3, 512, 512, 512) == (16, 144, 6, 0, 1, 1)
    assert j3d.j3d_tune_query_single(j3d.KIND_F32X3, 512, 512, 512) == (8, 48, 6, 0, 2, 1)
    for bad in [(1, 16, 20, 0, 1, 1), (4, 16, 16, 0, 1, 1), (4, 16, 20, 1, 1, 1), (4, 16, 20, 0, 1, 2),
                (16, 16, 20, 0, 1, 1), (3, 16, 20, 0, 1, 1), (5, 16, 20, 0, 1, 1), (6, 8, 6, 0, 1, 1),
                (7, 16, 20, 0, 1, 1), (4, 16, 6, 0, 3, 1)]:
        with pytest.raises(j3d.J3DError) as ei:
            j3d.j3d_tune_set_single(j3d.KIND_F64X3, 64, 64, 64, bad)
        assert ei.value.code == j3d.EINVAL
    for good in [(2, 16, 20, 0, 1, 1), (8, 8, 6, 0, 2, 1), (4, 48, 6, 0, 0, 1), (8, 24, 20, 0, 1, 1),
                 (16, 32, 6, 0, 1, 1)]:
        j3d.j3d_tune_set_single(j3d.KIND_F32X3, 64, 64, 64, good)
        assert j3d.j3d_tune_query_single(j3d.KIND_F32X3, 64, 64, 64) == good
    lib = j3d._lib
    a, b, c = fake_desc(10, 8, 6), fake_desc(10, 8, 6, base=0x900000), fake_desc(10, 8, 6, base=0x1900000)
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), -0.1, 0, None, None) == j3d.EINVAL
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(a), ctypes.byref(c), 0.1, 0, None, None) == j3d.EALIAS
    d = fake_desc(11, 8, 6, base=0x900000)
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(d), ctypes.byref(c), 0.1, 0, None, None) == j3d.EINVAL
    a32 = fake_desc(10, 8, 6, dtype=j3d.F32)
    b32 = fake_desc(10, 8, 6, dtype=j3d.F32, base=0x900000)
    c32 = fake_desc(10, 8, 6, dtype=j3d.F32, base=0x1900000)
    r = ctypes.c_double()
    assert lib.jacobi3d_sweep3(ctypes.byref(a32), ctypes.byref(b32), ctypes.byref(c32), 0.1, j3d.HOST_RESULT,
                               ctypes.cast(ctypes.byref(r), ctypes.c_void_p), None) == j3d.EDTYPE
    rp = ctypes.cast(ctypes.byref(r), ctypes.c_void_p)
    both = j3d.HOST_RESULT | j3d.RESID_AFTER_1 | j3d.RESID_AFTER_2
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, both, rp, None) == j3d.EINVAL
    assert "exclusive" in j3d.last_error()
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, j3d.RESID_AFTER_2, None,
                               None) == j3d.EINVAL
    assert "resid_out" in j3d.last_error()
    assert lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, 8, rp, None) == j3d.EINVAL
    assert lib.jacobi3d_sweep3(ctypes.byref(a32), ctypes.byref(b32), ctypes.byref(c32), 0.1,
                               j3d.HOST_RESULT | j3d.RESID_AFTER_1, rp, None) == j3d.EDTYPE
    # the other sweep entries know no residual-stage flags
    assert lib.jacobi3d_sweep2(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, j3d.RESID_AFTER_1, rp,
                               None) == j3d.EINVAL



@pytest.mark.skipif(__import__("torch").cuda.is_available(),
                    reason="fake device addresses: only where no GPU could run a kernel on them")
def test_noalloc_sweep3_validation():
    """jacobi3d_sweep3_noalloc rejects, before any device work: a null or host
    result, FP32 arrays, and a grid whose tiling needs more tile partials than
    its static device array holds (65536)."""
    lib = j3d._lib
    a, b, c = fake_desc(10, 8, 6), fake_desc(10, 8, 6, base=0x900000), fake_desc(10, 8, 6, base=0x1900000)
    r = ctypes.c_double()
    rp = ctypes.cast(ctypes.byref(r), ctypes.c_void_p)
    dev = ctypes.c_void_p(0x7000000)
    assert lib.jacobi3d_sweep3_noalloc(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, 0, None,
                                       None) == j3d.EINVAL
    assert lib.jacobi3d_sweep3_noalloc(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), 0.1, j3d.HOST_RESULT,
                                       rp, None) == j3d.EINVAL
    assert "J3D_HOST_RESULT" in j3d.last_error()
    a32 = fake_desc(10, 8, 6, dtype=j3d.F32)
    b32 = fake_desc(10, 8, 6, dtype=j3d.F32, base=0x900000)
    c32 = fake_desc(10, 8, 6, dtype=j3d.F32, base=0x1900000)
    assert lib.jacobi3d_sweep3_noalloc(ctypes.byref(a32), ctypes.byref(b32), ctypes.byref(c32), 0.1, 0, dev,
                                       None) == j3d.EDTYPE
    assert lib.jacobi3d_sweep3_noalloc(ctypes.byref(a), ctypes.byref(a), ctypes.byref(c), 0.1, 0, dev,
                                       None) == j3d.EALIAS
    # 59 x 1021 x 2049 points with a pinned shape of 58 columns, 4 rows and
    # 16 planes per tile: 2 x 256 x 129 = 66048 tiles
    nx, ny, nz = 59, 1021, 2049
    j3d.j3d_tune_set_single(j3d.KIND_F64X3, nx, ny, nz, (4, 16, 6, 0, 0, 1))
    span = (nx + 2) * (ny + 2) * (nz + 2) * 8
    base = 1 << 40
    big = [fake_desc(nx, ny, nz, base=base + q * (span + 4096)) for q in range(3)]
    assert lib.jacobi3d_sweep3_noalloc(*[ctypes.byref(x) for x in big], 1e-4, 0, dev, None) == j3d.EINVAL
    assert "66048 tile partials" in j3d.last_error()


def test_serve_create_validation_before_device_work():
    """poisson_serve_create checks its options (precision, reserved, counts)
    before it looks for a device."""
    lib = j3d._lib
    h = ctypes.c_void_p()

    def opts(**kw):
        o = j3d.ServeOpts(1 << 30, 4, 50, 0, 16, 0, j3d.SERVE_MIXED, 0)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    for bad in (dict(precision=2), dict(precision=-1), dict(reserved=1), dict(max_slots=0), dict(cycle_sweeps=0),
                dict(hbm_budget_bytes=0), dict(queue_cap=0)):
        assert lib.poisson_serve_create(ctypes.byref(opts(**bad)), ctypes.byref(h)) == j3d.EINVAL, bad
    assert "precision" in (lib.poisson_serve_create(ctypes.byref(opts(precision=7)), ctypes.byref(h)) and
                           j3d.last_error())
