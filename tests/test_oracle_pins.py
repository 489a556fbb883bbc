"""Pins of the CPU oracle against what the mathematics fixes (CPU only).

Each test ties an oracle function to something outside the oracle itself:
a closed form of the 7-point operator, an invariant, or a dense brute-force
matrix assembled from the operator's definition.  A plausible slip in the
oracle (a dropped or doubled neighbour, a swapped stride, a sign, the h^2
factor, the divisor) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import dense

PI = math.pi


def eigenmode(nx, ny, nz, a, b, c, dtype=np.float64):
    """phi = sin(a pi i/(nx+1)) sin(b pi j/(ny+1)) sin(c pi k/(nz+1)), zero halo."""
    si = np.sin(a * PI * np.arange(nx + 2) / (nx + 1))
    sj = np.sin(b * PI * np.arange(ny + 2) / (ny + 1))
    sk = np.sin(c * PI * np.arange(nz + 2) / (nz + 1))
    phi = sk[:, None, None] * sj[None, :, None] * si[None, None, :]
    phi[0], phi[-1] = 0, 0
    phi[:, 0], phi[:, -1] = 0, 0
    phi[:, :, 0], phi[:, :, -1] = 0, 0
    return phi.astype(dtype)


def lam(nx, ny, nz, a, b, c):
    return (math.cos(a * PI / (nx + 1)) + math.cos(b * PI / (ny + 1)) + math.cos(c * PI / (nz + 1))) / 3.0


# --------------------------------------------------------------------------
# Generator (shared input module)
# --------------------------------------------------------------------------

def test_splitmix64_published_vectors(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64_vectors.json")))
    for v in g["vectors"]:
        got = synth.splitmix64(v["seed"], 0, np.arange(len(v["outputs"]), dtype=np.uint64))
        assert [int(x) for x in got] == [int(s) for s in v["outputs"]]


def test_uniform_ranges_and_exactness():
    idx = np.arange(200000, dtype=np.uint64)
    u01 = synth.uniform(7, 1, idx, 0.0, 1.0)
    assert u01.min() >= 0.0 and u01.max() < 1.0
    um = synth.uniform(7, 1, idx, -1.0, 1.0)
    assert um.min() >= -1.0 and um.max() < 1.0
    # -1 + 2U is exact for U a multiple of 2^-53 in [0,1)
    assert np.array_equal((um + 1.0) / 2.0, u01)
    assert abs(u01.mean() - 0.5) < 0.005


def test_field_independent_of_padding():
    a = synth.uniform_field(5, 4, 3, 11, synth.STREAM_F, -1, 1)
    # interior linear index (i-1) + nx*((j-1) + ny*(k-1))
    k, j, i = 2, 3, 4
    lin = (i - 1) + 5 * ((j - 1) + 4 * (k - 1))
    assert a[k, j, i] == synth.uniform(11, synth.STREAM_F, np.array([lin], dtype=np.uint64), -1, 1)[0]
    assert np.all(a[0] == 0) and np.all(a[:, :, -1] == 0)


def test_workload_recipes_deterministic():
    s1 = synth.batch_shapes(256, 4)
    s2 = synth.batch_shapes(256, 4)
    assert [(g.nx, g.ny, g.nz) for g in s1] == [(g.nx, g.ny, g.nz) for g in s2]
    dims = np.array([(g.nx, g.ny, g.nz) for g in s1])
    assert dims.min() >= 32 and dims.max() <= 256
    reqs = synth.serve_requests(1000)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 384
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 3.5 < arr[-1] < 6.5  # 1000 arrivals at 200/s
    tols = np.array([r.rtol for r in reqs])
    assert 0.4 < np.mean(tols == 1e-8) < 0.6


# --------------------------------------------------------------------------
# P1: discrete eigenmodes (sweep and residual, non-cubic, distinct modes)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,mode", [((5, 7, 9), (2, 3, 1)), ((12, 5, 9), (1, 4, 7)), ((3, 4, 5), (3, 1, 2))])
def test_p1_sweep_eigenmode(shape, mode):
    nx, ny, nz = shape
    phi = eigenmode(nx, ny, nz, *mode)
    f = np.zeros_like(phi)
    out = oracle.sweep(phi, f, 0.37)
    want = lam(nx, ny, nz, *mode) * phi
    assert np.max(np.abs(out[1:-1, 1:-1, 1:-1] - want[1:-1, 1:-1, 1:-1])) < 1e-14


@pytest.mark.parametrize("shape,mode", [((5, 7, 9), (2, 3, 1)), ((12, 5, 9), (1, 4, 7))])
def test_p1_residual_eigenmode(shape, mode):
    nx, ny, nz = shape
    h = 0.37
    phi = eigenmode(nx, ny, nz, *mode)
    f = np.zeros_like(phi)
    a, b, c = mode
    th = [a * PI / (nx + 1), b * PI / (ny + 1), c * PI / (nz + 1)]
    norm_phi = math.sqrt((nx + 1) * (ny + 1) * (nz + 1) / 8.0)
    want = (2.0 / h ** 2) * sum(1 - math.cos(t) for t in th) * norm_phi
    got = oracle.residual_l2(phi, f, h)
    assert abs(got - want) <= 1e-12 * want
    assert abs(oracle.norm2(phi) - norm_phi) <= 1e-13 * norm_phi


def test_p1_sweep_f32_eigenmode():
    nx, ny, nz = 9, 6, 11
    phi = eigenmode(nx, ny, nz, 2, 1, 3, np.float32)
    r = np.zeros_like(phi)
    out = oracle.sweep_f32(phi, r, np.float32(0.01))
    want = lam(nx, ny, nz, 2, 1, 3) * phi.astype(np.float64)
    # six FP32 additions and a division: a few units of 2^-24 of the terms
    assert np.max(np.abs(out.astype(np.float64) - want)) < 8 * 2.0 ** -24
    # FP32 arithmetic really is FP32: it differs from the FP64 evaluation somewhere
    assert np.any(out.astype(np.float64) != want)


# --------------------------------------------------------------------------
# P2 / P3: manufactured solution closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 64])
def test_p2_manufactured_sweep(n):
    h = 1.0 / (n + 1)
    us = synth.manufactured_u(n, n, n, h)
    us[0], us[-1], us[:, 0], us[:, -1], us[:, :, 0], us[:, :, -1] = 0, 0, 0, 0, 0, 0
    f = synth.manufactured_f(n, n, n, h)
    out = oracle.sweep(us, f, h)
    g = math.cos(PI * h) + PI ** 2 * h ** 2 / 2
    assert np.max(np.abs(out - g * us)[1:-1, 1:-1, 1:-1]) < 1e-14


@pytest.mark.parametrize("n", [16, 64])
def test_p3_manufactured_residual_closed_form(n):
    h = 1.0 / (n + 1)
    us = synth.manufactured_u(n, n, n, h)
    us[0], us[-1], us[:, 0], us[:, -1], us[:, :, 0], us[:, :, -1] = 0, 0, 0, 0, 0, 0
    f = synth.manufactured_f(n, n, n, h)
    lam_h = (12.0 / h ** 2) * math.sin(PI * h / 2) ** 2
    want = (3 * PI ** 2 - lam_h) * ((n + 1) / 2.0) ** 1.5
    got = oracle.residual_l2(us, f, h)
    # cancellation floor: terms are O(3 pi^2), the residual is O(1e-3) of them
    assert abs(got - want) <= 1e-9 * want


# --------------------------------------------------------------------------
# P4: constant field with matching halo is a fixed point
# --------------------------------------------------------------------------

def test_p4_constant_fixed_point():
    u = np.full((7, 6, 9), 0.75)
    f = np.zeros_like(u)
    out = oracle.sweep(u, f, 0.1)
    assert np.array_equal(out, u)
    assert oracle.residual_l2(u, f, 0.1) == 0.0


def test_p4_zero_halo_breaks_fixed_point():
    u = np.full((7, 6, 9), 0.75)
    u[0] = 0.0
    out = oracle.sweep(u, np.zeros_like(u), 0.1)
    assert out[1, 3, 4] == 0.75 * 5 / 6 and out[2, 3, 4] == 0.75


# --------------------------------------------------------------------------
# P5: residual contracts by at most rho per sweep, and tends to rho
# --------------------------------------------------------------------------

def test_p5_monotone_residual():
    nx, ny, nz = 6, 7, 8
    u0 = synth.uniform_field(nx, ny, nz, 3, 1, 0, 1)
    f = synth.uniform_field(nx, ny, nz, 3, 2, -1, 1)
    h = 1.0 / 9
    _, res = oracle.solve_plain(u0, f, h, rtol=0.0, check_every=1, max_sweeps=150)
    hist = res.history
    assert len(hist) == 151 and res.sweeps == 150 and not res.converged
    rho = (math.cos(PI / (nx + 1)) + math.cos(PI / (ny + 1)) + math.cos(PI / (nz + 1))) / 3
    ratios = hist[1:] / hist[:-1]
    assert np.all(ratios <= rho * (1 + 1e-12))
    assert abs(ratios[-1] - rho) < 1e-3


def test_p5_rho_on_4cubed():
    rho = math.cos(PI / 5)
    assert abs(rho - 0.809017) < 1e-6
    u0 = synth.uniform_field(4, 4, 4, 9, 1, 0, 1)
    f = np.zeros_like(u0)
    _, res = oracle.solve_plain(u0, f, 0.2, rtol=0.0, check_every=1, max_sweeps=80)
    r = res.history
    assert abs(r[-1] / r[-2] - rho) < 1e-6


# --------------------------------------------------------------------------
# P6: dense brute force on tiny grids, with non-zero Dirichlet data
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(4, 4, 4), (3, 4, 5), (5, 3, 2)])
def test_p6_dense_bruteforce(shape):
    nx, ny, nz = shape
    h = 0.2
    halo = synth.uniform_field(nx, ny, nz, 21, 7, -1, 1, halo=0.0)
    rng_halo = synth.uniform(21, 8, np.arange((nx + 2) * (ny + 2) * (nz + 2), dtype=np.uint64), -1, 1)
    bdry = rng_halo.reshape(nz + 2, ny + 2, nx + 2)
    u = synth.uniform_field(nx, ny, nz, 21, 1, 0, 1)
    # Dirichlet data in the halo, random interior
    mask = np.ones_like(u, dtype=bool)
    mask[1:-1, 1:-1, 1:-1] = False
    u[mask] = bdry[mask]
    f = synth.uniform_field(nx, ny, nz, 21, 2, -1, 1)
    del halo
    A = dense.assemble(nx, ny, nz, h)
    b = dense.rhs(f, u, h)
    uv = dense.to_vec(u)
    # sweep
    want = dense.jacobi(A, b, uv)
    got = dense.to_vec(oracle.sweep(u, f, h))
    assert np.max(np.abs(got - want)) < 1e-13
    # residual field and norm
    rw = dense.residual(A, b, uv)
    rg = dense.to_vec(oracle.residual_field(u, f, h))
    assert np.max(np.abs(rg - rw)) <= 1e-12 * np.max(np.abs(rw))
    assert abs(oracle.residual_l2(u, f, h) - np.linalg.norm(rw)) <= 1e-12 * np.linalg.norm(rw)
    # solve: converges to the dense LU solution
    ustar = dense.exact(A, b)
    us, res = oracle.solve_plain(u, f, h, rtol=1e-12, check_every=5, max_sweeps=20000)
    assert res.converged and res.sweeps % 5 == 0
    assert res.resid <= 1e-12 * res.norm_f
    assert np.max(np.abs(dense.to_vec(us) - ustar)) < 1e-9 * np.max(np.abs(ustar))
    # halo untouched
    assert np.array_equal(us[mask], u[mask])


def test_p6_defect_step_dense():
    nx, ny, nz = 4, 3, 5
    h = 0.25
    u = synth.uniform_field(nx, ny, nz, 5, 1, 0, 1)
    f = synth.uniform_field(nx, ny, nz, 5, 2, -1, 1)
    e = synth.uniform_field(nx, ny, nz, 5, 3, -1e-3, 1e-3).astype(np.float32)
    un, r32, rn = oracle.defect(u, e, f, h)
    A = dense.assemble(nx, ny, nz, h)
    uv = dense.to_vec(u) + dense.to_vec(e).astype(np.float64)
    assert np.array_equal(dense.to_vec(un), uv)
    r = dense.residual(A, dense.rhs(f, u, h), uv)
    assert abs(rn - np.linalg.norm(r)) <= 1e-12 * np.linalg.norm(r)
    r32v = dense.to_vec(r32).astype(np.float64)
    assert np.all(np.abs(r32v - r) <= 2.0 ** -24 * np.abs(r) + 1e-12 * np.max(np.abs(r)))
    assert r32.dtype == np.float32


# --------------------------------------------------------------------------
# P7: mixed precision reaches the plain solve's iterate at cycle granularity
# --------------------------------------------------------------------------

def test_p7_mixed_matches_plain():
    n = 12
    h = 1.0 / (n + 1)
    u0 = synth.uniform_field(n, n, n, 2, 1, 0, 1)
    f = synth.manufactured_f(n, n, n, h)
    up, rp = oracle.solve_plain(u0, f, h, rtol=1e-8, check_every=50, max_sweeps=20000)
    um, rm = oracle.solve_mixed(u0, f, h, rtol=1e-8, inner=50, max_sweeps=20000)
    assert rp.converged and rm.converged
    assert rp.sweeps == rm.sweeps
    assert len(rp.history) == len(rm.history)
    # same iterate up to FP32 rounding of the corrections
    rel = np.abs(rm.history - rp.history) / rp.history
    assert np.max(rel) < 1e-4
    d = np.max(np.abs(um - up)) / np.max(np.abs(up))
    assert d < 1e-7
    # independent check of the reported residual with the dense operator
    A = dense.assemble(n, n, n, h)
    r = dense.residual(A, dense.rhs(f, u0, h), dense.to_vec(um))
    # Near convergence r is a difference of O(12 |u| / h^2) terms: the two
    # evaluation orders may differ by a few ulps of those terms per point.
    floor = 4 * 2.0 ** -52 * (12 * np.max(np.abs(um)) / h ** 2 + np.max(np.abs(f))) * math.sqrt(n ** 3)
    assert abs(np.linalg.norm(r) - rm.resid) <= floor
    assert rm.resid <= 1e-8 * rm.norm_f


def test_p7_mixed_cap_and_count():
    n = 10
    h = 1.0 / (n + 1)
    u0 = np.zeros((n + 2,) * 3)
    f = synth.uniform_field(n, n, n, 9, 2, -1, 1)
    um, rm = oracle.solve_mixed(u0, f, h, rtol=1e-14, inner=50, max_sweeps=120)
    assert not rm.converged and rm.sweeps == 120
    assert len(rm.history) == 4  # defects at 0, 50, 100, 120
    assert rm.resid0 == pytest.approx(rm.norm_f, rel=1e-14)  # u0 = 0 -> r0 = f


# --------------------------------------------------------------------------
# P8: Fortran addressing: leading-dimension padding does not change results
# --------------------------------------------------------------------------

def test_p8_padded_leading_dimension():
    nx, ny, nz = 6, 5, 4
    u = synth.uniform_field(nx, ny, nz, 8, 1, 0, 1)
    f = synth.uniform_field(nx, ny, nz, 8, 2, -1, 1)
    ld = nx + 2 + 7
    up = np.full((nz + 2, ny + 2, ld), np.nan)
    fp = np.full((nz + 2, ny + 2, ld), np.nan)
    up[:, :, :nx + 2] = u
    fp[:, :, :nx + 2] = f
    a = oracle.sweep(u, f, 0.3)
    b = oracle.sweep(up, fp, 0.3, nx=nx)
    assert np.array_equal(a, b[:, :, :nx + 2])
    assert oracle.residual_l2(u, f, 0.3) == oracle.residual_l2(up, fp, 0.3, nx=nx)


def test_p8_paper_index_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "fortran_index.json")))
    ex = g["paper_example"]
    data = np.zeros(ex["extent"], dtype=np.int32)
    data[ex["index"] - ex["lbound"]] = ex["value"]
    assert int(np.nonzero(data)[0][0]) == ex["offset"]
