"""Pins of the oracle's two multi-field stencils (CPU only).

Momentum advection (centred flux form of Piacsek and Williams on a staggered
grid, the stand-in for pw-advection): zero tendency of uniform flow, closed
forms for linear fields, second-order convergence to the continuous
-div(u q) of smooth fields, momentum and kinetic-energy conservation for
periodic, discretely non-divergent flow (the scheme's defining property),
and a face-flux-first brute force on a tiny grid.

Tracer advection (donor cell, the stand-in for tra-adv): exact shifts at
Courant number one in all six directions (also over several iterations,
with the inflow boundary entering), conservation of the volume-weighted
tracer, preservation of a uniform tracer and the maximum principle under
non-divergent transport, and a face-flux-first brute force.
"""
import math

import numpy as np
import pytest

import oracle

EPS = np.finfo(np.float64).eps
I3 = (slice(1, -1),) * 3


def grids(nx, ny, nz):
    """Index arrays k, j, i broadcast over a padded (nz+2, ny+2, nx+2) field."""
    k = np.arange(nz + 2, dtype=np.float64)[:, None, None]
    j = np.arange(ny + 2, dtype=np.float64)[None, :, None]
    i = np.arange(nx + 2, dtype=np.float64)[None, None, :]
    return k, j, i


def full(shape, a):
    return np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)


def wrap(a):
    """Periodic halo: every halo plane copies the interior plane on the other side."""
    nz, ny, nx = (s - 2 for s in a.shape)
    a[:, :, 0] = a[:, :, nx]
    a[:, :, nx + 1] = a[:, :, 1]
    a[:, 0, :] = a[:, ny, :]
    a[:, ny + 1, :] = a[:, 1, :]
    a[0] = a[nz]
    a[nz + 1] = a[1]
    return a


def back_diff(a, axis):
    """a(n) - a(n-1) along a numpy axis (0 = z, 1 = y, 2 = x); index 0 left zero."""
    r = np.zeros_like(a)
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[axis] = slice(1, None)
    sl_lo[axis] = slice(None, -1)
    r[tuple(sl_hi)] = a[tuple(sl_hi)] - a[tuple(sl_lo)]
    return r


def nondivergent(rng, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0):
    """Periodic staggered velocity (u, v, w) = curl of a random edge-centred
    vector potential: its discrete divergence vanishes up to rounding."""
    shape = (nz + 2, ny + 2, nx + 2)
    ax, ay, az = (wrap(rng.uniform(-1, 1, shape)) for _ in range(3))
    u = wrap(back_diff(az, 1) / dy - back_diff(ay, 0) / dz)
    v = wrap(back_diff(ax, 0) / dz - back_diff(az, 2) / dx)
    w = wrap(back_diff(ay, 2) / dx - back_diff(ax, 1) / dy)
    return u, v, w


def divergence(u, v, w, dx=1.0, dy=1.0, dz=1.0):
    return ((u[I3] - u[1:-1, 1:-1, :-2]) / dx + (v[I3] - v[1:-1, :-2, 1:-1]) / dy
            + (w[I3] - w[:-2, 1:-1, 1:-1]) / dz)


# ---------------------------------------------------------------------------
# Momentum advection
# ---------------------------------------------------------------------------

def test_uniform_flow_has_zero_tendency():
    shape = (9, 8, 11)
    u, v, w = full(shape, 0.3), full(shape, -1.7), full(shape, 2.9)
    for out in oracle.pw_advection(u, v, w, 0.1, 0.37, 2.3):
        assert np.all(out == 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_self_advection(axis):
    """q = a * (position of q along its own axis): the tendency of q is
    -d(q^2)/ds = -2 a^2 s at q's staggered point, the others vanish."""
    nx, ny, nz = 10, 9, 8
    d = (0.11, 0.07, 0.23)  # dx, dy, dz
    k, j, i = grids(nx, ny, nz)
    pos = [(i + 0.5) * d[0], (j + 0.5) * d[1], (k + 0.5) * d[2]][axis]
    a = 1.3
    shape = (nz + 2, ny + 2, nx + 2)
    fields = [np.zeros(shape) for _ in range(3)]
    fields[axis] = full(shape, a * pos)
    out = oracle.pw_advection(*fields, *d)
    want = full(shape, -2.0 * a * a * pos)
    scale = np.max(np.abs(want[I3]))
    for c in range(3):
        if c == axis:
            assert np.max(np.abs(out[c][I3] - want[I3])) <= 64 * EPS * scale
        else:
            assert np.all(out[c] == 0.0)


# (advected component, its coordinate axis, advecting component held constant)
CROSS = [(0, 1, 1), (0, 2, 2), (1, 0, 0), (1, 2, 2), (2, 0, 0), (2, 1, 1)]


@pytest.mark.parametrize("q,s,c", CROSS)
def test_cross_advection_constant_carrier(q, s, c):
    """q = b * s (s a coordinate transverse to q's face) carried by a constant
    velocity component c along s: tendency of q = -c0 * b, exactly in exact
    arithmetic; the carrier's own tendency vanishes."""
    nx, ny, nz = 9, 10, 11
    d = (0.2, 0.05, 0.125)
    k, j, i = grids(nx, ny, nz)
    coord = [i * d[0], j * d[1], k * d[2]][s]  # q sits at integer positions along s
    shape = (nz + 2, ny + 2, nx + 2)
    b, c0 = 0.7, -1.9
    fields = [np.zeros(shape) for _ in range(3)]
    fields[q] = full(shape, b * coord)
    fields[c] = full(shape, c0)
    out = oracle.pw_advection(*fields, *d)
    assert np.max(np.abs(out[q][I3] + c0 * b)) <= 64 * EPS * abs(c0 * b)
    assert np.all(out[c][I3] == 0.0)
    third = 3 - q - c
    assert np.all(out[third][I3] == 0.0)


def smooth_case(n):
    """Smooth fields on a grid of spacing 1/n and the exact tendencies
    -div(u q) at the staggered points of q."""
    h = 1.0 / n
    k, j, i = grids(n, n, n)
    X, Y, Z = i * h, j * h, k * h
    xh, yh, zh = X + 0.5 * h, Y + 0.5 * h, Z + 0.5 * h

    def U(x, y, z):
        return np.sin(x + 2 * y + 3 * z)

    def V(x, y, z):
        return np.cos(2 * x - y + z)

    def W(x, y, z):
        return 0.5 + np.sin(x - y + 2 * z)

    def grads(x, y, z):
        au, av, aw = x + 2 * y + 3 * z, 2 * x - y + z, x - y + 2 * z
        u, v, w = np.sin(au), np.cos(av), 0.5 + np.sin(aw)
        ux, uy, uz = np.cos(au), 2 * np.cos(au), 3 * np.cos(au)
        vx, vy, vz = -2 * np.sin(av), np.sin(av), -np.sin(av)
        wx, wy, wz = np.cos(aw), -np.cos(aw), 2 * np.cos(aw)
        return u, v, w, (ux, uy, uz), (vx, vy, vz), (wx, wy, wz)

    shape = (n + 2,) * 3
    u = full(shape, U(xh, Y, Z))
    v = full(shape, V(X, yh, Z))
    w = full(shape, W(X, Y, zh))
    uu, vv, ww, gu, gv, gw = grads(xh, Y, Z)
    su = -(2 * uu * gu[0] + gv[1] * uu + vv * gu[1] + gw[2] * uu + ww * gu[2])
    uu, vv, ww, gu, gv, gw = grads(X, yh, Z)
    sv = -(gu[0] * vv + uu * gv[0] + 2 * vv * gv[1] + gw[2] * vv + ww * gv[2])
    uu, vv, ww, gu, gv, gw = grads(X, Y, zh)
    sw = -(gu[0] * ww + uu * gw[0] + gv[1] * ww + vv * gw[1] + 2 * ww * gw[2])
    return (u, v, w), [full(shape, s) for s in (su, sv, sw)], h


def test_second_order_convergence():
    errs = []
    for n in (16, 32):
        fields, exact, h = smooth_case(n)
        got = oracle.pw_advection(*fields, h, h, h)
        errs.append([np.max(np.abs(got[c][I3] - exact[c][I3])) for c in range(3)])
    for c in range(3):
        rate = math.log2(errs[0][c] / errs[1][c])
        assert 1.85 < rate < 2.15, (c, errs, rate)
        assert errs[1][c] < 0.05


def test_periodic_momentum_and_energy_conservation():
    rng = np.random.default_rng(11)
    nx, ny, nz = 12, 10, 9
    d = (0.1, 0.13, 0.07)
    u, v, w = nondivergent(rng, nx, ny, nz, *d)
    assert np.max(np.abs(divergence(u, v, w, *d))) < 1e-11
    su, sv, sw = oracle.pw_advection(u, v, w, *d)
    for s in (su, sv, sw):
        assert abs(s[I3].sum()) <= 1e-13 * np.abs(s[I3]).sum()
    e = (u[I3] * su[I3]).sum() + (v[I3] * sv[I3]).sum() + (w[I3] * sw[I3]).sum()
    scale = np.abs(u[I3] * su[I3]).sum() + np.abs(v[I3] * sv[I3]).sum() + np.abs(w[I3] * sw[I3]).sum()
    assert abs(e) <= 1e-13 * scale
    # a divergent random field does not conserve energy (the pin has teeth)
    u2, v2, w2 = (wrap(rng.uniform(-1, 1, u.shape)) for _ in range(3))
    s2 = oracle.pw_advection(u2, v2, w2, *d)
    e2 = sum((f[I3] * s[I3]).sum() for f, s in zip((u2, v2, w2), s2))
    assert abs(e2) > 1e-4 * sum(np.abs(f[I3] * s[I3]).sum() for f, s in zip((u2, v2, w2), s2))


def test_face_flux_brute_force():
    """Tendencies from explicitly tabulated face fluxes (averages taken as
    half-sums, fluxes stored per face, then differenced), pure Python loops."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 3, 4, 2
    d = (0.3, 0.2, 0.5)
    shape = (nz + 2, ny + 2, nx + 2)
    F = [rng.uniform(-1, 1, shape) for _ in range(3)]
    got = oracle.pw_advection(*F, *d)

    def val(c, i, j, k):
        return F[c][k, j, i]

    def avg(c, p, axis):
        # component c averaged from its two nearest points in direction axis
        # onto position p (doubled coordinates, integer grid index = 2n)
        lo = list(p)
        hi = list(p)
        lo[axis] -= 1
        hi[axis] += 1
        return 0.5 * (at(c, lo) + at(c, hi))

    def at(c, p):
        # component c at doubled position p; c sits at odd doubled coordinate
        # along its own axis (2n+1 = face n+1/2), even along the others
        idx = [p[0] // 2, p[1] // 2, p[2] // 2]
        return val(c, *idx)

    def flux(a, q, p):
        # flux along axis a of component q through doubled position p
        return avg(a, p, q) * avg(q, p, a)

    want = [np.zeros(shape) for _ in range(3)]
    for q in range(3):
        for k in range(1, nz + 1):
            for j in range(1, ny + 1):
                for i in range(1, nx + 1):
                    p = [2 * i, 2 * j, 2 * k]
                    p[q] += 1  # q's own point
                    tot = 0.0
                    for a in range(3):
                        lo, hi = list(p), list(p)
                        lo[a] -= 1
                        hi[a] += 1
                        tot -= (flux(a, q, hi) - flux(a, q, lo)) / d[a]
                    want[q][k, j, i] = tot
    for q in range(3):
        assert np.max(np.abs(got[q][I3] - want[q][I3])) <= 1e-13 * np.max(np.abs(want[q][I3]))


# ---------------------------------------------------------------------------
# Tracer advection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("axis,sign", [(a, s) for a in (0, 1, 2) for s in (1, -1)])
@pytest.mark.parametrize("niter", [1, 4])
def test_courant_one_shift(axis, sign, niter):
    """Transport +-1 through every face of one axis, r = 1: each iteration
    moves the tracer one cell downstream, exactly (values in [1, 2) make every
    subtraction exact); the fixed halo flows in at the upstream boundary."""
    rng = np.random.default_rng(7 + axis)
    nx, ny, nz = 7, 6, 5
    shape = (nz + 2, ny + 2, nx + 2)
    t0 = rng.uniform(1.0, 2.0, shape)
    vel = [np.zeros(shape) for _ in range(3)]
    vel[axis] = np.full(shape, float(sign))
    r = np.ones(shape)
    got = oracle.tracer_advection(t0, *vel, r, niter)
    np_axis = 2 - axis  # numpy axis of Fortran axis
    n = shape[np_axis]
    want = t0.copy()
    for m in range(1, n - 1):
        src = max(m - niter, 0) if sign > 0 else min(m + niter, n - 1)
        sl_dst = [slice(1, -1)] * 3
        sl_src = [slice(1, -1)] * 3
        sl_dst[np_axis] = m
        sl_src[np_axis] = src
        want[tuple(sl_dst)] = t0[tuple(sl_src)]
    assert np.array_equal(got, want)


def test_volume_weighted_tracer_is_conserved():
    rng = np.random.default_rng(9)
    nx, ny, nz = 11, 8, 7
    shape = (nz + 2, ny + 2, nx + 2)
    t0 = rng.uniform(0.0, 1.0, shape)
    u, v, w = (rng.uniform(-0.1, 0.1, shape) for _ in range(3))
    # no transport through the domain's faces
    u[:, :, 0] = u[:, :, nx] = 0.0
    v[:, 0, :] = v[:, ny, :] = 0.0
    w[0] = w[nz] = 0.0
    vol = rng.uniform(0.5, 1.5, shape)
    r = 1.0 / vol
    t5 = oracle.tracer_advection(t0, u, v, w, r, 5)
    a, b = (vol[I3] * t0[I3]).sum(), (vol[I3] * t5[I3]).sum()
    assert abs(a - b) <= 1e-13 * a
    assert np.max(np.abs(t5[I3] - t0[I3])) > 1e-3  # it did move


def test_uniform_tracer_and_maximum_principle_nondivergent():
    rng = np.random.default_rng(10)
    nx, ny, nz = 10, 9, 8
    u, v, w = nondivergent(rng, nx, ny, nz)
    out = np.maximum(u[I3], 0) - np.minimum(u[1:-1, 1:-1, :-2], 0)
    out += np.maximum(v[I3], 0) - np.minimum(v[1:-1, :-2, 1:-1], 0)
    out += np.maximum(w[I3], 0) - np.minimum(w[:-2, 1:-1, 1:-1], 0)
    scale = 0.9 / np.max(out)  # r * outflow <= 0.9
    u, v, w = u * scale, v * scale, w * scale
    r = np.ones_like(u)
    c = np.full(u.shape, 0.625)
    tc = oracle.tracer_advection(c, u, v, w, r, 3)
    assert np.max(np.abs(tc - 0.625)) <= 1e-14
    t0 = wrap(rng.uniform(-1.0, 1.0, u.shape))
    t3 = oracle.tracer_advection(t0, u, v, w, r, 3)
    lo, hi = t0.min(), t0.max()
    assert t3[I3].min() >= lo - 1e-14 and t3[I3].max() <= hi + 1e-14


def test_tracer_face_flux_brute_force():
    """Two iterations from per-face donor-cell fluxes, pure Python loops."""
    rng = np.random.default_rng(12)
    nx, ny, nz = 4, 3, 3
    shape = (nz + 2, ny + 2, nx + 2)
    t = rng.uniform(-1, 1, shape)
    vel = [rng.uniform(-0.2, 0.2, shape) for _ in range(3)]
    r = rng.uniform(0.5, 2.0, shape)
    got = oracle.tracer_advection(t, *vel, r, 2)
    cur = t.copy()
    for _ in range(2):
        nxt = cur.copy()
        # flux through the upper face of cell (i,j,k) along Fortran axis a
        flux = {}
        for a in range(3):
            for k in range(0, nz + 1):
                for j in range(0, ny + 1):
                    for i in range(0, nx + 1):
                        nb = [i, j, k]
                        nb[a] += 1
                        if max(nb[0] - nx, nb[1] - ny, nb[2] - nz) > 1:
                            continue
                        q = vel[a][k, j, i]
                        donor = cur[k, j, i] if q > 0 else cur[nb[2], nb[1], nb[0]]
                        flux[(a, i, j, k)] = q * donor if q != 0 else 0.0
        for k in range(1, nz + 1):
            for j in range(1, ny + 1):
                for i in range(1, nx + 1):
                    dfl = []
                    for a in range(3):
                        lo = [i, j, k]
                        lo[a] -= 1
                        dfl.append(flux[(a, i, j, k)] - flux[(a, *lo)])
                    nxt[k, j, i] = cur[k, j, i] - r[k, j, i] * ((dfl[0] + dfl[1]) + dfl[2])
        cur = nxt
    assert np.max(np.abs(got - cur)) <= 1e-15
