"""Seeded synthetic inputs for the 3D Jacobi/Poisson workloads.

This module is shared by the tests, the benchmark and the oracle checks, and
holds none of the Jacobi method's arithmetic: it only draws random numbers and
builds right-hand sides.  Every field is returned as a NumPy array of shape
``(nz+2, ny+2, nx+2)`` in C order, which is byte-for-byte the Fortran array
``u(0:nx+1, 0:ny+1, 0:nz+1)`` in column-major order (x has unit stride), with
a one-cell halo.  ``a[k, j, i]`` is Fortran's ``u(i, j, k)``.

Random numbers come from a counter-based use of SplitMix64 (G. L. Steele,
D. Lea, C. H. Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): the value for counter ``n`` of a stream is the SplitMix64 output
number ``n+1`` of a generator whose 64-bit seed is ``seed XOR (stream << 40)``,
that is ``mix64(seed' + (n+1) * GAMMA)`` with the published constants.  The
counter of an interior point is its Fortran linear index over the interior,
``(i-1) + nx*((j-1) + ny*(k-1))``, so a field does not depend on padding,
leading dimension or thread count.  The device fill kernel implements the
same published definition on its own; tests compare the two bit for bit.

A uniform draw on [lo, hi) is ``lo + (hi - lo) * U`` with
``U = (bits >> 11) * 2**-53``; for [0,1) and [-1,1) every step is exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
TWO_M53 = 2.0 ** -53

# Stream identifiers (the "stream" part of a key).
STREAM_U0 = 1
STREAM_F = 2
STREAM_SIZES = 3
STREAM_ARRIVALS = 4
STREAM_TOL = 5
# multi-field stencils: velocities / transports, tracer, reciprocal volume
STREAM_ADV_U = 6
STREAM_ADV_V = 7
STREAM_ADV_W = 8
STREAM_TRACER = 9
STREAM_RVOL = 10


def _u64(x):
    return np.asarray(x, dtype=np.uint64)


def splitmix64(seed: int, stream: int, counter) -> np.ndarray:
    """SplitMix64 output for each counter of (seed, stream); uint64 array."""
    with np.errstate(over="ignore"):
        key = np.uint64((int(seed) ^ (int(stream) << 40)) & 0xFFFFFFFFFFFFFFFF)
        z = key + (_u64(counter) + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, counter, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform doubles on [lo, hi) for the given counters."""
    bits = splitmix64(seed, stream, counter)
    u = (bits >> np.uint64(11)).astype(np.float64) * TWO_M53
    return lo + (hi - lo) * u


def padded_zeros(nx: int, ny: int, nz: int, dtype=np.float64) -> np.ndarray:
    return np.zeros((nz + 2, ny + 2, nx + 2), dtype=dtype)


def uniform_field(nx: int, ny: int, nz: int, seed: int, stream: int,
                  lo: float = 0.0, hi: float = 1.0, halo: float = 0.0) -> np.ndarray:
    """Padded FP64 field: interior ~ U[lo,hi) from (seed, stream), halo = ``halo``."""
    a = np.full((nz + 2, ny + 2, nx + 2), halo, dtype=np.float64)
    # Chunk over planes so that 512^3 does not need several GB of temporaries.
    per_plane = nx * ny
    kchunk = max(1, (1 << 23) // max(per_plane, 1))
    for k0 in range(0, nz, kchunk):
        k1 = min(nz, k0 + kchunk)
        idx = np.arange(k0 * per_plane, k1 * per_plane, dtype=np.uint64)
        a[1 + k0:1 + k1, 1:ny + 1, 1:nx + 1] = uniform(seed, stream, idx, lo, hi).reshape(k1 - k0, ny, nx)
    return a


def uniform_box(nx: int, ny: int, nz: int, seed: int, stream: int, lo: float, hi: float, halo: float,
                i0: int, i1: int, j0: int, j1: int, k0: int, k1: int) -> np.ndarray:
    """The block [k0:k1, j0:j1, i0:i1] (padded indices, halo = index 0 and
    n+1) of ``uniform_field(nx, ny, nz, seed, stream, lo, hi, halo)``,
    computed without the rest of the field."""
    k = np.arange(k0, k1, dtype=np.int64)[:, None, None]
    j = np.arange(j0, j1, dtype=np.int64)[None, :, None]
    i = np.arange(i0, i1, dtype=np.int64)[None, None, :]
    inside = (i >= 1) & (i <= nx) & (j >= 1) & (j <= ny) & (k >= 1) & (k <= nz)
    lin = (i - 1) + nx * ((j - 1) + ny * (k - 1))
    lin = np.where(inside, lin, 0).astype(np.uint64)
    vals = uniform(seed, stream, lin, lo, hi)
    return np.where(inside, vals, halo)


def sine_factors(n: int, h: float) -> np.ndarray:
    """sin(pi * i * h) for i = 0 .. n+1 (grid coordinate x_i = i*h)."""
    return np.sin(np.pi * (np.arange(n + 2, dtype=np.float64) * h))


def manufactured_u(nx: int, ny: int, nz: int, h: float) -> np.ndarray:
    """u*(x,y,z) = sin(pi x) sin(pi y) sin(pi z) sampled at x_i = i*h (halo included)."""
    sx, sy, sz = sine_factors(nx, h), sine_factors(ny, h), sine_factors(nz, h)
    return (sz[:, None, None] * sy[None, :, None]) * sx[None, None, :]


def manufactured_f(nx: int, ny: int, nz: int, h: float, scale: float | None = None) -> np.ndarray:
    """Right-hand side ``scale * u*`` (default scale 3*pi^2, the continuous -Laplacian of u*).

    The halo is set to zero (no kernel reads the halo of f).
    """
    if scale is None:
        scale = 3.0 * math.pi ** 2
    f = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    sx, sy, sz = sine_factors(nx, h), sine_factors(ny, h), sine_factors(nz, h)
    for k in range(1, nz + 1):
        f[k, 1:ny + 1, 1:nx + 1] = ((scale * sz[k]) * sy[1:ny + 1, None]) * sx[None, 1:nx + 1]
    return f


# ----------------------------------------------------------------------------
# Workload recipes (one seed per workload).
# ----------------------------------------------------------------------------

def small_plain(n: int = 64, seed: int = 1):
    """64^3 FP64, u0 ~ U[0,1), f ~ U[-1,1), h = 1/(n+1), zero halo."""
    h = 1.0 / (n + 1)
    u0 = uniform_field(n, n, n, seed, STREAM_U0, 0.0, 1.0)
    f = uniform_field(n, n, n, seed, STREAM_F, -1.0, 1.0)
    return u0, f, h


def manufactured_problem(n: int = 512, seed: int = 2):
    """Cubic manufactured Poisson problem: u0 ~ U[0,1), f = 3 pi^2 u*, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    u0 = uniform_field(n, n, n, seed, STREAM_U0, 0.0, 1.0)
    f = manufactured_f(n, n, n, h)
    return u0, f, h


@dataclass
class BatchGrid:
    nx: int
    ny: int
    nz: int
    h: float
    seed: int


def batch_shapes(ngrids: int = 256, seed: int = 4, lo: int = 32, hi: int = 256):
    """Uneven grid shapes: each axis drawn independently and uniformly from {lo..hi}.

    Grid g draws counters 3g, 3g+1, 3g+2 of the sizes stream.  h = 1/(max(n)+1).
    Grid g's right-hand side uses the seed ``seed * 65536 + g``.
    """
    span = hi - lo + 1
    u = uniform(seed, STREAM_SIZES, np.arange(3 * ngrids, dtype=np.uint64))
    dims = lo + np.minimum(np.floor(u * span).astype(np.int64), span - 1)
    out = []
    for g in range(ngrids):
        nx, ny, nz = (int(d) for d in dims[3 * g:3 * g + 3])
        out.append(BatchGrid(nx, ny, nz, 1.0 / (max(nx, ny, nz) + 1), seed * 65536 + g))
    return out


def batch_rhs(g: BatchGrid) -> np.ndarray:
    return uniform_field(g.nx, g.ny, g.nz, g.seed, STREAM_F, -1.0, 1.0)


@dataclass
class ServeRequest:
    rid: int
    arrival_s: float
    n: int
    h: float
    rtol: float
    seed: int
    max_sweeps: int


def serve_requests(count: int = 1000, rate: float = 200.0, seed: int = 5,
                   nmin: int = 32, nmax: int = 384, max_sweeps: int = 5000,
                   tols=(1e-6, 1e-8)):
    """Poisson arrivals (exponential gaps at ``rate``/s), cubic n log-uniform in [nmin, nmax].

    n = round(nmin * (nmax/nmin)**U); the tolerance is tols[0] or tols[1] with
    probability 1/2 each.  Request r's right-hand side uses seed ``seed*65536 + r``.
    """
    idx = np.arange(count, dtype=np.uint64)
    ua = uniform(seed, STREAM_ARRIVALS, idx)
    us = uniform(seed, STREAM_SIZES, idx)
    ut = uniform(seed, STREAM_TOL, idx)
    gaps = -np.log1p(-ua) / rate
    t = np.cumsum(gaps)
    ratio = nmax / nmin
    out = []
    for r in range(count):
        n = int(round(nmin * ratio ** float(us[r])))
        n = max(nmin, min(nmax, n))
        out.append(ServeRequest(r, float(t[r]), n, 1.0 / (n + 1),
                                tols[0] if ut[r] < 0.5 else tols[1],
                                seed * 65536 + r, max_sweeps))
    return out


# Multi-field stencils (stand-ins for pw-advection and tra-adv).
PW_SHAPE = (2048, 1024, 1024)     # three fields
TRA_SHAPE = (1024, 512, 512)      # six fields, 20 iterations
TRA_ITERS = 20


@dataclass
class FieldRecipe:
    seed: int
    stream: int
    lo: float
    hi: float
    halo: float


def pw_recipe(seed: int = 6):
    """Velocities u, v, w ~ U[-1, 1), halo 0.25; spacing 1/1024 on every axis."""
    fields = [FieldRecipe(seed, s, -1.0, 1.0, 0.25) for s in (STREAM_ADV_U, STREAM_ADV_V, STREAM_ADV_W)]
    return fields, (1.0 / 1024, 1.0 / 1024, 1.0 / 1024)


def tracer_recipe(seed: int = 7):
    """Tracer t ~ U[0, 1) (halo 0.5); transports u, v, w ~ U[-0.1, 0.1) (halo
    0); r = step / volume ~ U[0.5, 1.5) (halo 1).  r times the outflow of a
    cell stays below 0.9, so the steps are stable."""
    t = FieldRecipe(seed, STREAM_TRACER, 0.0, 1.0, 0.5)
    vel = [FieldRecipe(seed, s, -0.1, 0.1, 0.0) for s in (STREAM_ADV_U, STREAM_ADV_V, STREAM_ADV_W)]
    r = FieldRecipe(seed, STREAM_RVOL, 0.5, 1.5, 1.0)
    return t, vel, r
