"""CPU oracle for the 3D 7-point Jacobi / Poisson hot path.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's CPU-baseline leg; the product package never imports it,
and the two share no code.

Two independent references live here:

* ``j3d_oracle.c`` (built with gcc into ``liboracle.so``): plain triple loops
  for the sweep, the residual and its norm, the plain and mixed-precision
  solves, the paper's 2D Laplace jacobi benchmark, and the two multi-field
  stencils standing in for pw-advection and tra-adv.  The functions below wrap it for NumPy arrays of shape
  ``(nz+2, ny+2, ld)`` (Fortran ``u(0:ld-1, 0:ny+1, 0:nz+1)``, x unit stride).
* ``dense`` : the operator assembled as a dense matrix from its definition,
  used to pin the loop oracle on tiny grids (brute force).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "j3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        F = ctypes.c_float
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_sweep_f64.argtypes = [P, P, P, I, I, I, I, I, D]
        L.oracle_sweep_f64.restype = None
        L.oracle_residual_field_f64.argtypes = [P, P, P, I, I, I, I, I, D]
        L.oracle_residual_field_f64.restype = None
        L.oracle_norm2_f64.argtypes = [P, I, I, I, I, I]
        L.oracle_norm2_f64.restype = D
        L.oracle_residual_l2_f64.argtypes = [P, P, I, I, I, I, I, D]
        L.oracle_residual_l2_f64.restype = D
        L.oracle_sweep_f32.argtypes = [P, P, P, I, I, I, I, I, F]
        L.oracle_sweep_f32.restype = None
        L.oracle_defect.argtypes = [P, P, P, P, I, I, I, I, I, I, I, D]
        L.oracle_defect.restype = D
        L.oracle_solve_plain.argtypes = [P, P, P, I, I, I, I, I, D, D, I, I, P, I, P]
        L.oracle_solve_plain.restype = None
        L.oracle_solve_mixed.argtypes = [P, P, P, P, P, I, I, I, I, I, I, I, D, D, I, I, P, I, P]
        L.oracle_solve_mixed.restype = None
        L.oracle_jacobi2d.argtypes = [P, P, I, I, I, I]
        L.oracle_jacobi2d.restype = None
        L.oracle_laplace2d_resid_l2.argtypes = [P, I, I, I, D]
        L.oracle_laplace2d_resid_l2.restype = D
        L.oracle_pw_advection.argtypes = [P, P, P, P, P, P, I, I, I, I, I, D, D, D]
        L.oracle_pw_advection.restype = None
        L.oracle_tracer_advection.argtypes = [P, P, P, P, P, P, I, I, I, I, I, I]
        L.oracle_tracer_advection.restype = None
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().oracle_threads())


def _geom(a: np.ndarray, dtype):
    if a.dtype != dtype or a.ndim != 3 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous 3-D %s array" % np.dtype(dtype).name)
    nz2, ny2, ld = a.shape
    return ld, ny2 - 2, nz2 - 2, ld, ld * ny2


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def sweep(u: np.ndarray, f: np.ndarray, h: float, nx: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """One FP64 Jacobi sweep; returns u' (halo copied from u)."""
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    nx = ld - 2 if nx is None else nx
    assert f.shape == u.shape
    un = u.copy() if out is None else out
    lib().oracle_sweep_f64(_p(u), _p(un), _p(f), nx, ny, nz, sy, sz, float(h))
    return un


def residual_field(u: np.ndarray, f: np.ndarray, h: float, nx: int | None = None) -> np.ndarray:
    """Per-point residual f - A u over the interior (halo left zero)."""
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    nx = ld - 2 if nx is None else nx
    r = np.zeros_like(u)
    lib().oracle_residual_field_f64(_p(u), _p(f), _p(r), nx, ny, nz, sy, sz, float(h))
    return r


def residual_l2(u: np.ndarray, f: np.ndarray, h: float, nx: int | None = None) -> float:
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    nx = ld - 2 if nx is None else nx
    return float(lib().oracle_residual_l2_f64(_p(u), _p(f), nx, ny, nz, sy, sz, float(h)))


def norm2(a: np.ndarray, nx: int | None = None) -> float:
    ld, ny, nz, sy, sz = _geom(a, np.float64)
    nx = ld - 2 if nx is None else nx
    return float(lib().oracle_norm2_f64(_p(a), nx, ny, nz, sy, sz))


def sweep_f32(e: np.ndarray, r32: np.ndarray, h2: np.float32, nx: int | None = None) -> np.ndarray:
    ld, ny, nz, sy, sz = _geom(e, np.float32)
    nx = ld - 2 if nx is None else nx
    en = e.copy()
    lib().oracle_sweep_f32(_p(e), _p(en), _p(r32), nx, ny, nz, sy, sz, float(np.float32(h2)))
    return en


def defect(u: np.ndarray, e: np.ndarray | None, f: np.ndarray, h: float):
    """FP64 defect step in place on a copy of u; returns (u_new, r32, ||r||)."""
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    nx = ld - 2
    u = u.copy()
    r32 = np.zeros(u.shape, dtype=np.float32)
    _, _, _, sy4, sz4 = _geom(r32, np.float32)
    rn = lib().oracle_defect(_p(u), _p(e) if e is not None else None, _p(f), _p(r32),
                             nx, ny, nz, sy, sz, sy4, sz4, float(h))
    return u, r32, float(rn)


class SolveResult:
    def __init__(self, out, hist):
        self.sweeps = int(out[0])
        self.resid = float(out[1])
        self.resid0 = float(out[2])
        self.norm_f = float(out[3])
        self.converged = bool(out[4])
        self.history = hist[: int(out[5])].copy()

    @property
    def rel(self):
        return self.resid / self.norm_f if self.norm_f > 0 else 0.0


def solve_plain(u0: np.ndarray, f: np.ndarray, h: float, rtol: float, check_every: int,
                max_sweeps: int, hist_cap: int = 1 << 16):
    u = u0.copy()
    work = u0.copy()
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    hist = np.zeros(hist_cap)
    out = np.zeros(6)
    lib().oracle_solve_plain(_p(u), _p(work), _p(f), ld - 2, ny, nz, sy, sz, float(h), float(rtol),
                             int(check_every), int(max_sweeps), _p(hist), hist_cap, _p(out))
    return u, SolveResult(out, hist)


def solve_mixed(u0: np.ndarray, f: np.ndarray, h: float, rtol: float, inner: int,
                max_sweeps: int, hist_cap: int = 1 << 16):
    u = u0.copy()
    ld, ny, nz, sy, sz = _geom(u, np.float64)
    r32 = np.zeros(u.shape, dtype=np.float32)
    ea = np.zeros(u.shape, dtype=np.float32)
    eb = np.zeros(u.shape, dtype=np.float32)
    _, _, _, sy4, sz4 = _geom(r32, np.float32)
    hist = np.zeros(hist_cap)
    out = np.zeros(6)
    lib().oracle_solve_mixed(_p(u), _p(f), _p(r32), _p(ea), _p(eb), ld - 2, ny, nz, sy, sz, sy4, sz4,
                             float(h), float(rtol), int(inner), int(max_sweeps), _p(hist), hist_cap, _p(out))
    return u, SolveResult(out, hist)


def _geom2(a: np.ndarray):
    if a.dtype != np.float64 or a.ndim != 2 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous 2-D float64 array")
    ny2, ld = a.shape
    return ld, ny2 - 2


def jacobi2d(u0: np.ndarray, nsweeps: int, nx: int | None = None) -> np.ndarray:
    """The paper's 2D Laplace Jacobi benchmark: nsweeps sweeps of u0 (shape
    (ny+2, ld), x unit stride, halo = boundary values); returns the result."""
    ld, ny = _geom2(u0)
    nx = ld - 2 if nx is None else nx
    a, b = u0.copy(), u0.copy()
    lib().oracle_jacobi2d(_p(a), _p(b), nx, ny, ld, int(nsweeps))
    return a if nsweeps % 2 == 0 else b


def laplace2d_resid_l2(u: np.ndarray, h: float, nx: int | None = None) -> float:
    ld, ny = _geom2(u)
    nx = ld - 2 if nx is None else nx
    return float(lib().oracle_laplace2d_resid_l2(_p(u), nx, ny, ld, float(h)))


def _same(*arrs):
    a0 = arrs[0]
    for a in arrs:
        if a.shape != a0.shape:
            raise ValueError("all fields must have the same shape")
    return _geom(a0, np.float64)


def pw_advection(u: np.ndarray, v: np.ndarray, w: np.ndarray, dx: float, dy: float, dz: float,
                 nx: int | None = None):
    """Momentum advection tendencies (su, sv, sw) of the staggered velocity
    (u, v, w), centred flux form; interior written, halo zero."""
    ld, ny, nz, sy, sz = _same(u, v, w)
    nx = ld - 2 if nx is None else nx
    su, sv, sw = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
    lib().oracle_pw_advection(_p(u), _p(v), _p(w), _p(su), _p(sv), _p(sw), nx, ny, nz, sy, sz,
                              float(dx), float(dy), float(dz))
    return su, sv, sw


def tracer_advection(t0: np.ndarray, u: np.ndarray, v: np.ndarray, w: np.ndarray, r: np.ndarray,
                     niter: int, nx: int | None = None) -> np.ndarray:
    """niter donor-cell advection steps of the tracer t0 (its halo = boundary
    values); returns the result."""
    ld, ny, nz, sy, sz = _same(t0, u, v, w, r)
    nx = ld - 2 if nx is None else nx
    a, b = t0.copy(), t0.copy()
    lib().oracle_tracer_advection(_p(a), _p(b), _p(u), _p(v), _p(w), _p(r), nx, ny, nz, sy, sz, int(niter))
    return a if niter % 2 == 0 else b
