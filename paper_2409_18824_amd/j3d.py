"""Python binding of libj3d (ctypes).  Argument marshalling only.

Every entry point here has the name of the C function it calls and does no
arithmetic of its own: all work runs in the library's HIP kernels.  PyTorch
provides device memory and streams.  If ``libj3d.so`` is missing the import
fails loudly; there is no CPU fallback.

Fortran arrays live in torch storage: ``FArray`` describes the array
``u(lb0:ub0, lb1:ub1, lb2:ub2)`` (halo included, x unit stride) over a 1-D
torch tensor, in the C ABI's ``j3d_array`` form.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libj3d.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libj3d.so is not built (expected at %s); run "
        "`python -m paper_2409_18824_amd.csrc.build` or __graft_entry__.build()" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

F64, F32 = 0, 1
OK, EINVAL, EDTYPE, EALIAS, ENOMEM, EBUDGET, EHIP, ENONFINITE, EAGAIN, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
HOST_RESULT = 1
RESID_AFTER_1 = 2  # jacobi3d_sweep3: residual of the iterate after the pass's first sweep
RESID_AFTER_2 = 4  # ... after its second sweep
MODE_FP64, MODE_MIXED = 0, 1
SERVE_MIXED, SERVE_FP64 = 0, 1  # server precision
KIND_F64X2 = 2  # tuning kind of the two-sweep FP64 pass
KIND_F32X2 = 3  # tuning kind of the two-sweep FP32 pass (also the mixed solve's correction sweeps)
KIND_F64X3 = 4  # tuning kind of the three-sweep FP64 pass
KIND_F32X3 = 5  # tuning kind of the three-sweep FP32 pass

_ERRNAMES = {0: "OK", -1: "EINVAL", -2: "EDTYPE", -3: "EALIAS", -4: "ENOMEM", -5: "EBUDGET",
             -6: "EHIP", -7: "ENONFINITE", -8: "EAGAIN", -9: "ESTATE"}


class J3DError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__("%s failed with %s: %s" % (func, _ERRNAMES.get(code, code), msg))
        self.code = code


class J3DArray(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lbound", ctypes.c_int64 * 3), ("ubound", ctypes.c_int64 * 3),
                ("stride", ctypes.c_int64 * 3)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("inner_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int64), ("rtol", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int64)]


class SolveResult(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("resid", ctypes.c_double), ("resid0", ctypes.c_double),
                ("norm_f", ctypes.c_double), ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("history_len", ctypes.c_int64)]


class Grid(ctypes.Structure):
    _fields_ = [("u_a", J3DArray), ("u_b", J3DArray), ("f", J3DArray), ("h", ctypes.c_double)]


class Tune(ctypes.Structure):
    """(rows, planes, variant, persistent, order, cols); see j3d_tune in include/j3d.h."""
    _fields_ = [("rows", ctypes.c_int32), ("planes", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("order", ctypes.c_int32), ("cols", ctypes.c_int32)]

    def as_tuple(self):
        return (self.rows, self.planes, self.variant, self.persistent, self.order, self.cols)


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("cycle_sweeps", ctypes.c_int32), ("device", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("max_active_points", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("h", ctypes.c_double),
                ("f_host", ctypes.POINTER(ctypes.c_double)), ("seed", ctypes.c_uint64),
                ("rtol", ctypes.c_double), ("max_sweeps", ctypes.c_int64),
                ("u_host", ctypes.POINTER(ctypes.c_double))]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("resid", ctypes.c_double), ("norm_f", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_P = ctypes.POINTER
_V = ctypes.c_void_p
_I32, _I64, _U32, _U64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double

_SIGS = {
    "j3d_abi_version": ([], ctypes.c_int),
    "j3d_last_error": ([], ctypes.c_char_p),
    "j3d_element_offset": ([_P(J3DArray), _I64, _I64, _I64, _P(_I64)], ctypes.c_int),
    "j3d_check_array": ([_P(J3DArray), _I32], ctypes.c_int),
    "jacobi3d_sweep": ([_P(J3DArray), _P(J3DArray), _P(J3DArray), _D, _U32, _V, _V], ctypes.c_int),
    "jacobi3d_sweep2": ([_P(J3DArray), _P(J3DArray), _P(J3DArray), _D, _U32, _V, _V], ctypes.c_int),
    "jacobi3d_sweep3": ([_P(J3DArray), _P(J3DArray), _P(J3DArray), _D, _U32, _V, _V], ctypes.c_int),
    "jacobi3d_sweep3_noalloc": ([_P(J3DArray), _P(J3DArray), _P(J3DArray), _D, _U32, _V, _V], ctypes.c_int),
    "residual_l2": ([_P(J3DArray), _P(J3DArray), _D, _U32, _V, _V], ctypes.c_int),
    "poisson_solve": ([_P(J3DArray), _P(J3DArray), _D, _P(SolveOpts), _P(SolveResult), _V], ctypes.c_int),
    "j3d_tune_count": ([], ctypes.c_int),
    "j3d_tune_get": ([_I32, _P(Tune)], ctypes.c_int),
    "jacobi3d_sweep_batch": ([_I32, _P(Grid), _I32, _I32, _V, _P(Tune), _V], ctypes.c_int),
    "j3d_autotune": ([_I32, _P(Grid), _P(Tune), _V], ctypes.c_int),
    "j3d_batch_last_plan": ([_P(_I32), _P(Tune)], ctypes.c_int),
    "j3d_autotune_single": ([_I32, _I32, _I32, _I32, _P(Tune), _V], ctypes.c_int),
    "j3d_tune_set_single": ([_I32, _I32, _I32, _I32, _P(Tune)], ctypes.c_int),
    "j3d_tune_query_single": ([_I32, _I32, _I32, _I32, _P(Tune)], ctypes.c_int),
    "j3d_request_bytes": ([_I32, _I32, _I32], _U64),
    "j3d_request_state_bytes": ([_I32, _I32, _I32, _I32], _U64),
    "poisson_serve_create": ([_P(ServeOpts), _P(_V)], ctypes.c_int),
    "poisson_serve_submit": ([_V, _P(Request), _P(_U64)], ctypes.c_int),
    "poisson_serve_poll": ([_V, _P(Result), _I32, _P(_I32)], ctypes.c_int),
    "poisson_serve_drain": ([_V, _D], ctypes.c_int),
    "poisson_serve_stats": ([_V, _P(_D), _P(_I32), _P(_I32), _P(_I64)], ctypes.c_int),
    "poisson_serve_destroy": ([_V], ctypes.c_int),
    "j3d_fill_uniform": ([_P(J3DArray), _U64, _U32, _D, _D, _D, _V], ctypes.c_int),
    "j3d_fill_const": ([_P(J3DArray), _D, _V], ctypes.c_int),
    "j3d_bandwidth_probe": ([_V, _V, _I64, _I32, _P(_D), _V], ctypes.c_int),
    "j3d_bandwidth_probe_triad": ([_V, _V, _V, _I64, _I32, _P(_D), _V], ctypes.c_int),
    "j3d_sum": ([_V, _I64, _U32, _V, _V], ctypes.c_int),
    "jacobi2d_sweeps": ([_P(J3DArray), _P(J3DArray), _I64, _D, _U32, _V, _V], ctypes.c_int),
    "j3d_dot": ([_V, _V, _I64, _U32, _V, _V], ctypes.c_int),
    "pw_advection": ([_P(J3DArray)] * 6 + [_D, _D, _D, _V], ctypes.c_int),
    "tracer_advection": ([_P(J3DArray)] * 6 + [_I64, _V], ctypes.c_int),
    "j3d_release_cache": ([], ctypes.c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


def last_error() -> str:
    s = _lib.j3d_last_error()
    return s.decode() if s else ""


def _check(rc, func):
    if rc != OK:
        raise J3DError(rc, func, last_error())
    return rc


def abi_version() -> int:
    return _lib.j3d_abi_version()


def _stream_handle(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ----------------------------------------------------------------------------
# Fortran arrays over torch storage
# ----------------------------------------------------------------------------

_TORCH_DT = {F64: torch.float64, F32: torch.float32}
_NP_DT = {F64: np.float64, F32: np.float32}


@dataclass
class FArray:
    """Fortran array u(lbound:ubound) (inclusive, halo included) in torch storage.

    ``storage`` is a 1-D tensor; element (lbound0, lbound1, lbound2) is at
    ``storage[offset]``; ``stride`` is in elements with stride[0] = 1.
    """
    storage: torch.Tensor
    offset: int
    lbound: tuple
    ubound: tuple
    stride: tuple
    dtype: int

    @classmethod
    def empty(cls, nx, ny, nz, dtype=F64, device="cuda", lbound=(0, 0, 0), align_bytes=128,
              ld_extra=0, plane_extra=0):
        """Allocate a padded array for an nx*ny*nz interior plus halo.

        Rows are padded so that element (lbound0+1, j, k) of every row is
        ``align_bytes``-aligned; ``ld_extra``/``plane_extra`` add more padding
        (to exercise strided layouts).
        """
        es = 8 if dtype == F64 else 4
        al = max(1, align_bytes // es)
        ex, ey, ez = nx + 2, ny + 2, nz + 2
        ld = (ex + al - 1) // al * al + ld_extra
        sz = ld * ey + plane_extra
        offset = al - 1
        n = offset + sz * ez + al
        st = torch.zeros(n, dtype=_TORCH_DT[dtype], device=device)
        lb = tuple(int(x) for x in lbound)
        ub = (lb[0] + ex - 1, lb[1] + ey - 1, lb[2] + ez - 1)
        return cls(st, offset, lb, ub, (1, ld, sz), dtype)

    @property
    def extents(self):
        return tuple(self.ubound[d] - self.lbound[d] + 1 for d in range(3))

    @property
    def interior(self):
        ex, ey, ez = self.extents
        return ex - 2, ey - 2, ez - 2

    def desc(self) -> J3DArray:
        d = J3DArray()
        d.base = self.storage.data_ptr() + self.offset * self.storage.element_size()
        d.dtype = self.dtype
        d.reserved = 0
        for k in range(3):
            d.lbound[k] = self.lbound[k]
            d.ubound[k] = self.ubound[k]
            d.stride[k] = self.stride[k]
        return d

    def view(self) -> torch.Tensor:
        """Strided torch view (nz+2, ny+2, nx+2) of the array (no copy)."""
        ex, ey, ez = self.extents
        return torch.as_strided(self.storage, (ez, ey, ex), (self.stride[2], self.stride[1], 1), self.offset)

    def to_numpy(self) -> np.ndarray:
        return self.view().cpu().numpy().copy()

    def copy_from(self, a: np.ndarray):
        ex, ey, ez = self.extents
        if a.shape != (ez, ey, ex):
            raise ValueError("shape %s does not match array extents %s" % (a.shape, (ez, ey, ex)))
        self.view().copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=_NP_DT[self.dtype])))
        return self

    @classmethod
    def empty2d(cls, nx, ny, dtype=F64, device="cuda", lbound=(0, 0), align_bytes=128, ld_extra=0):
        """A rank-2 array u(0:nx+1, 0:ny+1) (descriptor axis 2 of extent 1)."""
        es = 8 if dtype == F64 else 4
        al = max(1, align_bytes // es)
        ex, ey = nx + 2, ny + 2
        ld = (ex + al - 1) // al * al + ld_extra
        offset = al - 1
        st = torch.zeros(offset + ld * ey + al, dtype=_TORCH_DT[dtype], device=device)
        lb = (int(lbound[0]), int(lbound[1]), 0)
        ub = (lb[0] + ex - 1, lb[1] + ey - 1, 0)
        return cls(st, offset, lb, ub, (1, ld, ld * ey), dtype)

    @classmethod
    def from_numpy2d(cls, a: np.ndarray, dtype=None, device="cuda", **kw):
        ey, ex = a.shape
        if dtype is None:
            dtype = F32 if a.dtype == np.float32 else F64
        out = cls.empty2d(ex - 2, ey - 2, dtype=dtype, device=device, **kw)
        return out.copy_from(a[None, :, :])

    def to_numpy2d(self) -> np.ndarray:
        return self.to_numpy()[0]

    @classmethod
    def from_numpy(cls, a: np.ndarray, dtype=None, device="cuda", **kw):
        ez, ey, ex = a.shape
        if dtype is None:
            dtype = F32 if a.dtype == np.float32 else F64
        out = cls.empty(ex - 2, ey - 2, ez - 2, dtype=dtype, device=device, **kw)
        return out.copy_from(a)


# ----------------------------------------------------------------------------
# Entry points (names of the C ABI)
# ----------------------------------------------------------------------------

def j3d_element_offset(a: FArray, i: int, j: int, k: int) -> int:
    out = ctypes.c_int64()
    d = a.desc()
    _check(_lib.j3d_element_offset(ctypes.byref(d), i, j, k, ctypes.byref(out)), "j3d_element_offset")
    return out.value


def j3d_check_array(desc: J3DArray, dtype: int) -> int:
    return _lib.j3d_check_array(ctypes.byref(desc), dtype)


def jacobi3d_sweep(u_in: FArray, u_out: FArray, f: FArray, h: float, resid_out=None, host_result=False,
                   stream=None, flags: int = 0):
    """One sweep u_out = J(u_in).  ``resid_out``: torch float64 tensor (device) or None.

    With ``host_result=True`` returns the residual norm of u_in as a float.
    """
    a, b, c = u_in.desc(), u_out.desc(), f.desc()
    st = _stream_handle(stream)
    if host_result:
        out = ctypes.c_double()
        _check(_lib.jacobi3d_sweep(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h),
                                   flags | HOST_RESULT, ctypes.cast(ctypes.byref(out), ctypes.c_void_p), st),
               "jacobi3d_sweep")
        return out.value
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi3d_sweep(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h), flags, ptr, st),
           "jacobi3d_sweep")
    return None


def jacobi3d_sweep2(u_in: FArray, u_out: FArray, f: FArray, h: float, resid_out=None, host_result=False,
                    stream=None, flags: int = 0):
    """Two sweeps in one pass: u_out = J(J(u_in)).  Residual (of u_in) as in jacobi3d_sweep."""
    a, b, c = u_in.desc(), u_out.desc(), f.desc()
    st = _stream_handle(stream)
    if host_result:
        out = ctypes.c_double()
        _check(_lib.jacobi3d_sweep2(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h),
                                    flags | HOST_RESULT, ctypes.cast(ctypes.byref(out), ctypes.c_void_p), st),
               "jacobi3d_sweep2")
        return out.value
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi3d_sweep2(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h), flags, ptr, st),
           "jacobi3d_sweep2")
    return None


def jacobi3d_sweep3(u_in: FArray, u_out: FArray, f: FArray, h: float, resid_out=None, host_result=False,
                    stream=None, flags: int = 0, resid_after: int = 0):
    """Three sweeps in one pass: u_out = J(J(J(u_in))).  Residual as in jacobi3d_sweep, of u_in
    (resid_after=0) or of the iterate after the pass's first or second sweep (resid_after=1, 2)."""
    if resid_after:
        flags |= {1: RESID_AFTER_1, 2: RESID_AFTER_2}[resid_after]
    a, b, c = u_in.desc(), u_out.desc(), f.desc()
    st = _stream_handle(stream)
    if host_result:
        out = ctypes.c_double()
        _check(_lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h),
                                    flags | HOST_RESULT, ctypes.cast(ctypes.byref(out), ctypes.c_void_p), st),
               "jacobi3d_sweep3")
        return out.value
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi3d_sweep3(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h), flags, ptr, st),
           "jacobi3d_sweep3")
    return None


def jacobi3d_sweep3_noalloc(u_in: FArray, u_out: FArray, f: FArray, h: float, resid_out, stream=None,
                            flags: int = 0, resid_after: int = 0):
    """jacobi3d_sweep3 with its fused residual into ``resid_out`` (a device float64 tensor), the
    tile partials kept in the library's static device array instead of allocated scratch."""
    if resid_after:
        flags |= {1: RESID_AFTER_1, 2: RESID_AFTER_2}[resid_after]
    a, b, c = u_in.desc(), u_out.desc(), f.desc()
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi3d_sweep3_noalloc(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(h), flags, ptr,
                                        _stream_handle(stream)), "jacobi3d_sweep3_noalloc")


def residual_l2(u: FArray, f: FArray, h: float, out=None, stream=None):
    """||f - A u||_2.  With ``out`` (device float64 tensor) asynchronous; else returns a float."""
    a, c = u.desc(), f.desc()
    st = _stream_handle(stream)
    if out is None:
        v = ctypes.c_double()
        _check(_lib.residual_l2(ctypes.byref(a), ctypes.byref(c), float(h), HOST_RESULT,
                                ctypes.cast(ctypes.byref(v), ctypes.c_void_p), st), "residual_l2")
        return v.value
    _check(_lib.residual_l2(ctypes.byref(a), ctypes.byref(c), float(h), 0, ctypes.c_void_p(out.data_ptr()), st),
           "residual_l2")
    return None


def _vec(x, what):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise TypeError("%s: a contiguous float64 CUDA tensor is required" % what)
    return ctypes.c_void_p(x.data_ptr()), x.numel()


def jacobi2d_sweeps(u_a: FArray, u_b: FArray, nsweeps: int, h: float = 1.0, resid_out=None, host_result=False,
                    stream=None):
    """The paper's 2D Laplace jacobi benchmark: nsweeps sweeps alternating
    u_a -> u_b -> ...; the result is in u_a when nsweeps is even.  With
    ``host_result`` returns ||r||_2 of the result; with ``resid_out`` (one
    device float64) stores it asynchronously."""
    a, b = u_a.desc(), u_b.desc()
    st = _stream_handle(stream)
    if host_result:
        v = ctypes.c_double()
        _check(_lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(b), int(nsweeps), float(h), HOST_RESULT,
                                    ctypes.cast(ctypes.byref(v), ctypes.c_void_p), st), "jacobi2d_sweeps")
        return v.value
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi2d_sweeps(ctypes.byref(a), ctypes.byref(b), int(nsweeps), float(h), 0, ptr, st),
           "jacobi2d_sweeps")
    return None


def pw_advection(u: FArray, v: FArray, w: FArray, su: FArray, sv: FArray, sw: FArray,
                 dx: float, dy: float, dz: float, stream=None):
    """Momentum advection tendencies (su, sv, sw) of the staggered velocity
    (u, v, w), centred flux form; asynchronous."""
    d = [a.desc() for a in (u, v, w, su, sv, sw)]
    _check(_lib.pw_advection(*[ctypes.byref(x) for x in d], float(dx), float(dy), float(dz),
                             _stream_handle(stream)), "pw_advection")


def tracer_advection(t_a: FArray, t_b: FArray, u: FArray, v: FArray, w: FArray, r: FArray, niter: int,
                     stream=None):
    """niter donor-cell steps alternating t_a -> t_b -> ...; the result is in
    t_a when niter is even.  Asynchronous."""
    d = [a.desc() for a in (t_a, t_b, u, v, w, r)]
    _check(_lib.tracer_advection(*[ctypes.byref(x) for x in d], int(niter), _stream_handle(stream)),
           "tracer_advection")


def j3d_sum(x, out=None, stream=None):
    """Fortran sum(x) of a contiguous float64 CUDA tensor.  With ``out`` (a
    one-element device float64 tensor) asynchronous; else returns a float."""
    px, n = _vec(x, "j3d_sum")
    st = _stream_handle(stream)
    if out is None:
        v = ctypes.c_double()
        _check(_lib.j3d_sum(px, n, HOST_RESULT, ctypes.cast(ctypes.byref(v), ctypes.c_void_p), st), "j3d_sum")
        return v.value
    _check(_lib.j3d_sum(px, n, 0, ctypes.c_void_p(out.data_ptr()), st), "j3d_sum")
    return None


def j3d_dot(x, y, out=None, stream=None):
    """Fortran dot_product(x, y) of two contiguous float64 CUDA tensors of one size."""
    px, n = _vec(x, "j3d_dot")
    py, ny = _vec(y, "j3d_dot")
    if ny != n:
        raise ValueError("j3d_dot: x and y differ in size (%d vs %d)" % (n, ny))
    st = _stream_handle(stream)
    if out is None:
        v = ctypes.c_double()
        _check(_lib.j3d_dot(px, py, n, HOST_RESULT, ctypes.cast(ctypes.byref(v), ctypes.c_void_p), st), "j3d_dot")
        return v.value
    _check(_lib.j3d_dot(px, py, n, 0, ctypes.c_void_p(out.data_ptr()), st), "j3d_dot")
    return None


@dataclass
class Solve:
    sweeps: int
    resid: float
    resid0: float
    norm_f: float
    converged: bool
    status: int
    history: np.ndarray

    @property
    def rel(self):
        return self.resid / self.norm_f if self.norm_f > 0 else 0.0


def poisson_solve(u: FArray, f: FArray, h: float, mode=MODE_FP64, rtol=1e-8, max_sweeps=1000,
                  check_every=10, inner_sweeps=50, history_cap=1 << 16, stream=None, raise_nonfinite=True):
    a, c = u.desc(), f.desc()
    hist = np.zeros(max(history_cap, 1), dtype=np.float64)
    o = SolveOpts(mode, check_every, inner_sweeps, 0, max_sweeps, rtol,
                  hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), history_cap)
    r = SolveResult()
    rc = _lib.poisson_solve(ctypes.byref(a), ctypes.byref(c), float(h), ctypes.byref(o), ctypes.byref(r),
                            _stream_handle(stream))
    if rc != OK and not (rc == ENONFINITE and not raise_nonfinite):
        raise J3DError(rc, "poisson_solve", last_error())
    return Solve(r.sweeps, r.resid, r.resid0, r.norm_f, bool(r.converged), r.status,
                 hist[: r.history_len].copy())


def tune_list():
    out = []
    for i in range(_lib.j3d_tune_count()):
        t = Tune()
        _check(_lib.j3d_tune_get(i, ctypes.byref(t)), "j3d_tune_get")
        out.append(t.as_tuple())
    return out


def _tune(t):
    if t is None:
        return None
    if isinstance(t, Tune):
        return t
    t = tuple(int(v) for v in t)
    if len(t) == 5:  # one wavefront along x
        t = t + (1,)
    return Tune(*t)


def _grids(grids):
    arr = (Grid * len(grids))()
    for k, (ua, ub, f, h) in enumerate(grids):
        arr[k].u_a = ua.desc()
        arr[k].u_b = ub.desc()
        arr[k].f = f.desc()
        arr[k].h = float(h)
    return arr


def jacobi3d_sweep_batch(grids, nsweeps: int, resid_every: int = 1, resid_out=None, tune=None, stream=None):
    """``grids``: list of (u_a, u_b, f, h).  ``resid_out``: device float64 tensor or None."""
    arr = _grids(grids)
    t = _tune(tune)
    ptr = None if resid_out is None else ctypes.c_void_p(resid_out.data_ptr())
    _check(_lib.jacobi3d_sweep_batch(len(grids), arr, int(nsweeps), int(resid_every), ptr,
                                     None if t is None else ctypes.byref(t), _stream_handle(stream)),
           "jacobi3d_sweep_batch")


def j3d_autotune(grids, stream=None):
    arr = _grids(grids)
    t = Tune()
    _check(_lib.j3d_autotune(len(grids), arr, ctypes.byref(t), _stream_handle(stream)), "j3d_autotune")
    return t.as_tuple()


def j3d_batch_last_plan():
    """(sweeps per pass, tile shape) of this thread's most recent jacobi3d_sweep_batch call."""
    k = ctypes.c_int32()
    t = Tune()
    _check(_lib.j3d_batch_last_plan(ctypes.byref(k), ctypes.byref(t)), "j3d_batch_last_plan")
    return k.value, t.as_tuple()


def j3d_autotune_single(dtype, nx, ny, nz, stream=None):
    t = Tune()
    _check(_lib.j3d_autotune_single(dtype, nx, ny, nz, ctypes.byref(t), _stream_handle(stream)),
           "j3d_autotune_single")
    return t.as_tuple()


def j3d_tune_query_single(kind, nx, ny, nz):
    """The tile shape single-grid calls of this kind and shape use now."""
    t = Tune()
    _check(_lib.j3d_tune_query_single(kind, nx, ny, nz, ctypes.byref(t)), "j3d_tune_query_single")
    return t.as_tuple()


def j3d_tune_set_single(dtype, nx, ny, nz, tune):
    t = _tune(tune)
    _check(_lib.j3d_tune_set_single(dtype, nx, ny, nz, ctypes.byref(t)), "j3d_tune_set_single")


def j3d_fill_uniform(a: FArray, seed: int, stream_id: int, lo: float, hi: float, halo: float = 0.0, stream=None):
    d = a.desc()
    _check(_lib.j3d_fill_uniform(ctypes.byref(d), seed, stream_id, lo, hi, halo, _stream_handle(stream)),
           "j3d_fill_uniform")


def j3d_fill_const(a: FArray, value: float, stream=None):
    d = a.desc()
    _check(_lib.j3d_fill_const(ctypes.byref(d), value, _stream_handle(stream)), "j3d_fill_const")


def j3d_bandwidth_probe(src: torch.Tensor, dst: torch.Tensor, reps: int = 10, stream=None) -> float:
    g = ctypes.c_double()
    n = min(src.numel(), dst.numel())
    _check(_lib.j3d_bandwidth_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, reps,
                                    ctypes.byref(g), _stream_handle(stream)), "j3d_bandwidth_probe")
    return g.value


def j3d_bandwidth_probe_triad(a: torch.Tensor, b: torch.Tensor, dst: torch.Tensor, reps: int = 10,
                              stream=None) -> float:
    g = ctypes.c_double()
    n = min(a.numel(), b.numel(), dst.numel())
    _check(_lib.j3d_bandwidth_probe_triad(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                          ctypes.c_void_p(dst.data_ptr()), n, reps, ctypes.byref(g),
                                          _stream_handle(stream)), "j3d_bandwidth_probe_triad")
    return g.value


def j3d_release_cache():
    _check(_lib.j3d_release_cache(), "j3d_release_cache")


def j3d_request_bytes(nx, ny, nz) -> int:
    return int(_lib.j3d_request_bytes(nx, ny, nz))


def j3d_request_state_bytes(precision, nx, ny, nz) -> int:
    return int(_lib.j3d_request_state_bytes(precision, nx, ny, nz))


class Server:
    """poisson_serve_* over a server handle."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, cycle_sweeps: int = 50,
                 device: int = 0, queue_cap: int = 100000, max_active_points: int = 0,
                 precision: int = SERVE_MIXED):
        self._h = ctypes.c_void_p()
        o = ServeOpts(int(hbm_budget_bytes), max_slots, cycle_sweeps, device, queue_cap, int(max_active_points),
                      int(precision), 0)
        _check(_lib.poisson_serve_create(ctypes.byref(o), ctypes.byref(self._h)), "poisson_serve_create")
        self._keep = {}

    def submit(self, n, h, rtol, max_sweeps, seed=0, f_host: np.ndarray | None = None,
               u_out: np.ndarray | None = None, ny=None, nz=None):
        nx = n
        ny = n if ny is None else ny
        nz = n if nz is None else nz
        r = Request()
        r.nx, r.ny, r.nz, r.reserved = nx, ny, nz, 0
        r.h, r.seed, r.rtol, r.max_sweeps = float(h), int(seed), float(rtol), int(max_sweeps)
        keep = []
        if f_host is not None:
            fh = np.ascontiguousarray(f_host, dtype=np.float64)
            keep.append(fh)
            r.f_host = fh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if u_out is not None:
            if u_out.dtype != np.float64 or not u_out.flags.c_contiguous or u_out.shape != (nz + 2, ny + 2, nx + 2):
                raise ValueError("u_out must be a C-contiguous float64 array of shape (nz+2, ny+2, nx+2)")
            keep.append(u_out)
            r.u_host = u_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        t = ctypes.c_uint64()
        _check(_lib.poisson_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "poisson_serve_submit")
        if u_out is not None:
            self._keep[t.value] = keep
        return t.value

    def poll(self, cap: int = 1024):
        buf = (Result * cap)()
        n = ctypes.c_int32()
        _check(_lib.poisson_serve_poll(self._h, buf, cap, ctypes.byref(n)), "poisson_serve_poll")
        out = []
        for k in range(n.value):
            r = buf[k]
            self._keep.pop(r.ticket, None)
            out.append(dict(ticket=r.ticket, status=r.status, converged=bool(r.converged), sweeps=r.sweeps,
                            resid=r.resid, norm_f=r.norm_f, t_submit=r.t_submit, t_admit=r.t_admit,
                            t_done=r.t_done))
        return out

    def drain(self, timeout_s: float = 0.0):
        _check(_lib.poisson_serve_drain(self._h, timeout_s), "poisson_serve_drain")

    def stats(self):
        now, a, q, f = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib.poisson_serve_stats(self._h, ctypes.byref(now), ctypes.byref(a), ctypes.byref(q),
                                        ctypes.byref(f)), "poisson_serve_stats")
        return dict(now=now.value, active=a.value, queued=q.value, finished=f.value)

    def close(self):
        if self._h:
            _check(_lib.poisson_serve_destroy(self._h), "poisson_serve_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
