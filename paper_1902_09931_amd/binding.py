"""Python binding of the C ABI in include/mxsten.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device buffers
may be given as torch tensors (their data_ptr() is passed) or as integer
device addresses; streams as torch.cuda.Stream, integer hipStream_t, or None
for torch's current stream.  Host arrays (weights, coefficients, offsets)
may be any sequence or NumPy array.  A nonzero status raises MxsError with
the library's message.  All compute happens in libmxsten.so: when the library
is missing this module raises at import time.
"""
import ctypes
import os

import numpy as np

# torch (ROCm) ships its own copy of the HIP runtime under the same soname
# as the system one.  Loading torch first makes the library bind to that
# copy, so that torch's tensors and the library's kernels share one runtime;
# loaded the other way round, the process would hold two runtimes.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_LIBPATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmxsten.so")
if not os.path.exists(_LIBPATH):
    raise ImportError(f"{_LIBPATH} is missing: build it with `python -m paper_1902_09931_amd.build`")
_lib = ctypes.CDLL(_LIBPATH)

MXS_OK = 0
MXS_ERR_INVALID_ARG = -1
MXS_ERR_ALIAS = -2
MXS_ERR_UNSUPPORTED = -3
MXS_ERR_HIP = -4
MXS_ERR_OOM = -5
MXS_ERR_NONFINITE = -6
MXS_ERR_BAD_HANDLE = -7

MXS_X, MXS_Y, MXS_XY = 0, 1, 2
MXS_NP, MXS_P = 0, 1
MXS_F64, MXS_F32, MXS_BF16 = 0, 1, 2
MXS_LINES_RAGGED, MXS_LINES_ROWS, MXS_LINES_COLS = 0, 1, 2
MXS_CH_SEPARATE, MXS_CH_PERSISTENT, MXS_CH_FUSED = 0, 1, 2


class MxsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{mxs_status_string(status)}: {message}")
        self.status = status


class mxs_stencil2d_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("ld", ctypes.c_longlong),
                ("dir", ctypes.c_int), ("bc", ctypes.c_int), ("dtype", ctypes.c_int),
                ("left", ctypes.c_int), ("right", ctypes.c_int),
                ("top", ctypes.c_int), ("bottom", ctypes.c_int),
                ("weights", ctypes.POINTER(ctypes.c_double)),
                ("coe", ctypes.POINTER(ctypes.c_double)), ("ncoe", ctypes.c_int),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_int = ctypes.c_int
_ll = ctypes.c_longlong
_dp = ctypes.POINTER(ctypes.c_double)
_llp = ctypes.POINTER(ctypes.c_longlong)
_ip = ctypes.POINTER(ctypes.c_int)

class mxs_stencil2d_fn_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("ld", ctypes.c_longlong),
                ("dir", ctypes.c_int), ("bc", ctypes.c_int), ("dtype", ctypes.c_int),
                ("left", ctypes.c_int), ("right", ctypes.c_int),
                ("top", ctypes.c_int), ("bottom", ctypes.c_int),
                ("ninputs", ctypes.c_int), ("inputs", ctypes.POINTER(ctypes.c_void_p)),
                ("out", ctypes.c_void_p),
                ("coe", ctypes.POINTER(ctypes.c_double)), ("ncoe", ctypes.c_int),
                ("source", ctypes.c_char_p), ("name", ctypes.c_char_p)]


_SIGS = {
    "mxs_create_2d": [ctypes.POINTER(mxs_stencil2d_desc), ctypes.POINTER(_vp)],
    "mxs_create_2d_fn": [ctypes.POINTER(mxs_stencil2d_fn_desc), ctypes.POINTER(_vp)],
    "mxs_create_1d_batch": [_int, _llp, _int, _int, _int, _int, _dp, _dp, _int, _vp, _vp,
                            ctypes.POINTER(_vp)],
    "mxs_create_cyclic_solve": [_int, _dp, _int, _int, _int, _ll, _int, _llp, _int, _vp, _vp,
                                ctypes.POINTER(_vp)],
    "mxs_compute": [_vp, _vp],
    "mxs_swap": [_vp],
    "mxs_set_io": [_vp, _vp, _vp],
    "mxs_ch_create": [_int, _int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                      ctypes.c_double, ctypes.c_double, _int, _vp, _vp, _vp, ctypes.POINTER(_vp)],
    "mxs_ch_ensemble_create": [_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                               _int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                               ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "mxs_ch_step": [_vp, _int, _int, _vp],
    "mxs_ch_state": [_vp, _int, ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "mxs_ch_steps_taken": [_vp, _llp],
    "mxs_ch_mass": [_vp, _dp, _vp],
    "mxs_create_weno_adv": [_int, _int, _ll, ctypes.c_double, ctypes.c_double, _int, _vp, _vp, _vp, _vp,
                            ctypes.POINTER(_vp)],
    "mxs_ch_coarsening": [_vp, _int, _dp, _dp, _vp],
    "mxs_ch_set_step_mode": [_vp, _int],
    "mxs_ch_coarsening_noalloc": [_vp, _int, _dp, _dp, _vp],
    "mxs_destroy": [_vp],
    "mxs_autotune": [_vp, _vp],
    "mxs_plan_info": [_vp, ctypes.c_char_p, _int],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _int
_lib.mxs_last_error.restype = ctypes.c_char_p
_lib.mxs_last_error.argtypes = []
_lib.mxs_status_string.restype = ctypes.c_char_p
_lib.mxs_status_string.argtypes = [_int]
_lib.mxs_version.restype = _int
_lib.mxs_version.argtypes = []


def library_path():
    return _LIBPATH


def mxs_last_error():
    return _lib.mxs_last_error().decode()


def mxs_status_string(status):
    return _lib.mxs_status_string(int(status)).decode()


def mxs_version():
    return _lib.mxs_version()


def _check(status):
    if status != MXS_OK:
        raise MxsError(status, mxs_last_error())


def _ptr(buf):
    if buf is None:
        return None
    if hasattr(buf, "data_ptr"):
        return buf.data_ptr()
    return int(buf)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _dbl_array(values):
    if values is None:
        return None, 0
    a = np.ascontiguousarray(np.asarray(values, dtype=np.float64).ravel())
    return a, a.size


def _as_dp(arr):
    return None if arr is None else arr.ctypes.data_as(_dp)


def dtype_code(t):
    """MXS dtype code of a torch dtype or tensor."""
    import torch
    dt = t.dtype if hasattr(t, "dtype") else t
    return {torch.float64: MXS_F64, torch.float32: MXS_F32, torch.bfloat16: MXS_BF16}[dt]


# --- stencils ----------------------------------------------------------------

def mxs_create_2d(nx, ny, ld, dir, bc, dtype, left, right, top, bottom, weights, coe, in_, out):
    w, _ = _dbl_array(weights)
    c, nc = _dbl_array(coe)
    d = mxs_stencil2d_desc(nx, ny, ld, dir, bc, dtype, left, right, top, bottom, _as_dp(w),
                           _as_dp(c), nc, _ptr(in_), _ptr(out))
    plan = _vp()
    _check(_lib.mxs_create_2d(ctypes.byref(d), ctypes.byref(plan)))
    return plan.value


def mxs_create_2d_fn(nx, ny, ld, dir, bc, dtype, left, right, top, bottom, inputs, out, coe, source,
                     name):
    """Stencil with a user function compiled at plan creation (HIP source
    defining `__device__ mxs_real name(const mxs_real *const *w, const
    mxs_real *coe, int loc)`), over one or more inputs."""
    ins = (ctypes.c_void_p * len(inputs))(*[_ptr(t) for t in inputs])
    c, nc = _dbl_array(coe)
    d = mxs_stencil2d_fn_desc(nx, ny, ld, dir, bc, dtype, left, right, top, bottom, len(inputs),
                              ctypes.cast(ins, ctypes.POINTER(ctypes.c_void_p)), _ptr(out), _as_dp(c), nc,
                              source.encode(), name.encode())
    plan = _vp()
    _check(_lib.mxs_create_2d_fn(ctypes.byref(d), ctypes.byref(plan)))
    return plan.value


def mxs_create_weno_adv(nx, ny, ld, dx, dy, dtype, phi, u, v, out):
    """WENO advection plan (out = u phi_x + v phi_y, periodic)."""
    plan = _vp()
    _check(_lib.mxs_create_weno_adv(nx, ny, ld, dx, dy, dtype, _ptr(phi), _ptr(u), _ptr(v), _ptr(out),
                                    ctypes.byref(plan)))
    return plan.value


def mxs_create_1d_batch(offsets, bc, dtype, left, right, weights, coe, in_, out):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    w, _ = _dbl_array(weights)
    c, nc = _dbl_array(coe)
    plan = _vp()
    _check(_lib.mxs_create_1d_batch(off.size - 1, off.ctypes.data_as(_llp), bc, dtype, left, right,
                                    _as_dp(w), _as_dp(c), nc, _ptr(in_), _ptr(out),
                                    ctypes.byref(plan)))
    return plan.value


def mxs_create_cyclic_solve(bw, coef, geometry, nx, ny, ld, offsets, dtype, rhs, x):
    c, _ = _dbl_array(coef)
    if offsets is not None:
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        nb, offp = off.size - 1, off.ctypes.data_as(_llp)
    else:
        nb, offp = 0, None
    plan = _vp()
    _check(_lib.mxs_create_cyclic_solve(bw, _as_dp(c), geometry, nx, ny, ld, nb, offp, dtype,
                                        _ptr(rhs), _ptr(x), ctypes.byref(plan)))
    return plan.value


def mxs_compute(plan, stream=None):
    _check(_lib.mxs_compute(plan, _stream(stream)))


def mxs_swap(plan):
    _check(_lib.mxs_swap(plan))


def mxs_set_io(plan, in_, out):
    _check(_lib.mxs_set_io(plan, _ptr(in_), _ptr(out)))


def mxs_destroy(plan):
    _check(_lib.mxs_destroy(plan))


def mxs_autotune(plan, stream=None):
    _check(_lib.mxs_autotune(plan, _stream(stream)))


def mxs_plan_info(plan):
    buf = ctypes.create_string_buffer(1024)
    _check(_lib.mxs_plan_info(plan, buf, 1024))
    return buf.value.decode()


# --- Cahn-Hilliard ------------------------------------------------------------

def mxs_ch_create(nx, ny, dx, dy, dt, D, gamma, dtype, c_prev, c_cur, c_next):
    plan = _vp()
    _check(_lib.mxs_ch_create(nx, ny, dx, dy, dt, D, gamma, dtype, _ptr(c_prev), _ptr(c_cur),
                              _ptr(c_next), ctypes.byref(plan)))
    return plan.value


def mxs_ch_ensemble_create(nx, ny, dx, dy, dt, D, gamma, dtype, c_prev, c_cur, c_next):
    n = len(nx)
    ia = lambda v: (ctypes.c_int * n)(*[int(x) for x in v])
    da = lambda v: (ctypes.c_double * n)(*[float(x) for x in v])
    pa = lambda v: (_vp * n)(*[_ptr(x) for x in v])
    plan = _vp()
    _check(_lib.mxs_ch_ensemble_create(n, ia(nx), ia(ny), da(dx), da(dy), da(dt), D, gamma, dtype,
                                       pa(c_prev), pa(c_cur), pa(c_next), ctypes.byref(plan)))
    return plan.value


def mxs_ch_step(plan, nsteps, use_graph=True, stream=None):
    _check(_lib.mxs_ch_step(plan, int(nsteps), int(bool(use_graph)), _stream(stream)))


def mxs_ch_state(plan, k=0):
    """Device addresses (C^{n-1}, C^n) of instance k."""
    p, c = _vp(), _vp()
    _check(_lib.mxs_ch_state(plan, k, ctypes.byref(p), ctypes.byref(c)))
    return p.value, c.value


def mxs_ch_steps_taken(plan):
    n = ctypes.c_longlong()
    _check(_lib.mxs_ch_steps_taken(plan, ctypes.byref(n)))
    return n.value


def mxs_ch_mass(plan, count=1, stream=None):
    out = (ctypes.c_double * count)()
    _check(_lib.mxs_ch_mass(plan, out, _stream(stream)))
    return [out[k] for k in range(count)]


def mxs_ch_coarsening(plan, k=0, stream=None):
    """Coarsening diagnostics (s, k1) of instance k's current state."""
    sv, kv = ctypes.c_double(), ctypes.c_double()
    _check(_lib.mxs_ch_coarsening(plan, k, ctypes.byref(sv), ctypes.byref(kv), _stream(stream)))
    return sv.value, kv.value


def mxs_ch_set_step_mode(plan, mode):
    """MXS_CH_SEPARATE, MXS_CH_PERSISTENT (one launch per step) or MXS_CH_FUSED
    (the right-hand side formed inside the row solves)."""
    _check(_lib.mxs_ch_set_step_mode(plan, mode))


def mxs_ch_coarsening_noalloc(plan, k=0, stream=None):
    """mxs_ch_coarsening on the library's static scratch (allocates nothing)."""
    sv, kv = ctypes.c_double(), ctypes.c_double()
    _check(_lib.mxs_ch_coarsening_noalloc(plan, k, ctypes.byref(sv), ctypes.byref(kv),
                                          _stream(stream)))
    return sv.value, kv.value
