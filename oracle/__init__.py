"""The oracle: a plain, slow, double-precision CPU implementation of the method.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The library never
does, and this package imports nothing from it: the two share no code.

The arithmetic lives in ``oracle.c`` (built by ``oracle/build.py`` into
``liborc.so``); this module converts NumPy arrays for it.  ``fdweights``
derives finite-difference weights in exact rationals and ``window`` evaluates
the paper's general window-function form with Python loops for small grids.

Paper: "cuSten -- CUDA Finite Difference and Stencil Library", Gloster,
O Naraigh, Pham (arXiv 1902.09931).  Each function cites the passage it
follows.
"""
import ctypes
import os

import numpy as np

from .fdweights import as_floats, central_weights, fd_weights  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liborc.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_ll = ctypes.c_longlong
_int = ctypes.c_int
_dbl = ctypes.c_double
_vp = ctypes.c_void_p


def lib():
    """Load liborc.so, building it first when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from .build import build
            build()
        L = ctypes.CDLL(_LIBPATH)
        L.orc_stencil2d.argtypes = [_f64p, _f64p, _ll, _ll, _ll, _int, _int, _int, _int,
                                    _f64p, _int, _vp, _int]
        L.orc_stencil2d_at.argtypes = [_f64p, _ll, _ll, _ll, _int, _int, _int, _int,
                                       _f64p, _int, _vp, _int, _ll, _i64p, _i64p,
                                       _f64p, _i32p]
        L.orc_stencil1d_batch.argtypes = [_f64p, _f64p, _i64p, _ll, _int, _int, _f64p,
                                          _int, _vp, _int]
        L.orc_cyclic_solve_batch.argtypes = [_int, _f64p, _i64p, _ll, _f64p, _f64p]
        L.orc_cyclic_solve_grid.argtypes = [_int, _f64p, _int, _ll, _ll, _ll, _f64p, _f64p]
        L.orc_ch_step.argtypes = [_ll, _ll, _dbl, _dbl, _dbl, _dbl, _dbl, _int,
                                  _f64p, _f64p, _f64p]
        L.orc_ch_run.argtypes = [_ll, _ll, _dbl, _dbl, _dbl, _dbl, _dbl, _int, _ll,
                                 _f64p, _f64p]
        L.orc_ch_step_stored.argtypes = [_ll, _ll, _dbl, _dbl, _dbl, _dbl, _dbl, _int, _int,
                                         _f64p, _f64p, _f64p]
        L.orc_ch_run_stored.argtypes = [_ll, _ll, _dbl, _dbl, _dbl, _dbl, _dbl, _int, _int, _ll,
                                        _f64p, _f64p]
        L.orc_round_storage.argtypes = [_f64p, _f64p, _ll, _int]
        L.orc_ch_run_nudged.argtypes = [_ll, _ll, _dbl, _dbl, _dbl, _dbl, _dbl, _int, _ll,
                                        ctypes.c_ulonglong, _f64p, _f64p]
        L.orc_weno_adv.argtypes = [_f64p, _f64p, _f64p, _f64p, _ll, _ll, _ll, _dbl, _dbl]
        L.orc_weno_derivatives.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p, _ll, _ll, _ll,
                                           _dbl, _dbl]
        L.orc_sum.argtypes = [_f64p, _ll]
        L.orc_sum.restype = _dbl
        for name in ("orc_stencil2d", "orc_stencil2d_at", "orc_stencil1d_batch",
                     "orc_cyclic_solve_batch", "orc_cyclic_solve_grid", "orc_ch_step",
                     "orc_ch_run", "orc_ch_step_stored", "orc_ch_run_stored",
                     "orc_round_storage", "orc_weno_adv", "orc_weno_derivatives",
                     "orc_ch_run_nudged"):
            getattr(L, name).restype = _int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _coe(coe):
    if coe is None or len(coe) == 0:
        return None, 0, None
    c = _f64(coe)
    return c.ctypes.data_as(_vp), len(c), c


def _check(st, what):
    if st != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def stencil2d(u, left, right, top, bottom, weights, periodic, coe=None, out=None):
    """2D stencil (Sec. 3): out[j,i] = sum_{b=-top..bottom} sum_{a=-left..right}
    w[(b+top)*(left+right+1) + a+left] * f(u[j+b, i+a]); periodic wrap, or the
    boundary cells of ``out`` left untouched (non-periodic).  f is the
    polynomial sum_m coe[m] c^m (the "Fun" form, Sec. 4.2) or the identity.

    ``out`` is updated in place when given (so untouched cells keep their
    value); otherwise a zero-filled array is used, as the example of Sec. 4.1
    zeroes its output."""
    u = _f64(u)
    ny, nx = u.shape
    w = _f64(weights).ravel()
    if w.size != (left + right + 1) * (top + bottom + 1):
        raise ValueError("weights size does not match the extents")
    if out is None:
        out = np.zeros_like(u)
    elif not (out.dtype == np.float64 and out.flags.c_contiguous and out.shape == u.shape):
        raise ValueError("out must be a C-contiguous float64 array shaped like u")
    cp, nc, _keep = _coe(coe)
    _check(lib().orc_stencil2d(u, out, nx, ny, nx, left, right, top, bottom, w,
                               int(bool(periodic)), cp, nc), "stencil2d")
    return out


def stencil2d_at(u, left, right, top, bottom, weights, periodic, js, is_, coe=None):
    """The stencil2d definition at chosen points; returns (values, written)."""
    u = _f64(u)
    ny, nx = u.shape
    w = _f64(weights).ravel()
    js = np.ascontiguousarray(js, dtype=np.int64)
    is_ = np.ascontiguousarray(is_, dtype=np.int64)
    vals = np.zeros(js.size, dtype=np.float64)
    written = np.zeros(js.size, dtype=np.int32)
    cp, nc, _keep = _coe(coe)
    _check(lib().orc_stencil2d_at(u, nx, ny, nx, left, right, top, bottom, w,
                                  int(bool(periodic)), cp, nc, js.size, js, is_,
                                  vals, written), "stencil2d_at")
    return vals, written.astype(bool)


def stencil1d_batch(values, offsets, left, right, weights, periodic, coe=None, out=None):
    """Batched 1D stencils over uneven signals stored back to back; signal b
    is values[offsets[b]:offsets[b+1]] and wraps onto itself when periodic
    (the batched 1D form of the abstract)."""
    v = _f64(values)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if out is None:
        out = np.zeros_like(v)
    cp, nc, _keep = _coe(coe)
    _check(lib().orc_stencil1d_batch(v, out, off, off.size - 1, left, right,
                                     _f64(weights).ravel(), int(bool(periodic)), cp, nc),
           "stencil1d_batch")
    return out


def circulant_bands(diag_and_offdiag):
    """Band values a[-bw..bw] of a symmetric circulant from [c0, c1, ..., c_bw]."""
    c = [float(v) for v in diag_and_offdiag]
    return np.array(c[:0:-1] + c, dtype=np.float64)


def cyclic_solve_batch(bands, offsets, r):
    """Solve A_b x_b = r_b for uneven lines stored back to back, A_b the
    circulant of length n_b with rows a[-bw..bw] (the periodic line inversions
    of Sec. 5.1); banded LU without pivoting plus a Woodbury correction for
    the wrapped corners."""
    a = _f64(bands).ravel()
    bw = (a.size - 1) // 2
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    r = _f64(r)
    x = np.zeros_like(r)
    _check(lib().orc_cyclic_solve_batch(bw, a, off, off.size - 1, r, x), "cyclic_solve_batch")
    return x


def cyclic_solve_grid(bands, axis, r):
    """Cyclic solves along every row (axis=1, x) or column (axis=0, y) of a
    2D grid, following NumPy's axis naming for an array shaped (ny, nx)."""
    a = _f64(bands).ravel()
    bw = (a.size - 1) // 2
    r = _f64(r)
    ny, nx = r.shape
    x = np.zeros_like(r)
    _check(lib().orc_cyclic_solve_grid(bw, a, 0 if axis in (1, -1) else 1, nx, ny, nx, r, x),
           "cyclic_solve_grid")
    return x


def ch_step(c_prev, c_cur, dx, dy, dt, D=1.0, gamma=0.01, nonlinear=True):
    """One ADI Cahn-Hilliard step (Sec. 5.1): returns C^{n+1} from C^{n-1},
    C^n on a periodic grid shaped (ny, nx)."""
    cp = _f64(c_prev)
    cc = _f64(c_cur)
    ny, nx = cc.shape
    out = np.zeros_like(cc)
    _check(lib().orc_ch_step(nx, ny, dx, dy, dt, D, gamma, int(bool(nonlinear)), cp, cc, out),
           "ch_step")
    return out


def ch_run(c_prev, c_cur, nsteps, dx, dy, dt, D=1.0, gamma=0.01, nonlinear=True):
    """nsteps ADI steps; returns (C^{n-1}, C^n) after the last one.  The start
    rule of Sec. 5.1 is c_prev = c_cur = C^0."""
    cp = _f64(c_prev).copy()
    cc = _f64(c_cur).copy()
    ny, nx = cc.shape
    _check(lib().orc_ch_run(nx, ny, dx, dy, dt, D, gamma, int(bool(nonlinear)),
                            int(nsteps), cp, cc), "ch_run")
    return cp, cc


def ch_run_nudged(c_prev, c_cur, nsteps, dx, dy, dt, seed, D=1.0, gamma=0.01, nonlinear=True):
    """ch_run with every window weight and band value of the step moved by
    one ulp, up or down by a seeded sequence (seed != 0): another equally
    valid double rounding of the scheme's coefficients."""
    cp = _f64(c_prev).copy()
    cc = _f64(c_cur).copy()
    ny, nx = cc.shape
    _check(lib().orc_ch_run_nudged(nx, ny, dx, dy, dt, D, gamma, int(bool(nonlinear)),
                                   int(nsteps), int(seed), cp, cc), "ch_run_nudged")
    return cp, cc


STORAGE = {"f64": 0, "f32": 1, "bf16": 2}


def round_storage(x, storage):
    """x rounded to the storage dtype ("f32" or "bf16"), nearest value, ties
    to even, in one step from double."""
    x = _f64(x)
    y = np.empty_like(x)
    _check(lib().orc_round_storage(x.ravel(), y.ravel(), x.size, STORAGE[storage]),
           "round_storage")
    return y


def ch_step_stored(c_prev, c_cur, dx, dy, dt, storage, D=1.0, gamma=0.01, nonlinear=True):
    """One ADI step (Sec. 5.1) in double arithmetic whose stored quantities
    are rounded as a reduced-precision implementation stores them: the
    right-hand side R and the x-sweep result w to float, C^{n+1} to the
    storage dtype ("f32" or "bf16"; "f64" is ch_step)."""
    cp = _f64(c_prev)
    cc = _f64(c_cur)
    ny, nx = cc.shape
    out = np.zeros_like(cc)
    _check(lib().orc_ch_step_stored(nx, ny, dx, dy, dt, D, gamma, int(bool(nonlinear)),
                                    STORAGE[storage], cp, cc, out), "ch_step_stored")
    return out


def ch_run_stored(c_prev, c_cur, nsteps, dx, dy, dt, storage, D=1.0, gamma=0.01,
                  nonlinear=True):
    """nsteps of ch_step_stored; returns (C^{n-1}, C^n)."""
    cp = _f64(c_prev).copy()
    cc = _f64(c_cur).copy()
    ny, nx = cc.shape
    _check(lib().orc_ch_run_stored(nx, ny, dx, dy, dt, D, gamma, int(bool(nonlinear)),
                                   STORAGE[storage], int(nsteps), cp, cc), "ch_run_stored")
    return cp, cc


def mass(x):
    """Grid mass sum_ij C_ij with compensated summation."""
    x = _f64(x).ravel()
    return float(lib().orc_sum(x, x.size))


def weno_adv(phi, u, v, dx, dy):
    """The WENO advection variant of Sec. 4.3 on a periodic grid shaped (ny,
    nx): out = u phi_x + v phi_y with fifth-order Hamilton-Jacobi WENO
    derivatives upwinded by the sign of each velocity."""
    phi, u, v = _f64(phi), _f64(u), _f64(v)
    ny, nx = phi.shape
    out = np.zeros_like(phi)
    _check(lib().orc_weno_adv(phi, u, v, out, nx, ny, nx, dx, dy), "weno_adv")
    return out


def weno_derivatives(phi, u, v, dx, dy):
    """The upwind WENO derivatives (phi_x, phi_y) the advection term uses."""
    phi, u, v = _f64(phi), _f64(u), _f64(v)
    ny, nx = phi.shape
    px, py = np.zeros_like(phi), np.zeros_like(phi)
    _check(lib().orc_weno_derivatives(phi, u, v, px, py, nx, ny, nx, dx, dy),
           "weno_derivatives")
    return px, py
