"""The general window-function form of the "Fun" stencils, with Python loops.

TEST INFRASTRUCTURE (part of the oracle).  In the paper the user function is
handed the input data, its coefficients and the location of the current point
inside the window, and returns the output value for that point (Sec. 4.2).
Here the function receives the window itself, a (top+bottom+1) x
(left+right+1) array whose element [b+top, a+left] is the input at offset
(a, b), plus the coefficient list.  Small grids only.
"""
import numpy as np


def stencil2d_window(u, left, right, top, bottom, fun, coe, periodic, out=None):
    u = np.asarray(u, dtype=np.float64)
    ny, nx = u.shape
    if out is None:
        out = np.zeros_like(u)
    win = np.empty((top + bottom + 1, left + right + 1))
    for j in range(ny):
        for i in range(nx):
            if not periodic and (i < left or i > nx - 1 - right
                                 or j < top or j > ny - 1 - bottom):
                continue  # boundary cells stay untouched (Sec. 3)
            for b in range(-top, bottom + 1):
                for a in range(-left, right + 1):
                    J = (j + b) % ny if periodic else j + b
                    I = (i + a) % nx if periodic else i + a
                    win[b + top, a + left] = u[J, I]
            out[j, i] = fun(win, coe)
    return out


def stencil2d_window_multi(inputs, left, right, top, bottom, fun, coe, periodic, out=None):
    """The window-function form over several input grids of one shape (the
    multi-input function variants of Sec. 4.2: the function takes one data
    set per input).  fun(wins, coe, loc) receives, per input, the window
    flattened in window order (row by row from the top left, left to right:
    element (b+top)*(left+right+1) + (a+left) is the input at offset (a, b)),
    the coefficients, and loc = top*(left+right+1) + left, the position of
    the point itself, so that the function indexes relative to loc as the
    paper's does.  Boundary cells of a non-periodic grid stay untouched."""
    us = [np.asarray(u, dtype=np.float64) for u in inputs]
    ny, nx = us[0].shape
    if any(u.shape != (ny, nx) for u in us):
        raise ValueError("inputs must share one shape")
    if out is None:
        out = np.zeros_like(us[0])
    width = left + right + 1
    loc = top * width + left
    wins = [np.empty((top + bottom + 1) * width) for _ in us]
    for j in range(ny):
        for i in range(nx):
            if not periodic and (i < left or i > nx - 1 - right
                                 or j < top or j > ny - 1 - bottom):
                continue
            for b in range(-top, bottom + 1):
                for a in range(-left, right + 1):
                    J = (j + b) % ny if periodic else j + b
                    I = (i + a) % nx if periodic else i + a
                    for w, u in zip(wins, us):
                        w[(b + top) * width + (a + left)] = u[J, I]
            out[j, i] = fun(wins, coe, loc)
    return out
