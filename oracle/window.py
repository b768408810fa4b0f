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
