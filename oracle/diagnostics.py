"""Coarsening diagnostics of a Cahn-Hilliard state (Sec. 5.3), in plain NumPy.

TEST INFRASTRUCTURE (part of the oracle): only the test suite and the
CPU-baseline leg of the benchmark use it.

* ``simpson_mean(f, ...)``: the spatial average of a periodic grid function by
  Simpson's rule.  The composite rule over one period [0, N h] (N even) with
  the end node identified with node 0 gives node i the weight 2h/3 (i even)
  or 4h/3 (i odd); dividing by the period length N h gives average weights
  2/3 and 4/3.  Along both axes the weights multiply.
* ``coarsening_s(c)``: s = 1 / (1 - <C^2>).
* ``coarsening_k1(c, dx, dy)``: k1 = sum |C^(k)|^2 / sum |k|^-1 |C^(k)|^2, with
  C^ the discrete Fourier transform (NumPy's FFT as the transform step) and
  the sums over every nonzero wavevector k = (2 pi mx / (nx dx),
  2 pi my / (ny dy)); the integral over k of the paper becomes the sum over
  the grid's modes (the constant mode spacing cancels in the ratio), and the
  k = 0 mode, where |k|^-1 is undefined, is left out (reading).
"""
import numpy as np


def simpson_weights(n):
    """Average weights of Simpson's rule on a periodic grid of n (even) nodes."""
    if n % 2:
        raise ValueError("Simpson's rule on a periodic grid needs an even number of nodes")
    return np.where(np.arange(n) % 2 == 0, 2.0, 4.0) / 3.0


def simpson_mean(f):
    """<f> over a periodic grid shaped (ny, nx) by Simpson's rule in both
    directions."""
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape
    return float(simpson_weights(ny) @ f @ simpson_weights(nx)) / (nx * ny)


def coarsening_s(c):
    """s(t) = 1 / (1 - <C^2>) (Sec. 5.3)."""
    c = np.asarray(c, dtype=np.float64)
    return 1.0 / (1.0 - simpson_mean(c * c))


def coarsening_k1(c, dx, dy):
    """k1(t) = sum |C^|^2 / sum |k|^-1 |C^|^2 over the nonzero wavevectors
    (Sec. 5.3)."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    power = np.abs(np.fft.fft2(c)) ** 2
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    kmag = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    nz = kmag > 0
    return float(power[nz].sum() / (power[nz] / kmag[nz]).sum())
