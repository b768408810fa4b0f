"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws and lays out input data: grids, random fields, signal
lengths and the stencil coefficient tables fed to the library.  It performs
none of the method's arithmetic.

Input recipe (the paper uses no dataset: its examples differentiate
trigonometric fields and its Cahn-Hilliard runs start from uniform random
data in (-0.1, 0.1), Sec. 4 and Sec. 5.3):

  seed 0  256 x 256 field sin(2 pi x) sin(2 pi y) + 1e-3 U(-1, 1) on [0,1)^2
  seed 1  8192 x 8192 field c ~ U(-1, 1)
  seed 2  Cahn-Hilliard initial data 0.1 U(-1, 1), 1024^2 and 4096^2
  seed 3  65536 signal lengths ~ U{64..4096}
  seed 4  signal values ~ U(-1, 1)
  seed 5  right-hand sides of the batched cyclic solves ~ U(-1, 1)
  seed 6  ensemble grid sizes: multiples of 32 in [256, 1024]
  seed 7  ensemble initial data 0.1 U(-1, 1)

All draws are numpy.random.default_rng(seed) in float64 on the host.
"""
import math

import numpy as np

# Stencil coefficient tables used as inputs (per unit spacing).
D2_2ND = (1.0, -2.0, 1.0)                             # second derivative, 2nd order
D2_4TH = (-1.0 / 12, 16.0 / 12, -30.0 / 12, 16.0 / 12, -1.0 / 12)   # 2nd deriv, 4th order
D1_4TH = (1.0 / 12, -8.0 / 12, 0.0, 8.0 / 12, -1.0 / 12)            # 1st deriv, 4th order
CROSS_XXYY = ((1.0, -2.0, 1.0), (-2.0, 4.0, -2.0), (1.0, -2.0, 1.0))  # Fig. 1 window
LAPLACE_3X3 = ((0.0, 1.0, 0.0), (1.0, -4.0, 1.0), (0.0, 1.0, 0.0))    # 5-point, dx = dy
CUBIC_MINUS_LINEAR = (0.0, -1.0, 0.0, 1.0)            # f(c) = c^3 - c as coefficients


def scaled(table, factor):
    """A coefficient table multiplied by a scalar (e.g. 1/dx**2)."""
    return np.asarray(table, dtype=np.float64) * factor


def periodic_field_cfg0(n=256, seed=0):
    """u = sin(2 pi x) sin(2 pi y) + 1e-3 U(-1,1) on an n x n grid of [0,1)^2;
    returns (u, smooth part, dx)."""
    dx = 1.0 / n
    x = np.arange(n) * dx
    smooth = np.outer(np.sin(2 * math.pi * x), np.sin(2 * math.pi * x))
    noise = 1e-3 * np.random.default_rng(seed).uniform(-1.0, 1.0, (n, n))
    return smooth + noise, smooth, dx


def uniform_grid(ny, nx, lo=-1.0, hi=1.0, seed=1):
    return np.random.default_rng(seed).uniform(lo, hi, (ny, nx))


def ragged_lengths(nbatch=65536, lo=64, hi=4096, seed=3):
    """Signal lengths ~ U{lo..hi} and the back-to-back offsets (int64, nbatch+1)."""
    lengths = np.random.default_rng(seed).integers(lo, hi + 1, nbatch, dtype=np.int64)
    offsets = np.zeros(nbatch + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    return lengths, offsets


def ragged_values(total, seed=4):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, total)


def ch_initial(ny, nx, seed=2, amplitude=0.1):
    """Deep-quench initial data amplitude * U(-1, 1) (Sec. 5.3)."""
    return amplitude * np.random.default_rng(seed).uniform(-1.0, 1.0, (ny, nx))


def ch_grid_spacing(n):
    """Spacing of n nodes on the periodic interval [0, 2 pi) (Sec. 5.1)."""
    return 2.0 * math.pi / n


def ensemble_sizes(count=64, lo=256, hi=1024, step=32, seed=6):
    choices = np.arange(lo, hi + 1, step)
    return [int(v) for v in np.random.default_rng(seed).choice(choices, count)]


def ensemble_initial(sizes, seed=7, amplitude=0.1):
    rng = np.random.default_rng(seed)
    return [amplitude * rng.uniform(-1.0, 1.0, (n, n)) for n in sizes]
