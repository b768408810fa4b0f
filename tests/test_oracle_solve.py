"""Pins of the oracle's cyclic banded solves (the periodic line inversions of
the ADI step, Sec. 5.1).

CPU only.  Independent routes to the same answer: dense Gaussian elimination
(numpy.linalg.solve) on the circulant built by scipy.linalg.circulant, the
FFT diagonalisation of a circulant, and the closed-form eigenvalues on
Fourier modes.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle


def _dense_circulant(bands, n):
    """Circulant whose row i holds bands[d+bw] at column (i+d) mod n."""
    bw = (len(bands) - 1) // 2
    col0 = np.zeros(n)
    for d in range(-bw, bw + 1):
        col0[(-d) % n] += bands[d + bw]   # scipy: C[i, j] = c[(i - j) mod n]
    return sla.circulant(col0)


def _lines(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)


@pytest.mark.parametrize("bands", [
    [-1.0, 2.5, -1.0],                        # the batched tridiagonal system, sigma = 0.5
    [0.3, 4.0, -1.2],                         # non-symmetric, diagonally dominant
    [17.7, -70.8, 107.2, -70.8, 17.7],        # I + beta*[1,-4,6,-4,1], beta = 17.7
    [0.5, -1.0, 5.0, 0.7, -0.2],              # non-symmetric pentadiagonal
])
def test_cyclic_solve_matches_dense_solve(bands):
    bw = (len(bands) - 1) // 2
    lengths = [n for n in (3, 4, 5, 7, 16, 64, 129, 256) if n >= 2 * bw + 1]
    off = _lines(lengths)
    r = np.random.default_rng(21).uniform(-1, 1, off[-1])
    x = oracle.cyclic_solve_batch(bands, off, r)
    for b, n in enumerate(lengths):
        A = _dense_circulant(bands, n)
        ref = np.linalg.solve(A, r[off[b]:off[b + 1]])
        got = x[off[b]:off[b + 1]]
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), n
        assert np.abs(A @ got - r[off[b]:off[b + 1]]).max() < 1e-13 * np.abs(A).sum(1).max() * np.abs(got).max() * n


@pytest.mark.parametrize("n", [1000, 4096])
def test_cyclic_solve_matches_fft_diagonalisation(n):
    bands = oracle.circulant_bands([1 + 6 * 283.0, -4 * 283.0, 283.0])
    r = np.random.default_rng(22).uniform(-1, 1, n)
    x = oracle.cyclic_solve_batch(bands, np.array([0, n]), r)
    col0 = _dense_circulant(bands, n)[:, 0]
    ref = np.real(np.fft.ifft(np.fft.fft(r) / np.fft.fft(col0)))
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,m", [(64, 1), (65, 7), (4096, 1000), (300, 150)])
def test_fourier_mode_eigenvalues(n, m):
    """cos(2 pi m j / n) is an eigenvector: tridiagonal circ(-1, 2+sigma, -1)
    has eigenvalue 2 + sigma - 2 cos(2 pi m/n); the pentadiagonal
    circ(b, -4b, 1+6b, -4b, b) has 1 + 16 b sin^4(pi m/n)."""
    j = np.arange(n)
    r = np.cos(2 * math.pi * m * j / n)
    sigma, beta = 0.5, 283.0
    x = oracle.cyclic_solve_batch([-1.0, 2 + sigma, -1.0], np.array([0, n]), r)
    lam = 2 + sigma - 2 * math.cos(2 * math.pi * m / n)
    assert np.abs(x - r / lam).max() < 1e-14 * n
    x = oracle.cyclic_solve_batch(oracle.circulant_bands([1 + 6 * beta, -4 * beta, beta]),
                                  np.array([0, n]), r)
    lam = 1 + 16 * beta * math.sin(math.pi * m / n) ** 4
    assert np.abs(x - r / lam).max() < 1e-13 / lam * n


def test_grid_solves_along_rows_and_columns():
    """Row and column solves of a grid equal the line solves of its rows and
    of its columns (dense references)."""
    ny, nx = 9, 12
    bands = oracle.circulant_bands([1 + 6 * 2.0, -4 * 2.0, 2.0])
    r = np.random.default_rng(23).uniform(-1, 1, (ny, nx))
    xr = oracle.cyclic_solve_grid(bands, 1, r)
    xc = oracle.cyclic_solve_grid(bands, 0, r)
    Ax, Ay = _dense_circulant(bands, nx), _dense_circulant(bands, ny)
    assert np.abs(xr - np.linalg.solve(Ax, r.T).T).max() < 1e-14
    assert np.abs(xc - np.linalg.solve(Ay, r)).max() < 1e-14


def test_mass_sum_is_compensated():
    """The mass sum agrees with math.fsum (exactly rounded) where a plain
    left-to-right sum would not."""
    x = np.array([1e16, 1.0, -1e16, 1.0, 3.0, 1e-3] * 1000)
    u = 2.0 ** -53
    exact = math.fsum(x)
    # Neumaier's bound: 2u|S| + O(n u^2) sum|x|; a plain sum loses whole units here.
    bound = 2 * u * abs(exact) + 2 * x.size * u * u * np.abs(x).sum()
    assert abs(oracle.mass(x) - exact) <= bound
    assert abs(float(np.cumsum(x)[-1]) - exact) > 1.0
    y = np.random.default_rng(24).uniform(-0.1, 0.1, 1 << 16)
    assert abs(oracle.mass(y) - math.fsum(y)) <= 1e-18
