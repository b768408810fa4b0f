"""Pins of the oracle's coarsening diagnostics (Sec. 5.3) against what the
mathematics fixes.  CPU only."""
import math

import numpy as np
import pytest

from oracle.diagnostics import coarsening_k1, coarsening_s, simpson_mean


def test_simpson_mean_is_the_composite_rule_over_one_period():
    """The periodic weights equal SciPy's composite Simpson rule over the
    closed period [0, N h] with the end node set to node 0, divided by the
    period, in each direction."""
    integrate = pytest.importorskip("scipy.integrate")
    rng = np.random.default_rng(4)
    ny, nx = 10, 16
    f = rng.uniform(-1, 1, (ny, nx))
    closed = np.concatenate([f, f[:1]], axis=0)
    closed = np.concatenate([closed, closed[:, :1]], axis=1)
    hx, hy = 0.3, 0.7
    inner = integrate.simpson(closed, x=np.arange(nx + 1) * hx, axis=1)
    total = integrate.simpson(inner, x=np.arange(ny + 1) * hy)
    assert simpson_mean(f) == pytest.approx(total / (nx * hx * ny * hy), rel=1e-14)


def test_simpson_mean_closed_forms():
    """Exact on low trigonometric modes (the mean of cos^2 3x cos^2 2y is
    1/4), and weights 2/3, 4/3: an alternating field averages to -1/3 (the
    trapezoid rule would give 0)."""
    n = 64
    x = np.arange(n) * 2 * math.pi / n
    f = np.outer(np.cos(2 * x) ** 2, np.cos(3 * x) ** 2)
    assert simpson_mean(f) == pytest.approx(0.25, abs=1e-15)
    alt = np.tile((-1.0) ** np.arange(n), (n, 1))
    assert simpson_mean(alt) == pytest.approx(-1.0 / 3.0, abs=1e-15)
    assert simpson_mean(np.full((6, 8), 0.3)) == pytest.approx(0.3, abs=1e-15)
    with pytest.raises(ValueError):
        simpson_mean(np.ones((5, 8)))


def test_s_of_uniform_fields():
    for a in (0.0, 0.5, -0.9):
        assert coarsening_s(np.full((8, 8), a)) == pytest.approx(1.0 / (1.0 - a * a), rel=1e-15)


@pytest.mark.parametrize("shape", [(32, 32), (64, 48)])
def test_k1_closed_forms(shape):
    """Single modes give their own wavenumber; two modes of equal amplitude
    at |k| = 3 and 4 give 24/7 (the ratio of 2 + 2 to 2/3 + 2/4); the mean
    does not enter; on a domain of length 4 pi the index-2 mode has k = 1."""
    ny, nx = shape
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    y, x = np.meshgrid(np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    assert coarsening_k1(np.cos(3 * x), dx, dy) == pytest.approx(3.0, rel=1e-13)
    assert coarsening_k1(0.7 + np.cos(3 * x) * np.cos(4 * y), dx, dy) == pytest.approx(5.0, rel=1e-13)
    assert coarsening_k1(np.cos(3 * x) + np.sin(4 * y), dx, dy) == pytest.approx(24.0 / 7.0, rel=1e-13)
    big = 4 * math.pi / nx
    xb = np.arange(nx) * big
    assert coarsening_k1(np.tile(np.cos(xb), (ny, 1)), big, dy) == pytest.approx(1.0, rel=1e-13)
