"""Pins of the oracle's multi-input window-function form (Sec. 4.2).

The function receives each input's window in window order plus loc, the
position of the point itself.  Pinned against closed forms (pointwise
products, the Sec. 4.1/4.2 example on sin x) and against the independently
pinned weighted-sum stencil of the C oracle (linear functions of one or two
inputs, which must reproduce a weighted stencil exactly up to rounding)."""
import math

import numpy as np
import pytest

import oracle
from oracle.window import stencil2d_window_multi


def test_pointwise_product_of_two_inputs():
    rng = np.random.default_rng(1)
    u, v = rng.uniform(-1, 1, (7, 9)), rng.uniform(-1, 1, (7, 9))
    for periodic in (True, False):
        out = stencil2d_window_multi([u, v], 1, 2, 1, 1, lambda w, c, loc: c[0] * w[0][loc] * w[1][loc],
                                     [3.0], periodic)
        ref = 3.0 * u * v
        if not periodic:
            mask = np.zeros_like(u, dtype=bool)
            mask[1:-1, 1:-2] = True
            assert np.array_equal(out[~mask], np.zeros_like(u)[~mask])
            out, ref = out[mask], ref[mask]
        assert np.array_equal(out, ref)


def test_central_difference_relative_to_loc():
    """The second-order central difference written relative to loc, on sin x:
    -(4/dx^2) sin^2(dx/2) sin x exactly (the Sec. 4.2 example's closed form)."""
    nx = 64
    dx = 2 * math.pi / nx
    x = np.arange(nx) * dx
    u = np.tile(np.sin(x), (3, 1))
    out = stencil2d_window_multi([u], 1, 1, 0, 0,
                                 lambda w, c, loc: c[0] * (w[0][loc - 1] - 2 * w[0][loc] + w[0][loc + 1]),
                                 [1 / dx ** 2], True)
    ref = -(4 / dx ** 2) * math.sin(dx / 2) ** 2 * np.sin(x)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max() / dx


@pytest.mark.parametrize("ext", [(1, 1, 1, 1), (2, 0, 1, 2), (0, 3, 0, 0)])
@pytest.mark.parametrize("periodic", [True, False])
def test_linear_functions_reproduce_weighted_stencils(ext, periodic):
    """sum_k w_k u_k + sum_k z_k v_k over the windows equals the C oracle's
    weighted stencils of u and v added, in the window index convention."""
    L, R, T, B = ext
    rng = np.random.default_rng(sum(ext) + periodic)
    u, v = rng.uniform(-1, 1, (9, 11)), rng.uniform(-1, 1, (9, 11))
    n = (L + R + 1) * (T + B + 1)
    wu, wv = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    out = stencil2d_window_multi([u, v], L, R, T, B,
                                 lambda w, c, loc: float(np.dot(wu, w[0]) + np.dot(wv, w[1])), [], periodic)
    ref = oracle.stencil2d(u, L, R, T, B, wu, periodic) + oracle.stencil2d(v, L, R, T, B, wv, periodic)
    assert np.allclose(out, ref, rtol=0, atol=1e-14)
