"""Pins of the oracle's WENO advection (the periodic xy advection variant of
Sec. 4.3; fifth-order Hamilton-Jacobi WENO upwinded by the velocity sign).

Each pin fixes a part of the oracle independently of its own formulas:
fifth-order convergence on a smooth field (the candidate coefficients and
the weights), exactness on a locally quadratic field where the three
smoothness indicators are equal (the optimal weights reduce the scheme to
the fifth-order upwind finite difference, whose weights fd_weights derives
in exact rationals), the non-oscillatory response to a jump (the smoothness
indicators), the upwind window (the sign convention), and the x/y symmetry
under transposition (the orientation of the y derivative).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.fdweights import as_floats, fd_weights


def periodic_x(n):
    return np.arange(n) * 2 * math.pi / n


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_fifth_order_convergence_on_a_smooth_field(sign):
    """phi = sin(x + 0.3), u = +-1: the error of u phi_x against u cos(x +
    0.3) falls 2^5 times per halving of dx (measured ratios 31.6-32.0)."""
    errs = []
    for n in (20, 40, 80, 160):
        x = periodic_x(n)
        phi = np.tile(np.sin(x + 0.3), (6, 1))
        u = np.full_like(phi, sign)
        out = oracle.weno_adv(phi, u, np.zeros_like(phi), 2 * math.pi / n, 1.0)
        errs.append(np.abs(out - sign * np.cos(x + 0.3)).max())
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(orders) > 4.8, orders
    assert errs[-1] < 2e-8


def test_exact_on_a_locally_quadratic_field():
    """On a quadratic the one-sided differences are linear, the three
    smoothness indicators are equal, the weights are the optimal 1/10, 6/10,
    3/10 and the scheme is the fifth-order upwind-biased difference, exact
    for quadratics.  Away from the periodic seam of a field that is
    quadratic over most of the period, phi_x must equal both the exact
    derivative and that difference with fd_weights' rational weights."""
    n = 64
    h = 2 * math.pi / n
    x = np.arange(n) * h
    a, b, c = 0.7, -1.3, 0.2
    row = a * x * x + b * x + c
    phi = np.tile(row, (6, 1))
    for sign, offsets in ((1.0, range(-3, 3)), (-1.0, range(-2, 4))):
        u = np.full_like(phi, sign)
        px, _ = oracle.weno_derivatives(phi, u, np.ones_like(phi), h, 1.0)
        w = as_floats(fd_weights(1, list(offsets)))
        for i in range(8, n - 8):
            lin = sum(wk * row[i + o] for wk, o in zip(w, offsets)) / h
            assert px[2, i] == pytest.approx(2 * a * x[i] + b, rel=1e-12, abs=1e-11)
            assert px[2, i] == pytest.approx(lin, rel=1e-12, abs=1e-11)


def test_non_oscillatory_at_a_jump():
    """A unit step (two jumps on the periodic line): phi_x vanishes (to
    rounding) wherever one candidate stencil avoids the jump, i.e.
    everywhere except the cell of each jump, where the value lies between 0
    and the jump over dx (no overshoot), with opposite signs at the two
    jumps; a linear fifth-order difference instead rings over six cells."""
    n = 64
    h = 2 * math.pi / n
    x = periodic_x(n)
    phi = np.tile((x >= math.pi).astype(float), (6, 1))
    for sign in (1.0, -1.0):
        u = np.full_like(phi, sign)
        px, _ = oracle.weno_derivatives(phi, u, np.ones_like(phi), h, 1.0)
        d = px[3] * h
        jumps = [0, n // 2] if sign > 0 else [n - 1, n // 2 - 1]
        others = np.delete(d, jumps)
        assert np.abs(others).max() < 1e-9
        up, down = d[n // 2 if sign > 0 else n // 2 - 1], d[0 if sign > 0 else n - 1]
        assert 0.5 < up <= 1.0 and -1.0 <= down < -0.5


def test_upwind_window():
    """With u > 0, phi_x at i reads phi at i-3 .. i+2 only (backward
    differences at i-2 .. i+2); with u < 0, at i-2 .. i+3."""
    rng = np.random.default_rng(11)
    phi = rng.uniform(-1, 1, (8, 16))
    i, j = 7, 3
    for sign, untouched in ((1.0, i + 3), (-1.0, i - 3)):
        u = np.full_like(phi, sign)
        v = np.zeros_like(phi)
        base = oracle.weno_adv(phi, u, v, 0.3, 0.4)[j, i]
        q = phi.copy()
        q[j, untouched] += 5.0
        assert oracle.weno_adv(q, u, v, 0.3, 0.4)[j, i] == base
        inside = i + 2 if sign > 0 else i - 2
        q = phi.copy()
        q[j, inside] += 5.0
        assert oracle.weno_adv(q, u, v, 0.3, 0.4)[j, i] != base


def test_transpose_symmetry_and_velocity_scaling():
    """Transposing the field and swapping u and v transposes the result (with
    dx = dy); the term is linear in the velocities at fixed signs and zero
    where they vanish."""
    rng = np.random.default_rng(12)
    phi = rng.uniform(-1, 1, (24, 40))
    u = rng.uniform(-1, 1, phi.shape)
    v = rng.uniform(-1, 1, phi.shape)
    out = oracle.weno_adv(phi, u, v, 0.25, 0.25)
    outT = oracle.weno_adv(phi.T.copy(), v.T.copy(), u.T.copy(), 0.25, 0.25)
    assert np.array_equal(out, outT.T)
    assert np.allclose(oracle.weno_adv(phi, 2 * u, 2 * v, 0.25, 0.25), 2 * out, rtol=1e-14, atol=1e-14)
    assert np.array_equal(oracle.weno_adv(phi, 0 * u, 0 * v, 0.25, 0.25), np.zeros_like(phi))
