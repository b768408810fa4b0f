"""Pins of the oracle's stencils against what the paper and the mathematics fix.

CPU only.  Each test states what it pins: the printed weights of the paper,
its worked examples, discrete Fourier symbols (closed forms), polynomial
exactness, single-tap shifts that reduce to numpy.roll, and linearity.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import fd_weights
from oracle.window import stencil2d_window
from paper_1902_09931_amd import workloads as wl
from tests.conftest import golden


# --- weights --------------------------------------------------------------

def test_fd_weights_reproduce_printed_central_differences():
    """The moment-system derivation reproduces the two central differences
    printed in Sec. 5.1 and the cross stencil of Fig. 1 (outer product of
    the printed second differences)."""
    g = golden("central_differences.json")
    assert fd_weights(2, g["d2"]["offsets"]) == [Fraction(v) for v in g["d2"]["weights"]]
    assert fd_weights(4, g["d4"]["offsets"]) == [Fraction(v) for v in g["d4"]["weights"]]
    fig1 = np.array(golden("fig1_cross_stencil.json")["weights"], dtype=float)
    d2 = np.array([float(v) for v in fd_weights(2, [-1, 0, 1])])
    assert np.array_equal(fig1, np.outer(d2, d2))


@pytest.mark.parametrize("m,half", [(2, 4), (1, 2), (2, 2), (4, 3)])
def test_fd_weights_moment_conditions(m, half):
    """Exactness on monomials a**q for q below the number of points."""
    offs = list(range(-half, half + 1))
    w = fd_weights(m, offs)
    for q in range(len(offs)):
        lhs = sum(wa * Fraction(a) ** q for wa, a in zip(w, offs))
        assert lhs == (math.factorial(m) if q == m else 0)


# --- the paper's worked examples ------------------------------------------

def test_example_2d_x_np_standard_weights():
    """Sec. 4.1: 8th-order 9-point d2/dx2 of sin(x) on 1024 x 512, lx = 2 pi,
    non-periodic; the answer is -sin(x) and the 4 cells on each side stay
    0.0 because the output was zeroed."""
    g = golden("example_2d_x_np.json")
    nx, ny, L, R = g["nx"], g["ny"], g["numStenLeft"], g["numStenRight"]
    dx = 2 * math.pi / nx
    w = oracle.as_floats(fd_weights(2, range(-L, R + 1)), dx, 2)
    assert len(w) == g["numSten"]
    x = np.arange(nx) * dx
    u = np.tile(np.sin(x), (ny, 1))
    out = np.zeros_like(u)
    oracle.stencil2d(u, L, R, 0, 0, w, periodic=False, out=out)
    nb = g["boundary_cells_each_side"]
    assert np.all(out[:, :nb] == g["boundary_value"])
    assert np.all(out[:, nx - nb:] == g["boundary_value"])
    inner = out[:, nb:nx - nb]
    # truncation ~ dx^8 (negligible); rounding ~ sum|w| * eps * |u|.
    assert np.abs(inner + np.sin(x[nb:nx - nb])).max() < 5e-10


def test_example_2d_x_np_fun_window_function():
    """Sec. 4.2: the second-order central difference supplied as a function
    with one coefficient 1/dx^2.  The discrete answer is exactly
    -(4/dx^2) sin^2(dx/2) sin(x), within dx^2/12 of -sin(x).  The window form
    agrees with the polynomial point-function form (identity f, weights
    [1,-2,1] * coe)."""
    g = golden("example_2d_x_np_fun.json")
    nx = g["nx"]
    dx = 2 * math.pi / nx
    x = np.arange(nx) * dx
    u = np.tile(np.sin(x), (2, 1))      # every row is the same x-line

    def central_difference(win, coe):
        return (win[0, 0] - 2.0 * win[0, 1] + win[0, 2]) * coe[0]

    out = stencil2d_window(u, 1, 1, 0, 0, central_difference, [1.0 / dx ** 2], periodic=False)
    inner = out[:, 1:-1]
    discrete = -(4.0 / dx ** 2) * math.sin(dx / 2) ** 2 * np.sin(x[1:-1])
    assert np.abs(inner - discrete).max() < 1e-9
    assert np.abs(inner + np.sin(x[1:-1])).max() < dx ** 2 / 12 * 1.01 + 1e-9
    assert np.all(out[:, 0] == 0.0) and np.all(out[:, -1] == 0.0)
    poly = oracle.stencil2d(u, 1, 1, 0, 0, [1.0, -2.0, 1.0], periodic=False, coe=[0.0, 1.0 / dx ** 2])
    assert np.abs(poly - out).max() < 1e-9


# --- closed forms (discrete Fourier symbols) ------------------------------

def test_cfg0_second_derivative_symbol():
    """256^2 periodic X stencil [1,-2,1]/dx^2 on sin(2 pi x) sin(2 pi y) + noise:
    the smooth part is an eigenfunction with eigenvalue -4 sin^2(pi dx)/dx^2,
    within (pi dx)^2/3 of the continuous -4 pi^2; the noise part enters
    linearly."""
    u, smooth, dx = wl.periodic_field_cfg0()
    w = wl.scaled(wl.D2_2ND, 1.0 / dx ** 2)
    s_u = oracle.stencil2d(u, 1, 1, 0, 0, w, True)
    s_smooth = oracle.stencil2d(smooth, 1, 1, 0, 0, w, True)
    s_noise = oracle.stencil2d(u - smooth, 1, 1, 0, 0, w, True)
    sigma = -4.0 * math.sin(math.pi * dx) ** 2 / dx ** 2
    assert np.abs(s_smooth - sigma * smooth).max() < 1e-9
    assert abs(sigma + 4 * math.pi ** 2) / (4 * math.pi ** 2) <= (math.pi * dx) ** 2 / 3
    assert np.abs(s_u - s_smooth - s_noise).max() < 1e-9


def _symbol(w, left, right, top, bottom, k, l, nx, ny):
    w = np.asarray(w, dtype=float).reshape(top + bottom + 1, left + right + 1)
    s = 0j
    for b in range(-top, bottom + 1):
        for a in range(-left, right + 1):
            s += w[b + top, a + left] * np.exp(2j * math.pi * (k * a / nx + l * b / ny))
    return s


@pytest.mark.parametrize("ext", [(2, 1, 1, 2), (0, 3, 2, 0), (1, 1, 0, 0), (0, 0, 3, 1)])
def test_asymmetric_window_symbol(ext):
    """Any window acting on the Fourier mode exp(i(k x + l y)) multiplies it by
    its symbol sum_ab w_ab exp(i(k a dx + l b dy)).  Running the oracle on cos
    and sin of the phase pins the index convention (top = smaller j, weights
    counted from the top left, left to right, row by row: Sec. 5.3), since a
    flipped or transposed window changes the symbol."""
    L, R, T, B = ext
    ny, nx = 10, 12
    rng = np.random.default_rng(11)
    w = rng.uniform(-1, 1, (T + B + 1) * (L + R + 1))
    k, l = 3, 2
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    theta = 2 * math.pi * (k * ii / nx + l * jj / ny)
    sc = oracle.stencil2d(np.cos(theta), L, R, T, B, w, True)
    ss = oracle.stencil2d(np.sin(theta), L, R, T, B, w, True)
    expect = _symbol(w, L, R, T, B, k, l, nx, ny) * np.exp(1j * theta)
    assert np.abs((sc + 1j * ss) - expect).max() < 1e-13


def test_fig1_cross_symbol():
    """Fig. 1 / (dx^2 dy^2) has the symbol 16 sin^2(k dx/2) sin^2(l dy/2)/(dx^2 dy^2),
    the product of the two second-difference symbols, and tends to
    d4/dx2dy2 of cos(kx)cos(ly) = k^2 l^2 cos cos."""
    fig1 = np.array(golden("fig1_cross_stencil.json")["weights"], dtype=float)
    ny, nx = 24, 40
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    k, l = 2, 3
    y, x = np.meshgrid(np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    u = np.cos(k * x) * np.cos(l * y)
    out = oracle.stencil2d(u, 1, 1, 1, 1, fig1 / (dx * dx * dy * dy), True)
    sym = 16 * math.sin(k * dx / 2) ** 2 * math.sin(l * dy / 2) ** 2 / (dx * dx * dy * dy)
    assert np.abs(out - sym * u).max() < 1e-11
    # second-order truncation: relative error below ((k dx)^2 + (l dy)^2) / 12
    assert abs(sym - k * k * l * l) / (k * k * l * l) < ((k * dx) ** 2 + (l * dy) ** 2) / 12


# --- special cases that reduce to library routines ------------------------

@pytest.mark.parametrize("a,b", [(2, 0), (-1, 0), (0, 2), (0, -3), (1, -2), (-2, 1)])
def test_single_tap_is_a_roll(a, b):
    """A window with one nonzero weight at offset (a, b) returns the input
    shifted: out[j, i] = w * u[j+b, i+a] = w * roll(u, (-b, -a))."""
    L, R, T, B = max(-a, 0), max(a, 0), max(-b, 0), max(b, 0)
    w = np.zeros((T + B + 1, L + R + 1))
    w[b + T, a + L] = 2.5
    u = np.random.default_rng(5).uniform(-1, 1, (9, 11))
    out = oracle.stencil2d(u, L, R, T, B, w, True)
    assert np.array_equal(out, 2.5 * np.roll(u, (-b, -a), axis=(0, 1)))


def test_single_tap_non_periodic_interior_and_untouched_border():
    u = np.random.default_rng(6).uniform(-1, 1, (9, 11))
    L, R, T, B = 0, 2, 1, 0
    w = np.zeros((2, 3))
    w[0, 2] = 1.0                       # offset (a, b) = (2, -1)
    out = np.full_like(u, np.nan)
    oracle.stencil2d(u, L, R, T, B, w, False, out=out)
    assert np.array_equal(out[1:, :9], u[:-1, 2:])
    assert np.all(np.isnan(out[0, :])) and np.all(np.isnan(out[:, 9:]))


# --- polynomial exactness --------------------------------------------------

def test_polynomial_exactness_non_periodic():
    """Order-p stencils for the m-th derivative are exact on polynomials of
    degree <= p + m - 1, on the interior; the boundary cells stay untouched."""
    ny, nx = 17, 19
    h = 0.1
    y, x = np.meshgrid(np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
    d2 = oracle.as_floats(fd_weights(2, range(-2, 3)), h, 2)         # 4th order
    u = x ** 5 - 2 * x ** 3 + x ** 2
    out = np.full_like(u, np.nan)
    oracle.stencil2d(u, 2, 2, 0, 0, d2, False, out=out)
    assert np.abs(out[:, 2:-2] - (20 * x ** 3 - 12 * x + 2)[:, 2:-2]).max() < 1e-9
    assert np.all(np.isnan(out[:, :2])) and np.all(np.isnan(out[:, -2:]))
    # y direction, asymmetric one-sided first derivative (offsets 0..3, 3rd order)
    d1 = oracle.as_floats(fd_weights(1, range(0, 4)), h, 1)
    v = y ** 3 + y
    out = np.full_like(v, np.nan)
    oracle.stencil2d(v, 0, 0, 0, 3, d1, False, out=out)
    assert np.abs(out[:-3] - (3 * y ** 2 + 1)[:-3]).max() < 1e-10
    assert np.all(np.isnan(out[-3:]))
    # xy: the corner cross derivative on x^2 y^2 + x y gives 4xy + 1 exactly
    cross = np.array([[1, 0, -1], [0, 0, 0], [-1, 0, 1]]) / (4 * h * h)
    p = x ** 2 * y ** 2 + x * y
    out = np.full_like(p, np.nan)
    oracle.stencil2d(p, 1, 1, 1, 1, cross, False, out=out)
    assert np.abs(out[1:-1, 1:-1] - (4 * x * y + 1)[1:-1, 1:-1]).max() < 1e-10
    fig1 = np.array(golden("fig1_cross_stencil.json")["weights"], dtype=float) / h ** 4
    out = oracle.stencil2d(x ** 2 * y ** 2, 1, 1, 1, 1, fig1, False)
    assert np.abs(out[1:-1, 1:-1] - 4.0).max() < 1e-8


# --- point function ---------------------------------------------------------

def test_point_function_laplacian_of_cubic():
    """lap_h (u^3 - u) for u = A cos(kx) cos(ly): the cubic splits into the
    modes (p k, q l), p, q in {1, 3} (cos^3 = (3 cos + cos 3)/4), each scaled
    by the 5-point Laplacian symbol -(Sx + Sy), Sx = 4 sin^2(p k dx/2)/dx^2."""
    ny, nx = 32, 48
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    A, k, l = 0.7, 2, 3
    y, x = np.meshgrid(np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    u = A * np.cos(k * x) * np.cos(l * y)
    lap = np.zeros((5, 5))
    lap[2, 1:4] += np.array([1, -2, 1]) / dx ** 2
    lap[1:4, 2] += np.array([1, -2, 1]) / dy ** 2
    out = oracle.stencil2d(u, 2, 2, 2, 2, lap, True, coe=wl.CUBIC_MINUS_LINEAR)

    def S(kappa, h):
        return 4 * math.sin(kappa * h / 2) ** 2 / h ** 2

    F = {(1, 1): 9 * A ** 3 / 16 - A, (1, 3): 3 * A ** 3 / 16, (3, 1): 3 * A ** 3 / 16,
         (3, 3): A ** 3 / 16}
    expect = sum(-(S(p * k, dx) + S(q * l, dy)) * c * np.cos(p * k * x) * np.cos(q * l * y)
                 for (p, q), c in F.items())
    assert np.abs(out - expect).max() < 1e-12 * np.abs(expect).max() * 100


# --- linearity and shift equivariance ---------------------------------------

def test_linearity_and_shift_equivariance():
    rng = np.random.default_rng(8)
    u, v = rng.uniform(-1, 1, (2, 13, 17))
    w = rng.uniform(-1, 1, (3, 5))
    S = lambda z: oracle.stencil2d(z, 2, 2, 1, 1, w, True)
    assert np.abs(S(2.0 * u - 3.0 * v) - (2.0 * S(u) - 3.0 * S(v))).max() < 1e-13
    assert np.array_equal(S(np.roll(u, (3, -5), axis=(0, 1))), np.roll(S(u), (3, -5), axis=(0, 1)))


# --- ragged 1D ---------------------------------------------------------------

def test_ragged_first_derivative_symbol_per_signal():
    """Each signal wraps onto itself: with h = 2 pi / n and u = sin(m x), the
    4th-order first derivative returns (8 sin(mh) - sin(2mh))/(6h) cos(m x)."""
    lengths = np.array([5, 64, 65, 97, 200], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    ms = [1, 3, 7, 2, 11]
    vals = np.concatenate([np.sin(m * np.arange(n) * 2 * math.pi / n) for n, m in zip(lengths, ms)])
    w = np.array([float(v) for v in fd_weights(1, range(-2, 3))])
    out = oracle.stencil1d_batch(vals, offs, 2, 2, w, True)
    outs = np.zeros_like(vals)
    for b, (n, m) in enumerate(zip(lengths, ms)):
        h = 2 * math.pi / n
        x = np.arange(n) * h
        expect = (8 * math.sin(m * h) - math.sin(2 * m * h)) / (6 * h) * np.cos(m * x)
        got = out[offs[b]:offs[b + 1]] / h
        assert np.abs(got - expect).max() < 1e-12 / h
        outs[offs[b]:offs[b + 1]] = 1
    # non-periodic: L and R cells of each signal untouched
    out = np.full_like(vals, np.nan)
    oracle.stencil1d_batch(vals, offs, 2, 2, w, False, out=out)
    for b in range(len(lengths)):
        seg = out[offs[b]:offs[b + 1]]
        assert np.all(np.isnan(seg[:2])) and np.all(np.isnan(seg[-2:]))
        assert not np.any(np.isnan(seg[2:-2]))


# --- the point-sampled definition and the workload tables -------------------

@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("ext,coe", [((2, 2, 0, 0), None), ((0, 0, 1, 3), None),
                                     ((2, 1, 2, 1), None), ((1, 1, 1, 1), (0.0, -1.0, 0.0, 1.0))])
def test_stencil2d_at_equals_the_whole_grid_definition(ext, coe, periodic):
    """orc_stencil2d_at (the reference of the sampled full-size parity tests)
    returns, at random, corner and border points, exactly the values of
    orc_stencil2d over the whole grid, and marks as unwritten exactly the
    cells that the whole-grid call leaves untouched."""
    L, R, T, B = ext
    rng = np.random.default_rng(31)
    ny, nx = 41, 57
    u = rng.uniform(-1, 1, (ny, nx))
    w = rng.uniform(-1, 1, (L + R + 1) * (T + B + 1))
    full = np.full_like(u, np.nan)
    oracle.stencil2d(u, L, R, T, B, w, periodic, coe=coe, out=full)
    js = np.concatenate([rng.integers(0, ny, 400), [0, 0, ny - 1, ny - 1],
                         np.arange(ny), np.full(nx, T), np.full(nx, ny - 1 - B)])
    is_ = np.concatenate([rng.integers(0, nx, 400), [0, nx - 1, 0, nx - 1],
                          np.full(ny, L), np.arange(nx), np.arange(nx)])
    vals, written = oracle.stencil2d_at(u, L, R, T, B, w, periodic, js, is_, coe=coe)
    expect = full[js, is_]
    assert np.array_equal(written, ~np.isnan(expect))
    assert np.array_equal(vals[written], expect[written])
    assert periodic or not written.all()


def test_workload_weight_tables_are_the_derived_stencils():
    """The coefficient tables the workloads feed to the library are the
    moment-system weights: D2_4TH the 5-point 4th-order second derivative,
    D1_4TH the 5-point 4th-order first derivative, D2_2ND the 3-point
    second difference, LAPLACE_3X3 the x and y second differences summed
    in a 3x3 window (dx = dy), CROSS_XXYY the outer product of two second
    differences (Fig. 1)."""
    d2_4 = [float(v) for v in fd_weights(2, range(-2, 3))]
    d1_4 = [float(v) for v in fd_weights(1, range(-2, 3))]
    d2_2 = [float(v) for v in fd_weights(2, range(-1, 2))]
    assert list(wl.D2_4TH) == d2_4
    assert list(wl.D1_4TH) == d1_4
    assert list(wl.D2_2ND) == d2_2
    lap = np.zeros((3, 3))
    lap[1, :] += d2_2
    lap[:, 1] += d2_2
    assert np.array_equal(np.array(wl.LAPLACE_3X3), lap)
    assert np.array_equal(np.array(wl.CROSS_XXYY), np.outer(d2_2, d2_2))
    # the 4th-order label: the second-derivative table is exact on monomials
    # up to degree p + m - 1 = 5 ...
    h = np.arange(-2, 3, dtype=float)
    for q in range(6):
        target = 2.0 if q == 2 else 0.0
        assert abs(np.dot(d2_4, h ** q) - target) < 1e-12, q
    # ... and not on x^6 (so it is 4th order, not higher)
    assert abs(np.dot(d2_4, h ** 6)) > 1.0
