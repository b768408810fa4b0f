"""Pins of the oracle's ADI Cahn-Hilliard step (Sec. 5.1).

CPU only.  The closed forms follow from the discrete Fourier symbols of the
second-order central differences of Sec. 5.1: on the mode cos(kx) cos(ly),
the 5-point Laplacian acts as -(Sx + Sy), Sx = 4 sin^2(k dx/2)/dx^2, the
biharmonic as (Sx + Sy)^2, d_xxxx as Sx^2, and the ADI operator L_x L_y as
(1 + a Sx^2)(1 + a Sy^2) with a = 2/3 D gamma dt.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1902_09931_amd import workloads as wl
from tests.conftest import golden


def _S(kappa, h):
    return 4.0 * math.sin(kappa * h / 2) ** 2 / h ** 2


def _grid(ny, nx):
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    y, x = np.meshgrid(np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    return x, y, dx, dy


def test_first_step_spectral_closed_form():
    """One nonlinear step from C^{-1} = C^0 = A cos(kx) cos(ly) (the start rule
    of Sec. 5.1): Cbar = C^0, the difference term vanishes, and every one of
    the modes (pk, ql), p, q in {1, 3}, created by the cubic is updated by a
    scalar formula.  Pins the biharmonic window, the nonlinear Laplacian,
    the signs and factors of the right-hand side and the two line solves."""
    p = golden("ch_parameters.json")
    D, gamma = p["D"], p["gamma"]
    ny, nx = 32, 48
    x, y, dx, dy = _grid(ny, nx)
    A, k, l = 0.6, 2, 3
    dt = 0.1 * dx
    c0 = A * np.cos(k * x) * np.cos(l * y)
    got = oracle.ch_step(c0, c0, dx, dy, dt, D, gamma)

    a = 2.0 / 3.0 * D * gamma * dt
    F = {(1, 1): 9 * A ** 3 / 16 - A, (1, 3): 3 * A ** 3 / 16, (3, 1): 3 * A ** 3 / 16,
         (3, 3): A ** 3 / 16}
    expect = c0.copy()
    for (pp, qq), f in F.items():
        sx, sy = _S(pp * k, dx), _S(qq * l, dy)
        r = 2.0 / 3.0 * D * dt * (-(sx + sy)) * f
        if (pp, qq) == (1, 1):
            r += -a * (sx + sy) ** 2 * A
        v = r / ((1 + a * sx ** 2) * (1 + a * sy ** 2))
        expect += v * np.cos(pp * k * x) * np.cos(qq * l * y)
    assert np.abs(got - expect).max() <= 1e-14 * np.abs(c0).max() * 10


def test_linear_problem_follows_scalar_recurrence():
    """Without the cubic term one mode evolves by the scalar recurrence
        abar = 2 a_n - a_{n-1},
        a_{n+1} = abar + (-2/3 (a_n - a_{n-1}) - a s4 abar) / ((1 + a Sx^2)(1 + a Sy^2)),
    s4 = (Sx + Sy)^2, over many steps and from unequal levels (exercises the
    difference term)."""
    ny, nx = 16, 20
    x, y, dx, dy = _grid(ny, nx)
    k, l = 3, 2
    D, gamma, dt = 1.0, 0.05, 0.02
    mode = np.cos(k * x + 0.3) * np.cos(l * y - 0.2)
    a0, am1 = 0.8, 0.9
    cp, cc = oracle.ch_run(am1 * mode, a0 * mode, 50, dx, dy, dt, D, gamma, nonlinear=False)
    aa = 2.0 / 3.0 * D * gamma * dt
    sx, sy = _S(k, dx), _S(l, dy)
    an, anm1 = a0, am1
    for _ in range(50):
        abar = 2 * an - anm1
        v = (-2.0 / 3.0 * (an - anm1) - aa * (sx + sy) ** 2 * abar) / ((1 + aa * sx ** 2) * (1 + aa * sy ** 2))
        anm1, an = an, abar + v
    assert np.abs(cc - an * mode).max() < 1e-13
    assert np.abs(cp - anm1 * mode).max() < 1e-13


def test_mass_is_conserved():
    """Periodic stencils with zero-sum weights and line operators with unit
    row sums make M^{n+1} = M^n + (M^n - M^{n-1})/3, so M stays at M^0 from
    the start rule C^{-1} = C^0 (Sec. 5.1): drift only from rounding."""
    n = 64
    c0 = wl.ch_initial(n, n, seed=2)
    dx = wl.ch_grid_spacing(n)
    cp, cc = oracle.ch_run(c0, c0, 200, dx, dx, 0.1 * dx * dx)
    drift = abs(oracle.mass(cc) - oracle.mass(c0)) / np.abs(c0).sum()
    assert drift < 1e-13
    assert np.abs(cc - c0).max() > 1e-3        # the field did evolve


def test_second_order_convergence_in_time():
    """For the linear problem (the hyperdiffusion scheme the method is built
    on, Sec. 5.1) started from exact levels, the error at fixed T shrinks
    four-fold when dt halves.  This holds only when the right-hand
    biharmonic carries the factor D gamma of the equation and of L_x:
    without it the scheme is consistent with a different equation."""
    ny = nx = 16
    x, y, dx, dy = _grid(ny, nx)
    D, gamma = 1.0, 0.01
    k, l = 1, 1
    lam = D * gamma * (_S(k, dx) + _S(l, dy)) ** 2      # semi-discrete decay rate
    mode = np.cos(k * x) * np.cos(l * y)
    T = 10.0
    errs = []
    for nsteps in (20, 40, 80, 160):
        dt = T / nsteps
        cp, cc = oracle.ch_run(math.exp(lam * dt) * mode, mode.copy(), nsteps, dx, dy, dt, D,
                               gamma, nonlinear=False)
        errs.append(np.abs(cc - math.exp(-lam * T) * mode).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.9 < r < 4.1 for r in ratios), errs
    assert errs[-1] < 1e-6 * math.exp(-lam * T)


@pytest.mark.parametrize("shape", [(24, 40), (33, 17)])
def test_rectangular_grids_solve_each_direction(shape):
    """On a rectangular grid the x and y operators use their own spacing; a
    mode constant in y is driven by the x operators only."""
    ny, nx = shape
    x, y, dx, dy = _grid(ny, nx)
    k = 2
    mode = np.cos(k * x)
    D, gamma, dt = 1.0, 0.01, 0.05
    cp, cc = oracle.ch_run(mode, mode, 3, dx, dy, dt, D, gamma, nonlinear=False)
    aa = 2.0 / 3.0 * D * gamma * dt
    sx = _S(k, dx)
    an, anm1 = 1.0, 1.0
    for _ in range(3):
        abar = 2 * an - anm1
        v = (-2.0 / 3.0 * (an - anm1) - aa * sx ** 2 * abar) / (1 + aa * sx ** 2)
        anm1, an = an, abar + v
    assert np.abs(cc - an * mode).max() < 1e-14


# --- the stored-precision form (reduced-precision reading) -------------------

def test_storage_rounding_is_nearest_even():
    """round_storage: float rounding equals NumPy's float32 cast; bfloat16
    rounding equals torch's float32 -> bfloat16 conversion (round to nearest
    even) on float values, and takes the documented ties: halfway between
    two bfloat16 values goes to the even one, just above halfway goes up."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))
    assert np.array_equal(oracle.round_storage(x, "f32"), x.astype(np.float32).astype(np.float64))
    xf = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(xf.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(oracle.round_storage(xf, "bf16"), ref)
    ulp = 2.0 ** -7
    ties = np.array([1 + ulp / 2, 1 + 3 * ulp / 2, -(1 + ulp / 2), 1 + ulp / 2 + 2.0 ** -40, 0.0])
    assert list(oracle.round_storage(ties, "bf16")) == [1.0, 1 + 2 * ulp, -1.0, 1 + ulp, 0.0]


def test_stored_step_rounds_the_stored_quantities():
    """The stored-precision step: storage "f64" is the plain step bit for
    bit; with "f32" or "bf16" every value of C^{n+1} is a value of that dtype,
    and after one step the result lies within the rounding of its storage
    (plus the float rounding of R and w carried through the two solves) of
    the double-precision step."""
    ny, nx = 40, 48
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    dt = 0.1 * dx * dx
    c0 = 0.1 * np.random.default_rng(8).uniform(-1, 1, (ny, nx))
    plain = oracle.ch_step(c0, c0, dx, dy, dt)
    assert np.array_equal(oracle.ch_step_stored(c0, c0, dx, dy, dt, "f64"), plain)
    for storage, u in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        cs = oracle.round_storage(c0, storage)
        ref = oracle.ch_step(cs, cs, dx, dy, dt)
        got = oracle.ch_step_stored(cs, cs, dx, dy, dt, storage)
        assert np.array_equal(oracle.round_storage(got, storage), got)
        # C^{n+1} rounded once (u |C|), w and R rounded to float and carried
        # through the two solves (each inverse has infinity norm about 1.1:
        # the sum of |entries| of the inverse of the symbol 1 + 16 beta sin^4)
        assert np.all(np.abs(got - ref) <= u * np.abs(ref) + 64 * 2.0 ** -24 * np.abs(c0).max())
        if storage == "bf16":
            assert np.abs(got - ref).max() > 2.0 ** -24 * np.abs(ref).max()


def test_stored_run_continues_the_stored_step():
    ny, nx = 24, 32
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    dt = 0.1 * dx * dx
    c0 = oracle.round_storage(0.1 * np.random.default_rng(9).uniform(-1, 1, (ny, nx)), "bf16")
    cp, cc = c0, c0
    for _ in range(5):
        cp, cc = cc, oracle.ch_step_stored(cp, cc, dx, dy, dt, "bf16")
    rp, rc = oracle.ch_run_stored(c0, c0, 5, dx, dy, dt, "bf16")
    assert np.array_equal(rc, cc) and np.array_equal(rp, cp)


def test_nudged_run_is_a_one_ulp_perturbation():
    """ch_run_nudged moves every coefficient of the step by one ulp: its run
    differs from ch_run, by no more than a few roundings of the step's terms
    per step, is fixed by its seed, and differs between seeds."""
    ny, nx = 32, 48
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    dt = 0.1 * dx * dx
    c0 = 0.1 * np.random.default_rng(4).uniform(-1, 1, (ny, nx))
    _, ref = oracle.ch_run(c0, c0, 6, dx, dy, dt)
    _, a = oracle.ch_run_nudged(c0, c0, 6, dx, dy, dt, seed=1)
    _, a2 = oracle.ch_run_nudged(c0, c0, 6, dx, dy, dt, seed=1)
    _, b = oracle.ch_run_nudged(c0, c0, 6, dx, dy, dt, seed=2)
    assert np.array_equal(a, a2)
    assert not np.array_equal(a, b)
    d = np.abs(a - ref).max()
    assert 0 < d <= 6 * 64 * 2.0 ** -52 * np.abs(c0).max(), d
    with pytest.raises(ValueError):
        oracle.ch_run_nudged(c0, c0, 1, dx, dy, dt, seed=0)
