"""GPU parity of stencils with a user function compiled at run time (the
function-pointer variants of Sec. 4.2, several inputs per function) against
the oracle's multi-input window form, evaluated with the same function
written in Python.

FP64 to 1e-12 normwise relative; FP32/BF16 (float arithmetic on the rounded
inputs) within a bound of 64 float roundings of the sum of the magnitudes of
the function's terms plus the final rounding to the storage dtype.
Untouched border cells of non-periodic plans keep their value.
"""
import math

import numpy as np
import pytest

from oracle.window import stencil2d_window_multi
from tests.gpu_util import code, round_to, to_device, to_host, torch

pytestmark = pytest.mark.gpu

b = pytest.importorskip("paper_1902_09931_amd.binding")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DIRS = {"X": b.MXS_X, "Y": b.MXS_Y, "XY": b.MXS_XY}
U_STORE = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8}

CENTRAL = """
__device__ mxs_real central(const mxs_real *const *w, const mxs_real *coe, int loc) {
    return coe[0] * (w[0][loc - 1] - 2 * w[0][loc] + w[0][loc + 1]);
}"""

VARDIFF = """
__device__ mxs_real vardiff(const mxs_real *const *w, const mxs_real *coe, int loc) {
    const mxs_real *c = w[0], *d = w[1];
    const mxs_real fx = (d[loc + 1] + d[loc]) * (c[loc + 1] - c[loc]) - (d[loc] + d[loc - 1]) * (c[loc] - c[loc - 1]);
    const mxs_real fy = (d[loc + 3] + d[loc]) * (c[loc + 3] - c[loc]) - (d[loc] + d[loc - 3]) * (c[loc] - c[loc - 3]);
    return coe[0] * fx + coe[1] * fy;
}"""

CUBIC_LAP = """
__device__ mxs_real cubic(mxs_real c) { return c * c * c - c; }
__device__ mxs_real cubic_lap(const mxs_real *const *w, const mxs_real *coe, int loc) {
    const mxs_real *c = w[0];
    return coe[0] * (cubic(c[loc - 1]) + cubic(c[loc + 1]) + cubic(c[loc - 3]) + cubic(c[loc + 3])
                     - 4 * cubic(c[loc]));
}"""

# three inputs on an asymmetric 4 x 4 window (left 2, right 1, top 1, bottom
# 2): reads the first and last window elements, so the window order shows
CORNERS = """
__device__ mxs_real corners(const mxs_real *const *w, const mxs_real *coe, int loc) {
    return coe[0] * w[0][0] + coe[1] * w[1][15] + w[2][loc] * w[0][loc + 5] - w[1][loc - 2] * coe[2];
}"""


def f_central(w, c, loc):
    return c[0] * (w[0][loc - 1] - 2 * w[0][loc] + w[0][loc + 1])


def m_central(w, c, loc):
    return abs(c[0]) * (abs(w[0][loc - 1]) + 2 * abs(w[0][loc]) + abs(w[0][loc + 1]))


def f_vardiff(w, c, loc):
    x, d = w
    fx = (d[loc + 1] + d[loc]) * (x[loc + 1] - x[loc]) - (d[loc] + d[loc - 1]) * (x[loc] - x[loc - 1])
    fy = (d[loc + 3] + d[loc]) * (x[loc + 3] - x[loc]) - (d[loc] + d[loc - 3]) * (x[loc] - x[loc - 3])
    return c[0] * fx + c[1] * fy


def m_vardiff(w, c, loc):
    x, d = [np.abs(v) for v in w]
    fx = (d[loc + 1] + d[loc]) * (x[loc + 1] + x[loc]) + (d[loc] + d[loc - 1]) * (x[loc] + x[loc - 1])
    fy = (d[loc + 3] + d[loc]) * (x[loc + 3] + x[loc]) + (d[loc] + d[loc - 3]) * (x[loc] + x[loc - 3])
    return abs(c[0]) * fx + abs(c[1]) * fy


def cub(v):
    return v * v * v - v


def f_cubic_lap(w, c, loc):
    x = w[0]
    return c[0] * (cub(x[loc - 1]) + cub(x[loc + 1]) + cub(x[loc - 3]) + cub(x[loc + 3]) - 4 * cub(x[loc]))


def m_cubic_lap(w, c, loc):
    a = np.abs(w[0])
    m = lambda v: v ** 3 + v
    return abs(c[0]) * (m(a[loc - 1]) + m(a[loc + 1]) + m(a[loc - 3]) + m(a[loc + 3]) + 4 * m(a[loc]))


def f_corners(w, c, loc):
    return c[0] * w[0][0] + c[1] * w[1][15] + w[2][loc] * w[0][loc + 5] - w[1][loc - 2] * c[2]


def m_corners(w, c, loc):
    return (abs(c[0] * w[0][0]) + abs(c[1] * w[1][15]) + abs(w[2][loc] * w[0][loc + 5]) +
            abs(w[1][loc - 2] * c[2]))


CASES = {
    "central": (CENTRAL, "central", f_central, m_central, "X", (1, 1, 0, 0), 1, [1e3]),
    "central_y": (CENTRAL, "central", f_central, m_central, "Y", (0, 0, 1, 1), 1, [2.0]),
    "vardiff": (VARDIFF, "vardiff", f_vardiff, m_vardiff, "XY", (1, 1, 1, 1), 2, [0.5, 0.25]),
    "cubic_lap": (CUBIC_LAP, "cubic_lap", f_cubic_lap, m_cubic_lap, "XY", (1, 1, 1, 1), 1, [3.0]),
    "corners": (CORNERS, "corners", f_corners, m_corners, "XY", (2, 1, 1, 2), 3, [0.7, -1.3, 2.1]),
}


def run_fn(case, shape, dt, periodic, ld_pad=0, seed=0):
    src, name, f, m, direction, ext, nin, coe = CASES[case]
    L, R, T, B = ext
    ny, nx = shape
    rng = np.random.default_rng(seed)
    ins = [rng.uniform(-1, 1, shape) for _ in range(nin)]
    ld = nx + ld_pad
    dins = [to_device(u, dt, ld) for u in ins]
    dout = torch.full_like(dins[0], float("nan"))
    p = b.mxs_create_2d_fn(nx, ny, ld, DIRS[direction], b.MXS_P if periodic else b.MXS_NP, code(dt),
                           L, R, T, B, dins, dout, coe, src, name)
    try:
        b.mxs_compute(p)
        torch.cuda.synchronize()
        info = b.mxs_plan_info(p)
    finally:
        b.mxs_destroy(p)
    got = to_host(dout, nx)
    rins = [round_to(u, dt) for u in ins]
    ref = np.full(shape, np.nan)
    stencil2d_window_multi(rins, L, R, T, B, f, coe, periodic, out=ref)
    mag = np.zeros(shape)
    stencil2d_window_multi(rins, L, R, T, B, m, coe, periodic, out=mag)
    return got, ref, mag, info


def _parity_cases():
    out = []
    for case in CASES:
        for periodic in (True, False):
            for dt in ("f64", "f32", "bf16"):
                out.append((case, (9, 13), 0, periodic, dt))
                out.append((case, (37, 300), 3, periodic, dt))
            out.append((case, (70, 530), 0, periodic, "f64"))
    return out


@pytest.mark.parametrize("case,shape,ld_pad,periodic,dt", _parity_cases())
def test_user_function_parity(case, shape, ld_pad, periodic, dt):
    got, ref, mag, info = run_fn(case, shape, dt, periodic, ld_pad, seed=len(case) * 100 + shape[0])
    written = ~np.isnan(ref)
    assert np.array_equal(~np.isnan(got), written), "written/untouched cells differ"
    err = np.abs(got - ref)[written]
    if dt == "f64":
        assert err.max() <= 1e-12 * max(np.abs(ref[written]).max(), 1e-300), info
    else:
        bound = (64 * 2.0 ** -24 * mag + U_STORE[dt] * np.abs(ref))[written]
        assert np.all(err <= bound), float((err / bound).max())


def test_paper_example_central_difference():
    """The Sec. 4.2 example: the second-order central difference of sin x
    written as the user function, non-periodic in x on 1024 x 512, matches
    -(4/dx^2) sin^2(dx/2) sin x and leaves one untouched cell on each side."""
    nx, ny = 1024, 512
    dx = 2 * math.pi / nx
    x = np.arange(nx) * dx
    u = np.tile(np.sin(x), (ny, 1))
    du = torch.from_numpy(u).cuda()
    dout = torch.zeros_like(du)
    p = b.mxs_create_2d_fn(nx, ny, nx, b.MXS_X, b.MXS_NP, b.MXS_F64, 1, 1, 0, 0, [du], dout,
                           [1 / dx ** 2], CENTRAL, "central")
    try:
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    got = dout.cpu().numpy()
    ref = -(4 / dx ** 2) * math.sin(dx / 2) ** 2 * np.sin(x)
    assert np.abs(got[:, 1:-1] - ref[1:-1]).max() <= 1e-9
    assert np.all(got[:, 0] == 0) and np.all(got[:, -1] == 0)


def test_compile_error_and_argument_errors():
    u = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(u)
    with pytest.raises(b.MxsError) as e:
        b.mxs_create_2d_fn(16, 16, 16, b.MXS_X, b.MXS_P, b.MXS_F64, 1, 1, 0, 0, [u], out, [1.0],
                           "__device__ mxs_real broken(const mxs_real *const *w) { return w[0][0] +; }",
                           "broken")
    assert e.value.status == b.MXS_ERR_INVALID_ARG and "compile" in str(e.value)
    for kw, st in ((dict(inputs=[u] * 5), b.MXS_ERR_INVALID_ARG), (dict(out=u), b.MXS_ERR_ALIAS),
                   (dict(name="not an identifier"), b.MXS_ERR_INVALID_ARG),
                   (dict(top=1), b.MXS_ERR_INVALID_ARG)):
        args = dict(inputs=[u], out=out, name="central", top=0)
        args.update(kw)
        with pytest.raises(b.MxsError) as e:
            b.mxs_create_2d_fn(16, 16, 16, b.MXS_X, b.MXS_P, b.MXS_F64, 1, 1, args["top"], 0, args["inputs"],
                               args["out"], [1.0], CENTRAL, args["name"])
        assert e.value.status == st


def test_swap_applies_the_function_again():
    nx = ny = 64
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, (ny, nx))
    du = torch.from_numpy(u).cuda()
    dout = torch.zeros_like(du)
    p = b.mxs_create_2d_fn(nx, ny, nx, b.MXS_XY, b.MXS_P, b.MXS_F64, 1, 1, 1, 1, [du], dout, [0.1],
                           CUBIC_LAP, "cubic_lap")
    try:
        b.mxs_compute(p)
        b.mxs_swap(p)
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    once = stencil2d_window_multi([u], 1, 1, 1, 1, f_cubic_lap, [0.1], True)
    twice = stencil2d_window_multi([once], 1, 1, 1, 1, f_cubic_lap, [0.1], True)
    assert np.abs(dout.cpu().numpy() - once).max() <= 1e-12 * np.abs(once).max()
    assert np.abs(du.cpu().numpy() - twice).max() <= 1e-12 * np.abs(twice).max()
