"""GPU parity of the 2D and ragged 1D stencils against the oracle.

FP64 plans must match the oracle to 1e-12 relative (normwise, over the cells
the plan writes) and leave every other cell bit-for-bit untouched; FP32 and
BF16 plans must stay inside the stated pointwise bound.  Inputs are seeded;
reduced-precision plans and the oracle see the same rounded input.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1902_09931_amd import workloads as wl
from tests.conftest import golden
from tests.gpu_util import (code, rel_err, round_to, stencil_bound, to_device, to_host,
                            torch)

pytestmark = pytest.mark.gpu

b = pytest.importorskip("paper_1902_09931_amd.binding")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DIRS = {"X": b.MXS_X, "Y": b.MXS_Y, "XY": b.MXS_XY}


def run_2d(u, direction, periodic, ext, w, coe, dt, ld_pad=0, fill=float("nan")):
    L, R, T, B = ext
    ny, nx = u.shape
    ld = nx + ld_pad
    din = to_device(u, dt, ld)
    dout = torch.full((ny, ld), fill, dtype=din.dtype, device="cuda")
    p = b.mxs_create_2d(nx, ny, ld, DIRS[direction], b.MXS_P if periodic else b.MXS_NP,
                        code(dt), L, R, T, B, w, coe, din, dout)
    try:
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    return to_host(dout, nx)


def check_against_oracle(u, got, direction, periodic, ext, w, coe, dt):
    L, R, T, B = ext
    uu = round_to(u, dt)
    ref = np.full_like(uu, np.nan)
    oracle.stencil2d(uu, L, R, T, B, w, periodic, coe=coe, out=ref)
    written = ~np.isnan(ref)
    assert np.array_equal(np.isnan(got), ~written), "written/untouched cells differ"
    if dt == "f64":
        assert rel_err(got, ref, written) <= 1e-12
    else:
        s_abs = oracle.stencil2d(np.abs(uu), L, R, T, B, np.abs(w), periodic,
                                 coe=None if coe is None else np.abs(coe))
        bound = stencil_bound(dt, s_abs, ref, (L + R + 1) * (T + B + 1),
                              0 if coe is None else len(coe))
        err = np.abs(got - ref)
        assert np.all(err[written] <= bound[written]), float((err / bound)[written].max())


WINDOWS = [("X", (2, 2, 0, 0)), ("X", (0, 3, 0, 0)), ("X", (4, 4, 0, 0)), ("X", (8, 7, 0, 0)),
           ("Y", (0, 0, 2, 2)), ("Y", (0, 0, 1, 0)), ("Y", (0, 0, 3, 5)), ("Y", (0, 0, 8, 8)),
           ("XY", (1, 1, 1, 1)), ("XY", (2, 1, 0, 2)), ("XY", (2, 2, 2, 2)), ("XY", (4, 3, 2, 4))]
SHAPES = [(37, 45), (70, 1030), (257, 129)]


def _cases():
    cases = []
    k = 0
    for shape in SHAPES:
        for direction, ext in WINDOWS:
            for periodic in (True, False):
                cases.append((shape, direction, ext, periodic, "f64", None, 0))
                dt = ("f32", "bf16", "f64")[k % 3]
                fun = (k // 3) % 2 == 1
                ld_pad = (0, 3, 1)[k % 3]
                cases.append((shape, direction, ext, periodic, dt,
                              wl.CUBIC_MINUS_LINEAR if fun else None, ld_pad))
                k += 1
    return cases


@pytest.mark.parametrize("shape,direction,ext,periodic,dt,coe,ld_pad", _cases())
def test_stencil2d_parity(shape, direction, ext, periodic, dt, coe, ld_pad):
    L, R, T, B = ext
    rng = np.random.default_rng(hash((shape, ext, periodic)) % (1 << 32))
    u = rng.uniform(-1, 1, shape)
    w = rng.uniform(-1, 1, (T + B + 1) * (L + R + 1))
    got = run_2d(u, direction, periodic, ext, w, coe, dt, ld_pad)
    check_against_oracle(u, got, direction, periodic, ext, w, coe, dt)


def test_cfg0_x_second_derivative():
    """256^2 periodic X [1,-2,1]/dx^2 on the seeded field: oracle parity and
    the closed form of the smooth part."""
    u, smooth, dx = wl.periodic_field_cfg0()
    w = wl.scaled(wl.D2_2ND, 1.0 / dx ** 2)
    got = run_2d(u, "X", True, (1, 1, 0, 0), w, None, "f64")
    ref = oracle.stencil2d(u, 1, 1, 0, 0, w, True)
    assert rel_err(got, ref) <= 1e-12
    sigma = -4.0 * math.sin(math.pi * dx) ** 2 / dx ** 2
    s_noise = oracle.stencil2d(u - smooth, 1, 1, 0, 0, w, True)
    assert np.abs(got - s_noise - sigma * smooth).max() < 1e-8


def test_example_2d_x_np_on_gpu():
    """Sec. 4.1 example on the GPU: 8th-order d2/dx2 of sin x, 1024 x 512, the
    4 boundary cells on each side stay 0.0 (zeroed output)."""
    g = golden("example_2d_x_np.json")
    nx, ny, L, R = g["nx"], g["ny"], g["numStenLeft"], g["numStenRight"]
    dx = 2 * math.pi / nx
    w = oracle.as_floats(oracle.fd_weights(2, range(-L, R + 1)), dx, 2)
    x = np.arange(nx) * dx
    u = np.tile(np.sin(x), (ny, 1))
    got = run_2d(u, "X", False, (L, R, 0, 0), w, None, "f64", fill=0.0)
    assert np.all(got[:, :4] == 0.0) and np.all(got[:, -4:] == 0.0)
    ref = oracle.stencil2d(u, L, R, 0, 0, w, False)
    # Differentiation amplifies rounding: sum|w||u| / |out| is about 2e5 here,
    # so the normwise 1e-12 is out of reach for any double evaluation.  Both
    # sides must sit within the dot-product bound (K + 2) u sum_k |w_k||u_k|.
    s_abs = oracle.stencil2d(np.abs(u), L, R, 0, 0, np.abs(w), False)
    assert np.all(np.abs(got - ref) <= (L + R + 3) * 2.0 ** -53 * s_abs)
    assert np.abs(got[:, 4:-4] + np.sin(x[4:-4])).max() < 5e-10


def test_swap_and_set_io():
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, (33, 70))
    w = [1.0, -2.0, 1.0]
    a = to_device(u, "f64")
    c = torch.zeros_like(a)
    p = b.mxs_create_2d(70, 33, 70, b.MXS_X, b.MXS_P, b.MXS_F64, 1, 1, 0, 0, w, None, a, c)
    try:
        b.mxs_compute(p)
        b.mxs_swap(p)                 # now reads c, writes a
        b.mxs_compute(p)
        torch.cuda.synchronize()
        ref = oracle.stencil2d(oracle.stencil2d(u, 1, 1, 0, 0, w, True), 1, 1, 0, 0, w, True)
        assert rel_err(to_host(a), ref) <= 1e-12
        d = torch.zeros_like(a)
        b.mxs_set_io(p, c, d)
        b.mxs_compute(p)
        torch.cuda.synchronize()
        assert rel_err(to_host(d), oracle.stencil2d(to_host(c), 1, 1, 0, 0, w, True)) <= 1e-12
        with pytest.raises(b.MxsError) as e:
            b.mxs_set_io(p, a, a)
        assert e.value.status == b.MXS_ERR_ALIAS
    finally:
        b.mxs_destroy(p)
    with pytest.raises(b.MxsError) as e:
        b.mxs_compute(p)
    assert e.value.status == b.MXS_ERR_BAD_HANDLE


# --- full-size grids, sampled outputs ------------------------------------------

def full_size_stencils(dx):
    """The 8192^2 stencil set: 4th-order 5-point d2 in x and in y, the Fig. 1
    cross derivative, and the Laplacian of c^3 - c."""
    d2 = wl.scaled(wl.D2_4TH, 1.0 / dx ** 2)
    return [("X", (2, 2, 0, 0), d2, None),
            ("Y", (0, 0, 2, 2), d2, None),
            ("XY", (1, 1, 1, 1), wl.scaled(wl.CROSS_XXYY, 1.0 / dx ** 4), None),
            ("XY", (1, 1, 1, 1), wl.scaled(wl.LAPLACE_3X3, 1.0 / dx ** 2), wl.CUBIC_MINUS_LINEAR)]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_size_8192_every_output(dt):
    """The 8192^2 stencil set in the layout the autotuner picks (the layout
    the benchmark times): every one of the 67M outputs of each of the eight
    stencils against the oracle over the whole grid, and every untouched
    border cell of the non-periodic ones still untouched.  The oracle calls
    run concurrently on the host cores (each releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    import os
    n = 8192
    dx = 1.0 / n
    u = wl.uniform_grid(n, n, seed=1)
    uu = round_to(u, dt)
    din = to_device(u, dt)
    dout = torch.empty_like(din)
    runs = []
    for direction, ext, w, coe in full_size_stencils(dx):
        L, R, T, B = ext
        for periodic in (True, False):
            p = b.mxs_create_2d(n, n, n, DIRS[direction], b.MXS_P if periodic else b.MXS_NP,
                                code(dt), L, R, T, B, w, coe, din, dout)
            try:
                b.mxs_autotune(p)
                layout = b.mxs_plan_info(p)
                dout.fill_(float("nan"))
                b.mxs_compute(p)
                torch.cuda.synchronize()
            finally:
                b.mxs_destroy(p)
            runs.append((direction, ext, w, coe, periodic, layout, to_host(dout)))
    del din, dout
    torch.cuda.empty_cache()

    def check(run):
        direction, ext, w, coe, periodic, layout, got = run
        L, R, T, B = ext
        ref = np.full_like(uu, np.nan)
        oracle.stencil2d(uu, L, R, T, B, w, periodic, coe=coe, out=ref)
        written = ~np.isnan(ref)
        if not np.array_equal(~np.isnan(got), written):
            return f"{direction} p={periodic} {layout}: written cells differ"
        if dt == "f64":
            err = rel_err(got, ref, written)
            return None if err <= 1e-12 else f"{direction} p={periodic} {layout}: {err:.3e}"
        s_abs = oracle.stencil2d(np.abs(uu), L, R, T, B, np.abs(w), periodic,
                                 coe=None if coe is None else np.abs(coe))
        bound = stencil_bound(dt, s_abs, ref, (L + R + 1) * (T + B + 1),
                              0 if coe is None else len(coe))
        ratio = float((np.abs(got - ref)[written] / bound[written]).max())
        return None if ratio <= 1.0 else f"{direction} p={periodic} {layout}: {ratio:.3f} of the bound"

    with ThreadPoolExecutor(max(1, min(8, len(os.sched_getaffinity(0))))) as pool:
        failures = [m for m in pool.map(check, runs) if m]
    assert not failures, failures


# --- ragged batched 1D ------------------------------------------------------------

def run_1d(vals, offsets, periodic, L, R, w, coe, dt, fill=float("nan")):
    din = to_device(vals, dt)
    dout = torch.full_like(din, fill)
    p = b.mxs_create_1d_batch(offsets, b.MXS_P if periodic else b.MXS_NP, code(dt), L, R, w, coe,
                              din, dout)
    try:
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    return dout.double().cpu().numpy()


@pytest.mark.parametrize("L,R", [(2, 2), (1, 1), (0, 3), (4, 4), (8, 8), (0, 0)])
@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("dt,fun", [("f64", False), ("f64", True), ("f32", False), ("bf16", True)])
def test_stencil1d_ragged_parity(L, R, periodic, dt, fun):
    rng = np.random.default_rng(L * 100 + R)
    # three shuffles of a spread of lengths and a run of short signals (many
    # signals per tile): several tiles of every dtype and a ragged tail
    base = [17, 18, 64, 65, 97, 200, 513, 1025, 4096, 19, 700, 31, 2049]
    lengths = np.concatenate([rng.permutation(base), rng.integers(17, 41, 600),
                              rng.permutation(base), rng.permutation(base)])
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    vals = rng.uniform(-1, 1, offs[-1])
    w = rng.uniform(-1, 1, L + R + 1)
    coe = wl.CUBIC_MINUS_LINEAR if fun else None
    got = run_1d(vals, offs, periodic, L, R, w, coe, dt)
    vv = round_to(vals, dt)
    ref = np.full_like(vv, np.nan)
    oracle.stencil1d_batch(vv, offs, L, R, w, periodic, coe=coe, out=ref)
    written = ~np.isnan(ref)
    assert np.array_equal(~np.isnan(got), written)
    if dt == "f64":
        assert rel_err(got, ref, written) <= 1e-12
    else:
        s_abs = oracle.stencil1d_batch(np.abs(vv), offs, L, R, np.abs(w), periodic,
                                       coe=None if coe is None else np.abs(coe))
        bound = stencil_bound(dt, s_abs, ref, L + R + 1, 0 if coe is None else len(coe))
        assert np.all(np.abs(got - ref)[written] <= bound[written])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_stencil1d_full_batch(dt):
    """65536 periodic signals, lengths U{64..4096}, 4th-order first
    derivative: every output against the oracle."""
    lengths, offs = wl.ragged_lengths()
    vals = wl.ragged_values(int(offs[-1]))
    w = list(wl.D1_4TH)
    got = run_1d(vals, offs, True, 2, 2, w, None, dt)
    vv = round_to(vals, dt)
    ref = oracle.stencil1d_batch(vv, offs, 2, 2, w, True)
    if dt == "f64":
        assert rel_err(got, ref) <= 1e-12
    else:
        s_abs = oracle.stencil1d_batch(np.abs(vv), offs, 2, 2, np.abs(w), True)
        assert np.all(np.abs(got - ref) <= stencil_bound(dt, s_abs, ref, 5, 0))


# --- launch layouts -------------------------------------------------------------

# rows per workgroup, tile order, threads per workgroup, streaming stores:
# a spread of shapes plus every layout the autotuner picked for the 8192^2
# FP64 and FP32 stencil sets on the GPU
LAYOUTS = ["2,1,256,1", "4,0,256,0", "8,1,128,1", "16,0,128,0", "64,1,256,1", "128,0,256,1",
           "3,1,64,0", "4,1,256,1", "16,1,256,1", "128,1,256,1", "8,0,256,1", "64,0,256,1",
           # block form (fifth field: input rows per workgroup; windows of 3 or 5
           # rows only, others keep their default layout)
           "1,1,256,1,8", "1,0,128,0,8", "1,1,128,1,16", "1,0,256,0,16", "1,1,64,1,16",
           "1,1,256,1,12",
           # block form, x neighbours by lane shifts (sixth field; centred windows)
           "1,1,256,1,8,1", "1,0,128,0,12,1", "1,1,64,1,16,1",
           # tile order 2 (a band of row chunks per XCD, row-major), both forms
           "4,2,256,1", "16,2,128,0", "1,2,256,1,8", "1,2,128,0,16", "1,2,256,1,8,1"]
LAYOUT_WINDOWS = [("X", (2, 2, 0, 0), None), ("Y", (0, 0, 2, 1), None), ("XY", (1, 2, 2, 1), None),
                  ("XY", (1, 1, 1, 1), wl.CUBIC_MINUS_LINEAR), ("XY", (2, 2, 1, 1), None)]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("direction,ext,coe", LAYOUT_WINDOWS, ids=["X", "Y", "XY", "XYfun", "XY5x3"])
def test_every_layout_keeps_parity(monkeypatch, layout, dt, direction, ext, coe):
    """Rows per workgroup, tile order, threads per workgroup and streaming
    stores change only the schedule: every layout matches the oracle in
    every storage dtype (FP64 to 1e-12, FP32/BF16 inside the stated bound)."""
    monkeypatch.setenv("MXS_STENCIL_TILE", layout)
    L, R, T, B = ext
    rng = np.random.default_rng(17)
    u = rng.uniform(-1, 1, (150, 1100))
    w = rng.uniform(-1, 1, (T + B + 1) * (L + R + 1))
    for periodic in (True, False):
        got = run_2d(u, direction, periodic, ext, w, coe, dt)
        check_against_oracle(u, got, direction, periodic, ext, w, coe, dt)


BLOCK_WINDOWS = [("Y", (0, 0, 1, 1)), ("Y", (0, 0, 2, 2)), ("Y", (0, 0, 3, 0)), ("XY", (1, 1, 1, 1)),
                 ("XY", (2, 1, 0, 2)), ("XY", (2, 2, 2, 2)), ("XY", (0, 1, 1, 0))]


@pytest.mark.parametrize("layout", ["1,1,64,1,8", "1,0,128,0,16", "1,1,64,1,8,1", "1,0,256,0,12,1",
                                    "1,1,128,1,16,1", "1,2,128,1,8"])
@pytest.mark.parametrize("shape", [(5, 9), (8, 70), (37, 45), (257, 129), (23, 1030)])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_block_form_small_and_ragged_grids(monkeypatch, layout, shape, dt):
    """The block form on grids with fewer rows than one chunk, ragged last
    chunks and strips, unaligned pitches and padded windows, periodic and
    not, with and without the point function; with x neighbours from LDS
    and, for the centred windows, from lane shifts (the other windows keep
    their default layout)."""
    monkeypatch.setenv("MXS_STENCIL_TILE", layout)
    rng = np.random.default_rng(hash((shape, layout, dt)) % (1 << 32))
    u = rng.uniform(-1, 1, shape)
    for k, (direction, ext) in enumerate(BLOCK_WINDOWS):
        L, R, T, B = ext
        if T + B >= shape[0] or L + R >= shape[1]:
            continue
        w = rng.uniform(-1, 1, (T + B + 1) * (L + R + 1))
        coe = wl.CUBIC_MINUS_LINEAR if k % 2 else None
        for periodic in (True, False):
            got = run_2d(u, direction, periodic, ext, w, coe, dt, ld_pad=k % 3)
            check_against_oracle(u, got, direction, periodic, ext, w, coe, dt)


def test_autotune_keeps_parity_and_reports_layout():
    rng = np.random.default_rng(18)
    u = rng.uniform(-1, 1, (300, 700))
    w = rng.uniform(-1, 1, 9)
    din = to_device(u, "f32")
    dout = torch.full_like(din, float("nan"))
    p = b.mxs_create_2d(700, 300, 700, b.MXS_XY, b.MXS_NP, b.MXS_F32, 1, 1, 1, 1, w, None, din, dout)
    try:
        b.mxs_autotune(p)
        info = b.mxs_plan_info(p)
        assert "rows=" in info and "threads=" in info
        dout.fill_(float("nan"))
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    check_against_oracle(u, to_host(dout), "XY", False, (1, 1, 1, 1), w, None, "f32")
