"""GPU parity of the batched cyclic banded solves against the oracle.

FP64: 1e-12 relative (normwise) against the oracle's banded LU + Woodbury
solve.  FP32/BF16 storage (elimination in double): the only extra error is
the rounding of the result to the storage dtype, so |err| <= u_s |x| +
1e-12 max|x|.  Both sides read the same rounded right-hand side.
"""
import numpy as np
import pytest

import oracle
from paper_1902_09931_amd import workloads as wl
from tests.gpu_util import U_STORE, code, rel_err, round_to, to_device, to_host, torch

pytestmark = pytest.mark.gpu

b = pytest.importorskip("paper_1902_09931_amd.binding")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

TRI = [2.5, -1.0]                                   # circ(-1, 2 + sigma, -1), sigma = 0.5
PENTA = [1 + 6 * 283.0, -4 * 283.0, 283.0]          # I + beta [1, -4, 6, -4, 1]
PENTA_SMALL = [1 + 6 * 17.7, -4 * 17.7, 17.7]
OTHER = [5.0, 1.0, 0.8]                             # a symmetric positive definite pentadiagonal


def check(got, ref, dt):
    if dt == "f64":
        assert rel_err(got, ref) <= 1e-12
    else:
        bound = U_STORE[dt] * np.abs(ref) + 1e-12 * np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("coef", [TRI, PENTA, OTHER])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_ragged_lines(coef, dt):
    bw = len(coef) - 1
    rng = np.random.default_rng(7 + bw)
    lengths = rng.permutation([5, 6, 7, 63, 64, 65, 127, 128, 129, 1000, 4096, 300, 2 * bw + 1])
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    r = rng.uniform(-1, 1, offs[-1])
    rr = round_to(r, dt)
    drhs = to_device(r, dt)
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(bw, coef, b.MXS_LINES_RAGGED, 0, 0, 0, offs, code(dt), drhs, dx)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    ref = oracle.cyclic_solve_batch(oracle.circulant_bands(coef), offs, rr)
    check(dx.double().cpu().numpy(), ref, dt)


@pytest.mark.parametrize("shape", [(37, 45), (70, 1030), (257, 129), (5, 7), (33, 64)])
@pytest.mark.parametrize("coef", [TRI, PENTA, PENTA_SMALL])
@pytest.mark.parametrize("geometry", ["rows", "cols"])
def test_grid_lines_f64(shape, coef, geometry):
    bw = len(coef) - 1
    ny, nx = shape
    if (nx if geometry == "rows" else ny) < 2 * bw + 1:
        pytest.skip("line shorter than the band")
    rng = np.random.default_rng(ny * 1000 + nx)
    r = rng.uniform(-1, 1, shape)
    drhs = to_device(r, "f64")
    dx = torch.empty_like(drhs)
    geo = b.MXS_LINES_ROWS if geometry == "rows" else b.MXS_LINES_COLS
    p = b.mxs_create_cyclic_solve(bw, coef, geo, nx, ny, nx, None, b.MXS_F64, drhs, dx)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    ref = oracle.cyclic_solve_grid(oracle.circulant_bands(coef), 1 if geometry == "rows" else 0, r)
    check(to_host(dx), ref, "f64")


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("geometry", ["rows", "cols"])
def test_grid_lines_reduced_storage_in_place_and_pitch(dt, geometry):
    """Reduced-precision storage, a row pitch larger than nx, and the in-place
    form (rhs == x)."""
    ny, nx, ld = 100, 77, 80
    rng = np.random.default_rng(5)
    r = rng.uniform(-1, 1, (ny, nx))
    rr = round_to(r, dt)
    buf = to_device(r, dt, ld)
    geo = b.MXS_LINES_ROWS if geometry == "rows" else b.MXS_LINES_COLS
    p = b.mxs_create_cyclic_solve(2, PENTA, geo, nx, ny, ld, None, code(dt), buf, buf)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    ref = oracle.cyclic_solve_grid(oracle.circulant_bands(PENTA), 1 if geometry == "rows" else 0, rr)
    check(to_host(buf, nx), ref, dt)


@pytest.mark.parametrize("form", ["units", "classes"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_full_batch_tridiagonal(monkeypatch, dt, form):
    """65536 periodic lines, lengths U{64..4096}, circ(-1, 2.5, -1): every
    output against the oracle, in one launch (work units) and in one launch
    per length class."""
    monkeypatch.setenv("MXS_RAGGED_FORM", form)
    lengths, offs = wl.ragged_lengths()
    r = np.random.default_rng(5).uniform(-1, 1, int(offs[-1]))
    rr = round_to(r, dt)
    drhs = to_device(r, dt)
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_RAGGED, 0, 0, 0, offs, code(dt), drhs, dx)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    ref = oracle.cyclic_solve_batch(oracle.circulant_bands(TRI), offs, rr)
    check(dx.double().cpu().numpy(), ref, dt)


def test_swap_solves_twice():
    r = np.random.default_rng(9).uniform(-1, 1, (40, 50))
    a = to_device(r, "f64")
    c = torch.empty_like(a)
    p = b.mxs_create_cyclic_solve(2, PENTA_SMALL, b.MXS_LINES_COLS, 50, 40, 50, None, b.MXS_F64, a, c)
    b.mxs_compute(p)
    b.mxs_swap(p)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    bands = oracle.circulant_bands(PENTA_SMALL)
    ref = oracle.cyclic_solve_grid(bands, 0, oracle.cyclic_solve_grid(bands, 0, r))
    check(to_host(a), ref, "f64")


def test_solve_argument_errors():
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    c = torch.zeros_like(a)
    with pytest.raises(b.MxsError) as e:      # not positive definite
        b.mxs_create_cyclic_solve(1, [1.0, 0.6], b.MXS_LINES_RAGGED, 0, 0, 0, [0, 64], b.MXS_F64, a, c)
    assert e.value.status == b.MXS_ERR_UNSUPPORTED
    with pytest.raises(b.MxsError) as e:      # line shorter than 2 bw + 1
        b.mxs_create_cyclic_solve(2, PENTA, b.MXS_LINES_RAGGED, 0, 0, 0, [0, 4, 64], b.MXS_F64, a, c)
    assert e.value.status == b.MXS_ERR_INVALID_ARG
    with pytest.raises(b.MxsError) as e:      # partial overlap
        b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_RAGGED, 0, 0, 0, [0, 32], b.MXS_F64, a, a[1:])
    assert e.value.status == b.MXS_ERR_ALIAS


@pytest.mark.parametrize("waves", ["1", "2", "4"])
def test_every_line_workgroup_shape(monkeypatch, waves):
    """The LDS kernel with one, two or four wavefronts per line gives the
    same solution."""
    monkeypatch.setenv("MXS_LINE_KERNEL", "lds")
    monkeypatch.setenv("MXS_LINE_WAVES", waves)
    rng = np.random.default_rng(31)
    lengths = rng.permutation([5, 64, 65, 129, 1000, 4096, 3001, 2048, 17])
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    r = rng.uniform(-1, 1, offs[-1])
    drhs = to_device(r, "f64")
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(2, PENTA, b.MXS_LINES_RAGGED, 0, 0, 0, offs, b.MXS_F64, drhs, dx)
    assert f"waves_per_line={waves}" in b.mxs_plan_info(p)
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    check(dx.double().cpu().numpy(), oracle.cyclic_solve_batch(oracle.circulant_bands(PENTA), offs, r), "f64")


def test_autotuned_solve_keeps_parity():
    rng = np.random.default_rng(32)
    r = rng.uniform(-1, 1, (64, 3000))
    drhs = to_device(r, "f64")
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_ROWS, 3000, 64, 3000, None, b.MXS_F64, drhs, dx)
    b.mxs_autotune(p)
    dx.zero_()
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    check(to_host(dx), oracle.cyclic_solve_grid(oracle.circulant_bands(TRI), 1, r), "f64")


# every register class (256, 512, 1024, 2048, 4096 elements), block edges,
# partial lanes, and lines longer than the register kernel holds
CLASS_LENGTHS = [5, 6, 7, 63, 64, 65, 255, 256, 257, 259, 511, 512, 513, 1000, 1023, 1025,
                 2047, 2048, 2049, 3001, 4093, 4095, 4096, 4097, 6000, 9001]


@pytest.mark.parametrize("kernel", ["register", "classes", "lds"])
@pytest.mark.parametrize("coef", [TRI, PENTA, OTHER])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_line_kernels_every_length_class(monkeypatch, kernel, coef, dt):
    """Every register class with partial lanes, and lines for the LDS kernel:
    the register lines in one launch of work units, in one launch per class,
    or every line in the LDS kernel."""
    if kernel == "lds":
        monkeypatch.setenv("MXS_LINE_KERNEL", "lds")
    if kernel == "classes":
        monkeypatch.setenv("MXS_RAGGED_FORM", "classes")
    bw = len(coef) - 1
    rng = np.random.default_rng(41 + bw)
    lengths = rng.permutation(CLASS_LENGTHS)
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    r = rng.uniform(-1, 1, offs[-1])
    rr = round_to(r, dt)
    drhs = to_device(r, dt)
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(bw, coef, b.MXS_LINES_RAGGED, 0, 0, 0, offs, code(dt), drhs, dx)
    info = b.mxs_plan_info(p)
    if kernel == "lds":
        assert "register_kernel" not in info
    else:
        for nb in (1, 2, 4, 8, 16):
            assert f"register_kernel(nb={nb}" in info
        assert "lds_kernel_lines=3 " in info     # 4097, 6000 and 9001
        assert ("form=classes launches=6 " if kernel == "classes" else "form=units launches=2 ") in info
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    ref = oracle.cyclic_solve_batch(oracle.circulant_bands(coef), offs, rr)
    check(dx.double().cpu().numpy(), ref, dt)


@pytest.mark.parametrize("kernel", ["register", "lds"])
@pytest.mark.parametrize("nx", [5, 200, 256, 700, 1024, 1500, 4096])
def test_row_kernels(monkeypatch, kernel, nx):
    if kernel == "lds":
        monkeypatch.setenv("MXS_LINE_KERNEL", "lds")
    ny = 37
    rng = np.random.default_rng(nx)
    r = rng.uniform(-1, 1, (ny, nx))
    drhs = to_device(r, "f64")
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(2, PENTA_SMALL, b.MXS_LINES_ROWS, nx, ny, nx, None, b.MXS_F64, drhs, dx)
    assert ("register_kernel" in b.mxs_plan_info(p)) == (kernel == "register")
    b.mxs_compute(p)
    torch.cuda.synchronize()
    b.mxs_destroy(p)
    check(to_host(dx), oracle.cyclic_solve_grid(oracle.circulant_bands(PENTA_SMALL), 1, r), "f64")


def test_ragged_autotune_times_both_forms():
    lengths, offs = wl.ragged_lengths(nbatch=4000, seed=15)
    r = np.random.default_rng(16).uniform(-1, 1, int(offs[-1]))
    drhs = to_device(r, "f32")
    dx = torch.empty_like(drhs)
    p = b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_RAGGED, 0, 0, 0, offs, b.MXS_F32, drhs, dx)
    try:
        b.mxs_autotune(p)
        info = b.mxs_plan_info(p)
        assert "tuned_us_units=" in info and "tuned_us_classes=" in info
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    check(dx.double().cpu().numpy(),
          oracle.cyclic_solve_batch(oracle.circulant_bands(TRI), offs, round_to(r, "f32")), "f32")


def test_ragged_solve_is_one_launch_and_graph_capturable():
    """The ragged solve of lines up to 4096 elements is one launch (every
    length class in one grid of work units), and it can be captured into a
    HIP graph: every replay, with eager work and synchronisation between
    replays, equals the eager result bit for bit."""
    lengths, offs = wl.ragged_lengths(nbatch=3000, seed=13)
    r = np.random.default_rng(14).uniform(-1, 1, int(offs[-1]))
    drhs = to_device(r, "f64")
    x_eager = torch.empty_like(drhs)
    x_graph = torch.full_like(drhs, float("nan"))
    pe = b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_RAGGED, 0, 0, 0, offs, b.MXS_F64, drhs, x_eager)
    pg = b.mxs_create_cyclic_solve(1, TRI, b.MXS_LINES_RAGGED, 0, 0, 0, offs, b.MXS_F64, drhs, x_graph)
    try:
        assert "launches=1 " in b.mxs_plan_info(pg)
        b.mxs_compute(pe)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            b.mxs_compute(pg)          # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            b.mxs_compute(pg)
        for k in range(4):
            x_graph.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            _ = torch.ones(1000, device="cuda").sum().item()
            assert torch.equal(x_graph, x_eager), k
    finally:
        b.mxs_destroy(pe)
        b.mxs_destroy(pg)
    ref = oracle.cyclic_solve_batch(oracle.circulant_bands(TRI), offs, r)
    check(x_eager.cpu().numpy(), ref, "f64")


@pytest.mark.parametrize("geometry", ["rows", "cols"])
def test_grid_swap_then_set_io(geometry):
    """Swap exchanges rhs and x without touching device memory (the tables of
    both orientations exist from the start); set_io rebinds after a swap."""
    ny, nx = 40, 50
    r = np.random.default_rng(19).uniform(-1, 1, (ny, nx))
    a = to_device(r, "f64")
    c = torch.empty_like(a)
    geo = b.MXS_LINES_ROWS if geometry == "rows" else b.MXS_LINES_COLS
    axis = 1 if geometry == "rows" else 0
    bands = oracle.circulant_bands(PENTA_SMALL)
    p = b.mxs_create_cyclic_solve(2, PENTA_SMALL, geo, nx, ny, nx, None, b.MXS_F64, a, c)
    try:
        b.mxs_compute(p)           # c = A^-1 a
        b.mxs_swap(p)
        b.mxs_compute(p)           # a = A^-1 c
        torch.cuda.synchronize()
        ref2 = oracle.cyclic_solve_grid(bands, axis, oracle.cyclic_solve_grid(bands, axis, r))
        check(to_host(a), ref2, "f64")
        d = torch.empty_like(a)
        b.mxs_set_io(p, c, d)      # d = A^-1 c
        b.mxs_compute(p)
        torch.cuda.synchronize()
        check(to_host(d), oracle.cyclic_solve_grid(bands, axis, to_host(c)), "f64")
    finally:
        b.mxs_destroy(p)
