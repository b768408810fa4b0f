"""GPU parity of the WENO advection variant (Sec. 4.3) against the oracle.

FP64 to 1e-12 normwise relative on seeded fields (smooth plus noise, jumps,
mixed-sign velocities including exact zeros) over grids that span several
tiles with ragged strips and chunks, in every launch layout; at 8192^2 on
sampled rows against the oracle evaluated on those rows.
"""
import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import rel_err, torch

pytestmark = pytest.mark.gpu

b = pytest.importorskip("paper_1902_09931_amd.binding")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def fields(ny, nx, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * 2 * math.pi / nx
    y = np.arange(ny) * 2 * math.pi / ny
    phi = np.sin(x)[None, :] * np.cos(2 * y)[:, None] + 0.05 * rng.uniform(-1, 1, (ny, nx))
    phi[:, nx // 3: nx // 2] += 1.0          # a jump in x
    phi[ny // 4: ny // 3, :] -= 0.5          # and one in y
    u = rng.uniform(-1, 1, (ny, nx))
    v = rng.uniform(-1, 1, (ny, nx))
    u[::7, ::5] = 0.0
    v[::5, ::3] = 0.0
    return phi, u, v


def run(phi, u, v, dx, dy, ld_pad=0, layout=None, autotune=False):
    ny, nx = phi.shape
    ld = nx + ld_pad

    def dev(a):
        t = torch.zeros((ny, ld), dtype=torch.float64, device="cuda")
        t[:, :nx] = torch.from_numpy(a)
        return t

    dphi, du, dv = dev(phi), dev(u), dev(v)
    dout = torch.full((ny, ld), float("nan"), dtype=torch.float64, device="cuda")
    p = b.mxs_create_weno_adv(nx, ny, ld, dx, dy, b.MXS_F64, dphi, du, dv, dout)
    try:
        if autotune:
            b.mxs_autotune(p)
        b.mxs_compute(p)
        torch.cuda.synchronize()
        info = b.mxs_plan_info(p)
    finally:
        b.mxs_destroy(p)
    return dout[:, :nx].cpu().numpy(), info


@pytest.mark.parametrize("shape,ld_pad", [((6, 6), 0), ((37, 45), 1), ((64, 512), 0), ((70, 1030), 2),
                                          ((257, 129), 0), ((130, 2048), 0)])
def test_weno_parity(shape, ld_pad):
    ny, nx = shape
    phi, u, v = fields(ny, nx, seed=ny * 1000 + nx)
    dx, dy = 2 * math.pi / nx, 2 * math.pi / ny
    got, _ = run(phi, u, v, dx, dy, ld_pad)
    ref = oracle.weno_adv(phi, u, v, dx, dy)
    assert not np.isnan(got).any()
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("layout", ["4,1,256,1", "8,0,128,0", "4,0,128,1", "8,1,256,0"])
def test_weno_every_layout(monkeypatch, layout):
    monkeypatch.setenv("MXS_WENO_TILE", layout)
    phi, u, v = fields(150, 1100, seed=3)
    got, info = run(phi, u, v, 0.01, 0.02)
    r, o, t, nt = layout.split(",")
    assert f"rows={r} order={o} threads={t} nt_store={nt}" in info
    assert rel_err(got, oracle.weno_adv(phi, u, v, 0.01, 0.02)) <= 1e-12


def test_weno_8192_sampled_rows_after_autotune():
    """The benchmark's workload (8192^2, phi ~ U(-1, 1), u, v ~ U(-1, 1)) in
    the autotuned layout: 24 whole rows (the first, the last and seeded
    others) against the oracle run on the band of 7 rows around each."""
    n = 8192
    rng = np.random.default_rng(21)
    phi = rng.uniform(-1, 1, (n, n))
    u = rng.uniform(-1, 1, (n, n))
    v = rng.uniform(-1, 1, (n, n))
    h = 1.0 / n
    got, info = run(phi, u, v, h, h, autotune=True)
    rows = sorted(set([0, n - 1] + list(rng.integers(0, n, 22))))
    for j in rows:
        idx = [(j + k) % n for k in range(-3, 4)]
        band = oracle.weno_adv(phi[idx], u[idx], v[idx], h, h)
        # the band's middle row sees its true y neighbours; its x is periodic
        assert rel_err(got[j], band[3]) <= 1e-12, (j, info)


def test_weno_swap_and_errors():
    phi, u, v = fields(32, 48, seed=4)
    dx = dy = 0.1
    tp = torch.from_numpy(phi).cuda()
    tu, tv = torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()
    out = torch.zeros_like(tp)
    p = b.mxs_create_weno_adv(48, 32, 48, dx, dy, b.MXS_F64, tp, tu, tv, out)
    try:
        b.mxs_compute(p)
        b.mxs_swap(p)                # now phi <- out, out <- phi
        b.mxs_compute(p)
        torch.cuda.synchronize()
    finally:
        b.mxs_destroy(p)
    first = oracle.weno_adv(phi, u, v, dx, dy)
    assert rel_err(out.cpu().numpy(), first) <= 1e-12
    assert rel_err(tp.cpu().numpy(), oracle.weno_adv(first, u, v, dx, dy)) <= 1e-12
    for kw, st in ((dict(dtype=b.MXS_F32), b.MXS_ERR_UNSUPPORTED), (dict(nx=5), b.MXS_ERR_INVALID_ARG),
                   (dict(out=tu), b.MXS_ERR_ALIAS), (dict(dx=0.0), b.MXS_ERR_INVALID_ARG)):
        args = dict(nx=48, ny=32, ld=48, dx=dx, dy=dy, dtype=b.MXS_F64, phi=tp, u=tu, v=tv, out=out)
        args.update(kw)
        with pytest.raises(b.MxsError) as e:
            b.mxs_create_weno_adv(args["nx"], args["ny"], args["ld"], args["dx"], args["dy"], args["dtype"],
                                  args["phi"], args["u"], args["v"], args["out"])
        assert e.value.status == st
