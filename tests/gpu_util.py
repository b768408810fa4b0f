"""Helpers of the GPU parity tests: move seeded inputs to the device, run a
plan through the C ABI, bring results back, and the error bounds of the
reduced-precision forms."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

DTYPES = ("f64", "f32", "bf16")
TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
U_STORE = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8}
U32 = 2.0 ** -24


def code(dt):
    from paper_1902_09931_amd import binding as b
    return {"f64": b.MXS_F64, "f32": b.MXS_F32, "bf16": b.MXS_BF16}[dt]


def round_to(a, dt):
    """Host float64 copy of `a` rounded to storage dtype dt (nearest even)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(TORCH[dt]).double().numpy()


def to_device(a, dt, ld=None, fill=0.0):
    """(ny, nx) host array -> device tensor (ny, ld) of dtype dt; columns
    beyond nx hold `fill`."""
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a).to(TORCH[dt]).cuda()
    ny, nx = a.shape
    ld = nx if ld is None else ld
    t = torch.full((ny, ld), fill, dtype=TORCH[dt], device="cuda")
    t[:, :nx] = torch.from_numpy(a).to(TORCH[dt]).cuda()
    return t


def to_host(t, nx=None):
    h = t.double().cpu().numpy()
    return h if nx is None else h[:, :nx]


def rel_err(got, ref, mask=None):
    """Normwise relative error max|got - ref| / max|ref| over mask."""
    if mask is not None:
        got, ref = got[mask], ref[mask]
    den = np.abs(ref).max()
    return np.abs(got - ref).max() / (den if den > 0 else 1.0)


def stencil_bound(dt, s_abs, ref, taps, ncoe):
    """Stated forward bound of a stencil evaluated in float with storage
    dtype dt, when the input is already in the storage dtype (both sides
    read the same stored values, so input rounding has no part in it):

        |err| <= (K + 2 ncoe + 2) u_32 sum_k |w_k| |f|(|u_k|) + u_s |out|

    K float roundings of the dot product, one for each weight rounded to
    float, 2 (ncoe - 1) for Horner's rule over ncoe coefficients plus one for
    each coefficient rounded to float (the standard forward error analysis
    of an inner product and of Horner's rule), and the final rounding of the
    output to the storage dtype, u_s = 2^-24 (FP32) or 2^-8 (BF16)."""
    return (taps + 2 * ncoe + 2) * U32 * s_abs + U_STORE[dt] * np.abs(ref)
