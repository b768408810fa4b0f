"""The stated error bound of the reduced-precision stencils tells the
precision form it promises (float accumulation of values stored in BF16 or
FP32) from plausible precision bugs.

CPU only.  Each stencil is evaluated in NumPy float32 arithmetic, one
rounding per product and per sum, from inputs already rounded to BF16; the
oracle gives the double-precision reference.  The correct form must pass the
bound everywhere; a form that rounds its weights to BF16, or keeps its
partial sums in BF16, must fail it.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import round_to, stencil_bound


def float_stencil(u, w, L, R, T, B, weight_round=None, acc_round=None):
    """Periodic XY stencil in float32 arithmetic (window order, no FMA);
    optional rounding of the weights and of every partial sum."""
    ny, nx = u.shape
    u32 = u.astype(np.float32)
    wt = np.asarray(w, dtype=np.float64)
    if weight_round:
        wt = weight_round(wt)
    wt = wt.astype(np.float32)
    acc = np.zeros((ny, nx), dtype=np.float32)
    k = 0
    for b in range(-T, B + 1):
        for a in range(-L, R + 1):
            shifted = np.roll(np.roll(u32, -b, axis=0), -a, axis=1)
            acc = (acc + wt[k] * shifted).astype(np.float32)
            if acc_round:
                acc = acc_round(acc.astype(np.float64)).astype(np.float32)
            k += 1
    return round_to(acc.astype(np.float64), "bf16")


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(41)
    L, R, T, B = 1, 1, 1, 1
    u = round_to(rng.uniform(-1, 1, (64, 96)), "bf16")
    w = rng.uniform(-1, 1, 9)
    ref = oracle.stencil2d(u, L, R, T, B, w, True)
    s_abs = oracle.stencil2d(np.abs(u), L, R, T, B, np.abs(w), True)
    bound = stencil_bound("bf16", s_abs, ref, 9, 0)
    return u, w, (L, R, T, B), ref, bound


def test_float_accumulation_passes(case):
    u, w, ext, ref, bound = case
    got = float_stencil(u, w, *ext)
    assert np.all(np.abs(got - ref) <= bound)


def test_bf16_weights_fail(case):
    u, w, ext, ref, bound = case
    got = float_stencil(u, w, *ext, weight_round=lambda x: round_to(x, "bf16"))
    assert (np.abs(got - ref) > bound).mean() > 0.05


def test_bf16_partial_sums_fail(case):
    u, w, ext, ref, bound = case
    got = float_stencil(u, w, *ext, acc_round=lambda x: round_to(x, "bf16"))
    assert (np.abs(got - ref) > bound).mean() > 0.05
