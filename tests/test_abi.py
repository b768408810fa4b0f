"""The C ABI library loads, exports every entry point of include/mxsten.h, and
rejects invalid arguments before touching a GPU.  CPU only: no compute call."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

b = pytest.importorskip("paper_1902_09931_amd.binding")

HEADER = os.path.join(ROOT, "include", "mxsten.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mxs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(b.library_path())
    syms = declared_symbols()
    assert len(syms) >= 15
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_and_version():
    assert b.mxs_status_string(0) == "MXS_OK"
    assert b.mxs_status_string(b.MXS_ERR_ALIAS) == "MXS_ERR_ALIAS"
    assert b.mxs_status_string(-99) == "MXS_ERR_UNKNOWN"
    assert b.mxs_version() >= 100


def test_destroy_null_is_ok_and_unknown_handle_is_rejected():
    b.mxs_destroy(None)
    with pytest.raises(b.MxsError) as e:
        b.mxs_destroy(0x1234)
    assert e.value.status == b.MXS_ERR_BAD_HANDLE
    with pytest.raises(b.MxsError) as e:
        b.mxs_compute(0x1234, stream=0)
    assert e.value.status == b.MXS_ERR_BAD_HANDLE


FAKE_IN, FAKE_OUT = 1 << 32, 1 << 33     # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,status", [
    (dict(nx=0), b.MXS_ERR_INVALID_ARG),
    (dict(ld=10), b.MXS_ERR_INVALID_ARG),
    (dict(dir=7), b.MXS_ERR_INVALID_ARG),
    (dict(bc=3), b.MXS_ERR_INVALID_ARG),
    (dict(dtype=9), b.MXS_ERR_INVALID_ARG),
    (dict(top=1, weights=[1.0] * 6), b.MXS_ERR_INVALID_ARG),          # X with top
    (dict(dir=1), b.MXS_ERR_INVALID_ARG),                               # Y with left/right
    (dict(left=40, right=30, weights=[1.0] * 71), b.MXS_ERR_INVALID_ARG),
    (dict(left=9, right=9, weights=[1.0] * 19), b.MXS_ERR_UNSUPPORTED),
    (dict(dir=2, left=5, right=5, top=1, bottom=1, weights=[1.0] * 33), b.MXS_ERR_UNSUPPORTED),
    (dict(coe=[1.0] * 9), b.MXS_ERR_UNSUPPORTED),
    (dict(out=FAKE_IN + 8), b.MXS_ERR_ALIAS),
    (dict(in_=None), b.MXS_ERR_INVALID_ARG),
])
def test_create_2d_validation(kw, status):
    args = dict(nx=64, ny=32, ld=64, dir=b.MXS_X, bc=b.MXS_P, dtype=b.MXS_F64, left=1, right=1,
                top=0, bottom=0, weights=[1.0, -2.0, 1.0], coe=None, in_=FAKE_IN, out=FAKE_OUT)
    args.update(kw)
    with pytest.raises(b.MxsError) as e:
        b.mxs_create_2d(**args)
    assert e.value.status == status
    assert b.mxs_last_error() != ""


def test_create_1d_batch_validation():
    with pytest.raises(b.MxsError) as e:
        b.mxs_create_1d_batch([0, 10, 13], b.MXS_P, b.MXS_F64, 2, 2, [1.0] * 5, None, FAKE_IN, FAKE_OUT)
    assert e.value.status == b.MXS_ERR_INVALID_ARG          # a signal shorter than the window
    with pytest.raises(b.MxsError) as e:
        b.mxs_create_1d_batch([1, 10], b.MXS_P, b.MXS_F64, 1, 1, [1.0] * 3, None, FAKE_IN, FAKE_OUT)
    assert e.value.status == b.MXS_ERR_INVALID_ARG
    with pytest.raises(b.MxsError) as e:
        b.mxs_create_1d_batch([0, 100], b.MXS_P, b.MXS_F64, 1, 1, [1.0] * 3, None, FAKE_IN, FAKE_IN + 64)
    assert e.value.status == b.MXS_ERR_ALIAS


def test_one_hip_runtime_in_the_process():
    """torch carries its own HIP runtime under the system soname; the binding
    loads torch first so that the library binds to the same copy (two
    runtimes in one process do not see each other's device state)."""
    import torch  # noqa: F401
    with open("/proc/self/maps") as f:
        libs = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    assert len(libs) == 1, libs
