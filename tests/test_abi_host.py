"""Host-only checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects bad arguments before any device work (these
calls return before touching a GPU, so they run on a machine without one)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbx.h")


@pytest.fixture(scope="module")
def bbx():
    from paper_1605_06015_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_1605_06015_amd import bbx as mod
    return mod


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbx_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("bbx_grid_create", "bbx_model_set", "bbx_stimulus_add", "bbx_step",
                 "bbx_readout", "bbx_grid_destroy", "bbx_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol(bbx):
    lib = C.CDLL(bbx.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(bbx.SIGNATURES)


def _err(fn, *a):
    with pytest.raises(Exception) as ei:
        fn(*a)
    return getattr(ei.value, "code", None)


def test_create_validation_before_device(bbx):
    m = np.ones((2, 3, 4), np.uint8)
    E = bbx.BBX_EINVAL
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.0, m, None, 1, 1, bbx.BBX_FP32) == E
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.1, m, None, -1, 1, bbx.BBX_FP32) == E
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.1, m, None, 1, 0.0, bbx.BBX_FP32) == E
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.1, m, None, 1, 1, 7) == E
    assert _err(bbx.bbx_grid_create, 0, 3, 2, 0.1, np.ones(0, np.uint8), None, 1, 1, 0) == E
    fib = np.ones((2, 3, 4, 3))
    fib[1, 2, 3] = 0.0
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.1, m, fib, 1, 0.1, bbx.BBX_FP32) == E
    assert "fibre" in bbx.bbx_last_error()
    fib[1, 2, 3] = np.nan
    assert _err(bbx.bbx_grid_create, 4, 3, 2, 0.1, m, fib, 1, 0.1, bbx.BBX_FP32) == E
    # raw NULL mask through the C ABI
    out = C.c_void_p()
    rc = bbx._lib.bbx_grid_create(4, 3, 2, 0.1, None, None, 1.0, 1.0, 0, None, C.byref(out))
    assert rc == bbx.BBX_EINVAL and not out.value


def test_null_grid_calls_fail_cleanly(bbx):
    lib = bbx._lib
    assert lib.bbx_step(None, 1) == bbx.BBX_EINVAL
    assert lib.bbx_model_set(None, 0, None, 0, 0.1, 0) == bbx.BBX_EINVAL
    assert lib.bbx_state_set(None, 0, None) == bbx.BBX_EINVAL
    assert lib.bbx_stimulus_add(None, None, 1.0, 0.0, 1.0, 0.0, 1) == bbx.BBX_EINVAL
    assert lib.bbx_recording_set(None, 0.5) == bbx.BBX_EINVAL
    assert lib.bbx_readout(None, 0, 0, None, None, 0, 0) == bbx.BBX_EINVAL
    v = C.c_int64()
    assert lib.bbx_info(None, 0, C.byref(v)) == bbx.BBX_EINVAL
    lib.bbx_grid_destroy(None)
    assert "NULL" in bbx.bbx_last_error()
