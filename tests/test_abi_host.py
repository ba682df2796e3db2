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
    assert lib.bbx_state_fill(None, 0, 1.0) == bbx.BBX_EINVAL
    assert lib.bbx_ecg_set(None, 0, None, 0, 0) == bbx.BBX_EINVAL
    assert lib.bbx_tabulation_set(None, 0.1) == bbx.BBX_EINVAL


def test_ensemble_validation_before_device(bbx):
    """Every argument check of bbx_ensemble_create runs before any device work."""
    E = bbx.BBX_EINVAL
    one = np.array([8], np.int32)
    p4 = np.array([[0.11, 30.0, 1.9, 200.0]])
    mk = lambda *a, **k: bbx.bbx_ensemble_create(*a, **k)
    # sizes, coefficients, model and parameter count
    assert _err(mk, np.array([0], np.int32), one, 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4, 0.05, 0) == E
    assert _err(mk, one, one, 0.0, 0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4, 0.05, 0) == E
    assert _err(mk, one, one, 0.25, -0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4, 0.05, 0) == E
    assert _err(mk, one, one, 0.25, 0.1, 0.1, np.nan, bbx.BBX_MODEL_FK4, p4, 0.05, 0) == E
    assert _err(mk, one, one, 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4[:, :3], 0.05, 0) == E
    assert _err(mk, one, one, 0.25, 0.1, 0.1, 0.0, 42, p4, 0.05, 0) == E
    assert _err(mk, one, one, 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4, 0.05, 3) == E
    assert _err(mk, one, one, 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_CRN, np.zeros((1, 0)), 0.05, 0) == \
        bbx.BBX_ENOTSUP
    assert _err(mk, one, one, 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_FK4, p4, 0.3, 0) == bbx.BBX_EUNSTABLE
    # more than 2^31 voxels in total (checked before any allocation)
    big = np.array([65536, 65536], np.int32)
    assert _err(mk, big, np.array([32768, 32768], np.int32), 0.25, 0.1, 0.1, 0.0, bbx.BBX_MODEL_NONE,
                np.zeros((2, 0)), 0.05, 0) == E
    assert "2^31" in bbx.bbx_last_error()
    lib = bbx._lib
    assert lib.bbx_ensemble_step(None, 1) == E
    assert lib.bbx_ensemble_state_set(None, 0, 0, None) == E
    assert lib.bbx_ensemble_graph_set(None, 2) == E
    assert lib.bbx_ensemble_variant_set(None, 0) == E
    assert lib.bbx_ensemble_tune(None, 1, None, None) == E
    assert lib.bbx_ensemble_recording_set(None, 0.5) == E
    assert lib.bbx_ensemble_stimulus_add(None, 0, 0, 1, 0, 1, 1.0, 0.0, 1.0, 0.0, 1) == E
    v = C.c_int64()
    assert lib.bbx_ensemble_info(None, 0, C.byref(v)) == E
    lib.bbx_ensemble_destroy(None)


def test_slab_bounds_tissue_balanced(bbx):
    """bbx_slab_bounds (host only): strictly increasing plane boundaries from 0 to nz,
    each at the plane boundary nearest to k/nslab of the tissue (brute force over all
    boundaries), on an uneven mask."""
    from paper_1605_06015_amd import workloads as WL
    g = WL.cup_shell(40, 36, 20, 0.25, 0.35, seed=2)
    mask = g["mask"]
    per_plane = mask.reshape(mask.shape[0], -1).sum(axis=1)
    cum = np.concatenate([[0], np.cumsum(per_plane)])
    for nslab in (1, 2, 3, 5, 8, 20):
        zb = bbx.bbx_slab_bounds(mask, nslab)
        assert zb[0] == 0 and zb[-1] == mask.shape[0]
        assert np.all(np.diff(zb) >= 1)
        for k in range(1, nslab):
            target = cum[-1] * k / nslab
            lo, hi = zb[k - 1] + 1, mask.shape[0] - (nslab - k)
            best = min(range(lo, hi + 1), key=lambda z: (abs(cum[z] - target), z))
            assert abs(cum[zb[k]] - target) <= abs(cum[best] - target) + 1e-9, (nslab, k)
    E = bbx.BBX_EINVAL
    assert _err(bbx.bbx_slab_bounds, mask, 0) == E
    assert _err(bbx.bbx_slab_bounds, mask, mask.shape[0] + 1) == E


def test_slab_validation_before_device(bbx):
    m = np.ones((6, 3, 4), np.uint8)
    E = bbx.BBX_EINVAL
    assert _err(bbx.bbx_slab_create, m, 3, 3, 0.1, None, 1, 1, bbx.BBX_FP32) == E
    assert _err(bbx.bbx_slab_create, m, -1, 3, 0.1, None, 1, 1, bbx.BBX_FP32) == E
    assert _err(bbx.bbx_slab_create, m, 2, 7, 0.1, None, 1, 1, bbx.BBX_FP32) == E
    lib = bbx._lib
    assert lib.bbx_halo_pack(None, 0, None, 0) == E
    assert lib.bbx_halo_unpack(None, 1, None, 0) == E


def test_log_switch_reports_failures(bbx):
    """BBX_LOG=1 makes a failing call write its code and message to stderr (a child
    process, so that the switch is read fresh); without it the library stays silent."""
    import subprocess
    import sys
    code = ("import numpy as np; from paper_1605_06015_amd import bbx as B\n"
            "try:\n"
            "    B.bbx_slab_bounds(np.ones((4, 3, 3), np.uint8), 9)\n"
            "except B.BBXError as e:\n"
            "    print('raised', e.code)\n")
    out = {}
    for flag in ("1", "0"):
        env = dict(os.environ, BBX_LOG=flag)
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        assert "raised" in r.stdout
        out[flag] = r.stderr
    assert "bbx: error -1: nslab must be in [1, nz]" in out["1"]
    assert "bbx:" not in out["0"]
