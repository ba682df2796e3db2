"""Degenerate boxes: a one-voxel-thick cable along x, y or z (fibres along the cable), a
stimulus at one end and a wave along it.  Dense boxes whose tiles are almost empty (a
64 x 4 tile holding one column) take the z-marching kernels for the light models and the
one-voxel-per-thread kernel for CRN; against the oracle: FP64 state <= 1e-10 normwise, FP32
activation times within 1 dt, and the conduction velocity the two runs imply (for ZFK also
within 1% of the equation's closed-form front speed)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL
from parity_util import Problem, gpu_state, make_gpu, rel_errs, run_oracle

pytestmark = pytest.mark.gpu

N = 160
TOL64 = 1e-10


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1605_06015_amd import bbx
    torch.cuda.set_device(0)
    return bbx


def cable(axis, model):
    shape = [1, 1, 1]
    shape[2 - axis] = N                               # (nz, ny, nx); axis 0 = x
    mask = np.ones(shape, np.uint8)
    fib = np.zeros(tuple(shape) + (3,))
    fib[..., axis] = 1.0
    stim = np.zeros_like(mask)
    idx = [0, 0, 0]
    for k in range(5):
        idx[2 - axis] = k
        stim[tuple(idx)] = 1
    if model == "crn":
        st = np.stack([np.full(shape, v) for v in WL.CRN_INITIAL])
        return Problem(mask, 0.25, fib, 0.3, 0.03, O.MODEL_CRN, [], 0.01, state=st, theta=-40.0,
                       stims=[(stim, 40.0, 0.0, 2.0, 0.0, 1)]), 4000
    st = np.zeros((1,) + tuple(shape))
    return Problem(mask, 0.25, fib, 1.0, 0.3, O.MODEL_ZFK, [0.13], 0.01, state=st, theta=0.5,
                   stims=[(stim, 2.0, 0.0, 0.5, 0.0, 1)]), 6000


@pytest.mark.parametrize("model", ["zfk", "crn"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cable_matches_oracle(B, axis, model):
    p, steps = cable(axis, model)
    nv = p.state.shape[0]
    s = run_oracle(p, steps)
    g64 = make_gpu(p, B.BBX_FP64)
    g64.step(steps)
    e = rel_errs(gpu_state(g64, nv), s.state, p.mask)
    assert np.all(e <= TOL64), e
    g32 = make_gpu(p, B.BBX_FP32)
    g32.step(steps)
    at_o = np.asarray(s.rec.at)
    at = g32.read(B.BBX_READ_ACT_TIME).ravel()
    fa = np.isfinite(at_o)
    assert fa.sum() > N // 3, fa.sum()                # the wave travelled
    # the activated sets agree, up to a voxel crossing the threshold in the last steps
    t_end = steps * p.dt
    differ = np.isfinite(at) != fa
    late = np.fmin(np.nan_to_num(at, nan=np.inf), np.nan_to_num(at_o, nan=np.inf)) >= t_end - 2 * p.dt
    assert not (differ & ~late).any()
    both = fa & np.isfinite(at)
    assert np.abs(at[both] - at_o[both]).max() <= p.dt
    k = np.flatnonzero(both)
    i1, i2 = k[len(k) // 3], k[-1]
    cv_o = (i2 - i1) * p.h / (at_o[i2] - at_o[i1])
    cv = (i2 - i1) * p.h / (at[i2] - at[i1])
    print(f"axis {axis} {model}: {fa.sum()} voxels activated, CV oracle {cv_o:.4f} FP32 {cv:.4f} mm/ms")
    assert abs(cv - cv_o) <= 1e-3 * cv_o
    if model == "zfk":
        # the continuum front speed sqrt(2 D) (1/2 - alpha) of the ZFK equation
        c = np.sqrt(2.0 * p.Dpar) * (0.5 - p.params[0])
        assert abs(cv - c) <= 0.01 * c, (cv, c)
