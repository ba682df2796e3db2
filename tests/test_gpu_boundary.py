"""C-ABI completions: the whole-state readout as a checkpoint (the paper's `dump` /
`load` of the state), and a surrogate attached from host BF16 weights."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL
from parity_util import Problem, gpu_state, make_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1605_06015_amd import bbx
    torch.cuda.set_device(0)
    return bbx


@pytest.mark.parametrize("prec", [0, 1])
def test_all_state_checkpoint_resume_bitwise(B, prec):
    """Run 300 steps, read BBX_READ_ALL_STATE and the step, restore into a new grid, run
    300 more: bit for bit the uninterrupted 600-step run; ALL_STATE equals the
    per-variable readouts."""
    g0 = WL.crn_cup(24, 24, 12, seed=4)
    p = Problem(g0["mask"], 0.25, g0["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01, state=g0["state"],
                stims=[(g0["stim"], 40.0, 0.0, 2.0, 0.0, 1), (g0["stim"], 40.0, 4.0, 1.0, 0.0, 1)])
    ref = make_gpu(p, prec)
    ref.step(600)
    a = make_gpu(p, prec)
    a.step(300)
    st, n = a.checkpoint()
    assert n == 300
    per = gpu_state(a, 21)
    assert np.array_equal(st, per, equal_nan=True)
    b = make_gpu(p, prec)
    b.restore(st, n)
    b.step(300)
    assert np.array_equal(gpu_state(b, 21), gpu_state(ref, 21), equal_nan=True)


def test_surrogate_import_equals_attached_network(B):
    """A network's parameters with the weights rounded to BF16 on the host: attached via
    bbx_surrogate_import (BF16 bit patterns + FP32 biases + normalisation) and via a
    bbx_mlp holding the same values, 200 steps of the CRN cup give identical states."""
    import torch
    g0 = WL.crn_cup(24, 24, 12, seed=4)
    p = Problem(g0["mask"], 0.25, g0["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01, state=g0["state"],
                stims=[(g0["stim"], 40.0, 0.0, 2.0, 0.0, 1)])
    m = B.Mlp(21, 21, seed=7)
    rest = np.array(WL.CRN_INITIAL, np.float32)
    jitter = 1.0 + np.random.default_rng(0).normal(0, 1e-3, (64, 21)).astype(np.float32)
    S = torch.from_numpy(rest * jitter).cuda()          # states near rest, all positive
    g = make_gpu(p, 0)
    S1 = torch.empty_like(S)
    g.ionic_map(S, S1)
    m.fit_norm(S, S1)
    theta = m.get_params()
    nw1, nw2, nw3 = 128 * 21, 128 * 128, 21 * 128
    o = [0, nw1, nw1 + 128, nw1 + 128 + nw2, nw1 + 256 + nw2, nw1 + 256 + nw2 + nw3]
    W = np.concatenate([theta[o[0]:o[1]], theta[o[2]:o[3]], theta[o[4]:o[5]]]).astype(np.float32)
    bits = W.view(np.uint32)
    bits = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)      # round to nearest even
    Wr = (bits.astype(np.uint32) << 16).view(np.float32)
    theta_r = theta.copy()
    theta_r[o[0]:o[1]], theta_r[o[2]:o[3]], theta_r[o[4]:o[5]] = Wr[:nw1], Wr[nw1:nw1 + nw2], Wr[nw1 + nw2:]
    biases = np.concatenate([theta[o[1]:o[2]], theta[o[3]:o[4]], theta[o[5]:]]).astype(np.float32)
    m.set_params(theta_r)
    lo, hi = np.full(21, -1e30, np.float32), np.full(21, 1e30, np.float32)
    lo[0], hi[0] = -90.0, -70.0
    a = make_gpu(p, 0)
    a.surrogate(m, lo, hi, 5.0)
    b = make_gpu(p, 0)
    B.bbx_surrogate_import(b.handle, 21, 21, bits, biases, m.get_norm(), lo, hi, 5.0)
    a.step(200)
    b.step(200)
    assert a.read(B.BBX_READ_FALLBACK_COUNT)[0] == b.read(B.BBX_READ_FALLBACK_COUNT)[0]
    assert a.read(B.BBX_READ_FALLBACK_COUNT)[0] < 200 * a.nact
    assert np.array_equal(gpu_state(a, 21), gpu_state(b, 21), equal_nan=True)
    bad = m.get_norm()
    bad[3, 0] = -1.0
    with pytest.raises(B.BBXError) as ei:
        B.bbx_surrogate_import(b.handle, 21, 21, bits, biases, bad, lo, hi, 5.0)
    assert ei.value.code == B.BBX_EINVAL
    with pytest.raises(B.BBXError) as ei:
        B.bbx_surrogate_import(b.handle, 19, 19, bits, biases, m.get_norm(), lo, hi, 5.0)
    assert ei.value.code == B.BBX_EINVAL
