"""Graph replay of bbx_step (bbx_graph_set): bitwise the results of direct launches,
with stimulus windows, recording and the clock handled on the device, across chunk
boundaries and odd remainders, for the plain step, RK4 and both coupling schemes."""
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


@pytest.mark.parametrize("prec,scheme,integ", [(0, 0, 0), (1, 1, 0), (0, 0, 1)])
def test_graph_replay_bitwise_equals_direct(B, prec, scheme, integ):
    import torch
    g0 = WL.crn_cup(24, 24, 12, seed=4)
    p = Problem(g0["mask"], 0.25, g0["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01, scheme,
                state=g0["state"], theta=-40.0, integrator=integ,
                stims=[(g0["stim"], 40.0, 0.0, 2.0, 0.0, 1),
                       (g0["stim"], 30.0, 3.05, 0.37, 1.3, 3)])    # periodic, windows inside chunks
    s = torch.cuda.Stream()
    a = make_gpu(p, prec, s)
    b = make_gpu(p, prec, s)
    b.graph(64)
    for n in (5, 200, 64, 129, 1, 300):      # remainders, several chunks, odd starts
        a.step(n)
        b.step(n)
    torch.cuda.synchronize()
    assert int(a.read(B.BBX_READ_STEP)[0]) == int(b.read(B.BBX_READ_STEP)[0]) == 699
    assert np.array_equal(gpu_state(a, 21), gpu_state(b, 21), equal_nan=True)
    for w in (B.BBX_READ_ACT_TIME, B.BBX_READ_APD90, B.BBX_READ_VMAX):
        assert np.array_equal(a.read(w), b.read(w), equal_nan=True)
    assert np.isfinite(a.read(B.BBX_READ_ACT_TIME)).any()
    # a change of the stimuli drops the captured graphs; replay stays equal
    for g in (a, b):
        g.stimulus(g0["stim"], 20.0, 7.2, 0.5)
        g.clock(690)
        g.step(200)
    assert np.array_equal(gpu_state(a, 21), gpu_state(b, 21), equal_nan=True)


def test_graph_replay_with_surrogate_bitwise_equals_direct(B):
    """A surrogate attached (network accepting states near rest, the rest falling back):
    the captured graph holds the classifier and network launches of every step and
    alternates their list counters with the step number; graph and direct runs stay
    bitwise equal, fallback counts included, also after a clock change flips the step
    number's parity (the graph is captured again)."""
    import torch
    g0 = WL.crn_cup(24, 24, 12, seed=4)
    p = Problem(g0["mask"], 0.25, g0["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01,
                state=g0["state"], theta=-40.0, stims=[(g0["stim"], 40.0, 0.0, 2.0, 0.0, 1)])
    rng = np.random.default_rng(7)
    rest = np.array(WL.CRN_INITIAL, np.float32)
    S = (rest * (1 + 0.01 * rng.standard_normal((4096, 21)))).astype(np.float32)
    S1 = (S + 1e-3 * np.abs(rest) * rng.standard_normal((4096, 21))).astype(np.float32)
    S, S1 = torch.from_numpy(S).cuda(), torch.from_numpy(S1).cuda()
    m = B.Mlp(21, 21, seed=5)
    m.fit_norm(S, S1)
    lo, hi = S.min(0).values.cpu().numpy(), S.max(0).values.cpu().numpy()
    s = torch.cuda.Stream()
    a = make_gpu(p, B.BBX_FP32, s)
    b = make_gpu(p, B.BBX_FP32, s)
    for g in (a, b):
        g.surrogate(m, lo, hi, 5.0)
    b.graph(64)
    for n in (5, 200, 64, 129, 1, 300):
        a.step(n)
        b.step(n)
    torch.cuda.synchronize()
    fa, fb = (int(g.read(B.BBX_READ_FALLBACK_COUNT)[0]) for g in (a, b))
    print("fallback", fa, "of", a.nact * 699)
    assert fa == fb and 0 < fa < a.nact * 699
    assert np.array_equal(gpu_state(a, 21), gpu_state(b, 21), equal_nan=True)
    assert np.array_equal(a.read(B.BBX_READ_ACT_TIME), b.read(B.BBX_READ_ACT_TIME), equal_nan=True)
    for g in (a, b):
        g.clock(690)
        g.step(200)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_state(a, 21), gpu_state(b, 21), equal_nan=True)
    assert int(a.read(B.BBX_READ_FALLBACK_COUNT)[0]) == int(b.read(B.BBX_READ_FALLBACK_COUNT)[0])


def test_graph_errors(B):
    g = B.Grid(np.ones((2, 2, 2), np.uint8), 0.25, None, 0.3, 0.03, B.BBX_FP32)
    g.model(B.BBX_MODEL_NONE, [], 0.01)
    with pytest.raises(B.BBXError) as ei:
        g.graph(64)
    assert ei.value.code == B.BBX_ENOTSUP          # the null stream cannot be captured
    import torch
    h = B.Grid(np.ones((2, 2, 2), np.uint8), 0.25, None, 0.3, 0.03, B.BBX_FP32, torch.cuda.Stream())
    for bad in (3, -2, 5000):
        with pytest.raises(B.BBXError) as ei:
            h.graph(bad)
        assert ei.value.code == B.BBX_EINVAL
