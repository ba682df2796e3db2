"""Batched 2D ensemble (many independent tissues, one launch per step) against the
FP64 oracle run tissue by tissue, plus the ensemble's own invariants: every tile
variant and the graph-replay mode give bitwise-identical results, and autotuning
leaves the state untouched."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL
from parity_util import rel_errs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
DT = 0.05
H = 0.25


@pytest.fixture(scope="module")
def B():
    from paper_1605_06015_amd import bbx
    return bbx


def small_ensemble(seed=11, sizes=((9, 13), (40, 33), (1, 17), (25, 1), (64, 5), (17, 70), (70, 66))):
    rng = np.random.default_rng(seed)
    n = len(sizes)
    nx = np.array([s[0] for s in sizes], np.int32)
    ny = np.array([s[1] for s in sizes], np.int32)
    Dp = 0.1171 * rng.uniform(0.8, 1.2, n)
    Dq = Dp / 4
    ang = rng.uniform(0, np.pi, n)
    prm = np.array(WL.FK4_EPI) * rng.uniform(0.8, 1.2, (n, 4))
    stims = []
    for i in range(n):
        stims.append((i, 0, min(3, int(nx[i])), 0, int(ny[i]), 1.0, 0.0, 2.0))
        if nx[i] > 8 and ny[i] > 8:
            stims.append((i, int(nx[i]) // 2, int(nx[i]), int(ny[i]) // 2, int(ny[i]), 0.6, 1.0, 1.5))
    return dict(nx=nx, ny=ny, Dpar=Dp, Dperp=Dq, angle=ang, params=prm, stims=stims)


def init_state(nx, ny, i, seed=3):
    """FK4 rest with a little seeded noise on u (so that every voxel differs)."""
    rng = np.random.default_rng(seed + i)
    st = np.stack([np.full((ny, nx), v) for v in WL.FK4_INITIAL])
    st[0] += rng.uniform(0, 0.004, (ny, nx))
    return st


def make_ens(B, w, prec, stream=None, theta=None):
    e = B.Ensemble(w["nx"], w["ny"], H, w["Dpar"], w["Dperp"], w["angle"], B.BBX_MODEL_FK4,
                   w["params"], DT, prec, stream)
    for i in range(len(w["nx"])):
        st = init_state(int(w["nx"][i]), int(w["ny"][i]), i)
        for v in range(4):
            e.set(i, v, st[v])
    for (i, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
        e.stimulus(i, x0, x1, y0, y1, amp, t0, dur)
    if theta is not None:
        e.record(theta)
    return e


def oracle_tissue(w, i, theta=None):
    nx, ny = int(w["nx"][i]), int(w["ny"][i])
    mask = np.ones((1, ny, nx), np.uint8)
    fib = np.zeros((1, ny, nx, 3))
    fib[..., 0] = np.cos(w["angle"][i])
    fib[..., 1] = np.sin(w["angle"][i])
    s = O.Sim(mask, H, fib, w["Dpar"][i], w["Dperp"][i], O.MODEL_FK4, list(w["params"][i]), DT)
    s.state[:] = init_state(nx, ny, i)[:, None]
    for (k, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
        if k != i:
            continue
        reg = np.zeros_like(mask)
        reg[0, y0:y1, x0:x1] = 1
        s.stimuli.append(O.Stimulus(reg, amp, int(round(t0 / DT)), int(round(dur / DT))))
    if theta is not None:
        s.start_recording(theta)
    return s, mask


def ens_state(e, i):
    return np.stack([e.get(i, v)[None] for v in range(4)])


def test_ensemble_fp64_matches_oracle_tissue_by_tissue(B):
    """Seven tissues (1 x 17 strips to 70 x 66, anisotropic, per-tissue D, angle and
    time constants, two stimuli each): 600 steps (30 ms, through the upstroke), every
    state variable within 1e-10 normwise; activation-time maps equal to 1e-9."""
    w = small_ensemble()
    e = make_ens(B, w, B.BBX_FP64, theta=0.5)
    e.step(600)
    for i in range(len(w["nx"])):
        s, mask = oracle_tissue(w, i, theta=0.5)
        s.step(600)
        err = rel_errs(ens_state(e, i), s.state, mask)
        assert np.all(err <= TOL64), (i, err)
        at_o = s.rec.at.reshape(mask.shape[1:])
        at_g = e.read(B.BBX_READ_ACT_TIME, i)
        assert np.array_equal(np.isnan(at_o), np.isnan(at_g)), i
        ok = ~np.isnan(at_o)
        if ok.any():
            assert np.abs(at_o[ok] - at_g[ok]).max() <= 1e-9, i
    assert e.read(B.BBX_READ_STEP, 0)[0] == 600


def test_ensemble_fp32_within_tolerance(B):
    """FP32 against the FP64 oracle over 60 ms: |du| <= 0.0075 (0.5 mV on the model's
    ~100 mV span of u ~ 1.5) sampled every 1 ms, activation times within 1 dt, equal
    activated sets."""
    w = small_ensemble(seed=12, sizes=((48, 40), (33, 57), (9, 9)))
    e = make_ens(B, w, B.BBX_FP32, theta=0.5)
    sims = [oracle_tissue(w, i, theta=0.5) for i in range(3)]
    worst = 0.0
    for _ in range(60):
        e.step(20)
        for i, (s, mask) in enumerate(sims):
            s.step(20)
            worst = max(worst, np.abs(e.get(i, 0) - s.state[0, 0]).max())
    print("ensemble fp32 max |du|:", worst)
    assert worst <= 0.0075
    for i, (s, mask) in enumerate(sims):
        at_o = s.rec.at.reshape(mask.shape[1:])
        at_g = e.read(B.BBX_READ_ACT_TIME, i)
        assert np.array_equal(np.isnan(at_o), np.isnan(at_g))
        ok = ~np.isnan(at_o)
        assert ok.sum() > 0.5 * ok.size
        assert np.abs(at_o[ok] - at_g[ok]).max() <= DT


@pytest.mark.parametrize("prec", [0, 1])
def test_tile_variants_bitwise_identical(B, prec):
    w = small_ensemble(seed=13)
    outs = []
    for v in range(B.BBX_ENS_NVARIANT):
        e = make_ens(B, w, prec, theta=0.5)
        e.variant(v)
        e.step(300)
        outs.append([np.concatenate([ens_state(e, i).ravel(), e.read(B.BBX_READ_ACT_TIME, i).ravel()])
                     for i in range(len(w["nx"]))])
        e.close()
    for v in range(1, len(outs)):
        for i in range(len(w["nx"])):
            assert np.array_equal(outs[0][i], outs[v][i], equal_nan=True), (v, i)


def test_graph_replay_equals_direct(B):
    """Graph mode (chunk 64) against direct launches, bitwise, over several step calls of
    mixed lengths with readouts in between (each graph replay is checked)."""
    w = small_ensemble(seed=14)
    a = make_ens(B, w, B.BBX_FP32, theta=0.5)
    b = make_ens(B, w, B.BBX_FP32, theta=0.5)
    b.graph(64)
    for n in (100, 37, 128, 64, 1, 200):
        a.step(n)
        b.step(n)
        for i in range(len(w["nx"])):
            assert np.array_equal(ens_state(a, i), ens_state(b, i)), (n, i)
            assert np.array_equal(a.read(B.BBX_READ_ACT_TIME, i), b.read(B.BBX_READ_ACT_TIME, i),
                                  equal_nan=True)
    assert a.read(B.BBX_READ_STEP, 0)[0] == b.read(B.BBX_READ_STEP, 0)[0] == 530


def test_tune_leaves_state_and_clock(B):
    w = small_ensemble(seed=15)
    e = make_ens(B, w, B.BBX_FP32, theta=0.5)
    e.step(50)
    before = [ens_state(e, i) for i in range(len(w["nx"]))]
    best, times = e.tune(10)
    assert 0 <= best < B.BBX_ENS_NVARIANT and e.variant() == best
    assert np.all(times > 0) and times[best] == times.min()
    assert e.read(B.BBX_READ_STEP, 0)[0] == 50
    for i in range(len(w["nx"])):
        assert np.array_equal(before[i], ens_state(e, i))
    # and stepping on continues exactly like an untuned ensemble
    ref = make_ens(B, w, B.BBX_FP32, theta=0.5)
    ref.step(50)
    e.step(70)
    ref.step(70)
    for i in range(len(w["nx"])):
        assert np.array_equal(ens_state(ref, i), ens_state(e, i))


def test_full_size_ensemble_few_steps(B):
    """The 96-tissue workload (24.0 M voxels, sides drawn from 64..768) in the launch configuration
    the benchmark times (graph mode, tuned tile): after 4 steps with S1 on, the smallest,
    a middle and the largest tissue match the FP64 oracle (FP32: |du| <= 1e-5, gates
    <= 1e-5 absolute and within 1e-3 of their own value)."""
    c = WL.FK4_ENSEMBLE
    w = WL.fk4_ensemble(n=c["n"], side_lo=c["side_lo"], side_hi=c["side_hi"], seed=c["seed"])
    e = B.Ensemble(w["nx"], w["ny"], c["h"], w["Dpar"], w["Dperp"], w["angle"], B.BBX_MODEL_FK4,
                   w["params"], c["dt"], B.BBX_FP32)
    for i in range(len(w["nx"])):
        s = int(w["nx"][i])
        for v, val in enumerate(WL.FK4_INITIAL):
            e.set(i, v, np.full(s * s, val))
    for (i, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
        e.stimulus(i, x0, x1, y0, y1, amp, t0, dur)
    e.record(c["theta"])
    e.tune(4)
    e.graph(2)
    e.step(4)
    order = np.argsort(w["nx"])
    for i in (order[0], order[len(order) // 2], order[-1]):
        s = int(w["nx"][i])
        mask = np.ones((1, s, s), np.uint8)
        fib = np.zeros((1, s, s, 3))
        fib[..., 0] = np.cos(w["angle"][i])
        fib[..., 1] = np.sin(w["angle"][i])
        o = O.Sim(mask, c["h"], fib, w["Dpar"][i], w["Dperp"][i], O.MODEL_FK4, list(w["params"][i]),
                  c["dt"], nthreads=8)
        for v, val in enumerate(WL.FK4_INITIAL):
            o.state[v] = val
        for (k, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
            if k == i:
                reg = np.zeros_like(mask)
                reg[0, y0:y1, x0:x1] = 1
                o.stimuli.append(O.Stimulus(reg, amp, int(round(t0 / c["dt"])), int(round(dur / c["dt"]))))
        o.step(4)
        for v in range(4):
            d = np.abs(e.get(i, v) - o.state[v, 0])
            assert d.max() <= 1e-5, (i, v)
            if v > 0:       # gates: also within 1e-3 of their own value
                assert np.all(d <= 1e-3 * np.abs(o.state[v, 0]) + 1e-9), (i, v)
    assert e.read(B.BBX_READ_NAN_FLAG, 0)[0] == 0


def test_grid_fk4_2d_fp64_matches_oracle(B):
    """The single-grid path runs the same model: a 2D anisotropic FK4 sheet with a ragged
    mask, FP64, 400 steps."""
    from parity_util import Problem, gpu_state, make_gpu, run_oracle
    mask = WL.random_blob_mask(50, 37, 1, seed=3)
    fib = WL.random_fibres(mask.shape, seed=4)
    fib[..., 2] = 0.0
    fib[..., 0] += 0.1
    st = np.stack([np.full(mask.shape, v) for v in WL.FK4_INITIAL])
    reg = np.zeros_like(mask)
    reg[:, :, :8] = 1
    p = Problem(mask, H, fib, 0.1171, 0.03, O.MODEL_FK4, list(WL.FK4_EPI), DT, state=st,
                stims=[(reg & mask, 1.0, 0.0, 2.0, 0.0, 1)])
    s = run_oracle(p, 400)
    g = make_gpu(p, 1)
    g.step(400)
    assert np.all(rel_errs(gpu_state(g, 4), s.state, mask) <= TOL64)


def test_ensemble_errors(B):
    one = np.array([8], np.int32)
    with pytest.raises(B.BBXError) as ex:
        B.Ensemble(one, one, H, 0.1, 0.1, 0.0, B.BBX_MODEL_CRN, np.zeros((1, 0)), DT)
    assert ex.value.code == B.BBX_ENOTSUP
    with pytest.raises(B.BBXError) as ex:
        B.Ensemble(one, one, H, 0.1, 0.1, 0.0, B.BBX_MODEL_FK4, np.zeros((1, 3)), DT)
    assert ex.value.code == B.BBX_EINVAL
    with pytest.raises(B.BBXError) as ex:
        B.Ensemble(one, one, H, 0.1, 0.1, 0.0, B.BBX_MODEL_FK4, [WL.FK4_EPI], 0.3)
    assert ex.value.code == B.BBX_EUNSTABLE
    with pytest.raises(B.BBXError) as ex:
        B.Ensemble(np.array([8, 0], np.int32), np.array([8, 8], np.int32), H, 0.1, 0.1, 0.0,
                   B.BBX_MODEL_FK4, [WL.FK4_EPI] * 2, DT)
    assert ex.value.code == B.BBX_EINVAL
    e = B.Ensemble(one, one, H, 0.1, 0.1, 0.0, B.BBX_MODEL_FK4, [WL.FK4_EPI], DT)
    for bad in (lambda: e.graph(3), lambda: e.variant(7), lambda: e.stimulus(0, 0, 9, 0, 1, 1.0, 0, 1),
                lambda: e.stimulus(1, 0, 1, 0, 1, 1.0, 0, 1), lambda: e.set(0, 4, np.zeros(64))):
        with pytest.raises(B.BBXError) as ex:
            bad()
        assert ex.value.code == B.BBX_EINVAL
    with pytest.raises(B.BBXError) as ex:
        e.read(B.BBX_READ_ACT_TIME, 0)
    assert ex.value.code == B.BBX_ESTATE


@pytest.mark.parametrize("model", ["none", "barkley", "zfk", "fhn"])
def test_ensemble_other_models_fp64(B, model):
    """The ensemble runs every 2D model: four tissues (13x9 to 1x11) with per-tissue
    parameters, D and fibre angle, random initial states, 300 steps, each tissue against
    the oracle within 1e-10 normwise per variable."""
    mid = {"none": O.MODEL_NONE, "barkley": O.MODEL_BARKLEY, "zfk": O.MODEL_ZFK, "fhn": O.MODEL_FHN}[model]
    base = {"none": [], "barkley": [0.75, 0.02, 0.02], "zfk": [0.13], "fhn": [0.3, 0.7, 0.5]}[model]
    nv = O.nvar(mid)
    sizes = [(13, 9), (30, 21), (1, 11), (17, 1)]
    rng = np.random.default_rng(21)
    n = len(sizes)
    nx = np.array([s[0] for s in sizes], np.int32)
    ny = np.array([s[1] for s in sizes], np.int32)
    Dp = rng.uniform(0.8, 1.2, n)
    Dq = Dp / 3
    ang = rng.uniform(0, np.pi, n)
    prm = np.array(base, float)[None, :] * rng.uniform(0.8, 1.2, (n, len(base))) if base else np.zeros((n, 0))
    h, dt = 0.5, 0.01
    e = B.Ensemble(nx, ny, h, Dp, Dq, ang, mid, prm, dt, B.BBX_FP64)
    states = []
    for i in range(n):
        st = np.stack([rng.uniform(0, 1 if v == 0 else 0.5, (int(ny[i]), int(nx[i]))) for v in range(nv)])
        states.append(st)
        for v in range(nv):
            e.set(i, v, st[v])
    e.step(300)
    for i in range(n):
        mask = np.ones((1, int(ny[i]), int(nx[i])), np.uint8)
        fib = np.zeros(mask.shape + (3,))
        fib[..., 0] = np.cos(ang[i])
        fib[..., 1] = np.sin(ang[i])
        s = O.Sim(mask, h, fib, Dp[i], Dq[i], mid, list(prm[i]), dt)
        s.state[:] = states[i][:, None]
        s.step(300)
        got = np.stack([e.get(i, v)[None] for v in range(nv)])
        err = rel_errs(got, s.state, mask)
        assert np.all(err <= TOL64), (model, i, err)
