"""GPU parity of the fourth-order Runge-Kutta integrator (the `rk4` solver of
"Kinetics solvers") against the oracle's RK4, through the C ABI.  FP64: normwise
relative error <= 1e-10 per state variable; FP32: the |dV| <= 0.5 mV and 1-dt
activation-time bars."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL
from parity_util import Problem, gpu_state, make_gpu, rec_arrays, rel_errs, run_oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
RK4 = O.INTEGRATOR_RK4


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_1605_06015_amd import bbx
    torch.cuda.set_device(0)
    return bbx


def cup(model, nx, ny, nz, scheme, seed=5):
    if model == O.MODEL_CRN:
        g = WL.crn_cup(nx, ny, nz, seed=seed)
        return Problem(g["mask"], 0.25, g["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01, scheme,
                       state=g["state"], stims=[(g["stim"], 40.0, 0.0, 2.0, 0.0, 1)],
                       theta=-40.0, integrator=RK4)
    # RK4 is only conditionally stable: TP06's sodium activation gate relaxes with
    # tau_m ~ 1e-3 ms near rest, so the step must stay below ~2.8 tau_m (0.02 ms, the
    # Rush-Larsen step of the TP06 workload, diverges)
    g = WL.tp06_cup(nx, ny, nz, seed=seed)
    return Problem(g["mask"], 0.25, g["fibre"], 0.3, 0.03, O.MODEL_TP06, [], 0.002, scheme,
                   state=g["state"], stims=[(g["stim"], 60.0, 0.0, 2.0, 0.0, 1)],
                   theta=-40.0, integrator=RK4)


@pytest.mark.parametrize("scheme", [O.SCHEME_ADDITIVE, O.SCHEME_SPLIT])
@pytest.mark.parametrize("model", [O.MODEL_CRN, O.MODEL_TP06])
def test_rk4_fp64_matches_oracle_through_upstroke(B, model, scheme):
    """A cup with rotating fibres, 8 ms (CRN) or 6 ms (TP06) from rest through the
    stimulus and the upstroke: every state variable and the recorder's activation
    times."""
    p = cup(model, 20, 20, 10, scheme)
    n = 800 if model == O.MODEL_CRN else 3000
    s = run_oracle(p, n)
    g = make_gpu(p, B.BBX_FP64)
    g.step(n)
    nv = s.state.shape[0]
    e = rel_errs(gpu_state(g, nv), s.state, p.mask)
    print("RK4 FP64 normwise errors", e.max())
    assert np.all(e <= TOL64), e
    ra = rec_arrays(s, p.mask)
    at = g.read(B.BBX_READ_ACT_TIME)
    m = p.mask == 1
    assert np.array_equal(np.isfinite(at[m]), np.isfinite(ra["at"][m]))
    fin = np.isfinite(ra["at"]) & m
    assert fin.sum() > 0
    assert np.abs(at[fin] - ra["at"][fin]).max() <= 1e-9


@pytest.mark.parametrize("model,params,dt,state_fn", [
    (O.MODEL_BARKLEY, [0.75, 0.02, 0.02], 0.008, "barkley"),
    (O.MODEL_FHN, [0.3, 0.7, 0.5], 0.01, "fhn"),
    (O.MODEL_ZFK, [0.13], 0.01, "zfk"),
    (O.MODEL_FK4, list(WL.FK4_EPI), 0.05, "fk4"),
    (O.MODEL_NONE, [], 0.01, "none"),
])
def test_rk4_fp64_light_models(B, model, params, dt, state_fn):
    """The light models on a random blob with random fibres (9-point 2D for Barkley,
    19-point 3D otherwise), 300 steps, both coupling schemes."""
    rng = np.random.default_rng(7)
    if state_fn == "barkley":
        mask = WL.random_blob_mask(40, 36, 1, seed=3, frac=0.7)
        h = 0.25
    else:
        mask = WL.random_blob_mask(18, 16, 12, seed=3, frac=0.6)
        h = 0.25 if state_fn == "fk4" else 0.5
    fib = WL.random_fibres(mask.shape, seed=4)
    Dp, Dt = (1.0, 0.3) if state_fn in ("barkley", "fhn", "zfk", "none") else (0.1171, 0.03)
    nv = O.nvar(model)
    st = np.zeros((nv,) + mask.shape)
    if state_fn == "fk4":
        st[0] = rng.uniform(0.0, 1.2, mask.shape)
        st[1] = rng.uniform(0.0, 1.0, mask.shape)
        st[2] = rng.uniform(0.0, 1.0, mask.shape)
        st[3] = rng.uniform(0.0, 1.0, mask.shape)
    else:
        for v in range(nv):
            st[v] = rng.uniform(-0.2, 1.0, mask.shape)
    st[:, mask == 0] = 0.0
    for scheme in (O.SCHEME_ADDITIVE, O.SCHEME_SPLIT):
        p = Problem(mask, h, fib, Dp, Dt, model, params, dt, scheme, state=st, integrator=RK4)
        s = run_oracle(p, 300)
        g = make_gpu(p, B.BBX_FP64)
        g.step(300)
        e = rel_errs(gpu_state(g, nv), s.state, mask)
        assert np.all(e <= TOL64), (scheme, e)
        g.close()


def test_rk4_fp32_bar_against_fp64_oracle(B):
    """FP32 RK4 on a CRN cup for 60 ms: |dV| <= 0.5 mV sampled every 1 ms, activation
    times within 1 dt, identical activated sets."""
    p = cup(O.MODEL_CRN, 24, 24, 12, O.SCHEME_ADDITIVE)
    s = run_oracle(p, 0)
    g = make_gpu(p, B.BBX_FP32)
    m = p.mask == 1
    worst = 0.0
    for k in range(60):
        s.step(100)
        g.step(100)
        worst = max(worst, np.abs(g.get(0)[m] - s.state[0][m]).max())
    ra = rec_arrays(s, p.mask)
    at = g.read(B.BBX_READ_ACT_TIME)
    print("RK4 FP32: max |dV| every 1 ms", worst)
    assert worst <= 0.5
    assert np.array_equal(np.isfinite(at[m]), np.isfinite(ra["at"][m]))
    fin = np.isfinite(ra["at"]) & m
    assert np.abs(at[fin] - ra["at"][fin]).max() <= p.dt


def test_rk4_full_size_crn_cup_sampled(B):
    """The 128x128x64 CRN workload under RK4 in FP64 for 3 steps with the stimulus on:
    every tissue voxel against the oracle's RK4 step (normwise <= 1e-10)."""
    c = WL.CRN_3D
    g0 = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"])
    p = Problem(g0["mask"], c["h"], g0["fibre"], c["Dpar"], c["Dperp"], O.MODEL_CRN, [], c["dt"],
                state=g0["state"], stims=[(g0["stim"], c["stim_amp"], 0.0, c["stim_ms"], 0.0, 1)],
                integrator=RK4)
    s = run_oracle(p, 3)
    g = make_gpu(p, B.BBX_FP64)
    g.step(3)
    e = rel_errs(gpu_state(g, 21), s.state, p.mask)
    assert np.all(e <= TOL64), e


def test_rk4_errors(B):
    g = B.Grid(np.ones((2, 2, 2), np.uint8), 0.25, None, 0.3, 0.03, B.BBX_FP32)
    g.model(B.BBX_MODEL_CRN, [], 0.01)
    with pytest.raises(B.BBXError) as ei:
        g.integrator(7)
    assert ei.value.code == B.BBX_EINVAL
    m = B.Mlp(21, 21, seed=1)
    g.surrogate(m, np.full(21, -1e30), np.full(21, 1e30), 1e30)
    with pytest.raises(B.BBXError) as ei:
        g.integrator(B.BBX_INTEGRATOR_RK4)
    assert ei.value.code == B.BBX_ENOTSUP
    g.surrogate(None)
    g.integrator(B.BBX_INTEGRATOR_RK4)
    with pytest.raises(B.BBXError) as ei:
        g.surrogate(m, np.full(21, -1e30), np.full(21, 1e30), 1e30)
    assert ei.value.code == B.BBX_ENOTSUP
    # tabulated CRN terms are ignored under RK4: same result as without the table
    g.tabulate(0.05)
    for v, val in enumerate(WL.CRN_INITIAL):
        g.fill(v, val)
    g.step(5)
    assert np.isfinite(g.get(0)).all()
