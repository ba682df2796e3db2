"""Pins of the oracle's fourth-order Runge-Kutta integrator (the `rk4` solver of
"Kinetics solvers"): the exact amplification factor on linear test equations, the
forcing held through the four stages, and fourth-order convergence on nonlinear
kinetics against a tight implicit ODE solve."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL

ONE = np.ones((1, 1, 1), np.uint8)
RK4 = O.INTEGRATOR_RK4


def rk4_factor(z):
    """One classical RK4 step of y' = lam y multiplies y by 1 + z + z^2/2 + z^3/6 + z^4/24,
    z = lam dt (the Taylor polynomial of e^z to fourth order)."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def cell(model, params, y0, dt, integrator=RK4, stim=None):
    s = O.Sim(ONE, 1.0, None, 1.0, 1.0, model, list(params), dt, integrator=integrator)
    for i, v in enumerate(y0):
        s.set_state(i, v)
    if stim:
        s.stimuli.extend(stim)
    return s


def test_fk4_subthreshold_linear_closed_forms():
    """Below every threshold of the four-variable minimal model, u' = -u/400 and
    v' = (1 - v)/60 are linear and decoupled: RK4 gives u_n = u0 R(-dt/400)^n and
    v_n - 1 = (v0 - 1) R(-dt/60)^n exactly (up to rounding)."""
    dt, n = 0.05, 400
    s = cell(O.MODEL_FK4, WL.FK4_EPI, (0.005, 0.3, 0.9, 0.1), dt)
    for k in range(1, n + 1, 57):
        s.step(57 if k + 57 <= n + 1 else n + 1 - k)
    m = s.n
    u, v = s.state[0, 0, 0, 0], s.state[1, 0, 0, 0]
    assert abs(u - 0.005 * rk4_factor(-dt / 400.0) ** m) <= 1e-15
    assert abs((v - 1.0) - (0.3 - 1.0) * rk4_factor(-dt / 60.0) ** m) <= 1e-13
    # forward Euler / Rush-Larsen differs visibly at this step count: the two integrators
    # are distinct code paths
    e = cell(O.MODEL_FK4, WL.FK4_EPI, (0.005, 0.3, 0.9, 0.1), dt, O.INTEGRATOR_EULER_RL)
    e.step(m)
    assert abs(e.state[0, 0, 0, 0] - u) > 1e-12


def test_two_voxel_diffusion_forcing_held_through_stages():
    """Pure diffusion: V' = (L V)_p is the forcing, held at its step-n value, so RK4
    reduces to V + dt L V; on two coupled voxels d_n = d0 (1 - 2 dt w)^n exactly."""
    mask = np.ones((1, 1, 2), np.uint8)
    D, h, k = 0.7, 0.5, 0.05
    s = O.Sim(mask, h, None, D, D, O.MODEL_NONE, [], k, integrator=RK4)
    s.set_state(0, np.array([[[1.0, -0.25]]]))
    w = D / h ** 2
    for n in range(1, 30):
        s.step(1)
        v = s.state[0, 0, 0]
        assert abs((v[0] - v[1]) - 1.25 * (1 - 2 * k * w) ** n) < 1e-14


def test_zfk_stimulus_forcing_closed_form():
    """ZFK at V = 0 with a constant stimulus A for one step: the right-hand side is
    V(V - a)(1 - V) + A.  The exact RK4 stages give
      k1 = A, k2 = f(dt A/2) + A, k3 = f(dt k2/2) + A, k4 = f(dt k3) + A
    with f(V) = V (V - a)(1 - V); the oracle must reproduce that step."""
    a, dt, A = 0.13, 0.1, 0.7

    def f(V):
        return V * (V - a) * (1.0 - V)
    k1 = A
    k2 = f(0.5 * dt * k1) + A
    k3 = f(0.5 * dt * k2) + A
    k4 = f(dt * k3) + A
    want = dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    s = cell(O.MODEL_ZFK, (a,), (0.0,), dt, stim=[O.Stimulus(ONE, A, 0, 1)])
    s.step(1)
    assert abs(s.state[0, 0, 0, 0] - want) <= 1e-16
    # the stimulus window ends: the next step has no forcing, V decays towards 0
    v1 = s.state[0, 0, 0, 0]
    s.step(1)
    k1 = f(v1)
    k2 = f(v1 + 0.5 * dt * k1)
    k3 = f(v1 + 0.5 * dt * k2)
    k4 = f(v1 + dt * k3)
    assert abs(s.state[0, 0, 0, 0] - (v1 + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4))) <= 1e-16


def _converge(model, params, y0, T, dts, gate0, stim_amp=0.0, stim_ms=0.0):
    """Max-norm relative error at time T of the RK4 oracle vs a tight implicit solve of
    the same kinetics (gates as y' = (inf - y)/tau)."""
    nv = len(y0)
    gate = np.zeros(nv, bool)
    gate[gate0:] = True

    def rhs(t, y):
        r, inf, tau = O.model_eval(model, params, y)
        d = r.copy()
        d[gate] = (inf[gate] - y[gate]) / tau[gate]
        if t < stim_ms:
            d[0] += stim_amp
        return d

    if stim_ms:
        a = solve_ivp(rhs, (0, stim_ms), y0, method="Radau", rtol=1e-13, atol=1e-15)
        ref = solve_ivp(rhs, (stim_ms, T), a.y[:, -1], method="Radau", rtol=1e-13, atol=1e-15)
    else:
        ref = solve_ivp(rhs, (0, T), y0, method="Radau", rtol=1e-13, atol=1e-15)
    want = ref.y[:, -1]
    scale = np.maximum(np.abs(want), 1e-12)
    errs = []
    for dt in dts:
        st = [O.Stimulus(ONE, stim_amp, 0, int(round(stim_ms / dt)))] if stim_amp else []
        s = cell(model, params, y0, dt, stim=st)
        s.step(int(round(T / dt)))
        errs.append(np.max(np.abs(s.state[:, 0, 0, 0] - want) / scale))
    return np.array(errs)


@pytest.mark.parametrize("model,params,y0,T,dts,gate0", [
    (O.MODEL_FHN, (0.3, 0.7, 0.5), (1.5, -0.3), 3.0, [0.04, 0.02, 0.01], 2),
    (O.MODEL_BARKLEY, (0.75, 0.02, 0.02), (0.6, 0.1), 0.5, [0.004, 0.002, 0.001], 2),
])
def test_fourth_order_convergence_simple_models(model, params, y0, T, dts, gate0):
    e = _converge(model, list(params), np.array(y0, float), T, dts, gate0)
    order = np.log2(e[:-1] / e[1:])
    print("errors", e, "orders", order)
    assert np.all(order > 3.7) and np.all(order < 4.3), (e, order)


def test_fourth_order_convergence_crn_upstroke():
    """The CRN action potential's upstroke (1 ms of 20 pA/pF, state at 3 ms): every
    variable, gates included, converges at fourth order."""
    y0 = np.array(WL.CRN_INITIAL, float)
    e = _converge(O.MODEL_CRN, [], y0, 3.0, [0.02, 0.01, 0.005], 6, stim_amp=20.0, stim_ms=1.0)
    order = np.log2(e[:-1] / e[1:])
    print("errors", e, "orders", order)
    assert np.all(order > 3.6) and np.all(order < 4.4), (e, order)


def test_rk4_and_euler_agree_to_first_order():
    """On a 3D cup with rotating fibres (CRN, 2 ms with the stimulus on), the RK4 and
    Euler / Rush-Larsen states differ by O(dt): the RK4 path shares the stencil,
    stimulus and coupling of the other."""
    g = WL.crn_cup(16, 16, 8, seed=3)
    out = []
    for integ in (O.INTEGRATOR_EULER_RL, RK4):
        s = O.Sim(g["mask"], 0.25, g["fibre"], 0.3, 0.03, O.MODEL_CRN, [], 0.01, integrator=integ)
        s.state[:] = g["state"]
        s.stimuli.append(O.Stimulus(g["stim"], 40.0, 0, 200))
        s.step(200)
        out.append(s.state[0][g["mask"] == 1].copy())
    d = np.abs(out[0] - out[1]).max()
    assert 1e-6 < d < 5.0, d
