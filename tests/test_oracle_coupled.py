"""Pins of the oracle's coupled reaction-diffusion step against closed forms:
the ZFK/Nagumo travelling front (eqs (ZFKsolnV), speed c = sqrt(2 D)(1/2 - alpha),
reduced to the monodomain case) with second-order convergence of the speed
under h-refinement at dt = 3h^2/(16 D_par); conservation of pure diffusion
under no-flux with a uniform tensor; and the Bessel-disk test of eqs
(HTestPDE)-(HTestSolution) with the convergence behaviour the paper reports."""
import numpy as np
import pytest
from scipy.special import j0, jn_zeros

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL


def front_position(V, h):
    """x where V crosses 1/2 (V decreasing in x), by linear interpolation."""
    i = np.nonzero((V[:-1] >= 0.5) & (V[1:] < 0.5))[0]
    assert i.size == 1
    i = i[0]
    return h * (i + (V[i] - 0.5) / (V[i] - V[i + 1]))


def zfk_speed(h, axis, angle_deg, scheme=O.SCHEME_ADDITIVE, alpha=0.13, Dpar=1.0, Dperp=0.25):
    L, T1, T2 = 40.0, 4.0, 24.0
    n = int(round(L / h)) + 1
    shape = [1, 1, 1]
    shape[2 - axis] = n
    mask = np.ones(shape, np.uint8)
    a = np.deg2rad(angle_deg)
    f = np.zeros(3)
    f[axis] = np.cos(a)
    f[(axis + 1) % 3] = np.sin(a)
    fib = np.broadcast_to(f, tuple(shape) + (3,)).copy()
    Deff = Dperp + (Dpar - Dperp) * np.cos(a) ** 2
    dt = 3 * h * h / (16 * Dpar)
    x = h * np.arange(n)
    V0 = 1.0 / (1.0 + np.exp((x - 8.0) / np.sqrt(2 * Deff)))
    s = O.Sim(mask, h, fib, Dpar, Dperp, O.MODEL_ZFK, [alpha], dt, scheme=scheme)
    s.set_state(0, V0.reshape(shape))
    n1, n2 = int(round(T1 / dt)), int(round(T2 / dt))
    s.step(n1)
    p1 = front_position(s.state[0].ravel(), h)
    s.step(n2 - n1)
    p2 = front_position(s.state[0].ravel(), h)
    c_num = (p2 - p1) / ((n2 - n1) * dt)
    c_ex = np.sqrt(2 * Deff) * (0.5 - alpha)
    return c_num, c_ex


@pytest.mark.parametrize("axis,angle", [(0, 0.0), (0, 90.0), (1, 30.0), (2, 60.0)])
def test_zfk_front_speed_second_order(axis, angle):
    errs = []
    for h in (0.4, 0.2, 0.1):
        c, cex = zfk_speed(h, axis, angle)
        errs.append(abs(c - cex) / cex)
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert errs[-1] < 3e-3
    assert np.all(order > 1.6) and np.all(order < 2.4), (errs, order)


def test_zfk_split_scheme_converges_to_same_speed():
    errs = []
    for h in (0.4, 0.2, 0.1):
        c, cex = zfk_speed(h, 0, 0.0, scheme=O.SCHEME_SPLIT)
        errs.append(abs(c - cex) / cex)
    assert errs[-1] < 3e-3 and errs[0] / errs[-1] > 8


def test_pure_diffusion_conserved_on_cup_uniform_tensor():
    g = WL.cup_shell(48, 48, 24, 0.25, 0.35, seed=2)
    mask = g["mask"]
    fib = np.broadcast_to(np.array([0.3, -0.5, 0.8]), mask.shape + (3,)).copy()
    s = O.Sim(mask, 0.25, fib, 0.3, 0.03, O.MODEL_NONE, [], 0.01)
    u0 = np.random.default_rng(3).uniform(-80, 20, mask.shape) * mask
    s.set_state(0, u0)
    tot0 = u0.sum()
    s.step(2000)
    assert abs(s.state[0].sum() - tot0) < 1e-12 * np.abs(u0).sum()
    # and diffusion decays the variance
    assert s.state[0][mask == 1].std() < 0.5 * u0[mask == 1].std()


def test_pure_diffusion_nonconservative_with_rotating_fibres():
    """Rotating fibres make Wtilde nonzero and L non-symmetric; the oracle must not be
    accidentally conservative there (guards against a dropped Wtilde term)."""
    g = WL.cup_shell(48, 48, 24, 0.25, 0.35, seed=2)
    s = O.Sim(g["mask"], 0.25, g["fibre"], 0.3, 0.03, O.MODEL_NONE, [], 0.01)
    u0 = np.random.default_rng(3).uniform(-80, 20, g["mask"].shape) * g["mask"]
    s.set_state(0, u0)
    s.step(200)
    assert abs(s.state[0].sum() - u0.sum()) > 1e-9 * np.abs(u0).sum()


def bessel_errors(h, off):
    """Unit disk centred at offset*h from a grid node, u_t = lap u, no-flux, dt = h^2/80,
    T = 0.2; returns (Linf, L2) over space and all time steps (trapezoid in time)."""
    jr = jn_zeros(1, 1)[0]
    n = int(np.ceil(2.0 / h)) + 5
    c = np.array([(n // 2 + off[0]) * h, (n // 2 + off[1]) * h])
    x = h * np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r = np.hypot(X - c[0], Y - c[1])
    inside = r <= 1.0
    mask = inside.astype(np.uint8)[None]
    T = 0.2
    nsteps = int(round(T / (h * h / 80.0)))
    dt = T / nsteps
    s = O.Sim(mask, h, None, 1.0, 1.0, O.MODEL_NONE, [], dt)
    u0 = np.where(inside, j0(jr * r), 0.0)
    s.set_state(0, u0[None])
    shape_ex = j0(jr * r[inside])
    linf, acc = 0.0, []
    for k in range(nsteps + 1):
        if k:
            s.step(1)
        e = s.state[0, 0][inside] - shape_ex * np.exp(-jr * jr * k * dt)
        linf = max(linf, np.abs(e).max())
        acc.append((e * e).sum() * h * h)
    acc = np.array(acc)
    integral = dt * (acc.sum() - 0.5 * (acc[0] + acc[-1]))
    l2 = np.sqrt(integral / (T * inside.sum() * h * h))
    return linf, l2


@pytest.mark.slow
def test_bessel_disk_convergence_between_first_and_second_order():
    hs = [0.1, 0.05, 0.025]
    offs = [(0, 0), (0.2, 0.2), (0.2, 0.6), (0.6, 0.6)]
    lh, linf, l2 = [], [], []
    for h in hs:
        for o in offs:
            a, b = bessel_errors(h, o)
            lh.append(np.log(h))
            linf.append(np.log(a))
            l2.append(np.log(b))
    s_inf = np.polyfit(lh, linf, 1)[0]
    s_2 = np.polyfit(lh, l2, 1)[0]
    # The paper: convergence worse than h^2 but better than h^1, and the L2 norm
    # converging faster than Linf (best-fit slopes 1.564 and 1.719).
    assert 1.0 < s_inf < 2.0 and 1.0 < s_2 < 2.1
    # (Measured here: 1.27 and 1.62 over h = 0.1..0.025; the paper's h range sits in a
    # figure that is not available, so the printed slopes are not asserted.)
    assert s_2 > s_inf + 0.1, (s_inf, s_2)
