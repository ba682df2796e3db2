"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  FP64 mode: normwise relative error <= 1e-10 per state
variable.  FP32 mode: the tolerances stated with each test."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL
from parity_util import Problem, gpu_state, make_gpu, rec_arrays, rel_errs, run_oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def B():
    from paper_1605_06015_amd import bbx
    return bbx


def crn_problem(nx, ny, nz, seed=5, stim_amp=40.0, stim_ms=2.0, dt=0.01, theta=None):
    g = WL.crn_cup(nx, ny, nz, seed=seed)
    return Problem(g["mask"], 0.25, g["fibre"], 0.3, 0.03, O.MODEL_CRN, [], dt,
                   state=g["state"], stims=[(g["stim"], stim_amp, 0.0, stim_ms, 0.0, 1)],
                   theta=theta)


# ------------------------------------------------------------------ geometry (weights)
@pytest.mark.parametrize("case", ["blob_random_fibres", "cup_rotating", "iso_blob", "dense_aniso",
                                  "plane_2d"])
@pytest.mark.parametrize("prec", [1, 0])
def test_weights_match_oracle(B, case, prec):
    if case == "blob_random_fibres":
        mask = WL.random_blob_mask(13, 11, 9, seed=11, frac=0.55)
        fib = WL.random_fibres(mask.shape, seed=12)
        Dp, Dt = 1.3, 0.2
    elif case == "cup_rotating":
        g = WL.cup_shell(40, 40, 20, 0.25, 0.35, seed=3)
        mask, fib, Dp, Dt = g["mask"], g["fibre"], 0.3, 0.03
    elif case == "iso_blob":
        mask, fib, Dp, Dt = WL.random_blob_mask(17, 9, 5, seed=2), None, 0.7, 0.7
    elif case == "dense_aniso":
        mask, fib = WL.full_box_rotating(11, 7, 5)
        Dp, Dt = 0.3, 0.03
    else:
        mask = WL.random_blob_mask(29, 23, 1, seed=4, frac=0.7)
        fib = WL.random_fibres(mask.shape, seed=5)
        Dp, Dt = 1.0, 0.25
    h = 0.25
    act, Wo = O.weights(mask, h, fib, Dp, Dt)
    g = B.Grid(mask, h, fib, Dp, Dt, prec)
    Wg = g.read(B.BBX_READ_WEIGHTS)
    assert Wg.shape == Wo.shape
    tol = 1e-13 if prec == 1 else 2e-6
    assert np.abs(Wg - Wo).max() <= tol * np.abs(Wo).max()
    g.close()


# ------------------------------------------------------------------ FP64 parity
def test_barkley_2d_cross_field_fp64_full_run():
    c = WL.BARKLEY_2D
    u, v = WL.barkley_cross_field(c["nx"], c["ny"], seed=0)
    mask = np.ones((1, c["ny"], c["nx"]), np.uint8)
    p = Problem(mask, c["h"], None, c["D"], c["D"], O.MODEL_BARKLEY, [c["a"], c["b"], c["eps"]],
                c["dt"], state=np.stack([u, v]))
    s = run_oracle(p, c["steps"])
    g = make_gpu(p, 1)
    g.step(c["steps"])
    e = rel_errs(gpu_state(g, 2), s.state, mask)
    assert np.all(e <= TOL64), e


def test_barkley_2d_fp32_against_fp64_oracle():
    """FP32: per-step rounding ~6e-8 relative, accumulated over 2000 explicit steps of a
    rotating spiral; the bound 5e-4 (normwise relative) is the FP32 contract for the
    dimensionless models."""
    c = WL.BARKLEY_2D
    u, v = WL.barkley_cross_field(c["nx"], c["ny"], seed=0)
    mask = np.ones((1, c["ny"], c["nx"]), np.uint8)
    p = Problem(mask, c["h"], None, c["D"], c["D"], O.MODEL_BARKLEY, [c["a"], c["b"], c["eps"]],
                c["dt"], state=np.stack([u, v]))
    s = run_oracle(p, c["steps"])
    g = make_gpu(p, 0)
    g.step(c["steps"])
    e = rel_errs(gpu_state(g, 2), s.state, mask)
    print("barkley fp32 normwise rel err", e)
    assert np.all(e <= 5e-4), e


@pytest.mark.parametrize("scheme", [0, 1])
def test_pure_diffusion_cup_rotating_fibres_fp64(scheme):
    gg = WL.cup_shell(40, 40, 20, 0.25, 0.35, seed=3)
    mask = gg["mask"]
    u0 = np.random.default_rng(7).uniform(-80, 20, mask.shape) * mask
    p = Problem(mask, 0.25, gg["fibre"], 0.3, 0.03, O.MODEL_NONE, [], 0.01, scheme=scheme,
                state=u0[None])
    s = run_oracle(p, 300)
    g = make_gpu(p, 1)
    g.step(300)
    e = rel_errs(gpu_state(g, 1), s.state, mask)
    assert e[0] <= TOL64, e


@pytest.mark.parametrize("scheme", [0, 1])
def test_zfk_random_fibres_3d_fp64(scheme):
    mask = WL.random_blob_mask(19, 15, 11, seed=21, frac=0.6)
    fib = WL.random_fibres(mask.shape, seed=22)
    rng = np.random.default_rng(23)
    V0 = (rng.uniform(0, 1, mask.shape) > 0.7).astype(float) * mask
    p = Problem(mask, 0.5, fib, 1.0, 0.2, O.MODEL_ZFK, [0.13], 0.02, scheme=scheme,
                state=V0[None])
    s = run_oracle(p, 400)
    g = make_gpu(p, 1)
    g.step(400)
    e = rel_errs(gpu_state(g, 1), s.state, mask)
    assert e[0] <= TOL64, e


def test_fhn_ragged_2d_anisotropic_fp64():
    mask = WL.random_blob_mask(37, 23, 1, seed=31, frac=0.75)
    fib = WL.random_fibres(mask.shape, seed=32)
    rng = np.random.default_rng(33)
    st = np.stack([rng.uniform(-2, 2, mask.shape), rng.uniform(-1, 1, mask.shape)]) * mask
    p = Problem(mask, 0.4, fib, 1.0, 0.25, O.MODEL_FHN, [0.3, 0.7, 0.5], 0.01, state=st)
    s = run_oracle(p, 500)
    g = make_gpu(p, 1)
    g.step(500)
    e = rel_errs(gpu_state(g, 2), s.state, mask)
    assert np.all(e <= TOL64), e


def test_crn_small_cup_fp64_through_upstroke():
    p = crn_problem(24, 24, 12)
    n = 1500
    s = run_oracle(p, n, nthreads=8)
    g = make_gpu(p, 1)
    g.step(n)
    e = rel_errs(gpu_state(g, 21), s.state, p.mask)
    assert np.all(e <= TOL64), e
    assert s.state[0][p.mask == 1].max() > -20.0      # the tissue is excited (plateau)


@pytest.mark.parametrize("prec,tol", [(1, TOL64), (0, None)])
def test_crn_full_size_few_steps(prec, tol):
    """The 128x128x64 cup (367k tissue voxels) in the launch configuration the benchmark
    times: every tissue voxel after 3 steps with the stimulus on.  FP32: |dV| <= 1e-3 mV
    and concentrations within 1e-5 normwise; gates within 1e-5 absolute and 1e-3 of their
    own value (so a gate that stays small, x_r ~ 3e-5 at rest, is checked too)."""
    p = crn_problem(128, 128, 64, seed=1)
    s = run_oracle(p, 3, nthreads=8)
    g = make_gpu(p, prec)
    g.step(3)
    x = gpu_state(g, 21)
    e = rel_errs(x, s.state, p.mask)
    if prec == 1:
        assert np.all(e <= tol), e
    else:
        # gates live in [0, 1]: absolute and pointwise relative error; concentrations:
        # normwise relative
        m = p.mask == 1
        assert np.abs(x[0][m] - s.state[0][m]).max() <= 1e-3
        assert np.all(e[1:6] <= 1e-5), e
        for v in range(6, 21):
            d = np.abs(x[v][m] - s.state[v][m])
            rel = (d / (np.abs(s.state[v][m]) + 1e-9)).max()
            print("gate", v, "abs", d.max(), "rel", rel)
            assert d.max() <= 1e-5 and rel <= 1e-3, (v, d.max(), rel)


def test_crn_fp32_within_0p5mV_and_1dt():
    """FP32 vs the FP64 oracle on a reduced cup over 60 ms (stimulus, upstroke,
    propagation): max |dV| <= 0.5 mV sampled every 1 ms; activation times within 1 dt
    on the voxels activated in both runs; same activated set."""
    p = crn_problem(24, 24, 12, theta=-40.0)
    s = run_oracle(p, 0, nthreads=8)
    g = make_gpu(p, 0)
    m = p.mask == 1
    worst = 0.0
    for _ in range(60):
        s.step(100)
        g.step(100)
        worst = max(worst, np.abs(g.get(0)[m] - s.state[0][m]).max())
    assert worst <= 0.5, worst
    ro = rec_arrays(s, p.mask)
    at_g = g.read(1)
    act_o = np.isfinite(ro["at"]) & m
    act_g = np.isfinite(at_g) & m
    assert np.array_equal(act_o, act_g)
    assert act_o.sum() > 0.5 * m.sum()
    assert np.abs(at_g[act_o] - ro["at"][act_o]).max() <= p.dt
    print("crn fp32 max |dV| (mV):", worst, " max |dAT| (ms):",
          np.abs(at_g[act_o] - ro["at"][act_o]).max())


def test_recording_crn_fp64_full_action_potential():
    p = crn_problem(12, 12, 6, seed=8, theta=-40.0)
    n = 36000
    s = run_oracle(p, n, nthreads=8)
    g = make_gpu(p, 1)
    g.step(n)
    ro = rec_arrays(s, p.mask)
    m = p.mask == 1
    st = g.read(4)
    assert np.array_equal(st, ro["status"])
    assert (st[m] == 3).all()
    for what, key in ((1, "at"), (2, "apd"), (3, "vmax")):
        x = g.read(what)
        assert np.array_equal(np.isnan(x), np.isnan(ro[key]))
        d = np.abs(x[m] - ro[key][m]).max()
        assert d <= 1e-9 * np.nanmax(np.abs(ro[key])), (key, d)


def test_stimulus_windows_periodic_fp64():
    mask = np.ones((1, 6, 9), np.uint8)
    r1 = np.zeros_like(mask)
    r1[0, :3] = 1
    r2 = np.zeros_like(mask)
    r2[0, 2:, 4:] = 1
    st = [(r1, 1.5, 0.1, 0.3, 1.0, 3), (r2, -0.75, 0.25, 0.2, 0.7, 0), (r1, 0.5, 2.0, 0.45, 0.0, 1)]
    p = Problem(mask, 0.5, None, 0.1, 0.1, O.MODEL_NONE, [], 0.05, state=np.zeros((1,) + mask.shape),
                stims=st)
    s = run_oracle(p, 0)
    g = make_gpu(p, 1)
    for _ in range(12):
        s.step(7)
        g.step(7)
        assert rel_errs(gpu_state(g, 1), s.state, mask)[0] <= TOL64


# ------------------------------------------------------------------ robustness
def test_checkpoint_resume_bitwise_fp32():
    """step(2N) == step(N) + state read/restore into a fresh grid + clock restore + step(N),
    bitwise, with the stimulus window straddling the checkpoint."""
    p = crn_problem(20, 20, 10, stim_ms=3.0)
    a = make_gpu(p, 0)
    a.step(400)
    b = make_gpu(p, 0)
    b.step(200)
    snap = gpu_state(b, 21)
    from paper_1605_06015_amd import bbx as B
    step = int(b.read(B.BBX_READ_STEP)[0])
    c = make_gpu(p, 0)
    for v in range(21):
        c.set(v, snap[v])
    c.clock(step)
    c.step(200)
    assert np.array_equal(gpu_state(a, 21), gpu_state(c, 21), equal_nan=True)


def test_determinism_bitwise():
    p = crn_problem(20, 20, 10)
    outs = []
    for _ in range(2):
        g = make_gpu(p, 0)
        g.step(300)
        outs.append(gpu_state(g, 21))
    assert np.array_equal(outs[0], outs[1], equal_nan=True)


def test_nan_detected(B):
    p = crn_problem(12, 12, 6, seed=8)
    st = p.state.copy()
    idx = np.argwhere(p.mask == 1)[7]
    st[3][tuple(idx)] = np.nan
    p.state = st
    g = make_gpu(p, 0)
    g.nan_check(50)
    with pytest.raises(B.BBXError) as ei:
        g.step(120)
    assert ei.value.code == B.BBX_ENUMERIC
    assert g.read(B.BBX_READ_NAN_FLAG)[0] == 1


def test_reductions_fp64(B):
    gg = WL.cup_shell(32, 32, 16, 0.25, 0.35, seed=9)
    mask = gg["mask"]
    u0 = np.random.default_rng(1).standard_normal(mask.shape) * mask
    p = Problem(mask, 0.25, gg["fibre"], 0.3, 0.03, O.MODEL_NONE, [], 0.01, state=u0[None])
    g = make_gpu(p, 1)
    g.step(10)
    x = g.get(0)
    m = mask == 1
    region = np.zeros_like(mask)
    region[:, :16] = 1
    assert g.read(B.BBX_READ_REDUCE_SUM)[0] == pytest.approx(x[m].sum(), rel=1e-13, abs=1e-12)
    assert g.read(B.BBX_READ_REDUCE_MAX)[0] == x[m].max()
    rm = m & (region == 1)
    assert g.read(B.BBX_READ_REDUCE_SUM, 0, region)[0] == pytest.approx(x[rm].sum(), rel=1e-13, abs=1e-12)
    assert g.read(B.BBX_READ_REDUCE_MAX, 0, region)[0] == x[rm].max()
    assert g.read(B.BBX_READ_STEP)[0] == 10
    assert np.isnan(x[~m]).all()


# ------------------------------------------------------------------ edge cases
def test_empty_tissue(B):
    mask = np.zeros((3, 4, 5), np.uint8)
    g = B.Grid(mask, 0.1, None, 1.0, 1.0, B.BBX_FP32)
    assert g.nact == 0
    g.model(B.BBX_MODEL_CRN, [], 0.01)
    g.step(5)
    assert np.isnan(g.get(0)).all()
    assert g.read(B.BBX_READ_REDUCE_SUM)[0] == 0.0


def test_single_voxel_matches_oracle_cell():
    mask = np.ones((1, 1, 1), np.uint8)
    st = np.array(WL.CRN_INITIAL, float).reshape(21, 1, 1, 1)
    p = Problem(mask, 0.25, None, 0.3, 0.03, O.MODEL_CRN, [], 0.01, state=st,
                stims=[(mask, 20.0, 0.0, 2.0, 0.0, 1)])
    s = run_oracle(p, 3000)
    g = make_gpu(p, 1)
    g.step(3000)
    assert np.all(rel_errs(gpu_state(g, 21), s.state, mask) <= TOL64)


@pytest.mark.parametrize("fibres", ["none", "rotating", "random", "random_2d", "random_wide"])
@pytest.mark.parametrize("prec", [1, 0])
def test_dense_box_light_model(fibres, prec):
    """Dense boxes with a light model take the z-marching kernels (register march when
    isotropic; an LDS ring of V planes when anisotropic, with the precomputed face
    coefficients of the tensor-gradient term).  Fibres rotating in z only leave those
    coefficients zero; random fibres exercise them everywhere, including the box faces;
    the wide box has tiles whose whole halo lies inside the box (the kernel's
    branch-free interior path).  FP64 <= 1e-10 normwise; FP32 <= 1e-5 normwise."""
    shape = {"random_2d": (1, 37, 45), "random_wide": (10, 14, 150)}.get(fibres, (7, 13, 21))
    nz, ny, nx = shape
    mask, fib = WL.full_box_rotating(nx, ny, nz)
    if fibres.startswith("random"):
        fib = WL.random_fibres(mask.shape, seed=43)
    elif fibres == "none":
        fib = None
    rng = np.random.default_rng(41)
    V0 = rng.uniform(0, 1, mask.shape)
    p = Problem(mask, 0.5, fib, 1.0, 0.3, O.MODEL_ZFK, [0.13], 0.02, state=V0[None])
    s = run_oracle(p, 200)
    g = make_gpu(p, prec)
    g.step(200)
    e = rel_errs(gpu_state(g, 1), s.state, mask)[0]
    print(fibres, prec, "normwise error", e)
    assert e <= (TOL64 if prec == 1 else 1e-5)


@pytest.mark.parametrize("prec,tol", [(1, TOL64), (0, None)])
def test_dense_box_crn(prec, tol):
    """A dense box with a many-variable model takes the one-voxel-per-thread path (the
    z-marching kernel serves light models): CRN on a 20x12x8 all-tissue box, rotating
    fibres, corner stimulus, 300 steps.  FP64 <= 1e-10 normwise; FP32 |dV| <= 1e-3 mV."""
    mask, fib = WL.full_box_rotating(20, 12, 8)
    st = np.stack([np.full(mask.shape, v) for v in WL.CRN_INITIAL])
    reg = np.zeros_like(mask)
    reg[:3, :4, :5] = 1
    p = Problem(mask, 0.25, fib, 0.3, 0.03, O.MODEL_CRN, [], 0.01, state=st,
                stims=[(reg, 40.0, 0.0, 2.0, 0.0, 1)])
    s = run_oracle(p, 300)
    g = make_gpu(p, prec)
    g.step(300)
    x = gpu_state(g, 21)
    if prec == 1:
        assert np.all(rel_errs(x, s.state, mask) <= tol)
    else:
        assert np.abs(x[0] - s.state[0]).max() <= 1e-3


def test_dt_above_stability_bound_rejected(B):
    mask = np.ones((1, 10, 10), np.uint8)
    g = B.Grid(mask, 0.2, None, 1.0, 1.0, B.BBX_FP64)
    # 5-point, D/h^2 = 25: Gershgorin bound 2 / (2 * 4 * 25) = 0.01
    g.model(B.BBX_MODEL_BARKLEY, [0.75, 0.02, 0.02], 0.0099)
    with pytest.raises(B.BBXError) as ei:
        g.model(B.BBX_MODEL_BARKLEY, [0.75, 0.02, 0.02], 0.0101)
    assert ei.value.code == B.BBX_EUNSTABLE
    with pytest.raises(B.BBXError) as ei:
        g.model(B.BBX_MODEL_BARKLEY, [0.75, 0.02], 0.005)
    assert ei.value.code == B.BBX_EINVAL
    with pytest.raises(B.BBXError):
        g.read(B.BBX_READ_ACT_TIME)


def test_state_order_errors(B):
    mask = np.ones((2, 2, 2), np.uint8)
    g = B.Grid(mask, 0.2, None, 1.0, 1.0, B.BBX_FP32)
    with pytest.raises(B.BBXError) as ei:
        g.step(1)
    assert ei.value.code == B.BBX_ESTATE
    with pytest.raises(B.BBXError):
        g.set(3, np.zeros(mask.shape))
