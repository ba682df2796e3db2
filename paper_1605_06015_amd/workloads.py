"""Seeded synthetic inputs shared by the GPU library's tests, the oracle's tests
and the benchmark.

This module only *generates inputs* (tissue masks, fibre fields, initial
states, stimulus regions).  It contains none of the method's arithmetic: no
stencil weights, no kinetics, no time stepping.  Both the oracle and the GPU
library consume the arrays it returns, byte for byte.

Array conventions: masks are uint8 of shape (nz, ny, nx) (x fastest in
memory), fibres float64 of shape (nz, ny, nx, 3).

The paper's anatomical meshes (rabbit ventricles, human atrium; "Parallel
scaling performance") are not available; the ellipsoidal shells below stand
in for them by active fraction and shape class.
"""
from __future__ import annotations

import numpy as np

# Published initial state of the Courtemanche-Ramirez-Nattel (1998) atrial cell
# model, in the state order V, Na_i, K_i, Ca_i, Ca_up, Ca_rel, m, h, j, oa, oi,
# ua, ui, xr, xs, d, f, fCa, u, v, w (units mV, mM, dimensionless).
CRN_NAMES = ("V", "Nai", "Ki", "Cai", "Caup", "Carel", "m", "h", "j", "oa", "oi",
             "ua", "ui", "xr", "xs", "d", "f", "fCa", "u", "v", "w")
CRN_INITIAL = (-81.18, 11.17, 139.0, 1.013e-4, 1.488, 1.488, 2.908e-3, 0.9649, 0.9775,
               3.043e-2, 0.9992, 4.966e-3, 0.9986, 3.296e-5, 1.869e-2, 1.367e-4, 0.9996,
               0.7755, 0.0, 1.0, 0.9992)


# --------------------------------------------------------------------------
# Barkley 2D: 100x100, cross-field initial condition + seeded uniform noise
# --------------------------------------------------------------------------
# Published initial state of the ten Tusscher-Panfilov (2006) ventricular model,
# epicardial cell, in the state order V, K_i, Na_i, Ca_i, Ca_ss, Ca_SR, Rbar, Xr1,
# Xr2, Xs, m, h, j, d, f, f2, fCass, s, r.
TP06_NAMES = ("V", "Ki", "Nai", "Cai", "Cass", "CaSR", "Rbar", "Xr1", "Xr2", "Xs", "m", "h",
              "j", "d", "f", "f2", "fCass", "s", "r")
TP06_INITIAL = (-85.23, 136.89, 8.604, 0.000126, 0.00036, 3.64, 0.9073, 0.00621, 0.4712,
                0.0095, 0.00172, 0.7444, 0.7045, 3.373e-5, 0.7888, 0.9755, 0.9953, 0.999998,
                2.42e-8)

BARKLEY_2D = dict(nx=100, ny=100, nz=1, h=0.2, dt=0.008, D=1.0, a=0.75, b=0.02, eps=0.02,
                  steps=2000)


def barkley_cross_field(nx: int = 100, ny: int = 100, seed: int = 0, noise: float = 1e-3):
    """u = 1 where the x index < nx/2, v = 0.5 where the y index < ny/2 (indices
    from 0), plus i.i.d. U(-noise, +noise) added to both fields at every voxel."""
    rng = np.random.default_rng(seed)
    u = np.zeros((1, ny, nx))
    v = np.zeros((1, ny, nx))
    u[0, :, : nx // 2] = 1.0
    v[0, : ny // 2, :] = 0.5
    u += rng.uniform(-noise, noise, size=u.shape)
    v += rng.uniform(-noise, noise, size=v.shape)
    return u, v


# --------------------------------------------------------------------------
# Ellipsoidal cup shell with transmural fibre rotation (atrial/ventricular stand-in)
# --------------------------------------------------------------------------
def _shell_s(nx, ny, nz, h, axes, centre):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = (x + 0.5) * h - centre[0]
    Y = (y + 0.5) * h - centre[1]
    Z = (z + 0.5) * h - centre[2]
    s = np.sqrt((X / axes[0]) ** 2 + (Y / axes[1]) ** 2 + (Z / axes[2]) ** 2)
    return s, X, Y, Z


def _fibres_from_normal(nx_, ny_, nz_, e, angle_lo=-60.0, angle_hi=60.0):
    """Fibre f = cos(a) c + sin(a) l with a = lo + (hi-lo) e, c the circumferential
    direction normalise(z x n) and l = n x c; c := x where n is parallel to z."""
    n = np.stack([nx_, ny_, nz_], axis=-1)
    n = n / np.maximum(np.linalg.norm(n, axis=-1, keepdims=True), 1e-30)
    zhat = np.array([0.0, 0.0, 1.0])
    c = np.cross(np.broadcast_to(zhat, n.shape), n)
    cn = np.linalg.norm(c, axis=-1, keepdims=True)
    xhat = np.broadcast_to(np.array([1.0, 0.0, 0.0]), n.shape)
    c = np.where(cn > 1e-9, c / np.maximum(cn, 1e-30), xhat)
    l = np.cross(n, c)
    a = np.deg2rad(angle_lo + (angle_hi - angle_lo) * np.clip(e, 0.0, 1.0))[..., None]
    f = np.cos(a) * c + np.sin(a) * l
    return f / np.linalg.norm(f, axis=-1, keepdims=True)


def cup_shell(nx=128, ny=128, nz=64, h=0.25, active_frac=0.35, seed=1, tol=0.005):
    """Half-ellipsoidal cup: outer semi-axes 0.97 x half the box width (15.5 mm for the
    32 mm box) x (1 +- 0.05, seeded), base at
    the top z face, apex at the bottom; inner scale s_in found by bisection so
    that the active fraction is active_frac +- tol.

    Returns dict(mask, fibre, apex (mm), s, s_in)."""
    rng = np.random.default_rng(seed)
    L = np.array([nx * h, ny * h, nz * h])
    base = 0.97 * 0.5 * min(L[0], L[1])
    axes = np.array([base, base, min(base, 0.97 * L[2])]) * (1.0 + rng.uniform(-0.05, 0.05, 3))
    axes = np.minimum(axes, [0.5 * L[0] - 0.25 * h, 0.5 * L[1] - 0.25 * h, L[2] - 0.25 * h])
    centre = np.array([0.5 * L[0], 0.5 * L[1], L[2]])
    s, X, Y, Z = _shell_s(nx, ny, nz, h, axes, centre)
    inside = (s <= 1.0) & (Z <= 0.0)
    target = active_frac * s.size
    lo, hi = 0.0, 1.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        cnt = np.count_nonzero(inside & (s >= mid))
        if cnt > target:
            lo = mid
        else:
            hi = mid
    s_in = 0.5 * (lo + hi)
    mask = (inside & (s >= s_in)).astype(np.uint8)
    frac = mask.mean()
    if abs(frac - active_frac) > tol:
        raise RuntimeError(f"cup_shell: active fraction {frac:.4f} misses {active_frac}")
    e = (s - s_in) / (1.0 - s_in)
    gx, gy, gz = X / axes[0] ** 2, Y / axes[1] ** 2, Z / axes[2] ** 2
    fibre = _fibres_from_normal(gx, gy, gz, e)
    fibre[mask == 0] = 0.0
    apex = centre - np.array([0.0, 0.0, axes[2]])
    return dict(mask=mask, fibre=fibre, apex=apex, s_in=s_in, axes=axes, centre=centre)


def region_near(mask, h, point_mm, radius_mm):
    """uint8 region: tissue voxels whose centre lies within radius of a point."""
    nz, ny, nx = mask.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (((x + 0.5) * h - point_mm[0]) ** 2 + ((y + 0.5) * h - point_mm[1]) ** 2
          + ((z + 0.5) * h - point_mm[2]) ** 2)
    return ((d2 <= radius_mm ** 2) & (mask != 0)).astype(np.uint8)


# The 3D CRN workload: 128x128x64 cup at 35% active, D_par 0.3, D_perp 0.03 mm^2/ms,
# h 0.25 mm, dt 0.01 ms, 2 ms of 40 pA/pF at the apex, 500 ms.
CRN_3D = dict(nx=128, ny=128, nz=64, h=0.25, dt=0.01, Dpar=0.3, Dperp=0.03, active=0.35,
              stim_amp=40.0, stim_ms=2.0, t_end=500.0, seed=1, theta=-40.0)


def crn_cup(nx=128, ny=128, nz=64, seed=1, active=0.35, h=0.25):
    """Geometry, stimulus region (within 1 mm of the apex) and the uniform
    resting initial state of the 3D CRN workload."""
    g = cup_shell(nx, ny, nz, h, active, seed)
    stim = region_near(g["mask"], h, g["apex"], 1.0)
    if stim.sum() == 0:
        raise RuntimeError("crn_cup: empty stimulus region")
    state = np.stack([np.full(g["mask"].shape, v) for v in CRN_INITIAL])
    state[:, g["mask"] == 0] = 0.0
    g.update(stim=stim, state=state)
    return g


def full_box_rotating(nx, ny, nz, angle_lo=-60.0, angle_hi=60.0):
    """All-tissue box; fibres lie in the xy plane at an angle rotating linearly
    with z from angle_lo to angle_hi degrees."""
    mask = np.ones((nz, ny, nx), np.uint8)
    zz = (np.arange(nz) + 0.5) / nz if nz > 1 else np.array([0.5])
    a = np.deg2rad(angle_lo + (angle_hi - angle_lo) * zz)
    fibre = np.zeros((nz, ny, nx, 3))
    fibre[..., 0] = np.cos(a)[:, None, None]
    fibre[..., 1] = np.sin(a)[:, None, None]
    return mask, fibre


def random_blob_mask(nx, ny, nz, seed, frac=0.6, smooth=2):
    """Smooth random tissue blob (a thresholded, box-filtered noise field)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((nz, ny, nx))
    for ax in range(3):
        if f.shape[ax] > 1:
            for _ in range(smooth):
                f = (np.roll(f, 1, ax) + f + np.roll(f, -1, ax)) / 3.0
    thr = np.quantile(f, 1.0 - frac)
    return (f >= thr).astype(np.uint8)


def random_fibres(shape, seed):
    """Unit fibre vectors of random direction at every voxel."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(tuple(shape) + (3,))
    return f / np.linalg.norm(f, axis=-1, keepdims=True)


# ---------------------------------------------------------------- batched 2D ensemble
# Epicardial parameters (tau_fi, tau_so1, tau_si, tau_w+) of the four-variable
# minimal model of the Fenton-Karma family (Bueno-Orovio, Cherry & Fenton 2008)
# and its published resting state (u, v, w) = (0, 1, 1); s starts at 0.
FK4_EPI = (0.11, 30.0181, 1.8875, 200.0)
FK4_INITIAL = (0.0, 1.0, 1.0, 0.0)
# Ensemble protocol: diffusion coefficient of the model publication
# (1.171 cm^2/s = 0.1171 mm^2/ms) along fibres, 4:1 anisotropy, h = 0.25 mm,
# dt = 0.05 ms, 20,000 steps (1 s).
FK4_ENSEMBLE = dict(n=96, side_lo=64, side_hi=768, h=0.25, dt=0.05, Dpar=0.1171, aniso=4.0,
                    spread=0.2, steps=20000, seed=4, s1_amp=1.0, s1_ms=2.0, theta=0.5,
                    apd_est_ms=270.0, cv_est_mm_ms=0.6)


def fk4_ensemble(n=96, side_lo=64, side_hi=768, seed=4, h=0.25, Dpar=0.1171, aniso=4.0,
                 spread=0.2, s1_amp=1.0, s1_ms=2.0, apd_est_ms=270.0, cv_est_mm_ms=0.6):
    """n square tissues with sides drawn uniformly from [side_lo, side_hi] (seeded); per tissue D_par scaled by U(1 - spread, 1 + spread) with
    D_perp = D_par / aniso, a fibre angle U(0, pi), and each model time constant scaled
    by its own U(1 - spread, 1 + spread).  S1-S2 cross-field protocol: S1 on the
    three leftmost columns at t = 0; S2 on the lower-left quadrant once the S1 wave
    back is estimated to have passed the middle (t = apd_est + (side/2) h / cv_est),
    which breaks the S2 front into a spiral where the tissue is large enough.
    Returns dict(nx, ny, Dpar, Dperp, angle, params (n, 4), stims [(tissue, x0, x1,
    y0, y1, amp, t0_ms, dur_ms)], h)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, n).astype(np.int32)
    dscale = rng.uniform(1 - spread, 1 + spread, n)
    Dp = Dpar * dscale
    Dq = Dp / aniso
    angle = rng.uniform(0.0, np.pi, n)
    params = np.array(FK4_EPI) * rng.uniform(1 - spread, 1 + spread, (n, 4))
    stims = []
    for i, s in enumerate(sides):
        s = int(s)
        stims.append((i, 0, 3, 0, s, s1_amp, 0.0, s1_ms))
        t2 = apd_est_ms + 0.5 * s * h / cv_est_mm_ms
        stims.append((i, 0, s // 2, 0, s // 2, s1_amp, float(np.round(t2, 1)), s1_ms))
    return dict(nx=sides.copy(), ny=sides.copy(), Dpar=Dp, Dperp=Dq, angle=angle,
                params=params, stims=stims, h=h)


# ---------------------------------------------------------------- biventricular-like double shell
def _ellipsoid_s(x, y, z, h, axes, centre):
    X = (x + 0.5) * h - centre[0]
    Y = (y + 0.5) * h - centre[1]
    Z = (z + 0.5) * h - centre[2]
    return np.sqrt((X / axes[0]) ** 2 + (Y / axes[1]) ** 2 + (Z / axes[2]) ** 2), X, Y, Z


def double_shell(nx=512, ny=512, nz=384, h=0.2, active_frac=0.25, seed=5, tol=0.005,
                 rv_ratio=0.45, with_fibres=True):
    """Bi-ventricular-like tissue: two half-ellipsoidal shells with their bases on the top z
    face.  The left shell (outer semi-axes about (0.30, 0.36, 0.95) of the box, seeded
    +-5%) has a wall of relative thickness tau; the right shell (about (0.44, 0.46, 0.85),
    centred further along x) wraps it with a wall of relative thickness rv_ratio * tau and
    keeps only what lies outside the left shell.  tau is found by bisection so that the
    active fraction is active_frac +- tol.  Fibres rotate from -60 to +60 degrees through
    each wall (transmural depth from the shell's own inner to outer surface).  Built slab
    by slab along z to bound host memory.

    Returns dict(mask, fibre (None unless with_fibres), tau, lv=(axes, centre),
    rv=(axes, centre), apex (mm, of the left shell))."""
    rng = np.random.default_rng(seed)
    L = np.array([nx * h, ny * h, nz * h])
    j = 1.0 + rng.uniform(-0.05, 0.05, 6)
    lv_ax = np.array([0.30, 0.36, 0.95]) * L * j[:3]
    lv_c = np.array([0.40, 0.50, 1.0]) * L
    rv_ax = np.array([0.44, 0.46, 0.85]) * L * j[3:]
    rv_c = np.array([0.54, 0.50, 1.0]) * L
    # keep both shells inside the box
    lv_ax = np.minimum(lv_ax, [min(lv_c[0], L[0] - lv_c[0]) - h, 0.5 * L[1] - h, L[2] - h])
    rv_ax = np.minimum(rv_ax, [min(rv_c[0], L[0] - rv_c[0]) - h, 0.5 * L[1] - h, L[2] - h])
    y2, x2 = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    s_lv = np.empty((nz, ny, nx), np.float32)
    s_rv = np.empty((nz, ny, nx), np.float32)
    for z in range(nz):
        s_lv[z] = _ellipsoid_s(x2, y2, z, h, lv_ax, lv_c)[0]
        s_rv[z] = _ellipsoid_s(x2, y2, z, h, rv_ax, rv_c)[0]

    def tissue(tau, zs=slice(None)):
        a, b = s_lv[zs], s_rv[zs]
        lv = (a <= 1.0) & (a >= 1.0 - tau)
        rv = (b <= 1.0) & (b >= 1.0 - rv_ratio * tau) & (a > 1.0)
        return lv, rv

    target = active_frac * s_lv.size
    lo, hi = 0.0, 1.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        cnt = 0
        for z0 in range(0, nz, 32):
            lv, rv = tissue(mid, slice(z0, z0 + 32))
            cnt += np.count_nonzero(lv) + np.count_nonzero(rv)
        if cnt < target:
            lo = mid
        else:
            hi = mid
    tau = 0.5 * (lo + hi)
    mask = np.zeros((nz, ny, nx), np.uint8)
    fibre = np.zeros((nz, ny, nx, 3), np.float64) if with_fibres else None
    for z in range(nz):
        lv, rv = tissue(tau, z)
        mask[z] = lv | rv
        if with_fibres and mask[z].any():
            for sel, ax, c, s, th in ((lv, lv_ax, lv_c, s_lv[z], tau), (rv, rv_ax, rv_c, s_rv[z], rv_ratio * tau)):
                if not sel.any():
                    continue
                _, X, Y, Z = _ellipsoid_s(x2[sel], y2[sel], z, h, ax, c)
                e = (s[sel].astype(np.float64) - (1.0 - th)) / th
                fibre[z][sel] = _fibres_from_normal(X / ax[0] ** 2, Y / ax[1] ** 2,
                                                    np.broadcast_to(Z / ax[2] ** 2, X.shape), e)
    frac = mask.mean()
    if abs(frac - active_frac) > tol:
        raise RuntimeError(f"double_shell: active fraction {frac:.4f} misses {active_frac}")
    apex = lv_c - np.array([0.0, 0.0, lv_ax[2]])
    return dict(mask=mask, fibre=fibre, tau=tau, lv=(lv_ax, lv_c), rv=(rv_ax, rv_c), apex=apex)


def region_near_slabs(mask, h, point_mm, radius_mm):
    """region_near computed one z plane at a time (for large boxes)."""
    nz, ny, nx = mask.shape
    y2, x2 = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros_like(mask)
    for z in range(nz):
        dz2 = ((z + 0.5) * h - point_mm[2]) ** 2
        if dz2 > radius_mm ** 2:
            continue
        d2 = ((x2 + 0.5) * h - point_mm[0]) ** 2 + ((y2 + 0.5) * h - point_mm[1]) ** 2 + dz2
        out[z] = (d2 <= radius_mm ** 2) & (mask[z] != 0)
    return out


# The 3D TP06 workload: 512x512x384 biventricular-like double shell at 25% active,
# h 0.2 mm, dt 0.02 ms, D_par 0.3 / D_perp 0.03 mm^2/ms, 1 s.  Scroll-wave initiation
# by a cross-field S1-S2 protocol: S1 on the tissue within the first s1_strip of the box's
# y extent (counted from the tissue's smallest y) at t = 0, a wave that crosses the shells
# along y; S2 on the upper half of the box (z >= nz/2) at t = s2_t, when the S1 wave back
# has passed about half of the y extent, so that S2 excites only the recovered side and
# its front gets a free end at the refractory side.  Eight pseudo-ECG electrodes 20 mm
# outside the box.  (Measured on the full-size shell: S1 alone leaves the tissue at rest
# by 420 ms; with S2 at 346, 361 or 376 ms 57-87% of the tissue is still depolarised at
# every 100 ms sample up to 1 s.)
TP06_3D = dict(nx=512, ny=512, nz=384, h=0.2, dt=0.02, Dpar=0.3, Dperp=0.03, active=0.25,
               seed=5, theta=-40.0, s1_amp=60.0, s1_ms=2.0, s1_strip=0.1, s2_amp=60.0,
               s2_t=360.0, s2_ms=2.0, t_end=1000.0, ecg_every_ms=1.0)
# The same protocol on a down-scaled shell (128x128x96 at the same h: 25.6 x 25.6 x 19.2 mm)
# for parity runs against the oracle.  Its S1 wave crosses the shell in 33 ms, so S2 comes
# earlier (310 ms: part of the upper half has recovered), and too little tissue remains to
# sustain re-entry: the S2 wave dies out by about 500 ms, and the run ends at 600 ms.
TP06_3D_SMALL = dict(TP06_3D, nx=128, ny=128, nz=96, s2_t=310.0, t_end=600.0)


def tp06_biv(nx=512, ny=512, nz=384, h=0.2, seed=5, active=0.25, s1_strip=0.1,
             with_fibres=True):
    """Geometry, stimulus regions (S1 y-strip, S2 upper half) and electrodes of the 3D
    TP06 workload."""
    g = double_shell(nx, ny, nz, h, active, seed, with_fibres=with_fibres)
    mask = g["mask"]
    ys = np.nonzero(mask.any(axis=(0, 2)))[0]
    y0 = int(ys.min())
    w = max(1, int(round(s1_strip * ny)))
    s1 = np.zeros_like(mask)
    s1[:, y0:y0 + w, :] = mask[:, y0:y0 + w, :]
    if s1.sum() == 0:
        raise RuntimeError("tp06_biv: empty S1 region")
    s2 = np.zeros_like(mask)
    s2[nz // 2:] = mask[nz // 2:]
    L = np.array([nx, ny, nz]) * h
    c = 0.5 * L
    d = 20.0
    electrodes = np.array([[-d, c[1], c[2]], [L[0] + d, c[1], c[2]], [c[0], -d, c[2]],
                           [c[0], L[1] + d, c[2]], [c[0], c[1], -d], [c[0], c[1], L[2] + d],
                           [-d, -d, c[2]], [L[0] + d, L[1] + d, -d]])
    g.update(s1=s1, s2=s2, electrodes=electrodes)
    return g


def tp06_cup(nx, ny, nz, seed=5, active=0.35, h=0.25):
    """A small TP06 test tissue: the ellipsoidal cup with an apex stimulus region and the
    published epicardial initial state."""
    g = cup_shell(nx, ny, nz, h, active, seed)
    stim = region_near(g["mask"], h, g["apex"], 1.0)
    if stim.sum() == 0:
        raise RuntimeError("tp06_cup: empty stimulus region")
    state = np.stack([np.full(g["mask"].shape, v) for v in TP06_INITIAL])
    g.update(stim=stim, state=state)
    return g
