"""Training pipeline of the surrogate ionic map (sequencing of library calls).

Every computation runs in libbbx kernels: the simulator produces states
(bbx_step with periodic stimuli), bbx_sample_states draws voxel states,
bbx_ionic_map applies the plain kinetic one-step map to them (the training
targets), bbx_mlp_fit_norm fits the normalisation, bbx_mlp_train runs the
BF16-MFMA forward/backward/Adam kernels, and bbx_surrogate_set attaches the
network to a grid.  This module only orders those calls; torch provides the
device buffers.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bbx as B
from . import workloads as WL


@dataclass
class Trained:
    mlp: "B.Mlp"
    stats: np.ndarray        # (7, 32): state mean/std/min/max, increment mean/std/max|.|
    loss: np.ndarray         # per-iteration training loss
    npairs: int


def _model_setup(model):
    """(model id, nvar, workload dict, geometry, resting state) of a surrogate workload."""
    if model == "crn":
        c = WL.CRN_3D
        return B.BBX_MODEL_CRN, 21, c, WL.crn_cup, WL.CRN_INITIAL, c["stim_amp"], c["stim_ms"]
    if model == "tp06":
        c = dict(WL.CRN_3D, dt=0.02, stim_amp=60.0, stim_ms=2.0)
        return B.BBX_MODEL_TP06, 19, c, WL.tp06_cup, WL.TP06_INITIAL, 60.0, 2.0
    raise ValueError(f"no surrogate workload for model {model!r}")


def generate_pairs(nx=128, ny=128, nz=64, runs=3, t_ms=1200.0, every_ms=1.0, per_sample=2048,
                   cl_range=(250.0, 1000.0), seed=2, stream=None, model="crn"):
    """States of the 3D cup (CRN or TP06 kinetics) paced from the apex at seeded cycle
    lengths, sampled every `every_ms` at `per_sample` random tissue voxels, and their
    plain kinetic one-step images.  Returns device tensors S, S1 of shape (N, nvar) (FP32)."""
    import torch
    mid, nv, c, geo, _, amp, dur = _model_setup(model)
    rng = np.random.default_rng(seed)
    g0 = geo(nx, ny, nz, seed=c["seed"], active=c["active"], h=c["h"])
    nsamp = int(round(t_ms / every_ms))
    S = torch.empty((runs * nsamp * per_sample, nv), dtype=torch.float32, device="cuda")
    S1 = torch.empty_like(S)
    k = 0
    every = int(round(every_ms / c["dt"]))
    for r in range(runs):
        cl = float(rng.uniform(*cl_range))
        grid = B.Grid(g0["mask"], c["h"], g0["fibre"], c["Dpar"], c["Dperp"], B.BBX_FP32, stream)
        grid.model(mid, [], c["dt"])
        for v in range(nv):
            grid.set(v, g0["state"][v])
        grid.stimulus(g0["stim"], amp, 0.0, dur, period=cl, count=0)
        grid.nan_check(0)
        for i in range(nsamp):
            grid.step(every)
            sl = S[k:k + per_sample]
            grid.sample_states(per_sample, int(rng.integers(1 << 62)), sl)
            grid.ionic_map(sl, S1[k:k + per_sample])
            k += per_sample
        grid.close()
    torch.cuda.synchronize()
    return S[:k], S1[:k]


# Learning-rate schedules of the benchmark's surrogates: (Adam steps, learning rate)
# stages.  Measured on the held-out cups: for CRN a single stage at 1e-3 (20,000 steps)
# leaves a network that meets the 1-dt activation-time bar only below the resting
# potential (0.01% of the voxel updates), and stepping the rate down to 3e-5 lets it take
# 1.9% at 0.26 dt; for TP06 the same steps made the network worse near rest (2.5% of
# the updates at 1.35 dt against 1.7% at 0.76 dt with the single stage).
SCHEDULES = {"crn": ((20000, 1e-3), (15000, 3e-4), (15000, 1e-4), (10000, 3e-5)),
             "tp06": ((20000, 1e-3),)}


def train(S, S1, iters=20000, batch=4096, lr=1e-3, seed=0, stream=None, anchor_grid=None,
          model="crn", schedule=None):
    """Fit the normalisation and train an nvar -> 128 -> 128 -> nvar network: `iters` Adam
    steps at `lr`, or the stages of `schedule` one after the other (Adam moments carried
    over).  If anchor_grid is given (a grid with the plain kinetics of `model`), the
    network is anchored so that the published resting state is an exact fixed point."""
    import torch
    _, nv, _, _, rest, _, _ = _model_setup(model)
    m = B.Mlp(nv, nv, seed=seed, stream=stream)
    stats = m.fit_norm(S, S1)
    stages = schedule if schedule is not None else ((iters, lr),)
    hist = np.concatenate([m.train(S, S1, batch, it, r, seed=seed + 1 + k)
                           for k, (it, r) in enumerate(stages)])
    if anchor_grid is not None:
        s0 = torch.tensor([rest], dtype=torch.float32, device="cuda")
        s1 = torch.empty_like(s0)
        anchor_grid.ionic_map(s0, s1)
        torch.cuda.synchronize()
        m.anchor(s0, s1)
    return Trained(m, stats, hist, int(S.shape[0]))


def accepted_box(stats, margin=0.02, dv_cap=None, nvar=21):
    """Accepted kinetic inputs: the training range widened by `margin` of its width;
    |dV| up to the training maximum (or dv_cap if smaller)."""
    lo = stats[2, :nvar].copy()
    hi = stats[3, :nvar].copy()
    # a feature that barely varied in training still gets a box of 1e-3 of its size
    w = np.maximum(hi - lo, 1e-3 * np.maximum(np.abs(lo), np.abs(hi)))
    w = np.maximum(w, 1e-12)
    lo -= margin * w
    hi += margin * w
    dv = stats[6, 0] * 1.1
    if dv_cap is not None:
        dv = min(dv, dv_cap)
    return lo.astype(np.float32), hi.astype(np.float32), float(dv)


def attach(grid, trained, margin=0.02, dv_cap=None):
    lo, hi, dv = accepted_box(trained.stats, margin, dv_cap, trained.mlp.nin)
    grid.surrogate(trained.mlp, lo, hi, dv)
    return lo, hi, dv


def run_pair(trained, model, geo_seed, nx=96, ny=96, nz=48, t_ms=500.0, v_his=(), stream=None):
    """The plain FP32 run and one surrogate run per acceptance threshold v_hi on a cup of
    the workload's shape (geometry seed geo_seed), t_ms long.  Returns the plain run's
    activation-time and APD90 maps (tissue order) and seconds and, per threshold, a dict of
    share, activation-time and APD90 errors against the plain run, seconds, and the
    surrogate run's own maps ("at", "apd")."""
    import torch
    mid, nv, c, geo, _, amp, dur = _model_setup(model)
    g = geo(nx, ny, nz, seed=geo_seed, active=c["active"], h=c["h"])
    m = g["mask"] == 1
    nsteps = int(round(t_ms / c["dt"]))

    def one(v_hi):
        grid = B.Grid(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], B.BBX_FP32, stream)
        grid.model(mid, [], c["dt"])
        for v in range(nv):
            grid.set(v, g["state"][v])
        grid.stimulus(g["stim"], amp, 0.0, dur)
        grid.record(-40.0)
        grid.nan_check(0)
        if v_hi is not None:
            lo, hi, dv = accepted_box(trained.stats, nvar=nv)
            hi[0] = v_hi
            grid.surrogate(trained.mlp, lo, hi, dv)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        s = stream or torch.cuda.current_stream()
        torch.cuda.synchronize()
        ev[0].record(s)
        grid.step(nsteps)
        ev[1].record(s)
        torch.cuda.synchronize()
        sec = ev[0].elapsed_time(ev[1]) / 1e3
        out = dict(at=grid.read(B.BBX_READ_ACT_TIME)[m], apd=grid.read(B.BBX_READ_APD90)[m], sec=sec,
                   fb=int(grid.read(B.BBX_READ_FALLBACK_COUNT)[0]) if v_hi is not None else 0,
                   nact=grid.nact)
        grid.close()
        return out

    plain = one(None)
    res = {}
    for v_hi in v_his:
        q = one(v_hi)
        both = np.isfinite(plain["at"]) & np.isfinite(q["at"])
        bapd = np.isfinite(plain["apd"]) & np.isfinite(q["apd"])
        dat = np.abs(plain["at"][both] - q["at"][both])
        dapd = np.abs(plain["apd"][bapd] - q["apd"][bapd])
        res[float(v_hi)] = dict(
            share=1.0 - q["fb"] / (q["nact"] * nsteps),
            same_activated=bool(np.array_equal(np.isfinite(plain["at"]), np.isfinite(q["at"]))),
            at_max=float(dat.max()) if dat.size else None, at_mean=float(dat.mean()) if dat.size else None,
            apd_max=float(dapd.max()) if dapd.size else None,
            apd_mean=float(dapd.mean()) if dapd.size else None,
            sec=q["sec"], speed_vs_plain=plain["sec"] / q["sec"], at=q["at"], apd=q["apd"])
    return plain, res, c["dt"]


def select_threshold(trained, model, geo_seed=11, margin=0.5, offsets=(-0.2, -0.1, -0.05, -0.02,
                     -0.01, 0.0, 0.01), stream=None):
    """Acceptance threshold v_hi chosen on a held-out cup (geometry seed geo_seed, not the
    benchmark's): among rest + offsets (mV), the one with the largest surrogate share whose
    activation times stay within margin * dt of the plain run's on every voxel, with the
    same activated set.  The default half step leaves room under the 1-dt bar for the spread
    between cups (measured: a TP06 threshold at 0.98 dt on the held-out cup gave 1.1 dt on
    the benchmark's).  Returns (v_hi or None, the sweep)."""
    rest = _model_setup(model)[4][0]
    cands = [round(rest + o, 4) for o in offsets]
    _, sweep, dt = run_pair(trained, model, geo_seed, v_his=cands, stream=stream)
    sweep = {v: {k: x for k, x in r.items() if k not in ("at", "apd")} for v, r in sweep.items()}
    ok = [v for v in cands if sweep[v]["same_activated"] and sweep[v]["at_max"] is not None
          and sweep[v]["at_max"] <= margin * dt]
    best = max(ok, key=lambda v: (sweep[v]["share"], -v)) if ok else None
    return best, sweep
