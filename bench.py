#!/usr/bin/env python3
"""Benchmark of the monodomain step on one MI355X.

A "step" is one pass of the whole hot path over the 3D atrial workload: the
fused anisotropic 19-point no-flux stencil + Courtemanche-Ramirez-Nattel
kinetics (Euler + Rush-Larsen) + stimulus + activation-time/APD90 recording,
FP32, on a 128x128x64 ellipsoidal-cup tissue at 35% active (367,000 tissue
voxels), dt 0.01 ms.  Inputs are resident in HBM before timing starts; the
timed region is K steps bracketed by synchronisations, timed with HIP events
on the stream the kernels are launched on.

Prints ONE JSON line (see the keys below).  --gpus N>1 is refused: the
benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-updates/s (FP32 plain vs surrogate) at ≤1dt activation-time error; %HBM roof"
HBM_PEAK_GBS = 8000.0
VALU_PEAK_GINST = 614.4   # 256 CUs x 2.4 GHz x one wave64 VALU instruction per CU-cycle
PROFILE_DIR = os.path.join(ROOT, "profiles")
STEP_SOURCES = [os.path.join(ROOT, "paper_1605_06015_amd", "csrc", f)
                for f in ("step_kernels.hip", "step_device.h", "kinetics.h", "bbx_internal.h")]

# Algorithmic HBM bytes per tissue-voxel update of the fused CRN step in FP32:
# 21 state values read + 21 written (4 B each) + geometry (box index 4, neighbour
# bits 4, unit fibre 12, tensor-gradient face coefficients 12) + status byte 1.
CRN_BYTES_PER_VOXEL = 21 * 4 * 2 + 32 + 1
# Pure-diffusion stencil, FP32, dense anisotropic box: V read + V written + fibre +
# face coefficients (no index / bit arrays on a dense box).
STENCIL_BYTES_PER_VOXEL = 4 + 4 + 12 + 12


def source_hash(paths=STEP_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_counters(name: str):
    """Counter figures per launch from a committed rocprofv3 summary, if they were taken on
    the current kernel sources; else None."""
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d


def time_steps(grid, stream, steps, warmup):
    import torch
    grid.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    grid.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def crn_workload(precision, stream, tab_dv=0.0):
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    grid = B.Grid(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], precision, stream)
    grid.model(B.BBX_MODEL_CRN, [], c["dt"])
    if tab_dv > 0:
        grid.tabulate(tab_dv)
    for v in range(21):
        grid.set(v, g["state"][v])
    grid.stimulus(g["stim"], c["stim_amp"], 0.0, c["stim_ms"])
    grid.record(c["theta"])
    return grid, g


def cpu_baseline(seconds_target=12.0):
    """The FP64 oracle on the same workload, timed on this host's cores over a bounded
    number of steps (per-step time by differencing two runs)."""
    from oracle import oracle as O
    from paper_1605_06015_amd import workloads as WL
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    try:
        ncpu = len(os.sched_getaffinity(0))
    except Exception:
        ncpu = os.cpu_count() or 1
    nthreads = max(1, min(16, ncpu))
    s = O.Sim(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], O.MODEL_CRN, [], c["dt"],
              nthreads=nthreads)
    s.state[:] = g["state"]
    s.stimuli.append(O.Stimulus(g["stim"], c["stim_amp"], 0, int(round(c["stim_ms"] / c["dt"]))))
    t0 = time.perf_counter()
    s.step(2)
    t1 = time.perf_counter()
    per = max((t1 - t0) / 2, 1e-4)
    n1 = 2
    n2 = n1 + max(4, int(seconds_target / per))
    t2 = time.perf_counter()
    s.step(n2 - n1)
    t3 = time.perf_counter()
    per_step = (t3 - t2) / (n2 - n1)
    nact = int(g["mask"].sum())
    # the same oracle on one core, a few steps (context: the scalar reference rate)
    s1 = O.Sim(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], O.MODEL_CRN, [], c["dt"],
               nthreads=1)
    s1.state[:] = s.state
    t4 = time.perf_counter()
    s1.step(3)
    serial = nact * 3 / (time.perf_counter() - t4)
    return {"value": nact / per_step, "unit": "voxel-updates/s", "cores": nthreads,
            "kind": "oracle", "serial_value": serial,
            "sample": f"CRN 128x128x64 cup ({nact} tissue voxels), FP64 oracle, {n2 - n1} steps "
                      f"after 2 warm-up steps, {t3 - t2:.1f} s, OpenMP over voxels "
                      f"(serial_value: 3 steps on one core)"}


_SHELL = {}


def shell_geometry():
    """The 512x512x384 double shell of the TP06 workload (generated once per process)."""
    from paper_1605_06015_amd import workloads as WL
    if "g" not in _SHELL:
        c = WL.TP06_3D
        _SHELL["g"] = WL.tp06_biv(c["nx"], c["ny"], c["nz"], c["h"], c["seed"], c["active"],
                                  c["s1_radius"])
    return _SHELL["g"]


def _stencil_case(stream, mask, h, fib, steps, warmup, bytes_per_voxel):
    from paper_1605_06015_amd import bbx as B
    grid = B.Grid(mask, h, fib, 0.3, 0.03, B.BBX_FP32, stream)
    grid.model(B.BBX_MODEL_NONE, [], 0.01)
    grid.fill(0, -40.0)
    grid.nan_check(0)
    sec = time_steps(grid, stream, steps, warmup)
    nact = grid.nact
    grid.close()
    per = sec / steps
    gbs = bytes_per_voxel * nact / per / 1e9
    return {"tissue_voxels": nact, "us_per_launch": round(per * 1e6, 2), "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": bytes_per_voxel,
            "voxel_updates_per_s": nact / per}


def stencil_cases(stream, steps=100, warmup=10):
    """The other two HBM-roofline stencil cases: the dense box with an isotropic tensor
    (7-point, V read + written: 8 B/voxel) and the 25%-active double shell through the
    tissue list (19-point: V read + written, index, neighbour bits, fibre, face
    coefficients: 40 B/voxel)."""
    nx, ny, nz = 512, 512, 384
    out = {"dense_isotropic_7pt": _stencil_case(stream, np.ones((nz, ny, nx), np.uint8), 0.2, None,
                                                steps, warmup, 8)}
    g = shell_geometry()
    out["double_shell_19pt"] = _stencil_case(stream, g["mask"], 0.2, g["fibre"], steps, warmup, 40)
    return out


def paper_shape_line(stream, n=300, steps=200, warmup=20):
    """The paper's full-box scaling workload shape on one GPU: CRN on a dense n^3 box with
    fibres rotating through z, FP32 (every voxel tissue: the z-marching dense kernel)."""
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    mask, fib = WL.full_box_rotating(n, n, n)
    grid = B.Grid(mask, 0.25, fib, 0.3, 0.03, B.BBX_FP32, stream)
    del fib
    grid.model(B.BBX_MODEL_CRN, [], 0.01)
    for v, val in enumerate(WL.CRN_INITIAL):
        grid.fill(v, val)
    grid.nan_check(0)
    sec = time_steps(grid, stream, steps, warmup)
    nact = grid.nact
    grid.close()
    per = sec / steps
    bpv = 21 * 4 * 2 + 24              # dense box: no index / neighbour-bit arrays, no recorder
    gbs = bpv * nact / per / 1e9
    return {"workload": f"CRN dense {n}^3 box, fibres rotating through z, FP32, {steps} steps",
            "value": nact / per, "unit": "voxel-updates/s", "ms_per_step": per * 1e3,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": bpv}}


def barkley_line(stream):
    """The 2D Barkley cross-field workload (100x100, FP64, 2,000 steps): 10^4 voxels make
    each step a few microseconds of launch and latency, not a roofline case."""
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    c = WL.BARKLEY_2D
    u, v = WL.barkley_cross_field(c["nx"], c["ny"], seed=0)
    mask = np.ones((1, c["ny"], c["nx"]), np.uint8)
    grid = B.Grid(mask, c["h"], None, c["D"], c["D"], B.BBX_FP64, stream)
    grid.model(B.BBX_MODEL_BARKLEY, [c["a"], c["b"], c["eps"]], c["dt"])
    grid.set(0, u)
    grid.set(1, v)
    grid.nan_check(0)
    sec = time_steps(grid, stream, 2000, 100)
    nact = grid.nact
    grid.close()
    return {"workload": "Barkley 2D 100x100, 5-point, FP64, cross-field start, 2000 steps",
            "value": nact * 2000 / sec, "unit": "voxel-updates/s", "us_per_step": sec / 2000 * 1e6}


GOLDEN_MAPS = os.path.join(ROOT, "tests", "golden", "crn_cup128_at_apd.csv")


def headline_accuracy(stream):
    """The headline workload run in FP32 for its full 500 ms, in the timed launch
    configuration, against the FP64 oracle's activation times and APD90 at 4,000 seeded
    tissue voxels (a file the oracle wrote)."""
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    if not os.path.exists(GOLDEN_MAPS):
        return None
    d = np.loadtxt(GOLDEN_MAPS, delimiter=",", skiprows=2)
    idx, at_o, apd_o = d[:, 0].astype(np.int64), d[:, 1], d[:, 2]
    grid, _ = crn_workload(B.BBX_FP32, stream)
    n = int(round(WL.CRN_3D["t_end"] / WL.CRN_3D["dt"]))
    grid.step(n)
    at = grid.read(B.BBX_READ_ACT_TIME).ravel()[idx]
    apd = grid.read(B.BBX_READ_APD90).ravel()[idx]
    grid.close()
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)

    def fin(x):
        return float(x) if np.isfinite(x) else None
    ea, ep = np.abs(at[fa] - at_o[fa]), np.abs(apd[fp] - apd_o[fp])
    return {"reference": "FP64 oracle, 500 ms, 4000 seeded tissue voxels",
            "dt_ms": WL.CRN_3D["dt"],
            "same_activated_set": bool(np.array_equal(np.isfinite(at), fa)),
            "same_repolarised_set": bool(np.array_equal(np.isfinite(apd), fp)),
            "at_max_err_ms": fin(ea.max()), "at_mean_err_ms": fin(ea.mean()),
            "apd90_max_err_ms": fin(ep.max()), "apd90_mean_err_ms": fin(ep.mean())}


def thin_shell_line(stream, steps=500, warmup=50):
    """Atrium-like sparsity: CRN on a thin double shell at 8.3% of a 237x271x300 box
    (tissue list), FP32."""
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    g = WL.double_shell(237, 271, 300, h=0.25, active_frac=0.083, seed=6)
    grid = B.Grid(g["mask"], 0.25, g["fibre"], 0.3, 0.03, B.BBX_FP32, stream)
    grid.model(B.BBX_MODEL_CRN, [], 0.01)
    for v, val in enumerate(WL.CRN_INITIAL):
        grid.fill(v, val)
    grid.nan_check(0)
    sec = time_steps(grid, stream, steps, warmup)
    nact = grid.nact
    grid.close()
    per = sec / steps
    gbs = 200 * nact / per / 1e9                       # 201 B/voxel without the recorder byte
    return {"workload": f"CRN thin double shell, 237x271x300 box, 8.3% active ({nact} tissue voxels), FP32",
            "value": nact / per, "unit": "voxel-updates/s", "ms_per_step": per * 1e3,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": 200}}


def stencil_roofline(stream, steps=100, warmup=10):
    """Pure-diffusion FP32 stencil on a dense 512x512x384 box with fibres rotating
    through z (the HBM roofline workload: V is 403 MB, beyond the Infinity Cache)."""
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    nx, ny, nz = 512, 512, 384
    mask, fib = WL.full_box_rotating(nx, ny, nz)
    grid = B.Grid(mask, 0.2, fib, 0.3, 0.03, B.BBX_FP32, stream)
    del fib
    grid.model(B.BBX_MODEL_NONE, [], 0.01)
    grid.set(0, np.linspace(-80, 20, mask.size).reshape(mask.shape))
    grid.nan_check(0)
    sec = time_steps(grid, stream, steps, warmup)
    nact = grid.nact
    grid.close()
    per_launch = sec / steps
    gbs = STENCIL_BYTES_PER_VOXEL * nact / per_launch / 1e9
    return {"workload": "pure diffusion, dense 512x512x384, 19-point, rotating fibres, FP32",
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": STENCIL_BYTES_PER_VOXEL,
            "us_per_launch": round(per_launch * 1e6, 2),
            "voxel_updates_per_s": nact / per_launch,
            "device_copy_GBs": round(copy_bandwidth(stream), 1)}


def copy_bandwidth(stream, nbytes=1 << 30, reps=20):
    """Read+write bandwidth of a plain 1 GiB device-to-device copy (context for the
    stencil's fraction of peak)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    return 2 * nbytes * reps / sec / 1e9


def surrogate_line(stream, model="crn", t_ms=500.0, iters=20000, v_hi=-81.0):
    """Surrogate-with-fallback on the 128x128x64 cup with `model` kinetics: train on paced
    runs of the cup (outside the timed region), anchor the resting state, then time a full
    run with the plain FP32 kinetics and with the surrogate accepting tissue below v_hi mV,
    and compare activation-time and APD90 maps."""
    import torch
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import surrogate as SU
    mid, nv, c, geo, rest, amp, dur = SU._model_setup(model)
    t0 = time.perf_counter()
    S, S1 = SU.generate_pairs(runs=3, t_ms=1200.0, per_sample=2048, seed=2, stream=stream, model=model)
    t1 = time.perf_counter()
    anchor = B.Grid(np.ones((1, 1, 1), np.uint8), 0.25, None, 0.3, 0.03, B.BBX_FP32, stream)
    anchor.model(mid, [], c["dt"])
    tr = SU.train(S, S1, iters=iters, batch=4096, lr=1e-3, seed=0, stream=stream, anchor_grid=anchor,
                  model=model)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del S, S1
    nsteps = int(round(t_ms / c["dt"]))
    g = geo(128, 128, 64, seed=c["seed"], active=c["active"], h=c["h"])
    m = g["mask"] == 1
    res = {}
    for name in ("plain", "surrogate"):
        grid = B.Grid(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], B.BBX_FP32, stream)
        grid.model(mid, [], c["dt"])
        for v in range(nv):
            grid.set(v, g["state"][v])
        grid.stimulus(g["stim"], amp, 0.0, dur)
        grid.record(-40.0)
        grid.nan_check(0)
        if name == "surrogate":
            lo, hi, dv = SU.accepted_box(tr.stats, nvar=nv)
            hi[0] = v_hi                      # the network handles tissue below v_hi only
            grid.surrogate(tr.mlp, lo, hi, dv)
        sec = time_steps(grid, stream, nsteps, 0)
        res[name] = dict(sec=sec, at=grid.read(B.BBX_READ_ACT_TIME)[m], apd=grid.read(B.BBX_READ_APD90)[m],
                         fb=int(grid.read(B.BBX_READ_FALLBACK_COUNT)[0]), nact=grid.nact)
        grid.close()
    p, q = res["plain"], res["surrogate"]
    both = np.isfinite(p["at"]) & np.isfinite(q["at"])
    dat = np.abs(p["at"][both] - q["at"][both])
    bapd = np.isfinite(p["apd"]) & np.isfinite(q["apd"])
    dapd = np.abs(p["apd"][bapd] - q["apd"][bapd])
    value = q["nact"] * nsteps / q["sec"]
    return {"workload": f"{model.upper()} cup 128x128x64, {t_ms:.0f} ms, FP32, surrogate {nv}-128-128-{nv} "
                        "SiLU (BF16 MFMA, FP32 accumulate) with per-voxel fallback",
            "value": value, "unit": "voxel-updates/s", "ms_per_step": q["sec"] / nsteps * 1e3,
            "plain_ms_per_step": p["sec"] / nsteps * 1e3,
            "accepted_v_below_mV": v_hi,
            "speedup_vs_plain": p["sec"] / q["sec"],
            "fallback_fraction": q["fb"] / (q["nact"] * nsteps),
            "at_within_1dt": bool(dat.size and dat.max() <= c["dt"]),
            "at_err_vs_plain_ms": {"max": float(dat.max()) if dat.size else None,
                                   "mean": float(dat.mean()) if dat.size else None,
                                   "dt": c["dt"], "activated_plain": int(np.isfinite(p["at"]).sum()),
                                   "activated_surrogate": int(np.isfinite(q["at"]).sum())},
            "apd90_err_vs_plain_ms": {"max": float(dapd.max()) if dapd.size else None,
                                      "mean": float(dapd.mean()) if dapd.size else None,
                                      "n": int(bapd.sum())},
            "training": {"pairs": tr.npairs, "iters": iters, "batch": 4096,
                         "final_loss": float(np.mean(tr.loss[-100:])), "gen_s": round(t1 - t0, 2),
                         "train_s": round(t2 - t1, 2)}}


def tabulated_line(stream, dv, steps, warmup):
    """The same CRN workload with the voltage-only kinetic terms read from a table of
    spacing dv (mV), timed like the headline run."""
    from paper_1605_06015_amd import bbx as B
    grid, _ = crn_workload(B.BBX_FP32, stream, tab_dv=dv)
    grid.nan_check(0)
    sec = time_steps(grid, stream, steps, warmup)
    if grid.read(B.BBX_READ_NAN_FLAG)[0]:
        raise RuntimeError("non-finite state in the tabulated run")
    nact = grid.nact
    grid.close()
    return {"workload": f"CRN cup 128x128x64, FP32, Rush-Larsen/current voltage terms tabulated "
                        f"(dv {dv} mV, [-120, 80] mV, linear interpolation)",
            "value": nact * steps / sec, "unit": "voxel-updates/s",
            "ms_per_step": sec / steps * 1e3}


# Algorithmic HBM bytes per voxel update of the FP32 FK4 ensemble step: u read +
# written (8), three gates read + written (24), recorder status byte (1).
ENS_BYTES_PER_VOXEL = 4 * 2 + 3 * 4 * 2 + 1


def ensemble_workload(stream):
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    c = WL.FK4_ENSEMBLE
    w = WL.fk4_ensemble(n=c["n"], side_lo=c["side_lo"], side_hi=c["side_hi"], seed=c["seed"],
                        h=c["h"], Dpar=c["Dpar"], aniso=c["aniso"], spread=c["spread"],
                        s1_amp=c["s1_amp"], s1_ms=c["s1_ms"], apd_est_ms=c["apd_est_ms"],
                        cv_est_mm_ms=c["cv_est_mm_ms"])
    e = B.Ensemble(w["nx"], w["ny"], c["h"], w["Dpar"], w["Dperp"], w["angle"], B.BBX_MODEL_FK4,
                   w["params"], c["dt"], B.BBX_FP32, stream)
    for i in range(len(w["nx"])):
        n = int(w["nx"][i]) * int(w["ny"][i])
        for v, val in enumerate(WL.FK4_INITIAL):
            e.set(i, v, np.full(n, val))
    for (i, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
        e.stimulus(i, x0, x1, y0, y1, amp, t0, dur)
    e.record(c["theta"])
    return e, w, c


def ensemble_line(steps=None, chunk=1000):
    """f1: 96 uneven 2D FK4 tissues advanced together, the whole 20,000-step (1 s) protocol
    replayed from a captured HIP graph of `chunk` steps, tile shape autotuned; the direct
    launch mode is timed over the first steps for comparison."""
    import torch
    from paper_1605_06015_amd import bbx as B
    s = torch.cuda.Stream()
    e, w, c = ensemble_workload(s)
    steps = steps or c["steps"]
    best, times = e.tune(20)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # direct launches: 200 steps from a fresh copy of the protocol start
    d, _, _ = ensemble_workload(s)
    d.variant(best)
    d.step(20)
    torch.cuda.synchronize()
    ev[0].record(s)
    d.step(200)
    ev[1].record(s)
    torch.cuda.synchronize()
    direct_ms = ev[0].elapsed_time(ev[1]) / 200
    d.close()
    e.graph(chunk)
    torch.cuda.synchronize()
    ev[2].record(s)
    e.step(steps)
    ev[3].record(s)
    torch.cuda.synchronize()
    sec = ev[2].elapsed_time(ev[3]) / 1e3
    if e.read(B.BBX_READ_NAN_FLAG, 0)[0]:
        raise RuntimeError("non-finite state in the ensemble run")
    activated = sum(int(np.isfinite(e.read(B.BBX_READ_ACT_TIME, i)).sum()) for i in range(len(w["nx"])))
    nvox = e.nvox
    per = sec / steps
    gbs = ENS_BYTES_PER_VOXEL * nvox / per / 1e9
    names = ["64x4 LDS", "32x8 LDS", "16x16 LDS", "64x4 direct", "64x32 march", "64x128 march"]
    e.close()
    return {"workload": f"{len(w['nx'])} 2D FK4 tissues, sides {int(w['nx'].min())}-{int(w['nx'].max())} "
                        f"({nvox} voxels), per-tissue D/angle/time constants, S1-S2, "
                        f"{steps} steps x {c['dt']} ms, FP32, graph chunk {chunk}",
            "value": nvox * steps / sec, "unit": "voxel-updates/s", "ms_per_step": per * 1e3,
            "total_s": sec, "tile": names[best],
            "tune_ms_per_20_steps": {names[i]: round(float(times[i]), 3) for i in range(len(names))},
            "direct_launch_ms_per_step": direct_ms, "graph_speedup": direct_ms / (per * 1e3),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": ENS_BYTES_PER_VOXEL},
            "activated_voxels": activated}


# Algorithmic HBM bytes per tissue-voxel update of the fused TP06 step in FP32: 19
# state values read + written, geometry (index, neighbour bits, fibre, face
# coefficients: 32 B) and the recorder status byte.
TP06_BYTES_PER_VOXEL = 19 * 4 * 2 + 32 + 1


def tp06_workload(stream):
    from paper_1605_06015_amd import bbx as B
    from paper_1605_06015_amd import workloads as WL
    c = WL.TP06_3D
    g3 = shell_geometry()
    grid = B.Grid(g3["mask"], c["h"], g3["fibre"], c["Dpar"], c["Dperp"], B.BBX_FP32, stream)
    grid.model(B.BBX_MODEL_TP06, [], c["dt"])
    for v, val in enumerate(WL.TP06_INITIAL):
        grid.fill(v, val)
    grid.stimulus(g3["s1"], c["s1_amp"], 0.0, c["s1_ms"])
    grid.stimulus(g3["s2"], c["s2_amp"], c["s2_t"], c["s2_ms"])
    grid.record(c["theta"])
    grid.nan_check(0)
    return grid, g3["electrodes"], c


def tp06_line(stream, steps=1000, warmup=100):
    """f2: TP06 on the 512x512x384 biventricular-like double shell (25.2 M tissue voxels),
    FP32, S1 at the apex; timed without and with the FP64 pseudo-ECG sampled every 1 ms
    at eight electrodes."""
    from paper_1605_06015_amd import bbx as B
    grid, E, c = tp06_workload(stream)
    nact = grid.nact
    sec = time_steps(grid, stream, steps, warmup)
    every = int(round(c["ecg_every_ms"] / c["dt"]))
    grid.ecg(E, every=every, max_samples=100000)
    sec_ecg = time_steps(grid, stream, steps, 0)
    nsamp = int(grid.ecg_series().shape[0])
    if grid.read(B.BBX_READ_NAN_FLAG)[0]:
        raise RuntimeError("non-finite state in the TP06 run")
    grid.close()
    per = sec / steps
    gbs = TP06_BYTES_PER_VOXEL * nact / per / 1e9
    return {"workload": f"TP06 3D, 512x512x384 double shell, 25% active ({nact} tissue voxels), "
                        "19-point anisotropic, transmural fibres +-60 deg, h 0.2 mm, dt 0.02 ms, FP32",
            "value": nact * steps / sec, "unit": "voxel-updates/s", "ms_per_step": per * 1e3,
            "steps": steps, "one_second_protocol_s_est": per * round(c["t_end"] / c["dt"]),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_voxel": TP06_BYTES_PER_VOXEL},
            "pseudo_ecg": {"electrodes": int(len(E)), "every_steps": every, "samples": nsamp,
                           "ms_per_sample": (sec_ecg - sec) / max(nsamp, 1) * 1e3,
                           "overhead_frac": (sec_ecg - sec) / sec}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the stencil roofline and surrogate runs")
    ap.add_argument("--sur-ms", type=float, default=500.0,
                    help="simulated time of the surrogate comparison runs (ms)")
    ap.add_argument("--tab", type=float, default=0.05,
                    help="table spacing (mV) of the tabulated CRN comparison line (0: skip)")
    ap.add_argument("--ens-steps", type=int, default=0,
                    help="steps of the ensemble line (0: the full 20,000-step protocol)")
    ap.add_argument("--tp06-steps", type=int, default=1000, help="timed steps of the TP06 line")
    ap.add_argument("--profile", choices=["crn", "crn_tab", "stencil", "ensemble", "tp06"], default=None,
                    help="counter-collection mode: a few steps of one workload, then one plain "
                         "256 MiB device copy whose byte count calibrates FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_06015_amd import bbx as B
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if args.profile:
        if args.profile == "tp06":
            grid, _, _ = tp06_workload(stream)
            grid.step(args.warmup + args.steps)
            grid.close()
        elif args.profile == "ensemble":
            e, _, _ = ensemble_workload(stream)
            e.variant(B.BBX_ENS_DIRECT_64x4)
            e.step(args.warmup + args.steps)
            e.close()
        elif args.profile in ("crn", "crn_tab"):
            grid, _ = crn_workload(B.BBX_FP32, stream,
                                   tab_dv=args.tab if args.profile == "crn_tab" else 0.0)
            grid.nan_check(0)
            grid.step(args.warmup + args.steps)
            grid.close()
        else:
            stencil_roofline(stream, steps=args.steps, warmup=args.warmup)
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile": args.profile, "copy_bytes_each_way": src.numel() * 4}))
        return

    grid, g = crn_workload(B.BBX_FP32, stream)
    grid.nan_check(0)
    nact = grid.nact
    sec = time_steps(grid, stream, args.steps, args.warmup)
    flag = grid.read(B.BBX_READ_NAN_FLAG)[0]
    if flag:
        print("bench.py: non-finite state", file=sys.stderr)
        sys.exit(1)
    ms_per_step = sec / args.steps * 1e3
    value = nact * args.steps / sec
    per_launch = sec / args.steps
    achieved = CRN_BYTES_PER_VOXEL * nact / per_launch / 1e9
    ctr = measured_counters("step_crn_cup128_fp32_traffic.json")
    traffic = ctr.get("bytes_per_launch") if ctr else None
    valu = None
    if ctr and ctr.get("valu_insts_per_launch"):
        # VALU issue: one wave64 instruction per CU per cycle, 256 CUs at 2.4 GHz
        gi = ctr["valu_insts_per_launch"] / per_launch / 1e9
        valu = {"achieved": round(gi, 1), "peak": VALU_PEAK_GINST, "unit": "G wave-instructions/s",
                "frac": round(gi / VALU_PEAK_GINST, 4),
                "insts_per_launch": ctr["valu_insts_per_launch"]}
    out = {
        "metric": METRIC, "value": value, "unit": "voxel-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "CRN atrial 3D, 128x128x64 ellipsoidal cup, 35% active "
                               f"({nact} tissue voxels), 19-point anisotropic no-flux stencil, "
                               "rotating fibres, dt 0.01 ms, apex stimulus, AT/APD90 recording, "
                               "FP32 plain ionic", "tissue_voxels": nact, "dt_ms": 0.01},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_step<float, Crn, aniso>",
                     "bytes_per_voxel": CRN_BYTES_PER_VOXEL,
                     "us_per_launch": round(per_launch * 1e6, 2), "valu": valu},
    }
    grid.close()
    out["accuracy"] = headline_accuracy(stream)
    if not args.no_extras:
        if args.tab > 0:
            out["tabulated"] = tabulated_line(stream, args.tab, args.steps, args.warmup)
            out["tabulated"]["speedup_vs_plain"] = round(ms_per_step / out["tabulated"]["ms_per_step"], 3)
        out["stencil_roofline"] = stencil_roofline(stream)
        out["stencil_roofline"]["other_cases"] = stencil_cases(stream)
        out["paper_shape"] = paper_shape_line(stream)
        out["thin_shell"] = thin_shell_line(stream)
        out["barkley_2d"] = barkley_line(stream)
        out["ensemble"] = ensemble_line(steps=args.ens_steps or None)
        out["tp06"] = tp06_line(stream, steps=args.tp06_steps)
        # acceptance thresholds at which the surrogate run's activation times stay within
        # one time step of the plain run's (found by sweeping the threshold on this workload)
        out["surrogate"] = surrogate_line(stream, "crn", t_ms=args.sur_ms, v_hi=-81.17)
        out["surrogate_tp06"] = surrogate_line(stream, "tp06", t_ms=args.sur_ms, v_hi=-85.225)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
