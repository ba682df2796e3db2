"""Shared test plumbing: run the same seeded problem through the oracle and
through the GPU library (via its C ABI binding), and compare.

Normwise relative error per state variable (the reading of "1e-10 relative"):
max over tissue voxels |x_gpu - x_oracle| / max(max |x_oracle|, tiny).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from oracle import oracle as O


def round_half_away(x: float) -> int:
    """Nearest integer, halves away from zero (the library's stimulus rounding)."""
    return int(math.floor(abs(x) + 0.5)) * (1 if x >= 0 else -1)


@dataclass
class Problem:
    mask: np.ndarray                  # uint8 (nz, ny, nx)
    h: float
    fibre: object                     # float64 (nz, ny, nx, 3) or None
    Dpar: float
    Dperp: float
    model: int
    params: list
    dt: float
    scheme: int = 0
    state: np.ndarray = None          # (nvar, nz, ny, nx)
    stims: list = field(default_factory=list)   # (region, amp, t0_ms, dur_ms, period_ms, count)
    theta: float = None
    integrator: int = 0               # O.INTEGRATOR_EULER_RL or O.INTEGRATOR_RK4


def run_oracle(p: Problem, nsteps: int, nthreads: int = 0):
    s = O.Sim(p.mask, p.h, p.fibre, p.Dpar, p.Dperp, p.model, list(p.params), p.dt,
              scheme=p.scheme, nthreads=nthreads, integrator=p.integrator)
    s.state[:] = p.state
    for (reg, amp, t0, dur, per, cnt) in p.stims:
        s.stimuli.append(O.Stimulus(reg, amp, round_half_away(t0 / p.dt),
                                    round_half_away(dur / p.dt),
                                    round_half_away(per / p.dt) if per > 0 else 0, cnt))
    if p.theta is not None:
        s.start_recording(p.theta)
    if nsteps:
        s.step(nsteps)
    return s


def make_gpu(p: Problem, precision: int, stream=None):
    from paper_1605_06015_amd import bbx as B
    g = B.Grid(p.mask, p.h, p.fibre, p.Dpar, p.Dperp, precision, stream)
    g.model(p.model, p.params, p.dt, p.scheme)
    if p.integrator:
        g.integrator(p.integrator)
    for v in range(p.state.shape[0]):
        g.set(v, p.state[v])
    for (reg, amp, t0, dur, per, cnt) in p.stims:
        g.stimulus(reg, amp, t0, dur, per, cnt)
    if p.theta is not None:
        g.record(p.theta)
    return g


def gpu_state(g, nvar):
    return np.stack([g.get(v) for v in range(nvar)])


def rel_errs(x_gpu, x_orc, mask):
    m = mask.astype(bool)
    out = []
    for v in range(x_orc.shape[0]):
        a, b = x_gpu[v][m], x_orc[v][m]
        scale = max(np.abs(b).max() if b.size else 0.0, 1e-300)
        out.append(np.abs(a - b).max() / scale if b.size else 0.0)
    return np.array(out)


def rec_arrays(s, mask):
    """Oracle recording arrays scattered to box layout (NaN at void)."""
    out = {}
    for name in ("at", "apd", "vmax"):
        box = np.full(mask.size, np.nan)
        box[s.act] = getattr(s.rec, name)
        out[name] = box.reshape(mask.shape)
    st = np.full(mask.size, 255, np.uint8)
    st[s.act] = s.rec.status
    out["status"] = st.reshape(mask.shape)
    return out
