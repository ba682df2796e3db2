"""Python access to the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It builds ``bbx_oracle.c`` with gcc (serial semantics;
OpenMP only splits the per-voxel loop, which writes disjoint outputs, so
threaded and serial runs are bitwise identical) and wraps it with ctypes.
Nothing here imports the GPU library.

Paper: Antonioletti et al., BeatBox (arXiv:1605.06015).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bbx_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# A build with AddressSanitizer and UndefinedBehaviorSanitizer, loaded instead when
# BBX_ORACLE_SANITIZE=1 (the process must preload gcc's sanitizer runtimes).
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]

MODEL_NONE, MODEL_BARKLEY, MODEL_ZFK, MODEL_FHN, MODEL_CRN, MODEL_FK4, MODEL_TP06 = \
    0, 1, 2, 3, 4, 5, 6
SCHEME_ADDITIVE, SCHEME_SPLIT = 0, 1
INTEGRATOR_EULER_RL, INTEGRATOR_RK4 = 0, 1


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle into a shared library next to its source (with sanitize: the
    AddressSanitizer / UndefinedBehaviorSanitizer build)."""
    lib = LIB_SAN if sanitize else LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               *(SAN_FLAGS if sanitize else []), "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, lib)
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("BBX_ORACLE_SANITIZE") == "1"
        L = C.CDLL(build(sanitize=san))
        P = C.c_void_p
        i64 = C.c_int64
        L.orc_weights.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, P, P, C.c_double,
                                  C.c_double, i64, P, P]
        L.orc_weights.restype = C.c_int
        L.orc_apply_L.argtypes = [C.c_int, C.c_int, C.c_int, i64, P, P, P, P]
        L.orc_apply_L.restype = None
        L.orc_nvar.argtypes = [C.c_int]
        L.orc_nvar.restype = C.c_int
        L.orc_nparams.argtypes = [C.c_int]
        L.orc_nparams.restype = C.c_int
        L.orc_model_eval.argtypes = [C.c_int, P, P, P, P, P]
        L.orc_model_eval.restype = C.c_int
        L.orc_run.argtypes = [C.c_int, C.c_int, C.c_int, i64, P, P,
                              C.c_int, P, C.c_double, C.c_int, C.c_int,
                              C.c_int, P, P, P, P, P, P,
                              P, P, i64, i64,
                              C.c_int, C.c_double, P, P, P, P, P, C.c_int]
        L.orc_run.restype = C.c_int
        L.orc_tips.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, P, P, C.c_double, P,
                               C.c_double, P, P, i64]
        L.orc_tips.restype = i64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def nvar(model: int) -> int:
    return lib().orc_nvar(model)


def weights(mask: np.ndarray, h: float, fibre, Dpar: float, Dperp: float):
    """Literal 27-point weights of every tissue voxel.

    mask: uint8 array of shape (nz, ny, nx); fibre: float64 (nz, ny, nx, 3) or None.
    Returns (act, W) with act the box indices of tissue voxels (increasing) and
    W of shape (nact, 27).
    """
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    act = np.flatnonzero(mask.ravel()).astype(np.int64)
    W = np.zeros((act.size, 27), dtype=np.float64)
    fib = None if fibre is None else np.ascontiguousarray(fibre, dtype=np.float64)
    rc = lib().orc_weights(nx, ny, nz, float(h), _p(mask), _p(fib), float(Dpar), float(Dperp),
                           act.size, _p(act), _p(W))
    if rc != 0:
        raise ValueError("oracle: a tissue voxel has a zero-length fibre vector")
    return act, W


def apply_L(mask: np.ndarray, act: np.ndarray, W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(L u) at every tissue voxel (u in box layout)."""
    nz, ny, nx = mask.shape
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    out = np.zeros(act.size, dtype=np.float64)
    lib().orc_apply_L(nx, ny, nz, act.size, _p(act), _p(W), _p(u), _p(out))
    return out


def pseudo_ecg(mask: np.ndarray, h: float, fibre, Dpar: float, Dperp: float, V: np.ndarray,
               electrodes, chunk: int = 1 << 20, return_scale: bool = False):
    """Pseudo-ECG of the field V (box layout) at each electrode position (mm):
        phi(x_e) = h^3 sum_{p in tissue} (L V)_p / |x_p - x_e|,   x_p = h (x, y, z),
    with L the scheme's discrete diffusion operator (the same weights as the step).
    With no-flux boundaries, summation by parts turns this into the volume integral
    of -D grad V . grad(1/r) of the classical pseudo-ECG, up to its constant factor.
    Evaluated in FP64 over chunks of tissue voxels (weights per chunk).  With
    return_scale, also returns h^3 sum_p (sum_q |W_q (V_{p+q} - V_p)|) / |x_p - x_e|,
    the size of the terms whose cancellation the sum performs (the yardstick for
    comparing evaluations in other precisions)."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    act_all = np.flatnonzero(mask.ravel()).astype(np.int64)
    E = np.atleast_2d(np.asarray(electrodes, np.float64))
    fib = None if fibre is None else np.ascontiguousarray(fibre, dtype=np.float64)
    u = np.ascontiguousarray(V, dtype=np.float64).ravel()
    out = np.zeros(E.shape[0])
    scale = np.zeros(E.shape[0])
    offs = np.array([dz * nx * ny + dy * nx + dx for dz in (-1, 0, 1) for dy in (-1, 0, 1)
                     for dx in (-1, 0, 1)], dtype=np.int64)
    for c0 in range(0, act_all.size, chunk):
        act = np.ascontiguousarray(act_all[c0:c0 + chunk])
        W = np.zeros((act.size, 27), dtype=np.float64)
        if lib().orc_weights(nx, ny, nz, float(h), _p(mask), _p(fib), float(Dpar), float(Dperp),
                             act.size, _p(act), _p(W)) != 0:
            raise ValueError("oracle: a tissue voxel has a zero-length fibre vector")
        LV = np.zeros(act.size, dtype=np.float64)
        lib().orc_apply_L(nx, ny, nz, act.size, _p(act), _p(W), _p(u), _p(LV))
        x = (act % nx) * h
        y = ((act // nx) % ny) * h
        z = (act // (nx * ny)) * h
        if return_scale:
            nb = np.clip(act[:, None] + offs[None, :], 0, u.size - 1)
            W[:, 13] = 0.0
            A = np.sum(np.abs(W * (u[nb] - u[act][:, None])), axis=1)
        for e in range(E.shape[0]):
            r = np.sqrt((x - E[e, 0]) ** 2 + (y - E[e, 1]) ** 2 + (z - E[e, 2]) ** 2)
            out[e] += np.sum(LV / r)
            if return_scale:
                scale[e] += np.sum(A / r)
    if return_scale:
        return out * h ** 3, scale * h ** 3
    return out * h ** 3


def tips(mask, h, u, u_level, v, v_level, max_points=100000):
    """Phase singularities in z cross-sections: intersections of the isolines
    u = u_level and v = v_level inside cells of four tissue voxels (the `singz` device).
    Returns (stats, points): stats = [count, mean x, mean y, mean z, std x, std y, std z]
    (mm, population standard deviation), points (n, 3) in mm in cell order."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    uu = np.ascontiguousarray(u, dtype=np.float64)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    sums = np.zeros(7)
    pts = np.zeros((max_points, 3))
    n = lib().orc_tips(nx, ny, nz, float(h), _p(mask), _p(uu), float(u_level), _p(vv),
                       float(v_level), _p(sums), _p(pts), int(max_points))
    stats = np.zeros(7)
    stats[0] = sums[0]
    if n > 0:
        mean = sums[1:4] / n
        stats[1:4] = mean
        stats[4:7] = np.sqrt(np.maximum(sums[4:7] / n - mean * mean, 0.0))
    return stats, pts[:min(n, max_points)].copy()


def model_eval(model: int, params, y):
    """Kinetic rates of one cell: (rate, inf, tau), each of length nvar."""
    nv = nvar(model)
    p = np.ascontiguousarray(params if params is not None else [0.0], dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    rate = np.zeros(nv)
    inf = np.zeros(nv)
    tau = np.zeros(nv)
    lib().orc_model_eval(model, _p(p), _p(y), _p(rate), _p(inf), _p(tau))
    return rate, inf, tau


@dataclass
class Stimulus:
    """One stimulus: region (uint8 box mask), amplitude, window in whole steps."""
    region: np.ndarray
    amp: float
    n0: int
    length: int
    period: int = 0
    count: int = 1


@dataclass
class Recording:
    theta: float
    status: np.ndarray
    at: np.ndarray
    vmax: np.ndarray
    apd: np.ndarray
    vrest: np.ndarray


@dataclass
class Sim:
    """An oracle simulation: geometry, model, state in box layout [nvar][nz][ny][nx]."""
    mask: np.ndarray
    h: float
    fibre: object
    Dpar: float
    Dperp: float
    model: int
    params: list
    dt: float
    scheme: int = SCHEME_ADDITIVE
    stimuli: list = field(default_factory=list)
    nthreads: int = 0
    integrator: int = INTEGRATOR_EULER_RL

    def __post_init__(self):
        self.mask = np.ascontiguousarray(self.mask, dtype=np.uint8)
        self.act, self.W = weights(self.mask, self.h, self.fibre, self.Dpar, self.Dperp)
        nv = nvar(self.model)
        self.state = np.zeros((nv,) + self.mask.shape, dtype=np.float64)
        self.vnext = np.zeros(self.mask.size, dtype=np.float64)
        self.n = 0
        self.rec = None

    def set_state(self, var: int, values) -> None:
        self.state[var] = np.asarray(values, dtype=np.float64).reshape(self.mask.shape)

    def start_recording(self, theta: float) -> None:
        na = self.act.size
        self.rec = Recording(theta, np.zeros(na, np.uint8), np.full(na, np.nan),
                             np.full(na, np.nan), np.full(na, np.nan),
                             self.state[0].ravel()[self.act].copy())

    def step(self, nsteps: int) -> None:
        nz, ny, nx = self.mask.shape
        ns = len(self.stimuli)
        if ns:
            reg = np.ascontiguousarray(np.stack([np.asarray(s.region, np.uint8).ravel()
                                                 for s in self.stimuli]))
            amp = np.array([s.amp for s in self.stimuli], np.float64)
            sn0 = np.array([s.n0 for s in self.stimuli], np.int64)
            sl = np.array([s.length for s in self.stimuli], np.int64)
            sp = np.array([s.period for s in self.stimuli], np.int64)
            sc = np.array([s.count for s in self.stimuli], np.int64)
        else:
            reg = amp = sn0 = sl = sp = sc = None
        p = np.ascontiguousarray(self.params if self.params else [0.0], dtype=np.float64)
        r = self.rec
        rc = lib().orc_run(nx, ny, nz, self.act.size, _p(self.act), _p(self.W),
                           self.model, _p(p), float(self.dt), int(self.scheme),
                           int(self.integrator),
                           ns, _p(reg), _p(amp), _p(sn0), _p(sl), _p(sp), _p(sc),
                           _p(self.state), _p(self.vnext), int(self.n), int(nsteps),
                           1 if r is not None else 0, r.theta if r else 0.0,
                           _p(r.status) if r else None, _p(r.at) if r else None,
                           _p(r.vmax) if r else None, _p(r.apd) if r else None,
                           _p(r.vrest) if r else None, int(self.nthreads))
        if rc != 0:
            raise RuntimeError("oracle run failed")
        self.n += nsteps
