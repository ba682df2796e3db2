"""ctypes binding of libbbx.so (the C ABI declared in include/bbx.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libbbx.so.  Importing this module fails loudly if the library has
not been built; there is no fallback path.

PyTorch is used only as plumbing: the caller may pass a torch stream (its
``cuda_stream`` handle is handed to the library) and device tensors as
readout targets.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# BBX_LIB may name another build of the library (the sanitized host build of the CPU
# checks); the default is the in-tree libbbx.so.
LIB_PATH = os.environ.get("BBX_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                     "libbbx.so")

BBX_OK, BBX_EINVAL, BBX_ENOMEM, BBX_EDEVICE, BBX_ESTATE, BBX_EUNSTABLE, BBX_ENUMERIC, BBX_ENOTSUP = \
    0, -1, -2, -3, -4, -5, -6, -7
BBX_FP32, BBX_FP64 = 0, 1
BBX_SCHEME_ADDITIVE, BBX_SCHEME_SPLIT = 0, 1
BBX_INTEGRATOR_EULER_RL, BBX_INTEGRATOR_RK4 = 0, 1
BBX_MODEL_NONE, BBX_MODEL_BARKLEY, BBX_MODEL_ZFK, BBX_MODEL_FHN, BBX_MODEL_CRN, BBX_MODEL_FK4, \
    BBX_MODEL_TP06 = 0, 1, 2, 3, 4, 5, 6
(BBX_READ_VAR, BBX_READ_ACT_TIME, BBX_READ_APD90, BBX_READ_VMAX, BBX_READ_STATUS,
 BBX_READ_REDUCE_MAX, BBX_READ_REDUCE_SUM, BBX_READ_NAN_FLAG, BBX_READ_STEP,
 BBX_READ_WEIGHTS, BBX_READ_FALLBACK_COUNT, BBX_READ_ECG, BBX_READ_ECG_SERIES,
 BBX_READ_ECG_COUNT, BBX_READ_ALL_STATE) = range(15)
(BBX_INFO_NACTIVE, BBX_INFO_NVAR, BBX_INFO_NBOX, BBX_INFO_DEVICE_BYTES, BBX_INFO_SEND_LO,
 BBX_INFO_SEND_HI, BBX_INFO_RECV_LO, BBX_INFO_RECV_HI) = range(8)
(BBX_ENS_TILE_64x4, BBX_ENS_TILE_32x8, BBX_ENS_TILE_16x16, BBX_ENS_DIRECT_64x4, BBX_ENS_MARCH_64x32,
 BBX_ENS_MARCH_64x128, BBX_ENS_NVARIANT) = range(7)
(BBX_ENS_INFO_VOXELS, BBX_ENS_INFO_TILES, BBX_ENS_INFO_VARIANT, BBX_ENS_INFO_DEVICE_BYTES,
 BBX_ENS_INFO_GRAPH_CHUNK, BBX_ENS_INFO_NVAR) = range(6)

# Every symbol the header declares, with (restype, argtypes).
_P, _I, _D, _I64, _SZ = C.c_void_p, C.c_int, C.c_double, C.c_int64, C.c_size_t
SIGNATURES = {
    "bbx_grid_create": (_I, [_I, _I, _I, _D, _P, _P, _D, _D, _I, _P, C.POINTER(_P)]),
    "bbx_slab_bounds": (_I, [_I, _I, _I, _P, _I, _P]),
    "bbx_slab_create": (_I, [_I, _I, _I, _I, _I, _D, _P, _P, _D, _D, _I, _P, C.POINTER(_P)]),
    "bbx_halo_pack": (_I, [_P, _I, _P, _I64]),
    "bbx_halo_unpack": (_I, [_P, _I, _P, _I64]),
    "bbx_model_set": (_I, [_P, _I, _P, _I, _D, _I]),
    "bbx_state_set": (_I, [_P, _I, _P]),
    "bbx_state_fill": (_I, [_P, _I, _D]),
    "bbx_stimulus_add": (_I, [_P, _P, _D, _D, _D, _D, _I]),
    "bbx_stimulus_clear": (_I, [_P]),
    "bbx_recording_set": (_I, [_P, _D]),
    "bbx_nan_check_set": (_I, [_P, _I64]),
    "bbx_clock_set": (_I, [_P, _I64]),
    "bbx_integrator_set": (_I, [_P, _I]),
    "bbx_graph_set": (_I, [_P, _I]),
    "bbx_tabulation_set": (_I, [_P, _D]),
    "bbx_ecg_set": (_I, [_P, _I, _P, _I64, _I64]),
    "bbx_step": (_I, [_P, _I64]),
    "bbx_readout": (_I, [_P, _I, _I, _P, _P, _SZ, _I]),
    "bbx_info": (_I, [_P, _I, C.POINTER(_I64)]),
    "bbx_tips": (_I, [_P, _I, _D, _I, _D, _P, _P, _I64, C.POINTER(_I64)]),
    "bbx_grid_destroy": (None, [_P]),
    "bbx_last_error": (C.c_char_p, []),
    "bbx_mlp_create": (_I, [_I, _I, C.c_uint64, _P, C.POINTER(_P)]),
    "bbx_mlp_params": (_I, [_P, _I, _P, _SZ]),
    "bbx_mlp_norm": (_I, [_P, _I, _P]),
    "bbx_mlp_fit_norm": (_I, [_P, _P, _P, _I64, _P]),
    "bbx_mlp_forward": (_I, [_P, _P, _I64, _P]),
    "bbx_mlp_grad": (_I, [_P, _P, _P, _I64, _P, _P]),
    "bbx_mlp_grad_static": (_I, [_P, _P, _P, _I64, _P, _P]),
    "bbx_mlp_adam": (_I, [_P, C.c_float, C.c_float, C.c_float, C.c_float]),
    "bbx_mlp_train": (_I, [_P, _P, _P, _I64, _I64, _I64, C.c_float, C.c_uint64, _P]),
    "bbx_mlp_anchor": (_I, [_P, _P, _P]),
    "bbx_mlp_destroy": (None, [_P]),
    "bbx_sample_states": (_I, [_P, _I64, C.c_uint64, _P]),
    "bbx_ionic_map": (_I, [_P, _P, _I64, _P]),
    "bbx_surrogate_set": (_I, [_P, _P, _P, _P, C.c_float]),
    "bbx_surrogate_import": (_I, [_P, _I, _I, _P, _P, _P, _P, _P, C.c_float]),
    "bbx_ensemble_create": (_I, [_I, _P, _P, _D, _P, _P, _P, _I, _P, _I, _D, _I, _P, C.POINTER(_P)]),
    "bbx_ensemble_state_set": (_I, [_P, _I, _I, _P]),
    "bbx_ensemble_stimulus_add": (_I, [_P, _I, _I, _I, _I, _I, _D, _D, _D, _D, _I]),
    "bbx_ensemble_recording_set": (_I, [_P, _D]),
    "bbx_ensemble_graph_set": (_I, [_P, _I]),
    "bbx_ensemble_variant_set": (_I, [_P, _I]),
    "bbx_ensemble_tune": (_I, [_P, _I, C.POINTER(_I), _P]),
    "bbx_ensemble_step": (_I, [_P, _I64]),
    "bbx_ensemble_readout": (_I, [_P, _I, _I, _I, _P, _SZ]),
    "bbx_ensemble_info": (_I, [_P, _I, C.POINTER(_I64)]),
    "bbx_ensemble_destroy": (None, [_P]),
}


class BBXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bbx error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libbbx.so not built ({path}); run python paper_1605_06015_amd/build.py")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def _check(rc: int) -> int:
    if rc != BBX_OK:
        raise BBXError(rc, _lib.bbx_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C-ABI names
def bbx_last_error() -> str:
    return _lib.bbx_last_error().decode()


def bbx_grid_create(nx, ny, nz, h, mask, fibre, D_par, D_perp, precision, hip_stream=None):
    """Returns an opaque grid handle (c_void_p).  mask: uint8 (nz,ny,nx);
    fibre: float64 (nz,ny,nx,3) or None."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    if mask.size != nx * ny * nz:
        raise ValueError("mask size does not match the box")
    fib = None if fibre is None else np.ascontiguousarray(fibre, dtype=np.float64)
    if fib is not None and fib.size != 3 * nx * ny * nz:
        raise ValueError("fibre size does not match the box")
    out = C.c_void_p()
    _check(_lib.bbx_grid_create(nx, ny, nz, float(h), _ptr(mask), _ptr(fib), float(D_par),
                                float(D_perp), int(precision), _stream_handle(hip_stream),
                                C.byref(out)))
    return out


def bbx_model_set(g, model, params, dt, scheme=BBX_SCHEME_ADDITIVE):
    p = np.ascontiguousarray(params if params is not None and len(params) else [0.0],
                             dtype=np.float64)
    n = 0 if params is None else len(params)
    _check(_lib.bbx_model_set(g, int(model), _ptr(p), n, float(dt), int(scheme)))


def bbx_state_set(g, var, box_values):
    v = np.ascontiguousarray(box_values, dtype=np.float64)
    _check(_lib.bbx_state_set(g, int(var), _ptr(v)))


def bbx_state_fill(g, var, value):
    _check(_lib.bbx_state_fill(g, int(var), float(value)))


def bbx_stimulus_add(g, region, amplitude, t_start, duration, period=0.0, count=1):
    r = np.ascontiguousarray(region, dtype=np.uint8)
    _check(_lib.bbx_stimulus_add(g, _ptr(r), float(amplitude), float(t_start), float(duration),
                                 float(period), int(count)))


def bbx_stimulus_clear(g):
    _check(_lib.bbx_stimulus_clear(g))


def bbx_recording_set(g, theta):
    _check(_lib.bbx_recording_set(g, float(theta)))


def bbx_nan_check_set(g, every):
    _check(_lib.bbx_nan_check_set(g, int(every)))


def bbx_ecg_set(g, xyz_mm, every=0, max_samples=0):
    E = np.ascontiguousarray(np.asarray(xyz_mm, np.float64).reshape(-1, 3))
    _check(_lib.bbx_ecg_set(g, E.shape[0], _ptr(E) if E.size else None, int(every),
                            int(max_samples)))


def bbx_tabulation_set(g, dv):
    _check(_lib.bbx_tabulation_set(g, float(dv)))


def bbx_integrator_set(g, integrator):
    _check(_lib.bbx_integrator_set(g, int(integrator)))


def bbx_clock_set(g, step):
    _check(_lib.bbx_clock_set(g, int(step)))


def bbx_step(g, nsteps):
    _check(_lib.bbx_step(g, int(nsteps)))


def bbx_readout(g, what, var=0, region=None, out=None, out_bytes=None, out_on_device=0):
    """Low-level readout into `out` (numpy array, or an int device address with
    out_on_device=1)."""
    reg = None if region is None else np.ascontiguousarray(region, dtype=np.uint8)
    if out_on_device:
        addr = C.c_void_p(int(out))
    else:
        addr = _ptr(out)
        out_bytes = out.nbytes if out_bytes is None else out_bytes
    _check(_lib.bbx_readout(g, int(what), int(var), _ptr(reg), addr, int(out_bytes),
                            int(out_on_device)))
    return out


def bbx_info(g, what) -> int:
    v = C.c_int64()
    _check(_lib.bbx_info(g, int(what), C.byref(v)))
    return v.value


def bbx_grid_destroy(g):
    _lib.bbx_grid_destroy(g)


def bbx_surrogate_import(g, nin, nout, weights_bf16, biases, norm, lo, hi, dv_max):
    """weights_bf16: uint16 array (W1, W2, W3 flat); biases float32 (b1, b2, b3); norm (4, 32)."""
    w = np.ascontiguousarray(weights_bf16, dtype=np.uint16)
    b = np.ascontiguousarray(biases, dtype=np.float32)
    nm = np.ascontiguousarray(norm, dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    _check(_lib.bbx_surrogate_import(g, int(nin), int(nout), _ptr(w), _ptr(b), _ptr(nm), _ptr(lo),
                                     _ptr(hi), float(dv_max)))


def bbx_tips(g, var_u, u_level, var_v, v_level, max_points=100000):
    """Phase singularities: (stats[7], points (n, 3) mm)."""
    stats = np.zeros(7)
    pts = np.zeros((max(int(max_points), 0), 3))
    n = C.c_int64()
    _check(_lib.bbx_tips(g, int(var_u), float(u_level), int(var_v), float(v_level), _ptr(stats),
                         _ptr(pts) if max_points else None, int(max_points), C.byref(n)))
    return stats, pts[:min(n.value, int(max_points))].copy()


def bbx_slab_bounds(mask, nslab):
    """Tissue-balanced z boundaries (nslab + 1 ints) of a (nz, ny, nx) mask."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    out = np.zeros(int(nslab) + 1, np.int32)
    _check(_lib.bbx_slab_bounds(nx, ny, nz, _ptr(mask), int(nslab), _ptr(out)))
    return out


def bbx_slab_create(mask, z0, z1, h, fibre, D_par, D_perp, precision, hip_stream=None):
    """Handle of the grid of global planes [z0, z1) of the whole box's mask / fibre."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    fib = None if fibre is None else np.ascontiguousarray(fibre, dtype=np.float64)
    out = C.c_void_p()
    _check(_lib.bbx_slab_create(nx, ny, nz, int(z0), int(z1), float(h), _ptr(mask), _ptr(fib),
                                float(D_par), float(D_perp), int(precision),
                                _stream_handle(hip_stream), C.byref(out)))
    return out


def bbx_halo_pack(g, side, buf, count):
    """buf: device tensor or address."""
    _check(_lib.bbx_halo_pack(g, int(side), _dptr(buf), int(count)))


def bbx_halo_unpack(g, side, buf, count):
    _check(_lib.bbx_halo_unpack(g, int(side), _dptr(buf), int(count)))


# ---------------------------------------------------------------- convenience
class Grid:
    """Owning wrapper: a grid on the GPU with its model, stimuli and recorder."""

    def __init__(self, mask, h, fibre=None, Dpar=1.0, Dperp=1.0, precision=BBX_FP32,
                 stream=None):
        mask = np.asarray(mask, dtype=np.uint8)
        if mask.ndim == 2:
            mask = mask[None]
        self.shape = mask.shape
        nz, ny, nx = mask.shape
        self.handle = bbx_grid_create(nx, ny, nz, h, mask, fibre, Dpar, Dperp, precision, stream)
        self.mask = mask

    @classmethod
    def slab(cls, mask, z0, z1, h, fibre=None, Dpar=1.0, Dperp=1.0, precision=BBX_FP32,
             stream=None):
        """The grid of global planes [z0, z1) of a box, with one halo plane each side;
        its box (self.shape) has z1 - z0 + 2 planes, plane 0 = global plane z0 - 1."""
        mask = np.asarray(mask, dtype=np.uint8)
        g = cls.__new__(cls)
        g.handle = bbx_slab_create(mask, z0, z1, h, fibre, Dpar, Dperp, precision, stream)
        nz, ny, nx = mask.shape
        g.shape = (z1 - z0 + 2, ny, nx)
        sl = np.zeros(g.shape, np.uint8)
        lo, hi = max(z0 - 1, 0), min(z1 + 1, nz)
        sl[lo - (z0 - 1):hi - (z0 - 1)] = mask[lo:hi]
        g.mask = sl
        return g

    def halo_counts(self):
        """(send lo, send hi, recv lo, recv hi) value counts of a slab grid."""
        return tuple(bbx_info(self.handle, w) for w in (BBX_INFO_SEND_LO, BBX_INFO_SEND_HI,
                                                         BBX_INFO_RECV_LO, BBX_INFO_RECV_HI))

    def pack(self, side, buf, count):
        bbx_halo_pack(self.handle, side, buf, count)

    def unpack(self, side, buf, count):
        bbx_halo_unpack(self.handle, side, buf, count)

    def close(self):
        if self.handle is not None:
            bbx_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nact(self):
        return bbx_info(self.handle, BBX_INFO_NACTIVE)

    def model(self, model, params, dt, scheme=BBX_SCHEME_ADDITIVE):
        bbx_model_set(self.handle, model, params, dt, scheme)

    def set(self, var, values):
        bbx_state_set(self.handle, var, np.broadcast_to(np.asarray(values, float), self.shape))

    def stimulus(self, region, amplitude, t_start, duration, period=0.0, count=1):
        bbx_stimulus_add(self.handle, region, amplitude, t_start, duration, period, count)

    def record(self, theta):
        bbx_recording_set(self.handle, theta)

    def nan_check(self, every):
        bbx_nan_check_set(self.handle, every)

    def step(self, n):
        bbx_step(self.handle, n)

    def clock(self, step):
        bbx_clock_set(self.handle, step)

    def tips(self, var_u, u_level, var_v, v_level, max_points=100000):
        return bbx_tips(self.handle, var_u, u_level, var_v, v_level, max_points)

    def integrator(self, integrator):
        bbx_integrator_set(self.handle, integrator)

    def graph(self, chunk):
        """Replay chunks of `chunk` steps from a captured HIP graph (0: direct launches)."""
        _check(_lib.bbx_graph_set(self.handle, int(chunk)))

    def fill(self, var, value):
        bbx_state_fill(self.handle, var, value)

    def tabulate(self, dv):
        bbx_tabulation_set(self.handle, dv)

    def ecg(self, xyz_mm, every=0, max_samples=0):
        """Set pseudo-ECG electrodes (mm); every > 0 samples after every `every` steps."""
        self._nelec = int(np.asarray(xyz_mm).size // 3)
        bbx_ecg_set(self.handle, xyz_mm, every, max_samples)

    def ecg_now(self):
        out = np.empty(getattr(self, "_nelec", 0), np.float64)
        return bbx_readout(self.handle, BBX_READ_ECG, 0, None, out)

    def ecg_series(self):
        cnt = np.empty(1, np.int64)
        bbx_readout(self.handle, BBX_READ_ECG_COUNT, 0, None, cnt)
        out = np.empty((int(cnt[0]), getattr(self, "_nelec", 0)), np.float64)
        if out.size:
            bbx_readout(self.handle, BBX_READ_ECG_SERIES, 0, None, out)
        return out

    def sample_states(self, n, seed, out):
        bbx_sample_states(self.handle, n, seed, out)

    def ionic_map(self, inp, out):
        bbx_ionic_map(self.handle, inp, inp.shape[0], out)

    def surrogate(self, mlp, lo=None, hi=None, dv_max=0.0):
        """Attach a trained Mlp with its accepted input box (None detaches)."""
        bbx_surrogate_set(self.handle, None if mlp is None else mlp.handle, lo, hi, dv_max)

    def checkpoint(self):
        """(state (nvar, nz, ny, nx) in box layout, step counter): BBX_READ_ALL_STATE and
        BBX_READ_STEP."""
        nv = bbx_info(self.handle, BBX_INFO_NVAR)
        out = np.empty((nv,) + tuple(self.shape), np.float64)
        bbx_readout(self.handle, BBX_READ_ALL_STATE, 0, None, out)
        return out, int(self.read(BBX_READ_STEP)[0])

    def restore(self, state, step):
        for v in range(state.shape[0]):
            bbx_state_set(self.handle, v, np.nan_to_num(state[v]))
        bbx_clock_set(self.handle, step)

    def get(self, var=0):
        out = np.empty(self.shape, np.float64)
        return bbx_readout(self.handle, BBX_READ_VAR, var, None, out)

    def read(self, what, var=0, region=None):
        if what == BBX_READ_STATUS:
            out = np.empty(self.shape, np.uint8)
        elif what in (BBX_READ_REDUCE_MAX, BBX_READ_REDUCE_SUM):
            out = np.empty(1, np.float64)
        elif what == BBX_READ_NAN_FLAG:
            out = np.empty(1, np.int32)
        elif what in (BBX_READ_STEP, BBX_READ_FALLBACK_COUNT):
            out = np.empty(1, np.int64)
        elif what == BBX_READ_WEIGHTS:
            out = np.empty((self.nact, 27), np.float64)
        else:
            out = np.empty(self.shape, np.float64)
        bbx_readout(self.handle, what, var, region, out)
        return out


# ---------------------------------------------------------------- surrogate network
def _dptr(t):
    """Device address of a contiguous torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return C.c_void_p(t)
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def bbx_mlp_create(nin, nout, seed, hip_stream=None):
    out = C.c_void_p()
    _check(_lib.bbx_mlp_create(int(nin), int(nout), int(seed) & (2 ** 64 - 1),
                               _stream_handle(hip_stream), C.byref(out)))
    return out


def bbx_mlp_params(m, set_, host):
    host = np.ascontiguousarray(host, dtype=np.float32) if set_ else host
    _check(_lib.bbx_mlp_params(m, int(set_), _ptr(host), host.size))
    return host


def bbx_mlp_norm(m, set_, host):
    _check(_lib.bbx_mlp_norm(m, int(set_), _ptr(host)))
    return host


def bbx_mlp_fit_norm(m, S, S1, n, stats=None):
    _check(_lib.bbx_mlp_fit_norm(m, _dptr(S), _dptr(S1), int(n), _ptr(stats)))
    return stats


def bbx_mlp_forward(m, X, n, Y):
    _check(_lib.bbx_mlp_forward(m, _dptr(X), int(n), _dptr(Y)))


def bbx_mlp_grad(m, X, T, n, grad_host=None):
    loss = np.zeros(1, np.float64)
    _check(_lib.bbx_mlp_grad(m, _dptr(X), _dptr(T), int(n), _ptr(grad_host), _ptr(loss)))
    return loss[0]


def bbx_mlp_grad_static(m, X, T, n, grad_dev=None, loss_dev=None):
    """Allocation-free gradient: X, T device inputs; grad_dev / loss_dev device outputs
    (torch tensors or addresses, may be None).  Stream-ordered, no synchronisation."""
    _check(_lib.bbx_mlp_grad_static(m, _dptr(X), _dptr(T), int(n), _dptr(grad_dev), _dptr(loss_dev)))


def bbx_mlp_adam(m, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_lib.bbx_mlp_adam(m, float(lr), float(beta1), float(beta2), float(eps)))


def bbx_mlp_train(m, S, S1, n, batch, iters, lr, seed, loss_hist=None):
    _check(_lib.bbx_mlp_train(m, _dptr(S), _dptr(S1), int(n), int(batch), int(iters), float(lr),
                              int(seed) & (2 ** 64 - 1), _ptr(loss_hist)))
    return loss_hist


def bbx_mlp_anchor(m, s0, s1):
    _check(_lib.bbx_mlp_anchor(m, _dptr(s0), _dptr(s1)))


def bbx_mlp_destroy(m):
    _lib.bbx_mlp_destroy(m)


def bbx_sample_states(g, n, seed, out):
    _check(_lib.bbx_sample_states(g, int(n), int(seed) & (2 ** 64 - 1), _dptr(out)))


def bbx_ionic_map(g, inp, n, out):
    _check(_lib.bbx_ionic_map(g, _dptr(inp), int(n), _dptr(out)))


def bbx_surrogate_set(g, m, lo=None, hi=None, dv_max=0.0):
    """Attach network m (None detaches)."""
    if m is None:
        _check(_lib.bbx_surrogate_set(g, None, None, None, 0.0))
        return
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    _check(_lib.bbx_surrogate_set(g, m, _ptr(lo), _ptr(hi), float(dv_max)))


class Mlp:
    """Owning wrapper of a surrogate network nin -> 128 -> 128 -> nout."""

    def __init__(self, nin, nout, seed=0, stream=None):
        self.nin, self.nout = nin, nout
        self.handle = bbx_mlp_create(nin, nout, seed, stream)

    def close(self):
        if self.handle is not None:
            bbx_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nparams(self):
        return 128 * self.nin + 128 + 128 * 128 + 128 + self.nout * 128 + self.nout

    def get_params(self):
        return bbx_mlp_params(self.handle, 0, np.empty(self.nparams, np.float32))

    def set_params(self, p):
        bbx_mlp_params(self.handle, 1, p)

    def get_norm(self):
        return bbx_mlp_norm(self.handle, 0, np.empty((4, 32), np.float32))

    def set_norm(self, norm):
        bbx_mlp_norm(self.handle, 1, np.ascontiguousarray(norm, dtype=np.float32))

    def fit_norm(self, S, S1):
        stats = np.zeros((7, 32), np.float64)
        return bbx_mlp_fit_norm(self.handle, S, S1, S.shape[0], stats)

    def forward(self, X, Y):
        bbx_mlp_forward(self.handle, X, X.shape[0], Y)

    def grad(self, X, T, with_host=True):
        gh = np.empty(self.nparams, np.float32) if with_host else None
        loss = bbx_mlp_grad(self.handle, X, T, X.shape[0], gh)
        return loss, gh

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        bbx_mlp_adam(self.handle, lr, beta1, beta2, eps)

    def anchor(self, s0, s1):
        bbx_mlp_anchor(self.handle, s0, s1)

    def train(self, S, S1, batch, iters, lr, seed=0):
        hist = np.empty(iters, np.float32)
        bbx_mlp_train(self.handle, S, S1, S.shape[0], batch, iters, lr, seed, hist)
        return hist


# ---------------------------------------------------------------- batched ensemble
def bbx_ensemble_create(nx, ny, h, Dpar, Dperp, angle, model, params, dt, precision,
                        hip_stream=None):
    """params: (ntissue, nparams) array (nparams = the model's count; may be 0 columns)."""
    nx = np.ascontiguousarray(nx, dtype=np.int32)
    ny = np.ascontiguousarray(ny, dtype=np.int32)
    n = nx.size
    if ny.size != n:
        raise ValueError("nx and ny differ in length")
    Dp = np.ascontiguousarray(np.broadcast_to(np.asarray(Dpar, np.float64), (n,)))
    Dq = np.ascontiguousarray(np.broadcast_to(np.asarray(Dperp, np.float64), (n,)))
    an = np.ascontiguousarray(np.broadcast_to(np.asarray(angle, np.float64), (n,)))
    P = np.ascontiguousarray(np.asarray(params, np.float64).reshape(n, -1))
    out = C.c_void_p()
    _check(_lib.bbx_ensemble_create(n, _ptr(nx), _ptr(ny), float(h), _ptr(Dp), _ptr(Dq), _ptr(an),
                                    int(model), _ptr(P) if P.size else None, P.shape[1], float(dt),
                                    int(precision), _stream_handle(hip_stream), C.byref(out)))
    return out


def bbx_ensemble_state_set(e, tissue, var, values):
    v = np.ascontiguousarray(values, dtype=np.float64)
    _check(_lib.bbx_ensemble_state_set(e, int(tissue), int(var), _ptr(v)))


def bbx_ensemble_stimulus_add(e, tissue, x0, x1, y0, y1, amplitude, t_start, duration,
                              period=0.0, count=1):
    _check(_lib.bbx_ensemble_stimulus_add(e, int(tissue), int(x0), int(x1), int(y0), int(y1),
                                          float(amplitude), float(t_start), float(duration),
                                          float(period), int(count)))


def bbx_ensemble_recording_set(e, theta):
    _check(_lib.bbx_ensemble_recording_set(e, float(theta)))


def bbx_ensemble_graph_set(e, chunk):
    _check(_lib.bbx_ensemble_graph_set(e, int(chunk)))


def bbx_ensemble_variant_set(e, variant):
    _check(_lib.bbx_ensemble_variant_set(e, int(variant)))


def bbx_ensemble_tune(e, steps):
    best = C.c_int()
    times = np.zeros(BBX_ENS_NVARIANT, np.float64)
    _check(_lib.bbx_ensemble_tune(e, int(steps), C.byref(best), _ptr(times)))
    return best.value, times


def bbx_ensemble_step(e, nsteps):
    _check(_lib.bbx_ensemble_step(e, int(nsteps)))


def bbx_ensemble_readout(e, what, tissue, var, out):
    _check(_lib.bbx_ensemble_readout(e, int(what), int(tissue), int(var), _ptr(out), out.size))
    return out


def bbx_ensemble_info(e, what) -> int:
    v = C.c_int64()
    _check(_lib.bbx_ensemble_info(e, int(what), C.byref(v)))
    return v.value


def bbx_ensemble_destroy(e):
    _lib.bbx_ensemble_destroy(e)


class Ensemble:
    """Owning wrapper of a batched ensemble of 2D rectangular tissues."""

    def __init__(self, nx, ny, h, Dpar, Dperp, angle, model, params, dt, precision=BBX_FP32,
                 stream=None):
        self.nx = np.asarray(nx, np.int32).copy()
        self.ny = np.asarray(ny, np.int32).copy()
        self.handle = bbx_ensemble_create(self.nx, self.ny, h, Dpar, Dperp, angle, model, params,
                                          dt, precision, stream)
        self.nvar = bbx_ensemble_info(self.handle, BBX_ENS_INFO_NVAR)
        self.nvox = bbx_ensemble_info(self.handle, BBX_ENS_INFO_VOXELS)

    def close(self):
        if self.handle:
            bbx_ensemble_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, tissue, var, values):
        bbx_ensemble_state_set(self.handle, tissue, var, values)

    def stimulus(self, tissue, x0, x1, y0, y1, amp, t0, dur, period=0.0, count=1):
        bbx_ensemble_stimulus_add(self.handle, tissue, x0, x1, y0, y1, amp, t0, dur, period, count)

    def record(self, theta):
        bbx_ensemble_recording_set(self.handle, theta)

    def graph(self, chunk):
        bbx_ensemble_graph_set(self.handle, chunk)

    def variant(self, v=None):
        if v is not None:
            bbx_ensemble_variant_set(self.handle, v)
        return bbx_ensemble_info(self.handle, BBX_ENS_INFO_VARIANT)

    def tune(self, steps=20):
        return bbx_ensemble_tune(self.handle, steps)

    def step(self, n=1):
        bbx_ensemble_step(self.handle, n)

    def get(self, tissue, var=0):
        """State variable `var` of tissue `tissue` as float64 (ny, nx)."""
        out = np.empty(int(self.nx[tissue]) * int(self.ny[tissue]), np.float64)
        bbx_ensemble_readout(self.handle, BBX_READ_VAR, tissue, var, out)
        return out.reshape(int(self.ny[tissue]), int(self.nx[tissue]))

    def read(self, what, tissue):
        if what == BBX_READ_STEP:
            out = np.empty(1, np.int64)
        elif what == BBX_READ_NAN_FLAG:
            out = np.empty(1, np.int32)
        elif what == BBX_READ_STATUS:
            out = np.empty(int(self.nx[tissue]) * int(self.ny[tissue]), np.uint8)
        else:
            out = np.empty(int(self.nx[tissue]) * int(self.ny[tissue]), np.float64)
        bbx_ensemble_readout(self.handle, what, tissue, 0, out)
        if out.size > 1:
            return out.reshape(int(self.ny[tissue]), int(self.nx[tissue]))
        return out
