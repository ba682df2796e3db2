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

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbbx.so")

BBX_OK, BBX_EINVAL, BBX_ENOMEM, BBX_EDEVICE, BBX_ESTATE, BBX_EUNSTABLE, BBX_ENUMERIC, BBX_ENOTSUP = \
    0, -1, -2, -3, -4, -5, -6, -7
BBX_FP32, BBX_FP64 = 0, 1
BBX_SCHEME_ADDITIVE, BBX_SCHEME_SPLIT = 0, 1
BBX_MODEL_NONE, BBX_MODEL_BARKLEY, BBX_MODEL_ZFK, BBX_MODEL_FHN, BBX_MODEL_CRN = 0, 1, 2, 3, 4
(BBX_READ_VAR, BBX_READ_ACT_TIME, BBX_READ_APD90, BBX_READ_VMAX, BBX_READ_STATUS,
 BBX_READ_REDUCE_MAX, BBX_READ_REDUCE_SUM, BBX_READ_NAN_FLAG, BBX_READ_STEP,
 BBX_READ_WEIGHTS) = range(10)
BBX_INFO_NACTIVE, BBX_INFO_NVAR, BBX_INFO_NBOX, BBX_INFO_DEVICE_BYTES = range(4)

# Every symbol the header declares, with (restype, argtypes).
_P, _I, _D, _I64, _SZ = C.c_void_p, C.c_int, C.c_double, C.c_int64, C.c_size_t
SIGNATURES = {
    "bbx_grid_create": (_I, [_I, _I, _I, _D, _P, _P, _D, _D, _I, _P, C.POINTER(_P)]),
    "bbx_model_set": (_I, [_P, _I, _P, _I, _D, _I]),
    "bbx_state_set": (_I, [_P, _I, _P]),
    "bbx_stimulus_add": (_I, [_P, _P, _D, _D, _D, _D, _I]),
    "bbx_stimulus_clear": (_I, [_P]),
    "bbx_recording_set": (_I, [_P, _D]),
    "bbx_nan_check_set": (_I, [_P, _I64]),
    "bbx_clock_set": (_I, [_P, _I64]),
    "bbx_step": (_I, [_P, _I64]),
    "bbx_readout": (_I, [_P, _I, _I, _P, _P, _SZ, _I]),
    "bbx_info": (_I, [_P, _I, C.POINTER(_I64)]),
    "bbx_grid_destroy": (None, [_P]),
    "bbx_last_error": (C.c_char_p, []),
}


class BBXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bbx error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libbbx.so not built ({path}); run __graft_entry__.build()")
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
        elif what == BBX_READ_STEP:
            out = np.empty(1, np.int64)
        elif what == BBX_READ_WEIGHTS:
            out = np.empty((self.nact, 27), np.float64)
        else:
            out = np.empty(self.shape, np.float64)
        bbx_readout(self.handle, what, var, region, out)
        return out
