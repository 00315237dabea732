"""Python binding of the swept2d HIP library (gfx950).

Argument marshalling only: every step of the stencil path runs in the HIP
kernels of ``libswept2d.so`` (built in place by ``build.py``). There is no
CPU fallback: importing works without a GPU, but every call that needs the
library raises if it is not built, and every call that needs a device fails
with the library's own error.

The functions carry the names of the C ABI in ``include/swept2d.h``;
``Swept2D`` wraps a handle for convenience and can bind a torch CUDA tensor as
the state (torch is used for device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

LIB_PATH = _build.LIB

OK = 0
EINVAL = -1
EHIP = -2
ENOMEM = -3
EUNSUPPORTED = -4
EABORTED = -5

HEAT5 = 1
WAVE_LF = 2
EULER_RUS_RK2 = 3
EULER_FD_RK4 = 4
TEST_HASH = 100
TEST_INCR = 101
TEST_PUSH5 = 102
TEST_HASH25 = 103
USER_PDE_BASE = 1000
SCHEME_ABI = 1

FP64 = 0
FP32C = 1
FP32R = 2

LAUNCH_DIRECT = 0
LAUNCH_GRAPH = 1

STAGING_AUTO = 0
STAGING_OFF = 1
STAGING_SINGLE_BRIDGES = 2
STAGING_ON = 3

TUNE_MODEL = 0
TUNE_MEASURE = 1

BATCH_PHASED = 0
BATCH_PERSISTENT = 1

KIND_NAMES = {0: "plain", 1: "up", 2: "bridge", 3: "oct"}

EXPORTS = [
    "swept2d_create", "swept2d_destroy", "swept2d_set_params", "swept2d_set_precision",
    "swept2d_set_tile", "swept2d_get_tile", "swept2d_set_rect", "swept2d_get_rect", "swept2d_bind",
    "swept2d_state_bytes",
    "swept2d_upload", "swept2d_download", "swept2d_upload_raw", "swept2d_download_raw",
    "swept2d_advance", "swept2d_plain_advance", "swept2d_synchronize",
    "swept2d_substep_counter", "swept2d_set_substep_counter", "swept2d_set_launch_mode",
    "swept2d_set_staging",
    "swept2d_set_timing", "swept2d_get_timing", "swept2d_last_error",
    "swept2d_batch_create", "swept2d_batch_destroy", "swept2d_batch_count", "swept2d_batch_set_tile",
    "swept2d_batch_get_tile", "swept2d_batch_set_rect", "swept2d_batch_get_rect", "swept2d_batch_autotune",
    "swept2d_batch_upload", "swept2d_batch_download",
    "swept2d_batch_advance", "swept2d_batch_synchronize", "swept2d_batch_substep_counter",
    "swept2d_batch_set_wait_limit", "swept2d_batch_set_mode", "swept2d_batch_get_mode",
    "swept2d_batch_launches", "swept2d_advance_noalloc", "swept2d_register_scheme", "swept2d_init_state",
    "swept3d_create", "swept3d_destroy", "swept3d_set_params", "swept3d_set_tile", "swept3d_get_tile",
    "swept3d_upload", "swept3d_download", "swept3d_advance", "swept3d_plain_advance", "swept3d_synchronize",
    "swept3d_get_step", "swept3d_set_step",
]

_lib = None


class Swept2DError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swept2d error {code}: {msg}")
        self.code = code


def load_library():
    """Load libswept2d.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1602_07558_amd/build.py "
                           "(or __graft_entry__.build())")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname as the system one); loading torch first makes the dynamic loader
    # bind this library to torch's copy, so torch streams and allocations
    # handed to the library belong to the runtime that executes its kernels.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, ll, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double
    sig = {
        "swept2d_create": (vp, [i, i, i, i, i]),
        "swept2d_destroy": (None, [vp]),
        "swept2d_set_params": (i, [vp, ctypes.POINTER(d), i]),
        "swept2d_set_precision": (i, [vp, i]),
        "swept2d_set_tile": (i, [vp, i]),
        "swept2d_get_tile": (i, [vp]),
        "swept2d_set_rect": (i, [vp, i]),
        "swept2d_get_rect": (i, [vp]),
        "swept2d_bind": (i, [vp, vp, vp]),
        "swept2d_state_bytes": (ctypes.c_size_t, [vp]),
        "swept2d_upload": (i, [vp, vp]),
        "swept2d_download": (i, [vp, vp]),
        "swept2d_upload_raw": (i, [vp, vp]),
        "swept2d_download_raw": (i, [vp, vp]),
        "swept2d_advance": (i, [vp, ll]),
        "swept2d_plain_advance": (i, [vp, ll]),
        "swept2d_synchronize": (i, [vp]),
        "swept2d_substep_counter": (ll, [vp]),
        "swept2d_set_substep_counter": (i, [vp, ll]),
        "swept2d_set_launch_mode": (i, [vp, i]),
        "swept2d_set_staging": (i, [vp, i]),
        "swept2d_set_timing": (i, [vp, i]),
        "swept2d_get_timing": (i, [vp, ctypes.POINTER(d), i]),
        "swept2d_last_error": (ctypes.c_char_p, []),
        "swept2d_batch_create": (vp, [i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                      ctypes.POINTER(i), ctypes.POINTER(d), i]),
        "swept2d_batch_destroy": (None, [vp]),
        "swept2d_batch_count": (i, [vp]),
        "swept2d_batch_set_tile": (i, [vp, i, i]),
        "swept2d_batch_get_tile": (i, [vp, i]),
        "swept2d_batch_set_rect": (i, [vp, i, i]),
        "swept2d_batch_get_rect": (i, [vp, i]),
        "swept2d_batch_autotune": (i, [vp, i]),
        "swept2d_batch_upload": (i, [vp, i, vp]),
        "swept2d_batch_download": (i, [vp, i, vp]),
        "swept2d_batch_advance": (i, [vp, ll]),
        "swept2d_batch_synchronize": (i, [vp]),
        "swept2d_batch_substep_counter": (ll, [vp, i]),
        "swept2d_batch_set_wait_limit": (i, [vp, ll]),
        "swept2d_batch_set_mode": (i, [vp, i]),
        "swept2d_batch_get_mode": (i, [vp]),
        "swept2d_batch_launches": (i, [vp, ll]),
        "swept2d_advance_noalloc": (i, [i, i, i, i, i, i, ctypes.POINTER(d), i, i, vp, ll, ll, vp]),
        "swept2d_register_scheme": (i, [vp]),
        "swept2d_init_state": (i, [vp]),
        "swept3d_create": (vp, [i, i, i, i]),
        "swept3d_destroy": (None, [vp]),
        "swept3d_set_params": (i, [vp, ctypes.POINTER(d), i]),
        "swept3d_set_tile": (i, [vp, i]),
        "swept3d_get_tile": (i, [vp]),
        "swept3d_upload": (i, [vp, vp]),
        "swept3d_download": (i, [vp, vp]),
        "swept3d_advance": (i, [vp, ll]),
        "swept3d_plain_advance": (i, [vp, ll]),
        "swept3d_synchronize": (i, [vp]),
        "swept3d_get_step": (ll, [vp]),
        "swept3d_set_step": (i, [vp, ll]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def swept2d_last_error() -> str:
    return load_library().swept2d_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise Swept2DError(rc, swept2d_last_error())
    return rc


def swept2d_create(nx: int, ny: int, nvars: int, pde: int, substeps: int) -> int:
    h = load_library().swept2d_create(nx, ny, nvars, pde, substeps)
    if not h:
        raise Swept2DError(EINVAL, swept2d_last_error())
    return h


def swept2d_destroy(h: int) -> None:
    load_library().swept2d_destroy(h)


def swept2d_set_params(h: int, params) -> int:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    return _check(load_library().swept2d_set_params(
        h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(p.size)))


def swept2d_set_precision(h: int, prec: int) -> int:
    return _check(load_library().swept2d_set_precision(h, prec))


def swept2d_set_tile(h: int, n: int) -> int:
    return _check(load_library().swept2d_set_tile(h, n))


def swept2d_get_tile(h: int) -> int:
    return _check(load_library().swept2d_get_tile(h))


def swept2d_set_rect(h: int, hh: int) -> int:
    return _check(load_library().swept2d_set_rect(h, hh))


def swept2d_get_rect(h: int) -> int:
    return _check(load_library().swept2d_get_rect(h))


# swept2d_bind's selector of the HIP null stream (stream handle 0, torch's
# default stream); None selects the library's own stream.
NULL_STREAM = ctypes.c_size_t(-1).value


def swept2d_bind(h: int, dev_ptr: int | None, stream: int | None) -> int:
    return _check(load_library().swept2d_bind(h, dev_ptr or None, stream or None))


def swept2d_state_bytes(h: int) -> int:
    return int(load_library().swept2d_state_bytes(h))


def swept2d_upload(h: int, host: np.ndarray) -> int:
    a = np.ascontiguousarray(host, dtype=np.float64)
    return _check(load_library().swept2d_upload(h, a.ctypes.data))


def swept2d_download(h: int, host: np.ndarray) -> int:
    assert host.dtype == np.float64 and host.flags.c_contiguous
    return _check(load_library().swept2d_download(h, host.ctypes.data))


def swept2d_upload_raw(h: int, host: np.ndarray) -> int:
    a = np.ascontiguousarray(host)
    if a.nbytes != swept2d_state_bytes(h):
        raise ValueError("raw state has the wrong size")
    return _check(load_library().swept2d_upload_raw(h, a.ctypes.data))


def swept2d_download_raw(h: int, host: np.ndarray) -> int:
    assert host.flags.c_contiguous and host.nbytes == swept2d_state_bytes(h)
    return _check(load_library().swept2d_download_raw(h, host.ctypes.data))


def swept2d_advance(h: int, nsteps: int) -> int:
    return _check(load_library().swept2d_advance(h, nsteps))


def swept2d_plain_advance(h: int, nsteps: int) -> int:
    return _check(load_library().swept2d_plain_advance(h, nsteps))


def swept2d_synchronize(h: int) -> int:
    return _check(load_library().swept2d_synchronize(h))


def swept2d_substep_counter(h: int) -> int:
    return _check(load_library().swept2d_substep_counter(h))


def swept2d_set_substep_counter(h: int, T: int) -> int:
    return _check(load_library().swept2d_set_substep_counter(h, T))


def swept2d_set_launch_mode(h: int, mode: int) -> int:
    return _check(load_library().swept2d_set_launch_mode(h, mode))


def swept2d_set_staging(h: int, mode: int) -> int:
    return _check(load_library().swept2d_set_staging(h, mode))


def swept2d_set_timing(h: int, on: bool) -> int:
    return _check(load_library().swept2d_set_timing(h, 1 if on else 0))


def swept2d_get_timing(h: int) -> list[dict]:
    buf = (ctypes.c_double * 16)()
    k = _check(load_library().swept2d_get_timing(h, buf, 4))
    out = []
    for r in range(k):
        kind = int(buf[4 * r])
        out.append({"kind": KIND_NAMES.get(kind, str(kind)), "launches": int(buf[4 * r + 1]),
                    "ms": float(buf[4 * r + 2]), "points": float(buf[4 * r + 3])})
    return out


def _ivec(v):
    a = (ctypes.c_int * len(v))(*[int(x) for x in v])
    return a


def swept2d_batch_create(nx, ny, pde, prec, params=None, params_stride: int = 0) -> int:
    count = len(nx)
    if not (len(ny) == len(pde) == len(prec) == count):
        raise ValueError("nx, ny, pde, prec must have one entry per grid")
    p = None
    if params is not None:
        flat = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
        p = flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    b = load_library().swept2d_batch_create(count, _ivec(nx), _ivec(ny), _ivec(pde), _ivec(prec), p,
                                            params_stride)
    if not b:
        raise Swept2DError(EINVAL, swept2d_last_error())
    return b


def swept2d_batch_destroy(b: int) -> None:
    load_library().swept2d_batch_destroy(b)


def swept2d_batch_count(b: int) -> int:
    return _check(load_library().swept2d_batch_count(b))


def swept2d_batch_set_tile(b: int, idx: int, n: int) -> int:
    return _check(load_library().swept2d_batch_set_tile(b, idx, n))


def swept2d_batch_get_tile(b: int, idx: int) -> int:
    return _check(load_library().swept2d_batch_get_tile(b, idx))


def swept2d_batch_set_rect(b: int, idx: int, hh: int) -> int:
    return _check(load_library().swept2d_batch_set_rect(b, idx, hh))


def swept2d_batch_get_rect(b: int, idx: int) -> int:
    return _check(load_library().swept2d_batch_get_rect(b, idx))


def swept2d_batch_autotune(b: int, mode: int) -> int:
    return _check(load_library().swept2d_batch_autotune(b, mode))


def swept2d_batch_upload(b: int, idx: int, host: np.ndarray) -> int:
    a = np.ascontiguousarray(host, dtype=np.float64)
    return _check(load_library().swept2d_batch_upload(b, idx, a.ctypes.data))


def swept2d_batch_download(b: int, idx: int, host: np.ndarray) -> int:
    assert host.dtype == np.float64 and host.flags["C_CONTIGUOUS"]
    return _check(load_library().swept2d_batch_download(b, idx, host.ctypes.data))


def swept2d_batch_advance(b: int, nsteps: int) -> int:
    return _check(load_library().swept2d_batch_advance(b, nsteps))


def swept2d_batch_synchronize(b: int) -> int:
    return _check(load_library().swept2d_batch_synchronize(b))


def swept2d_batch_substep_counter(b: int, idx: int) -> int:
    return _check(load_library().swept2d_batch_substep_counter(b, idx))


def swept2d_batch_set_wait_limit(b: int, microseconds: int) -> int:
    return _check(load_library().swept2d_batch_set_wait_limit(b, microseconds))


def swept2d_batch_set_mode(b: int, mode: int) -> int:
    return _check(load_library().swept2d_batch_set_mode(b, mode))


def swept2d_batch_get_mode(b: int) -> int:
    return _check(load_library().swept2d_batch_get_mode(b))


def swept2d_batch_launches(b: int, nsteps: int) -> int:
    return _check(load_library().swept2d_batch_launches(b, nsteps))


PDE_SHAPE = {HEAT5: (1, 1), WAVE_LF: (2, 1), EULER_RUS_RK2: (8, 2), EULER_FD_RK4: (12, 4), TEST_HASH: (1, 1),
             TEST_INCR: (1, 1), TEST_PUSH5: (5, 2), TEST_HASH25: (9, 2)}


class SchemeOps(ctypes.Structure):
    """The C swept2d_scheme_ops table (launchers as opaque pointers)."""
    _fields_ = [("abi", ctypes.c_int), ("nvars", ctypes.c_int), ("substeps", ctypes.c_int),
                ("nparams", ctypes.c_int), ("nv", ctypes.c_int), ("nw", ctypes.c_int), ("vbytes", ctypes.c_int)] + \
               [(n, ctypes.c_void_p) for n in ("up", "bridge", "oct", "plain", "lds", "fetch_ahead", "init")]


def swept2d_register_scheme(ops_ptr: int) -> int:
    """Register a user scheme from the address of its swept2d_scheme_ops
    table; returns its pde id."""
    return _check(load_library().swept2d_register_scheme(ops_ptr))


def swept2d_init_state(h: int) -> int:
    return _check(load_library().swept2d_init_state(h))


NOALLOC_SCRATCH_BYTES = 64 << 20


def swept2d_advance_noalloc(nx: int, ny: int, pde: int, prec: int, params, tile: int, dev_ptr: int, T: int,
                            nsteps: int, stream: int | None = None) -> int:
    """The swept advance without allocation (panels in the library's static
    device array) of a caller device state; `stream` a HIP stream handle,
    None or 0 for the null stream."""
    nvars, sub = PDE_SHAPE[pde]
    p = np.ascontiguousarray(np.asarray(params if params is not None else [], dtype=np.float64))
    pp = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if p.size else None
    return _check(load_library().swept2d_advance_noalloc(nx, ny, nvars, pde, sub, prec, pp, int(p.size), tile,
                                                         dev_ptr, T, nsteps, stream or NULL_STREAM))


# --------------------------------------------------------------------- 3D
HEAT7_3D = 1
TEST_HASH27_3D = 100


def swept3d_create(nx: int, ny: int, nz: int, pde: int):
    h = load_library().swept3d_create(nx, ny, nz, pde)
    if not h:
        raise Swept2DError(EINVAL, swept2d_last_error())
    return h


def swept3d_destroy(h) -> None:
    load_library().swept3d_destroy(h)


def swept3d_set_params(h, params) -> int:
    arr = (ctypes.c_double * len(params))(*[float(x) for x in params])
    return _check(load_library().swept3d_set_params(h, arr, len(params)))


def swept3d_set_tile(h, n: int) -> int:
    return _check(load_library().swept3d_set_tile(h, n))


def swept3d_get_tile(h) -> int:
    return _check(load_library().swept3d_get_tile(h))


def swept3d_upload(h, host_ptr: int) -> int:
    return _check(load_library().swept3d_upload(h, host_ptr))


def swept3d_download(h, host_ptr: int) -> int:
    return _check(load_library().swept3d_download(h, host_ptr))


def swept3d_advance(h, nsteps: int) -> int:
    return _check(load_library().swept3d_advance(h, nsteps))


def swept3d_plain_advance(h, nsteps: int) -> int:
    return _check(load_library().swept3d_plain_advance(h, nsteps))


def swept3d_synchronize(h) -> int:
    return _check(load_library().swept3d_synchronize(h))


def swept3d_get_step(h) -> int:
    return _check(load_library().swept3d_get_step(h))


def swept3d_set_step(h, T: int) -> int:
    return _check(load_library().swept3d_set_step(h, T))


class Swept3D:
    """Owner of one swept3d handle (state [nz][ny][nx] float64)."""

    def __init__(self, nx: int, ny: int, nz: int, pde: int, params=None, tile: int = 0):
        self.nx, self.ny, self.nz, self.pde = nx, ny, nz, pde
        self.h = swept3d_create(nx, ny, nz, pde)
        try:
            if params is not None and len(params):
                swept3d_set_params(self.h, params)
            if tile:
                swept3d_set_tile(self.h, tile)
        except Exception:
            self.close()
            raise

    def close(self):
        if getattr(self, "h", None):
            swept3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def tile(self) -> int:
        return swept3d_get_tile(self.h)

    @tile.setter
    def tile(self, n: int):
        swept3d_set_tile(self.h, n)

    @property
    def T(self) -> int:
        return swept3d_get_step(self.h)

    @T.setter
    def T(self, value: int):
        swept3d_set_step(self.h, value)

    def upload(self, state):
        import numpy as np
        a = np.ascontiguousarray(state, dtype=np.float64)
        if a.shape != (self.nz, self.ny, self.nx):
            raise ValueError(f"state must be ({self.nz}, {self.ny}, {self.nx})")
        swept3d_upload(self.h, a.ctypes.data)

    def download(self):
        import numpy as np
        a = np.empty((self.nz, self.ny, self.nx), dtype=np.float64)
        swept3d_download(self.h, a.ctypes.data)
        return a

    def advance(self, nsteps: int):
        swept3d_advance(self.h, nsteps)

    def plain_advance(self, nsteps: int):
        swept3d_plain_advance(self.h, nsteps)

    def synchronize(self):
        swept3d_synchronize(self.h)


class Swept2D:
    """Owner of one swept2d handle."""

    def __init__(self, nx: int, ny: int, pde: int, params=None, prec: int = FP64, tile: int = 0, shape=None):
        nvars, sub = shape if shape is not None else PDE_SHAPE[pde]
        self.nx, self.ny, self.pde, self.nvars, self.substeps = nx, ny, pde, nvars, sub
        self.h = swept2d_create(nx, ny, nvars, pde, sub)
        try:
            if params is not None and len(params):
                swept2d_set_params(self.h, params)
            if prec != FP64:
                swept2d_set_precision(self.h, prec)
            if tile:
                swept2d_set_tile(self.h, tile)
        except Exception:
            self.close()
            raise
        self.prec = prec

    def close(self):
        if getattr(self, "h", None):
            swept2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def tile(self) -> int:
        return swept2d_get_tile(self.h)

    @tile.setter
    def tile(self, n: int):
        swept2d_set_tile(self.h, n)

    @property
    def rect(self) -> int:
        """Half-cycle height of the rectangular tiles in use (0: square tiles)."""
        return swept2d_get_rect(self.h)

    @rect.setter
    def rect(self, hh: int):
        swept2d_set_rect(self.h, hh)

    def upload(self, state: np.ndarray):
        assert state.shape == (self.nvars, self.ny, self.nx)
        swept2d_upload(self.h, state)

    def download(self) -> np.ndarray:
        out = np.empty((self.nvars, self.ny, self.nx), dtype=np.float64)
        swept2d_download(self.h, out)
        return out

    def raw_shape(self):
        if self.prec == FP64:
            return (self.nvars, self.ny, self.nx), np.float64
        if self.prec == FP32R:
            return (self.nvars, self.ny, self.nx), np.float32
        return (2 * self.nvars, self.ny, self.nx), np.float32

    def upload_raw(self, a: np.ndarray):
        swept2d_upload_raw(self.h, a)

    def download_raw(self) -> np.ndarray:
        shape, dt = self.raw_shape()
        out = np.empty(shape, dtype=dt)
        swept2d_download_raw(self.h, out)
        return out

    def bind_tensor(self, t, stream=None):
        """Use a torch CUDA tensor as the state, and a torch stream (default:
        torch's current stream; its default stream is the HIP null stream,
        handle 0) for every launch."""
        import torch
        shape, dt = self.raw_shape()
        tdt = torch.float64 if dt == np.float64 else torch.float32
        if tuple(t.shape) != shape or t.dtype != tdt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"state tensor must be a contiguous CUDA {tdt} tensor of shape {shape}")
        s = stream if stream is not None else torch.cuda.current_stream(t.device)
        swept2d_bind(self.h, t.data_ptr(), s.cuda_stream if s.cuda_stream else NULL_STREAM)
        self._bound = t

    def unbind(self):
        swept2d_bind(self.h, None, None)
        self._bound = None

    def init_state(self):
        """Set the state with the scheme's device Init (user schemes)."""
        swept2d_init_state(self.h)

    def advance(self, nsteps: int):
        swept2d_advance(self.h, nsteps)

    def plain_advance(self, nsteps: int):
        swept2d_plain_advance(self.h, nsteps)

    def synchronize(self):
        swept2d_synchronize(self.h)

    @property
    def T(self) -> int:
        return swept2d_substep_counter(self.h)

    @T.setter
    def T(self, v: int):
        swept2d_set_substep_counter(self.h, v)

    def set_launch_mode(self, mode: int):
        swept2d_set_launch_mode(self.h, mode)

    def set_staging(self, mode: int):
        swept2d_set_staging(self.h, mode)

    def set_timing(self, on: bool):
        swept2d_set_timing(self.h, on)

    def timing(self) -> list[dict]:
        return swept2d_get_timing(self.h)


class Swept2DBatch:
    """Owner of one swept2d batch handle. `grids` is a list of dicts with
    keys nx, ny, pde and optionally prec (FP64) and params."""

    def __init__(self, grids):
        self.grids = [dict(g) for g in grids]
        nparams = max([len(g.get("params") or []) for g in self.grids] + [1])
        params = np.zeros((len(self.grids), nparams))
        for i, g in enumerate(self.grids):
            pv = list(g.get("params") or [])
            params[i, :len(pv)] = pv
        self.b = swept2d_batch_create([g["nx"] for g in self.grids], [g["ny"] for g in self.grids],
                                      [g["pde"] for g in self.grids], [g.get("prec", FP64) for g in self.grids],
                                      params, nparams)

    def close(self):
        if getattr(self, "b", None):
            swept2d_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __len__(self):
        return len(self.grids)

    def shape(self, i: int):
        g = self.grids[i]
        return (PDE_SHAPE[g["pde"]][0], g["ny"], g["nx"])

    def tile(self, i: int) -> int:
        return swept2d_batch_get_tile(self.b, i)

    def set_tile(self, i: int, n: int):
        swept2d_batch_set_tile(self.b, i, n)

    def rect(self, i: int) -> int:
        return swept2d_batch_get_rect(self.b, i)

    def set_rect(self, i: int, hh: int):
        swept2d_batch_set_rect(self.b, i, hh)

    def autotune(self, mode: int = TUNE_MODEL):
        swept2d_batch_autotune(self.b, mode)

    def upload(self, i: int, state: np.ndarray):
        assert state.shape == self.shape(i)
        swept2d_batch_upload(self.b, i, state)

    def download(self, i: int) -> np.ndarray:
        out = np.empty(self.shape(i), dtype=np.float64)
        swept2d_batch_download(self.b, i, out)
        return out

    def advance(self, nsteps: int):
        swept2d_batch_advance(self.b, nsteps)

    def synchronize(self):
        swept2d_batch_synchronize(self.b)

    def T(self, i: int) -> int:
        return swept2d_batch_substep_counter(self.b, i)

    def set_wait_limit(self, microseconds: int):
        swept2d_batch_set_wait_limit(self.b, microseconds)

    def set_mode(self, mode: int):
        swept2d_batch_set_mode(self.b, mode)

    @property
    def mode(self) -> int:
        return swept2d_batch_get_mode(self.b)

    def launches(self, nsteps: int) -> int:
        return swept2d_batch_launches(self.b, nsteps)
