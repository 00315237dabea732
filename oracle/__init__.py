"""Oracle for the swept-rule hot path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg use this package. The GPU library never imports, links or calls it, and
the two share no code; both start from the seeded fields of ``swept_inputs``.

* ``advance_f64`` / ``advance_f32c``: the plain FP64 (and FP32-compensated)
  step-by-step stepper written in C; ``advance_f32r`` the FP32 stepper whose
  compensation survives only within one residency of the swept schedule (``stepper.c``, built with
  ``-O2 -ffp-contract=off``). This is the definition that the swept rule
  reproduces exactly: no redundant computation, every point computed from its
  full 3x3 neighbourhood one level below (abstract; Sec. 4).
* ``swept_model``: the swept decomposition of Sec. 3-4 (the level function
  that assigns every point and level of a half cycle to an upward pyramid, a
  bridge or a downward pyramid) executed component by component on small
  grids in pure Python, with its dependency order checked; it pins the
  component sizes, the panels and the reading of the bridges' printed bound.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stepper.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle in place (gcc)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_advance_f64.restype = ctypes.c_int
        lib.oracle_advance_f64.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int,
        ]
        lib.oracle_advance_f32c.restype = ctypes.c_int
        lib.oracle_advance_f32c.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int,
        ]
        lib.oracle_advance_f32r.restype = ctypes.c_int
        lib.oracle_advance_f32r.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_longlong, ctypes.c_longlong, ctypes.c_int,
        ]
        lib.oracle_advance_hash25.restype = ctypes.c_int
        lib.oracle_advance_hash25.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong,
                                              ctypes.c_longlong, ctypes.c_int]
        lib.oracle_advance3d_f64.restype = ctypes.c_int
        lib.oracle_advance3d_f64.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong,
                                             ctypes.c_int]
        lib.oracle_residency.restype = ctypes.c_longlong
        lib.oracle_residency.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_longlong, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
        lib.oracle_point_wave_f32v.restype = None
        lib.oracle_point_wave_f32v.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_double]
        _lib = lib
    return _lib


def point_wave_f32v(nu, nc, c2: float):
    """One point of the FP32 wave's velocity form: nu, nc are [3][3][2]
    float32 neighbourhoods (rows north to south, slots u, v) of values and
    compensations; returns the new (u, v) and their compensations."""
    lib = _load()
    a = np.ascontiguousarray(nu, dtype=np.float32).reshape(18)
    b = np.ascontiguousarray(nc, dtype=np.float32).reshape(18)
    ou, oc = np.zeros(2, np.float32), np.zeros(2, np.float32)
    lib.oracle_point_wave_f32v(a.ctypes.data, b.ctypes.data, ou.ctypes.data, oc.ctypes.data, float(c2))
    return ou, oc


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def advance_f64(pde: int, state: np.ndarray, params, nsub: int, t0: int = 0, threads: int | None = None) -> np.ndarray:
    """Return the state after ``nsub`` sub-steps starting at global sub-step t0.

    ``state`` is ``[nvars][ny][nx]`` float64; it is not modified."""
    lib = _load()
    s = np.ascontiguousarray(state, dtype=np.float64).copy()
    nvars, ny, nx = s.shape
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    rc = lib.oracle_advance_f64(int(pde), nx, ny, nvars, p.ctypes.data if p.size else None, int(p.size),
                                s.ctypes.data, int(t0), int(nsub), int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle_advance_f64 failed with {rc}")
    return s


def advance3d_f64(pde: int, state: np.ndarray, params, nsub: int, t0: int = 0,
                  threads: int | None = None) -> np.ndarray:
    """3D: the state ``[nz][ny][nx]`` float64 after ``nsub`` sub-steps from
    global sub-step t0 (pde 1: 7-point heat, params {r}; 100: 27-point
    hash). ``state`` is not modified."""
    lib = _load()
    s = np.ascontiguousarray(state, dtype=np.float64).copy()
    nz, ny, nx = s.shape
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    rc = lib.oracle_advance3d_f64(int(pde), nx, ny, nz, p.ctypes.data if p.size else None, int(p.size),
                                  s.ctypes.data, int(t0), int(nsub), int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle_advance3d_f64 failed with {rc}")
    return s


def advance_f32c(pde: int, u: np.ndarray, c: np.ndarray, params, nsub: int, t0: int = 0,
                 threads: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """FP32-compensated stepper; ``u`` and ``c`` are ``[nvars][ny][nx]`` float32."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float32).copy()
    cc = np.ascontiguousarray(c, dtype=np.float32).copy()
    nvars, ny, nx = uu.shape
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    rc = lib.oracle_advance_f32c(int(pde), nx, ny, nvars, p.ctypes.data, int(p.size),
                                 uu.ctypes.data, cc.ctypes.data, int(t0), int(nsub),
                                 int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle_advance_f32c failed with {rc}")
    return uu, cc


def advance_f32r(pde: int, u: np.ndarray, params, nsub: int, tile: int, t0: int = 0,
                 threads: int | None = None) -> np.ndarray:
    """FP32 state whose compensation lives only within a residency of the
    swept schedule on tiles of side ``tile`` (0: the per-step method; -1: one
    residency for the whole advance, the compensation kept everywhere), as
    one advance of ``nsub`` sub-steps; ``u`` is ``[nvars][ny][nx]`` float32 in
    the form of ``split_f32r`` (the wave as displacement and velocity)."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float32).copy()
    nvars, ny, nx = uu.shape
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    rc = lib.oracle_advance_f32r(int(pde), nx, ny, nvars, p.ctypes.data, int(p.size), uu.ctypes.data, int(tile),
                                 int(t0), int(nsub), int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle_advance_f32r failed with {rc}")
    return uu


def advance_hash25(u: np.ndarray, nsteps: int, k0: int = 0, threads: int | None = None) -> np.ndarray:
    """The 25-point test hash (a stencil reaching two rings) applied directly
    nsteps times to the scalar field u ([ny][nx] float64), the first with step
    index k0."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    ny, nx = uu.shape
    rc = lib.oracle_advance_hash25(nx, ny, uu.ctypes.data, int(k0), int(nsteps), int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle_advance_hash25 failed with {rc}")
    return uu


def split_f32r(pde: int, state64: np.ndarray) -> np.ndarray:
    """FP32 values of the residency-confined form from an FP64 state: u =
    fl32(x); the wave keeps (u, v) with v = fl32(u^n - u^(n-1))."""
    u = state64.astype(np.float32)
    if pde == 2:  # wave, velocity form
        u[1] = (state64[0] - state64[1]).astype(np.float32)
    return u


def join_f32r(pde: int, u: np.ndarray) -> np.ndarray:
    """FP64 state from the residency-confined form (the wave's previous
    level as u - v)."""
    x = u.astype(np.float64)
    if pde == 2:
        x[1] = x[0] - x[1]
    return x


def residency(x: int, y: int, L: int, tile: int, nx: int, ny: int) -> int:
    """Residency number of point (x, y) at level L of a swept advance."""
    return int(_load().oracle_residency(x, y, L, tile, nx, ny))


def split_f32c(state64: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Initial FP32-compensated state from an FP64 field: u = fl32(x), c = 0."""
    u = state64.astype(np.float32)
    return u, np.zeros_like(u)
