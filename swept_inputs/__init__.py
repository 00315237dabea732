"""Seeded synthetic initial fields for the swept-rule stepper.

This module is shared by the tests, the benchmark and the smoke check. It
creates initial states only and holds none of the stepping arithmetic. All
fields are produced on the host in FP64 (numpy), so the GPU path and the CPU
oracle start from the same bits.

State layout everywhere: structure of arrays ``[nvars][ny][nx]``, x fastest,
row ``j = 0`` is the north edge (the paper's grid point ``(i, j)`` is
``state[:, j, i]``; the grid is doubly periodic, Sec. 2 assumption 1).

Workload recipes (the paper runs a wave and an Euler problem, Sec. 7-8;
the heat problem and the exact field recipes below are synthetic stand-ins
with the shapes of those workloads):

* heat: sum of 8 Fourier modes, integer wavenumbers kx, ky in 1..8,
  amplitude U(-1, 1), phase U(0, 2 pi).
* wave: 16 Gaussian pulses of amplitude 1 and width sigma = 20 cells at
  uniform random centres (minimum-image distance on the torus), zero
  initial velocity (previous level equal to the current one).
* euler: 4 isentropic vortices (strength beta = 5) on a uniform flow
  rho = 1, p = 1, (u, v) = (1, 1), on a periodic square of side 20, vortex
  centres drawn with minimum-image separation of at least a quarter side.
* euler_fd: the paper's wind-tunnel free stream (rho = 1.084, Mach 0.2 along
  x, v = 0, p = 101325, cells of 50/1024 on both axes) with a seeded
  isentropic pressure pulse of 1 % (Gaussian, width 16 cells) in place of
  the obstacle; slots 4..7 (the Runge-Kutta stage) start as a copy of the
  conserved variables, slots 8..11 at zero.
* hash: uniform random integers in [0, 2^52) stored exactly as doubles.
* incr: constant field (the paper's worked example starts at value 1).
* push5: random small integers in slot 0, zeros in slots 1..4.
* hash25: random integers in [0, 2^52) in slot 0, zeros in slots 1..8.
"""
from __future__ import annotations

import math

import numpy as np

HEAT5 = 1
WAVE_LF = 2
EULER_RUS_RK2 = 3
EULER_FD_RK4 = 4
TEST_HASH = 100
TEST_INCR = 101
TEST_PUSH5 = 102
TEST_HASH25 = 103

PDE_NAMES = {
    HEAT5: "heat5",
    WAVE_LF: "wave_lf",
    EULER_RUS_RK2: "euler_rus_rk2",
    EULER_FD_RK4: "euler_fd_rk4",
    TEST_HASH: "test_hash",
    TEST_INCR: "test_incr",
    TEST_PUSH5: "test_push5",
    TEST_HASH25: "test_hash25",
}

# (nvars, substeps) per pde; hash and incr are scalar single-step stencils.
PDE_SHAPE = {
    HEAT5: (1, 1),
    WAVE_LF: (2, 1),
    EULER_RUS_RK2: (8, 2),
    EULER_FD_RK4: (12, 4),
    TEST_HASH: (1, 1),
    TEST_INCR: (1, 1),
    TEST_PUSH5: (5, 2),
    TEST_HASH25: (9, 2),
}

HEAT_R = 0.2          # r = alpha dt / h^2
WAVE_C2 = 0.25        # (c dt / h)^2 for Courant number 0.5
EULER_GAMMA = 1.4
EULER_CFL = 0.4
EULER_SIDE = 20.0
EULER_BETA = 5.0
# The paper's Euler experiment (Sec. 8): a 50 x 25 tunnel on 1024 x 512
# cells, dt = 1e-6, free stream rho = 1.084, Mach 0.2, v = 0, p = 101325.
EULERFD_H = 50.0 / 1024.0
EULERFD_DT = 1e-6
EULERFD_RHO = 1.084
EULERFD_MACH = 0.2
EULERFD_P = 101325.0


def default_params(pde: int, state: np.ndarray | None = None) -> np.ndarray:
    """Physical parameters passed to both sides for a pde id."""
    if pde == HEAT5:
        return np.array([HEAT_R], dtype=np.float64)
    if pde == WAVE_LF:
        return np.array([WAVE_C2], dtype=np.float64)
    if pde == EULER_RUS_RK2:
        if state is None:
            raise ValueError("euler parameters need the initial state for dt")
        return np.array([EULER_GAMMA, euler_dt_over_h(state)], dtype=np.float64)
    if pde == EULER_FD_RK4:
        return np.array([EULER_GAMMA, EULERFD_DT / EULERFD_H], dtype=np.float64)
    return np.zeros(0, dtype=np.float64)


def heat_field(nx: int, ny: int, seed: int = 0, modes: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    kx = rng.integers(1, 9, size=modes)
    ky = rng.integers(1, 9, size=modes)
    amp = rng.uniform(-1.0, 1.0, size=modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=modes)
    i = np.arange(nx, dtype=np.float64)[None, :]
    j = np.arange(ny, dtype=np.float64)[:, None]
    u = np.zeros((ny, nx), dtype=np.float64)
    for m in range(modes):
        u += amp[m] * np.cos(2.0 * math.pi * (kx[m] * i / nx + ky[m] * j / ny) + phase[m])
    return u[None, :, :].copy()


def heat_single_mode(nx: int, ny: int, kx: int, ky: int, amp: float = 1.0) -> np.ndarray:
    i = np.arange(nx, dtype=np.float64)[None, :]
    j = np.arange(ny, dtype=np.float64)[:, None]
    u = amp * np.cos(2.0 * math.pi * (kx * i / nx + ky * j / ny))
    return u[None, :, :].copy()


def _min_image(d: np.ndarray, period: float) -> np.ndarray:
    return d - period * np.round(d / period)


def wave_field(nx: int, ny: int, seed: int = 0, pulses: int = 16, sigma: float = 20.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, nx, size=pulses)
    cy = rng.uniform(0.0, ny, size=pulses)
    i = np.arange(nx, dtype=np.float64)[None, :]
    j = np.arange(ny, dtype=np.float64)[:, None]
    u = np.zeros((ny, nx), dtype=np.float64)
    for m in range(pulses):
        dx = _min_image(i - cx[m], nx)
        dy = _min_image(j - cy[m], ny)
        u += np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
    return np.stack([u, u.copy()])


def euler_field(nx: int, ny: int, seed: int = 0, vortices: int = 4) -> np.ndarray:
    """Isentropic vortices on uniform flow; conserved variables in slots 0..3,
    slots 4..7 (the Runge-Kutta stage) start as a copy."""
    gamma = EULER_GAMMA
    side = EULER_SIDE
    beta = EULER_BETA
    rng = np.random.default_rng(seed)
    centres: list[tuple[float, float]] = []
    while len(centres) < vortices:
        c = (rng.uniform(0.0, side), rng.uniform(0.0, side))
        ok = True
        for q in centres:
            ddx = _min_image(np.array(c[0] - q[0]), side)
            ddy = _min_image(np.array(c[1] - q[1]), side)
            if math.hypot(float(ddx), float(ddy)) < side / 4.0:
                ok = False
                break
        if ok:
            centres.append(c)
    hx = side / nx
    hy = side / ny
    x = (np.arange(nx, dtype=np.float64)[None, :] + 0.5) * hx
    y = (np.arange(ny, dtype=np.float64)[:, None] + 0.5) * hy
    du = np.zeros((ny, nx))
    dv = np.zeros((ny, nx))
    dT = np.zeros((ny, nx))
    for (xc, yc) in centres:
        ddx = _min_image(x - xc, side)
        ddy = _min_image(y - yc, side)
        r2 = ddx * ddx + ddy * ddy
        e = np.exp(0.5 * (1.0 - r2))
        du += -beta / (2.0 * math.pi) * ddy * e
        dv += beta / (2.0 * math.pi) * ddx * e
        dT += -(gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi * math.pi) * np.exp(1.0 - r2)
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    u = 1.0 + du
    v = 1.0 + dv
    en = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    cons = np.stack([rho, rho * u, rho * v, en])
    return np.concatenate([cons, cons.copy()]).copy()


def eulerfd_conserved(rho, u, v, p, gamma: float = EULER_GAMMA) -> np.ndarray:
    """(rho, rho u, rho v, E) from primitive fields."""
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def eulerfd_state(cons: np.ndarray) -> np.ndarray:
    """The 12-slot state of the four-stage scheme from (rho, mx, my, E):
    the stage slots a copy, the derivative sum zero."""
    return np.concatenate([cons, cons.copy(), np.zeros_like(cons)]).copy()


def eulerfd_field(nx: int, ny: int, seed: int = 0, amp: float = 0.01, width: float = 16.0) -> np.ndarray:
    gamma = EULER_GAMMA
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(0.0, nx), rng.uniform(0.0, ny)
    i = np.arange(nx, dtype=np.float64)[None, :]
    j = np.arange(ny, dtype=np.float64)[:, None]
    dx = _min_image(i - cx, nx)
    dy = _min_image(j - cy, ny)
    c0 = math.sqrt(gamma * EULERFD_P / EULERFD_RHO)
    p = EULERFD_P * (1.0 + amp * np.exp(-(dx * dx + dy * dy) / (2.0 * width * width)))
    rho = EULERFD_RHO * (p / EULERFD_P) ** (1.0 / gamma)
    u = np.full((ny, nx), EULERFD_MACH * c0)
    v = np.zeros((ny, nx))
    return eulerfd_state(eulerfd_conserved(rho, u, v, p, gamma))


def euler_dt_over_h(state: np.ndarray, cfl: float = EULER_CFL, gamma: float = EULER_GAMMA) -> float:
    """Fixed time step from the initial field: dt = cfl / max((|u|+c)/h + (|v|+c)/h)
    on a square grid; returned as dt/h (the only combination the scheme uses)."""
    rho, mx, my, en = state[0], state[1], state[2], state[3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (en - 0.5 * (mx * mx + my * my) / rho)
    c = np.sqrt(gamma * p / rho)
    smax = float(np.max(np.abs(u) + c + np.abs(v) + c))
    return cfl / smax


def hash_field(nx: int, ny: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.integers(0, 1 << 52, size=(1, ny, nx), dtype=np.int64)
    return v.astype(np.float64)


def incr_field(nx: int, ny: int, value: float = 1.0) -> np.ndarray:
    return np.full((1, ny, nx), value, dtype=np.float64)


def push5_field(nx: int, ny: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    s = np.zeros((5, ny, nx), dtype=np.float64)
    s[0] = rng.integers(-8, 9, size=(ny, nx)).astype(np.float64)
    return s


def hash25_field(nx: int, ny: int, seed: int = 0) -> np.ndarray:
    """The two-ring test stencil's state: random integers below 2^52 in slot
    0 (the value), zeros in the 8 slots of pushed values."""
    s = np.zeros((9, ny, nx), dtype=np.float64)
    s[0] = hash_field(nx, ny, seed)[0]
    return s


# ------------------------------------------------------------------- 3D
# 3D schemes (their own ids): 7-point heat and the 27-point test hash.
HEAT7_3D = 1
TEST_HASH27_3D = 100
HEAT3D_R = 0.125


def heat3d_field(nx: int, ny: int, nz: int, seed: int = 0, modes: int = 8) -> np.ndarray:
    """Sum of seeded Fourier modes, k in U{1..4} per axis, on [nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, None, :] / nx
    y = np.arange(ny)[None, :, None] / ny
    z = np.arange(nz)[:, None, None] / nz
    u = np.zeros((nz, ny, nx))
    for _ in range(modes):
        kx, ky, kz = rng.integers(1, 5, 3)
        a, ph = rng.uniform(-1.0, 1.0), rng.uniform(0.0, 2.0 * math.pi)
        u += a * np.cos(2.0 * math.pi * (kx * x + ky * y + kz * z) + ph)
    return u


def hash3d_field(nx: int, ny: int, nz: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 52, size=(nz, ny, nx), dtype=np.int64).astype(np.float64)


def initial_state(pde: int, nx: int, ny: int, seed: int = 0) -> np.ndarray:
    if pde == HEAT5:
        return heat_field(nx, ny, seed)
    if pde == WAVE_LF:
        return wave_field(nx, ny, seed)
    if pde == EULER_RUS_RK2:
        return euler_field(nx, ny, seed)
    if pde == EULER_FD_RK4:
        return eulerfd_field(nx, ny, seed)
    if pde == TEST_HASH:
        return hash_field(nx, ny, seed)
    if pde == TEST_INCR:
        return incr_field(nx, ny)
    if pde == TEST_PUSH5:
        return push5_field(nx, ny, seed)
    if pde == TEST_HASH25:
        return hash25_field(nx, ny, seed)
    raise ValueError(f"unknown pde {pde}")


def batch_specs(count: int = 256, seed: int = 0, lo: int = 64, hi: int = 512, quantum: int = 16) -> list[dict]:
    """Uneven batch: side lengths drawn uniformly from the multiples of
    `quantum` in lo..hi (independently in x and y; quantum 1 draws any
    integer), heat or wave and FP64 or FP32-compensated by fair seeded
    draws. Each spec carries the seed of its initial field."""
    rng = np.random.default_rng(seed)
    sides = np.arange(lo, hi + 1)
    sides = sides[sides % quantum == 0]
    specs = []
    for g in range(count):
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        pde = HEAT5 if rng.integers(0, 2) == 0 else WAVE_LF
        prec = int(rng.integers(0, 2))
        specs.append({"nx": nx, "ny": ny, "pde": pde, "prec": prec, "seed": seed * 1000 + g})
    return specs
