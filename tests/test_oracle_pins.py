"""Pins of the oracle against what the paper and the mathematics fix.

CPU only. Each test checks the oracle (``oracle/``) against something other
than itself: closed forms (von Neumann factors, discrete energy), exact
arithmetic on small inputs, conservation, symmetry, mutation-sensitive
closed forms (linear modes, a stationary contact), the worked example of the
paper (``tests/golden/worked_example.json``) and the swept decomposition of
Sec. 3-4 executed component by component (``oracle.swept_model``).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import swept_inputs as si
from oracle import swept_model as sm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ------------------------------------------------------------------ heat

@pytest.mark.parametrize("nx,ny,kx,ky,steps", [(32, 16, 3, 2, 50), (64, 64, 8, 1, 200), (16, 48, 1, 7, 30)])
def test_heat_single_mode_von_neumann(nx, ny, kx, ky, steps):
    """A Fourier mode is an eigenvector of the 5-point FTCS update with factor
    G = 1 - 4 r (sin^2(pi kx / nx) + sin^2(pi ky / ny)); nx != ny so that an
    x/y mix-up changes G."""
    r = si.HEAT_R
    u0 = si.heat_single_mode(nx, ny, kx, ky)
    u = oracle.advance_f64(si.HEAT5, u0, [r], steps)
    G = 1.0 - 4.0 * r * (math.sin(math.pi * kx / nx) ** 2 + math.sin(math.pi * ky / ny) ** 2)
    assert np.max(np.abs(u - G ** steps * u0)) < 1e-12


def test_heat_eight_modes_superposition():
    """The 64x64 heat workload (8 seeded modes, 1000 steps) equals the sum of
    the modes times their amplification factors (linearity)."""
    nx = ny = 64
    rng = np.random.default_rng(0)
    kx = rng.integers(1, 9, size=8)
    ky = rng.integers(1, 9, size=8)
    amp = rng.uniform(-1.0, 1.0, size=8)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=8)
    u0 = si.heat_field(nx, ny, seed=0)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    steps = 1000
    exact = np.zeros((ny, nx))
    for m in range(8):
        G = 1.0 - 4.0 * si.HEAT_R * (math.sin(math.pi * kx[m] / nx) ** 2 + math.sin(math.pi * ky[m] / ny) ** 2)
        exact += amp[m] * G ** steps * np.cos(2 * math.pi * (kx[m] * i / nx + ky[m] * j / ny) + phase[m])
    u = oracle.advance_f64(si.HEAT5, u0, [si.HEAT_R], steps)[0]
    assert np.max(np.abs(u - exact)) < 1e-11


def test_heat_impulse_response():
    """One step of a unit impulse gives 1-4r at the centre, r on the four
    edge neighbours (with periodic wrap) and 0 elsewhere."""
    nx, ny = 7, 5
    r = 0.125
    for (ci, cj) in [(0, 0), (6, 4), (3, 2), (0, 4)]:
        u0 = np.zeros((1, ny, nx))
        u0[0, cj, ci] = 1.0
        u = oracle.advance_f64(si.HEAT5, u0, [r], 1)[0]
        want = np.zeros((ny, nx))
        want[cj, ci] = 1 - 4 * r
        for di, dj in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
            want[(cj + dj) % ny, (ci + di) % nx] = r
        assert np.array_equal(u, want)


def test_heat_mass_conserved():
    u0 = si.heat_field(64, 32, seed=4)
    steps = 300
    u = oracle.advance_f64(si.HEAT5, u0, [si.HEAT_R], steps)
    drift = abs(float(u.sum()) - float(u0.sum()))
    bound = steps * 8 * np.finfo(np.float64).eps * float(np.abs(u0).sum())
    assert drift < bound


def test_heat_exact_dyadic_8x8():
    """With r = 1/8 and integer data in [-8, 8] every FP64 operation of 15 steps
    is exact (denominators 8^15 = 2^45, magnitudes <= 8), so the oracle must
    equal exact rational arithmetic."""
    rng = np.random.default_rng(11)
    n = 8
    u0 = rng.integers(-8, 9, size=(1, n, n)).astype(np.float64)
    got = oracle.advance_f64(si.HEAT5, u0, [0.125], 15)[0]
    r = Fraction(1, 8)
    q = [[Fraction(int(u0[0, j, i])) for i in range(n)] for j in range(n)]
    for _ in range(15):
        q = [[q[j][i] + r * (q[j][(i - 1) % n] + q[j][(i + 1) % n] + q[(j - 1) % n][i] + q[(j + 1) % n][i]
                             - 4 * q[j][i]) for i in range(n)] for j in range(n)]
    exact = np.array([[float(x) for x in row] for row in q])
    assert np.array_equal(got, exact)


def test_heat_r02_within_rounding_bound():
    """r = 0.2 is not dyadic: compare with exact rational arithmetic on the
    FP64 value of 0.2 and bound the rounding error (max norm is non-increasing
    for r <= 1/4, each step adds at most a few ulps)."""
    rng = np.random.default_rng(12)
    n = 8
    steps = 10
    u0 = rng.integers(-8, 9, size=(1, n, n)).astype(np.float64)
    got = oracle.advance_f64(si.HEAT5, u0, [0.2], steps)[0]
    r = Fraction(0.2)
    q = [[Fraction(int(u0[0, j, i])) for i in range(n)] for j in range(n)]
    for _ in range(steps):
        q = [[q[j][i] + r * (q[j][(i - 1) % n] + q[j][(i + 1) % n] + q[(j - 1) % n][i] + q[(j + 1) % n][i]
                             - 4 * q[j][i]) for i in range(n)] for j in range(n)]
    exact = np.array([[float(x) for x in row] for row in q])
    assert np.max(np.abs(got - exact)) < steps * 16 * 8 * np.finfo(np.float64).eps


# ------------------------------------------------------------------ wave

def _lap(u):
    return (np.roll(u, 1, 1) + np.roll(u, -1, 1) + np.roll(u, 1, 0) + np.roll(u, -1, 0)) - 4.0 * u


def test_wave_discrete_energy_conserved():
    """Leapfrog conserves E = |u^{n+1} - u^n|^2 - C2 <u^{n+1}, L u^n> exactly in
    exact arithmetic (L symmetric); here to rounding."""
    s = si.wave_field(64, 48, seed=2, sigma=4.0)
    energies = []
    for _ in range(40):
        s = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], 5)
        u, p = s[0], s[1]
        energies.append(float(np.sum((u - p) ** 2) - si.WAVE_C2 * np.sum(u * _lap(p))))
    e = np.array(energies)
    assert e[0] > 1e-3
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-12


@pytest.mark.parametrize("nx,ny,kx,ky", [(32, 24, 2, 3), (64, 64, 5, 1)])
def test_wave_single_mode_closed_form(nx, ny, kx, ky):
    """With u^{-1} = u^0 a mode evolves as cos(w (n + 1/2)) / cos(w / 2), where
    cos w = 1 - 2 C2 (sin^2(pi kx / nx) + sin^2(pi ky / ny))."""
    u0 = si.heat_single_mode(nx, ny, kx, ky)[0]
    s = np.stack([u0, u0])
    steps = 300
    out = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], steps)
    w = math.acos(1.0 - 2.0 * si.WAVE_C2 * (math.sin(math.pi * kx / nx) ** 2 + math.sin(math.pi * ky / ny) ** 2))
    a = math.cos(w * (steps + 0.5)) / math.cos(w / 2)
    ap = math.cos(w * (steps - 0.5)) / math.cos(w / 2)
    assert np.max(np.abs(out[0] - a * u0)) < 1e-11
    assert np.max(np.abs(out[1] - ap * u0)) < 1e-11


def test_wave_previous_level_is_carried():
    s = si.wave_field(32, 32, seed=1, sigma=3.0)
    one = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], 1)
    two = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], 2)
    assert np.array_equal(two[1], one[0])
    assert np.array_equal(one[1], s[0])


def test_wave_momentum_conserved():
    s = si.wave_field(48, 32, seed=3, sigma=4.0)
    s[1] = s[0] - 0.01 * np.cos(np.arange(48)[None, :] * 2 * math.pi / 48)
    m0 = float(np.sum(s[0] - s[1]))
    out = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], 200)
    assert abs(float(np.sum(out[0] - out[1])) - m0) < 1e-11


# ----------------------------------------------------------------- euler

def test_euler_uniform_state_preserved_bitwise():
    s = np.zeros((8, 12, 10))
    vals = [1.3, 0.7, -0.4, 3.1]
    for k in range(4):
        s[k] = vals[k]
        s[4 + k] = vals[k]
    out = oracle.advance_f64(si.EULER_RUS_RK2, s, [1.4, 0.05], 20)
    assert np.array_equal(out, s)


def test_euler_conservation_and_positivity():
    s = si.euler_field(48, 48, seed=0)
    prm = si.default_params(si.EULER_RUS_RK2, s)
    out = oracle.advance_f64(si.EULER_RUS_RK2, s, prm, 2 * 40)
    for k in range(4):
        t0 = float(np.sum(s[k]))
        t1 = float(np.sum(out[k]))
        scale = float(np.sum(np.abs(s[k])))
        assert abs(t1 - t0) <= 1e-13 * scale
    rho = out[0]
    p = 0.4 * (out[3] - 0.5 * (out[1] ** 2 + out[2] ** 2) / rho)
    assert rho.min() > 0 and p.min() > 0
    assert np.array_equal(out[4:], out[:4])


def test_euler_transpose_symmetry_bitwise():
    """Swapping x and y (and the two momenta) commutes with the update."""
    s = si.euler_field(32, 32, seed=5)
    prm = si.default_params(si.EULER_RUS_RK2, s)
    t = s.transpose(0, 2, 1).copy()
    t[[1, 2]] = t[[2, 1]]
    t[[5, 6]] = t[[6, 5]]
    a = oracle.advance_f64(si.EULER_RUS_RK2, s, prm, 6)
    b = oracle.advance_f64(si.EULER_RUS_RK2, t, prm, 6)
    b = b.transpose(0, 2, 1).copy()
    b[[1, 2]] = b[[2, 1]]
    b[[5, 6]] = b[[6, 5]]
    assert np.array_equal(a, b)


def _euler_at_rest(nx, ny, rho=1.0, p=1.0, gamma=1.4):
    s = np.zeros((8, ny, nx))
    s[0] = rho
    s[3] = p / (gamma - 1.0)
    return s


@pytest.mark.parametrize("mode,kx,dtoh,steps", [("acoustic", 3, 0.3, 20), ("acoustic", 5, 0.25, 12),
                                                 ("entropy", 4, 0.3, 20)])
def test_euler_linear_modes_von_neumann(mode, kx, dtoh, steps):
    """Small Fourier modes on a fluid at rest (rho = 1, p = 1). Linearised,
    the Rusanov flux at rest is 1/2 A (U_R + U_L) - 1/2 c (U_R - U_L), with A
    the flux Jacobian and c = sqrt(gamma p / rho) the sound speed, so along x
    the semi-discrete operator acts on a mode exp(i theta i) as
    -(1/h) (i sin(theta) A + c (1 - cos(theta))). On an eigenvector of A
    (eigenvalue lambda = +c for the acoustic mode (1, c, H), H = c^2 /
    (gamma - 1); lambda = 0 for the entropy mode (1, 0, 0)) one two-stage
    Heun step multiplies the mode by 1 + z + z^2 / 2 with
    z = dt/h (-i lambda sin(theta) - c (1 - cos(theta))).

    This fixes the sound speed in the dissipation (gamma inside the square
    root), the 1/2 dissipation coefficient and the Runge-Kutta weights."""
    gamma, nx, ny, eps = 1.4, 24, 3, 1e-6
    c = math.sqrt(gamma * 1.0 / 1.0)
    H = c * c / (gamma - 1.0)
    lam, r = (c, np.array([1.0, c, H])) if mode == "acoustic" else (0.0, np.array([1.0, 0.0, 0.0]))
    theta = 2.0 * math.pi * kx / nx
    i = np.arange(nx)
    s = _euler_at_rest(nx, ny, gamma=gamma)
    base = s.copy()
    for k, slot in enumerate((0, 1, 3)):
        s[slot] += eps * r[k] * np.cos(theta * i)[None, :]
    s[4:] = s[:4]
    out = oracle.advance_f64(si.EULER_RUS_RK2, s, [gamma, dtoh], 2 * steps)
    z = dtoh * complex(-c * (1.0 - math.cos(theta)), -lam * math.sin(theta))
    g = 1.0 + z + z * z / 2.0
    want = np.real(g ** steps * np.exp(1j * theta * i))
    for k, slot in enumerate((0, 1, 3)):
        got = (out[slot, 1] - base[slot, 1]) / eps
        assert np.max(np.abs(got - r[k] * want)) < 2e-5 * max(1.0, abs(r[k]))
    assert np.max(np.abs(out[2])) < 1e-20 and abs(abs(g) - 1.0) > 0.05


def test_euler_stationary_contact_diffuses_at_the_larger_sound_speed():
    """A density jump at rest under uniform pressure. The physical fluxes on
    both sides are (0, p, 0, 0), so the Rusanov flux reduces to momentum p
    and a pure density flux -1/2 a (rho_R - rho_L) with the face speed
    a = max(c_L, c_R), c = sqrt(gamma p / rho): momentum stays zero, energy
    and pressure stay uniform, and the first Runge-Kutta stage moves
    1/2 a dt/h (rho_L - rho_R) of density across each jump, from the dense
    side to the light one. a is the larger sound speed, that of the lighter
    fluid."""
    gamma, p, dtoh, nx, ny = 1.4, 1.0, 0.2, 16, 2
    rl, rr = 1.0, 0.25
    s = _euler_at_rest(nx, ny, gamma=gamma)
    s[0, :, nx // 2:] = rr
    s[4:] = s[:4]
    one = oracle.advance_f64(si.EULER_RUS_RK2, s, [gamma, dtoh], 1)
    pb = (gamma - 1.0) * (p / (gamma - 1.0))  # the pressure the bits of E give
    a = max(math.sqrt(gamma * pb / rl), math.sqrt(gamma * pb / rr))
    moved = 0.5 * a * (rl - rr) * dtoh
    want = s[0].copy()
    for dense, light in ((nx // 2 - 1, nx // 2), (0, nx - 1)):
        want[:, dense] -= moved
        want[:, light] += moved
    assert np.max(np.abs(one[4] - want)) < 4e-16
    assert np.array_equal(one[:4], s[:4])
    assert not np.any(one[5]) and not np.any(one[6])
    assert np.array_equal(one[7], s[3])
    # The whole Heun step: the same reduction applied to the stage state.
    def diffuse(rho):
        cs = np.sqrt(gamma * pb / rho)
        flux = -0.5 * np.maximum(cs, np.roll(cs, -1)) * (np.roll(rho, -1) - rho)  # face i + 1/2
        return rho - dtoh * (flux - np.roll(flux, 1))
    r0 = s[0, 0]
    r1 = 0.5 * r0 + 0.5 * diffuse(diffuse(r0))
    two = oracle.advance_f64(si.EULER_RUS_RK2, s, [gamma, dtoh], 2)
    assert not np.any(two[1]) and not np.any(two[2]) and np.array_equal(two[3], s[3])
    assert np.max(np.abs(two[0] - r1[None, :])) < 1e-15
    assert np.count_nonzero(two[0, 0] != r0) == 8


def test_euler_vortex_advects_with_the_flow():
    """One isentropic vortex on a (1, 1) stream moves by (t, t): the density
    minimum after time t sits within a cell of its start shifted by t."""
    nx = 64
    s = si.euler_field(nx, nx, seed=0, vortices=1)
    prm = si.default_params(si.EULER_RUS_RK2, s)
    h = si.EULER_SIDE / nx
    dt = prm[1] * h
    steps = 60
    out = oracle.advance_f64(si.EULER_RUS_RK2, s, prm, 2 * steps)

    def centre(rho):
        j, i = np.unravel_index(np.argmin(rho), rho.shape)
        return (i + 0.5) * h, (j + 0.5) * h

    x0, y0 = centre(s[0])
    x1, y1 = centre(out[0])
    dist = steps * dt
    L = si.EULER_SIDE
    ex = (x1 - x0 - dist + L / 2) % L - L / 2
    ey = (y1 - y0 - dist + L / 2) % L - L / 2
    assert dist > 3 * h
    assert abs(ex) <= 1.01 * h and abs(ey) <= 1.01 * h


# ----------------------------------------------------------- test stencils

# ------------------------------------------------- euler, central / rk4

EFD = si.EULER_FD_RK4


def _efd_state(rho, u, v, p, gamma=1.4):
    return si.eulerfd_state(si.eulerfd_conserved(rho, u, v, p, gamma))


def _efd_prim(s, gamma=1.4):
    rho = s[0]
    u, v = s[1] / rho, s[2] / rho
    p = (gamma - 1.0) * (s[3] - 0.5 * (s[1] ** 2 + s[2] ** 2) / rho)
    return np.stack([rho, u, v, p])


def test_eulerfd_uniform_free_stream_preserved_bitwise():
    """The paper's tunnel free stream: every face flux is the same, so no
    sub-step changes a bit and the stage slots return to their entry values."""
    s = si.eulerfd_state(si.eulerfd_conserved(*(np.full((10, 14), x) for x in (
        si.EULERFD_RHO, si.EULERFD_MACH * math.sqrt(1.4 * si.EULERFD_P / si.EULERFD_RHO), 0.0, si.EULERFD_P))))
    out = oracle.advance_f64(EFD, s, si.default_params(EFD), 4 * 5)
    assert np.array_equal(out, s)


def test_eulerfd_rest_with_uniform_pressure_is_steady_bitwise():
    """At rest with uniform pressure every mass flux is zero and the pressure
    terms cancel exactly, however the density varies (a stationary contact)."""
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, (12, 16))
    z = np.zeros_like(rho)
    s = _efd_state(rho, z, z, np.full_like(rho, 0.8))
    out = oracle.advance_f64(EFD, s, [1.4, 0.3], 4 * 7)
    assert np.array_equal(out, s)


def test_eulerfd_first_substep_is_the_split_form():
    """Sub-step 0 leaves -r in the derivative slots, r = h div F. Written out
    independently as the skew-symmetric split form of the convective terms,
    per direction d with mass flux m = rho u_d and phi in (1, u, v, H):
    r = sum_d 1/4 [D(m phi) + m D(phi) + phi D(m)] + 1/2 D(p) e_d,
    D f = f(+1) - f(-1), a central difference (Sec. 8; the face-flux form
    in the oracle is algebraically the same and conservative)."""
    gamma = 1.4
    rng = np.random.default_rng(11)
    ny, nx = 9, 13
    rho = rng.uniform(0.8, 1.3, (ny, nx))
    u, v = rng.uniform(-0.4, 0.4, (2, ny, nx))
    p = rng.uniform(0.6, 1.1, (ny, nx))
    s = _efd_state(rho, u, v, p, gamma)
    out = oracle.advance_f64(EFD, s, [gamma, 0.1], 1)
    got = -out[8:12]
    H = (s[3] + p) / rho

    def D(f, ax):
        return np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)

    want = np.zeros((4, ny, nx))
    scale = np.zeros((4, ny, nx))
    for ax, m in ((1, s[1]), (0, s[2])):
        for k, phi in enumerate((np.ones_like(rho), u, v, H)):
            want[k] += 0.25 * (D(m * phi, ax) + m * D(phi, ax) + phi * D(m, ax))
            scale[k] += np.abs(m * phi) + np.abs(m) + np.abs(phi)
        want[2 if ax == 0 else 1] += 0.5 * D(p, ax)
        scale[2 if ax == 0 else 1] += np.abs(p)
    assert np.all(np.abs(got - want) <= 1e-14 * scale)
    # the plain average flux (f_L + f_R) / 2 differs from the split form
    plain = 0.5 * (D(s[1], 1) + D(s[2], 0))
    assert np.allclose(got[0], plain, rtol=0, atol=1e-13)
    plain_mx = 0.5 * (D(s[1] * u + p, 1) + D(s[2] * u, 0))
    assert np.max(np.abs(got[1] - plain_mx)) > 1e-3


def test_eulerfd_conservation_and_stage_slots():
    s = si.eulerfd_field(48, 32, seed=2, amp=0.2, width=4.0)
    out = oracle.advance_f64(EFD, s, [1.4, 2e-4], 4 * 30)
    for k in range(4):
        t0, t1 = float(np.sum(s[k])), float(np.sum(out[k]))
        scale = float(np.sum(np.abs(s[1 if k == 2 else k])))  # my starts at zero: use mx's scale
        assert abs(t1 - t0) <= 1e-14 * scale
    assert not np.array_equal(out[:4], s[:4]) and np.max(np.abs(out[2])) > 1e-3 * np.max(np.abs(s[1]))
    assert np.array_equal(out[4:8], out[:4]) and not np.any(out[8:])


def test_eulerfd_transpose_symmetry_bitwise():
    s = si.eulerfd_field(24, 24, seed=4, amp=0.1, width=3.0)
    s[2] += 0.3 * s[0] * np.sin(np.arange(24) / 3.0)[:, None]
    s[6] = s[2]
    t = s.transpose(0, 2, 1).copy()
    for a, b in ((1, 2), (5, 6), (9, 10)):
        t[[a, b]] = t[[b, a]]
    prm = [1.4, 1e-4]
    a = oracle.advance_f64(EFD, s, prm, 4 * 3 + 2)
    b = oracle.advance_f64(EFD, t, prm, 4 * 3 + 2)
    b = b.transpose(0, 2, 1).copy()
    for x, y in ((1, 2), (5, 6), (9, 10)):
        b[[x, y]] = b[[y, x]]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("family", ["acoustic+", "acoustic-", "entropy", "shear"])
def test_eulerfd_linear_modes_rk4_amplification(family):
    """Small modes on a uniform stream (rho = 1, u0 = 0.3, p = 1/gamma, so
    c = 1). The face flux is a symmetric two-point flux, so linearised it is
    A (U_L + U_R) / 2 and the semi-discrete operator on exp(i theta i) is
    -(i sin(theta) / h) A: each characteristic family (eigenvalue u0 - c, u0,
    u0, u0 + c of A) is multiplied per step by the four-stage Runge-Kutta
    polynomial 1 + z + z^2/2 + z^3/6 + z^4/24, z = -i lambda sin(theta) dt/h.
    The difference of the runs from +eps and -eps removes the even orders of
    the nonlinearity."""
    gamma, nx, ny, eps, dth, steps = 1.4, 32, 3, 1e-5, 0.8, 16
    rho0, u0, p0 = 1.0, 0.3, 1.0 / gamma
    c = 1.0
    r, lam = {"acoustic+": ((1.0, 1.0, 0.0, 1.0), u0 + c), "acoustic-": ((1.0, -1.0, 0.0, 1.0), u0 - c),
              "entropy": ((1.0, 0.0, 0.0, 0.0), u0), "shear": ((0.0, 0.0, 1.0, 0.0), u0)}[family]
    theta = 2.0 * math.pi * 7 / nx
    wave = np.cos(theta * np.arange(nx))[None, :] * np.ones((ny, 1))
    base = [np.full((ny, nx), x) for x in (rho0, u0, 0.0, p0)]

    def run(e):
        w = [base[k] + e * r[k] * wave for k in range(4)]
        return _efd_prim(oracle.advance_f64(EFD, _efd_state(*w, gamma), [gamma, dth], 4 * steps), gamma)

    got = (run(eps) - run(-eps)) / (2.0 * eps)
    z = complex(0.0, -lam * math.sin(theta) * dth)
    g = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    want = np.real(g ** steps * np.exp(1j * theta * np.arange(nx)))
    for k in range(4):
        assert np.max(np.abs(got[k] - r[k] * want[None, :])) < 1e-8
    # the bound separates the polynomial from its third-order truncation
    g3 = 1 + z + z ** 2 / 2 + z ** 3 / 6
    assert abs(g ** steps - g3 ** steps) > 1e-5


def test_push5_two_substeps_equal_wide_stencil():
    """Eq. (2)-(3) reproduce Eq. (1) bit for bit (same values, same order)."""
    s = si.push5_field(24, 20, seed=7)
    s[0] = np.random.default_rng(7).standard_normal((20, 24))
    out = oracle.advance_f64(si.TEST_PUSH5, s, [], 2)
    u = s[0]
    wide = (np.roll(u, 2, 1) + np.roll(u, -2, 1)) + np.roll(u, 2, 0)
    wide = wide + np.roll(u, -2, 0)
    wide = wide - 4.0 * u
    assert np.array_equal(out[0], wide)
    assert not np.any(out[1:])


def test_hash_is_local_and_position_sensitive():
    """One step of the hash stencil changes exactly the 3x3 neighbourhood of a
    changed input, and swapping two inputs of a neighbourhood changes the
    output."""
    s = si.hash_field(9, 7, seed=1)
    base = oracle.advance_f64(si.TEST_HASH, s, [], 1, t0=3)
    t = s.copy()
    t[0, 0, 0] += 1.0
    moved = oracle.advance_f64(si.TEST_HASH, t, [], 1, t0=3)
    diff = moved[0] != base[0]
    want = np.zeros_like(diff)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            want[dj % 7, di % 9] = True
    assert np.array_equal(diff, want)
    w = s.copy()
    w[0, 3, 3], w[0, 3, 4] = s[0, 3, 4], s[0, 3, 3]
    swapped = oracle.advance_f64(si.TEST_HASH, w, [], 1, t0=3)
    assert swapped[0, 3, 3] != base[0, 3, 3]
    other_level = oracle.advance_f64(si.TEST_HASH, s, [], 1, t0=4)
    assert np.all(other_level != base)
    assert np.all(base < 2.0 ** 52) and np.all(base == np.floor(base))


def test_incr_every_value_equals_its_level():
    s = si.incr_field(12, 10)
    out = oracle.advance_f64(si.TEST_INCR, s, [], 17)
    assert np.all(out == 18.0)
    s[0, 4, 4] = 5.0
    out = oracle.advance_f64(si.TEST_INCR, s, [], 1)
    assert np.isnan(out[0, 4, 4]) and np.isnan(out[0, 3, 5]) and out[0, 0, 0] == 2.0


# ------------------------------------------------------------------ FP32C

def _norm_rel(a, ref):
    return max(float(np.max(np.abs(a[v] - ref[v])) / np.max(np.abs(ref[v]))) for v in range(ref.shape[0]))


def test_f32c_heat_exact_when_fp32_is_exact():
    """Integer data, r = 1/8, 6 steps: every FP32 operation is exact, so the
    compensated stepper equals the FP64 oracle and every compensation is 0."""
    rng = np.random.default_rng(3)
    u0 = rng.integers(-8, 9, size=(1, 8, 8)).astype(np.float64)
    u, c = oracle.split_f32c(u0)
    u6, c6 = oracle.advance_f32c(si.HEAT5, u, c, [0.125], 6)
    ref = oracle.advance_f64(si.HEAT5, u0, [0.125], 6)
    assert np.array_equal(u6.astype(np.float64), ref)
    assert not np.any(c6)


def test_f32c_heat_error_and_benefit():
    """Compensated FP32 stays within 1e-6 (normwise, per variable) of FP64 and
    beats plain FP32 (the same stepper with the compensation reset every step).
    256^2 keeps the field from decaying below the FP32 floor of its initial
    rounding within 2000 steps."""
    s = si.heat_field(256, 256, seed=0)
    steps = 2000
    ref = oracle.advance_f64(si.HEAT5, s, [si.HEAT_R], steps)
    u, c = oracle.split_f32c(s)
    uc, _ = oracle.advance_f32c(si.HEAT5, u, c, [si.HEAT_R], steps)
    err_c = _norm_rel(uc.astype(np.float64), ref)
    up = u.copy()
    for _ in range(steps):
        up, _ = oracle.advance_f32c(si.HEAT5, up, np.zeros_like(up), [si.HEAT_R], 1, threads=1)
    err_p = _norm_rel(up.astype(np.float64), ref)
    assert err_c < 1e-6
    assert err_c < 0.3 * err_p


def test_f32c_wave_error():
    s = si.wave_field(64, 64, seed=0, sigma=6.0)
    steps = 500
    ref = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], steps)
    u, c = oracle.split_f32c(s)
    uc, _ = oracle.advance_f32c(si.WAVE_LF, u, c, [si.WAVE_C2], steps)
    assert _norm_rel(uc.astype(np.float64), ref) < 1e-6


def test_f32c_wave_error_and_benefit():
    """Leapfrog adds every error of the velocity to the displacement for
    good, so the compensated form must keep both the velocity (the
    compensated difference of the two levels) and the Laplacian (of the
    compensated values) accurate. Against plain FP32 (the same stepper with
    the compensations reset every step) it must cut the error by far more
    than either half alone does: on 256^2 after 1000 steps the full form
    stays below 2e-7 and under a tenth of plain FP32's error, while dropping
    either correction leaves about half of plain FP32's error."""
    s = si.wave_field(256, 256, seed=0)
    steps = 1000
    ref = oracle.advance_f64(si.WAVE_LF, s, [si.WAVE_C2], steps)
    u, c = oracle.split_f32c(s)
    uc, cc = oracle.advance_f32c(si.WAVE_LF, u, c, [si.WAVE_C2], steps)
    err_c = _norm_rel(uc.astype(np.float64) - cc.astype(np.float64), ref)
    up = u.copy()
    for _ in range(steps):
        up, _ = oracle.advance_f32c(si.WAVE_LF, up, np.zeros_like(up), [si.WAVE_C2], 1)
    err_p = _norm_rel(up.astype(np.float64), ref)
    assert err_c < 2e-7
    assert err_c < 0.1 * err_p


def test_f32c_euler_error():
    s = si.euler_field(32, 32, seed=1)
    prm = si.default_params(si.EULER_RUS_RK2, s)
    steps = 50
    ref = oracle.advance_f64(si.EULER_RUS_RK2, s, prm, 2 * steps)
    u, c = oracle.split_f32c(s)
    uc, cc = oracle.advance_f32c(si.EULER_RUS_RK2, u, c, prm, 2 * steps)
    got = uc.astype(np.float64) - cc.astype(np.float64)
    assert _norm_rel(got[:4], ref[:4]) < 1e-6


def test_f32c_eulerfd_error_and_benefit():
    """The paper's Euler discretisation on compensated FP32 slots: every value
    is widened to u - c and the FP64 sub-step applied, so from the same
    (FP32-representable) start it tracks the FP64 stepper to FP64 rounding
    over 100 steps (400 sub-steps), about 2^-48 relative per variable, while
    the same stepper with the compensations dropped after every sub-step is
    plain FP32 and off by over 1e-6."""
    s = si.eulerfd_field(48, 32, seed=2, amp=0.2, width=4.0)
    prm, steps = [1.4, 2e-4], 100
    u, c = oracle.split_f32c(s)
    ref = oracle.advance_f64(EFD, u.astype(np.float64), prm, 4 * steps)
    uc, cc = oracle.advance_f32c(EFD, u, c, prm, 4 * steps)
    err_c = _norm_rel(uc[:4].astype(np.float64) - cc[:4].astype(np.float64), ref[:4])
    up = u.copy()
    for t in range(4 * steps):
        up, _ = oracle.advance_f32c(EFD, up, np.zeros_like(up), prm, 1, t0=t, threads=1)
    err_p = _norm_rel(up[:4].astype(np.float64), ref[:4])
    assert err_c < 2e-12
    assert err_p > 1e-6 and err_c < 1e-5 * err_p


def test_f32c_eulerfd_stage_slots():
    """Sub-steps 0-2 of a step leave both halves of the U slots untouched;
    after the last one Y equals U in both halves and K is zero in both."""
    s = si.eulerfd_field(32, 16, seed=5, amp=0.2, width=3.0)
    prm = [1.4, 2e-4]
    u, c = oracle.advance_f32c(EFD, *oracle.split_f32c(s), prm, 4 * 3)
    assert np.any(c[:4])
    for k in (1, 2, 3):
        uk, ck = oracle.advance_f32c(EFD, u, c, prm, k, t0=12)
        assert np.array_equal(uk[:4], u[:4]) and np.array_equal(ck[:4], c[:4])
        assert np.any(uk[8:]) and not np.array_equal(uk[4:8], u[4:8])
    u4, c4 = oracle.advance_f32c(EFD, u, c, prm, 4, t0=12)
    assert np.array_equal(u4[4:8], u4[:4]) and np.array_equal(c4[4:8], c4[:4])
    assert not np.any(u4[8:]) and not np.any(c4[8:])
    assert not np.array_equal(u4[:4], u[:4])


# ------------------------------------- the swept decomposition (Sec. 3-4)

@pytest.mark.parametrize("nx,ny,n", [(16, 16, 8), (8, 8, 8), (16, 16, 4), (24, 16, 8), (12, 12, 4), (8, 12, 2)])
def test_decomposition_equals_plain_stepping(nx, ny, n):
    """Every half cycle of the component-by-component model (pyramids, then
    bridges, then downward pyramids, the tiling shifted by n/2 between half
    cycles) lands on the plain result; the hash stencil makes any misplaced
    neighbour or level visible."""
    g = si.hash_field(nx, ny, seed=3)
    got = {}
    sm.swept2d(sm.st_hash, g[0], n, cycles=2, T0=5, after_half=lambda T, grid: got.__setitem__(T, grid))
    assert sorted(got) == [5 + k * (n // 2) for k in range(1, 5)]
    for T, grid in got.items():
        ref = oracle.advance_f64(si.TEST_HASH, g, [], T - 5, t0=5)[0]
        assert np.array_equal(grid, ref)


def test_decomposition_heat_and_reduced_half_cycle():
    g = si.heat_field(16, 24, seed=2)
    out = sm.swept2d(sm.st_heat(si.HEAT_R), g[0], 8, cycles=2)
    assert np.array_equal(out, oracle.advance_f64(si.HEAT5, g, [si.HEAT_R], 16)[0])
    # a half cycle of reduced height H < n/2 (the remainder of a step count)
    h3 = sm.half_cycle(sm.st_heat(si.HEAT_R), g[0], 8, 4, 0, 3)
    assert np.array_equal(h3, oracle.advance_f64(si.HEAT5, g, [si.HEAT_R], 3)[0])


def test_printed_bridge_band_does_not_cover_the_half_cycle(monkeypatch):
    """The bridges' compute loop as printed (a two-point band on one side of
    the edge at every level) leaves points of the bridges' space-time
    uncomputed, so a downward pyramid or the next level needs a value nothing
    produced."""
    monkeypatch.setattr(sm, "LITERAL_BRIDGE_BAND", True)
    g = si.hash_field(16, 16, seed=3)
    with pytest.raises(sm.ModelError):
        sm.swept2d(sm.st_hash, g[0], 8, cycles=1)


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_component_sizes(n):
    """Points computed per tile and half cycle: up n(n-1)(n-2)/6, each bridge
    (n^3-4n)/12, down n(n+1)(n+2)/6; together n^2 * n/2 (Sec. 5: a half cycle
    performs n/2 sub-steps on n^2 points)."""
    nx = ny = 2 * n
    st = sm.Stats()
    sm.swept2d(sm.st_hash, si.hash_field(nx, ny)[0], n, cycles=1, stats=st)
    tiles_halves = (nx // n) * (ny // n) * 2
    assert st.computed.get(sm.UP, 0) == tiles_halves * n * (n - 1) * (n - 2) // 6
    assert st.computed.get(sm.YB, 0) == tiles_halves * (n ** 3 - 4 * n) // 12
    assert st.computed.get(sm.XB, 0) == tiles_halves * (n ** 3 - 4 * n) // 12
    assert st.computed[sm.DOWN] == tiles_halves * n * (n + 1) * (n + 2) // 6
    assert sum(st.computed.values()) == tiles_halves * n * n * (n // 2)


def test_downward_pyramid_ring():
    """At each level k a downward pyramid reads a ring two wide around its
    level-k square: 16k values from the four bridges' bands and the four 2x2
    corners (16 values) from the upward pyramids."""
    n = 8
    st = sm.Stats()
    sm.half_cycle(sm.st_hash, si.hash_field(16, 16)[0], n, 0, 0, n // 2, st)
    corners = 4
    for k in range(n // 2):
        from_bridges = sum(len(v) for key, v in st.crossing.items()
                           if key[1] == sm.DOWN and key[2] == k and key[0] in (sm.XB, sm.YB))
        from_up = sum(len(v) for key, v in st.crossing.items() if key[1] == sm.DOWN and key[2] == k and key[0] == sm.UP)
        assert from_bridges == corners * 16 * k
        assert from_up == corners * 16


def _square(n, k):
    return {(x, y) for x in range(k, n - k) for y in range(k, n - k)}


def test_worked_example_values():
    gold = json.load(open(GOLDEN))
    n = gold["upward_panel_values_per_level"]["n"]
    h = n // 2
    # What an upward pyramid sends at level k is the band two wide along the
    # edges of its level-k square (a 2x2 tip at the last level); each side's
    # strip holds 16, 12, 8, 4 values for n = 8.
    st = sm.Stats()
    sm.half_cycle(sm.st_hash, si.hash_field(2 * n, 2 * n)[0], n, 0, 0, h, st)
    per_level = []
    for k in range(h):
        sent = st.up_sent[((0, 0), k)]
        assert sent == _square(n, k) - _square(n, k + 2)
        per_level.append(len({p for p in sent if p[1] in (k, k + 1)}))
    assert per_level == gold["upward_panel_values_per_level"]["values"]
    # From level 1 on 8x8 subdomains the tip of each upward pyramid (2x2) is
    # at level 4.
    start = gold["pyramid_tip_level"]["start_level"]
    assert start + h - 1 == gold["pyramid_tip_level"]["tip_level"]
    assert len(_square(n, h - 1)) == 4
    # A full cycle on 8x8 subdomains advances 8 levels with 4 communications.
    cyc = gold["cycle"]
    st = sm.Stats()
    out = sm.swept2d(sm.st_incr, np.full((2 * n, 2 * n), float(cyc["start_level"])), cyc["n"], cycles=1, stats=st)
    assert np.all(out == cyc["start_level"] + cyc["levels_advanced"])
    assert st.exchanges == cyc["communications"]
    # The downward pyramid computes squares of side 2, 4, ..., n.
    sq = gold["downward_first_square"]["computed_squares"]
    st = sm.Stats()
    sm.half_cycle(sm.st_hash, si.hash_field(n, n)[0], n, 0, 0, h, st)
    assert st.computed[sm.DOWN] == sum(s * s for s in sq) == n * (n + 1) * (n + 2) // 6
    half = gold["half_cycle_substeps"]
    got = {}
    st = sm.Stats()
    sm.swept2d(sm.st_incr, np.ones((2 * n, 2 * n)), half["n"], cycles=1, stats=st,
               after_half=lambda T, grid: got.__setitem__(T, grid))
    assert sorted(got)[0] == half["substeps"]
    assert np.all(got[half["substeps"]] == 1 + half["substeps"])
    assert st.exchanges == 2 * half["communications"]


# ------------------------------------ FP32 with the compensation in a residency

def _model_residency_keys(nx, ny, n, S):
    """Residency of every point at levels 0..S of one swept advance, from the
    level-function model: the first upward pyramid (with level 0); each half
    cycle's bridges one by one; a downward pyramid together with the upward
    pyramid of the next half cycle whose tile is exactly the set of points
    the downward pyramid holds at its last level."""
    h = n // 2
    keys = {}
    for y in range(ny):
        for x in range(nx):
            keys[(x, y, 0)] = ("first",)
    k = 0
    prev_down_sets = None
    while k * h < S:
        off = (k % 2) * h
        H = min(h, S - k * h)
        comp = {(x, y, l): sm.component(x, y, l, n, off, nx, ny)
                for l in range(0, H + 1) for y in range(ny) for x in range(nx)}
        # upward pyramids of this half cycle: which downward pyramid of the
        # previous one (if any) covers exactly the same points
        up_home = {}
        tiles = {}
        for (x, y, l), c in comp.items():
            if l == 0:
                tiles.setdefault(c[1], set()).add((x, y))
        for t, pts in tiles.items():
            if k == 0:
                up_home[t] = ("first",)
            else:
                match = [d for d, dpts in prev_down_sets.items() if dpts == pts]
                assert len(match) == 1
                up_home[t] = ("oct", k - 1, match[0])
        down_sets = {}
        for (x, y, l), c in comp.items():
            if l == 0:
                continue
            L = k * h + l
            if c[0] == sm.UP:
                keys[(x, y, L)] = up_home[c[1]]
            elif c[0] == sm.DOWN:
                keys[(x, y, L)] = ("oct", k, c[1])
                if l == h:
                    down_sets.setdefault(c[1], set()).add((x, y))
            else:
                keys[(x, y, L)] = ("bridge", k, c)
        prev_down_sets = down_sets
        k += 1
    return keys


@pytest.mark.parametrize("nx,ny,n,S", [(16, 24, 8, 11), (12, 12, 4, 9), (8, 8, 8, 4), (6, 10, 2, 3)])
def test_residency_rule_matches_the_decomposition(nx, ny, n, S):
    """The oracle's residency numbers (a formula in the edge distances) give,
    for every point, level and neighbour, the same answer to "computed in the
    same window as the point reading it" as the model's components."""
    keys = _model_residency_keys(nx, ny, n, S)
    res = {(x, y, L): oracle.residency(x, y, L, n, nx, ny) for (x, y, L) in keys}
    for (x, y, L), key in keys.items():
        if L == 0:
            continue
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                q = ((x + di) % nx, (y + dj) % ny, L - 1)
                assert (keys[q] == key) == (res[q] == res[(x, y, L)]), ((x, y, L), q)


def test_f32r_per_step_method_is_plain_fp32():
    """Tile side 0 (a launch per sub-step) keeps no compensation across a
    sub-step: for heat it equals the compensated stepper with c reset every
    step."""
    s0 = si.initial_state(si.HEAT5, 48, 32, seed=2)
    p = si.default_params(si.HEAT5)
    u = s0.astype(np.float32)
    got = oracle.advance_f32r(si.HEAT5, u, p, 25, 0)
    ref = u.copy()
    for _ in range(25):
        ref, _ = oracle.advance_f32c(si.HEAT5, ref, np.zeros_like(ref), p, 1)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("pde,shape", [(si.HEAT5, (48, 32)), (si.WAVE_LF, (32, 48))])
def test_f32r_per_step_method_restarts_every_sub_step(pde, shape):
    """At tile side 0 every sub-step is a residency of its own: one advance
    of 25 sub-steps equals 25 advances of one (each starting its
    compensations at zero); at tile side 8 it does not."""
    s0 = si.initial_state(pde, *shape, seed=2)
    p = si.default_params(pde)
    u = oracle.split_f32r(pde, s0)
    got = oracle.advance_f32r(pde, u, p, 25, 0)
    ref = u.copy()
    for k in range(25):
        ref = oracle.advance_f32r(pde, ref, p, 1, 0, t0=k)
    assert np.array_equal(got, ref)
    ref8 = u.copy()
    for k in range(25):
        ref8 = oracle.advance_f32r(pde, ref8, p, 1, 8, t0=k)
    assert not np.array_equal(oracle.advance_f32r(pde, u, p, 25, 8), ref8)


def test_f32r_wave_velocity_form_exact_on_dyadic_data():
    """The wave's velocity form (v = u^n - u^(n-1); v' = v + C2 lap,
    u' = u + v') is leapfrog in exact arithmetic: on small integers with
    C2 = 1/4 every value of 4 steps is exact in FP32, and the converted
    result equals the FP64 leapfrog oracle for every tile side, the
    conversions to and from (u^n, u^(n-1)) included."""
    rng = np.random.default_rng(8)
    u0 = rng.integers(-2, 3, size=(16, 16)).astype(np.float64)
    s0 = np.stack([u0, u0 + rng.integers(-1, 2, size=(16, 16))])
    ref = oracle.advance_f64(si.WAVE_LF, s0, [0.25], 4)
    for n in (4, 8, 16, 0):
        got = oracle.join_f32r(si.WAVE_LF, oracle.advance_f32r(si.WAVE_LF, oracle.split_f32r(si.WAVE_LF, s0), [0.25], 4, n))
        assert np.array_equal(got, ref), n


def test_f32r_wave_velocity_compensations_give_exact_leapfrog_on_one_point():
    """The pairs stand for u - c_u and v - c_v, so one point of the velocity
    form must be leapfrog on those values, which dyadic data makes exact.
    Neighbours 0 (no compensation), the point's u = 0 with c_u = 2^-25 and
    v = 1 with c_v = 0, C2 = 1/4: U = -2^-25, V = 1, lap U = 4 * 2^-25, so
    V' = V + C2 lap U = 1 + 2^-25 and U' = U + V' = 1 exactly. The new
    velocity rounds to tv = 1 with compensation -2^-25, and the displacement
    takes the increment V' - c_u = tv - (c_u + c_v'): taking that
    compensation with the other sign gives U' = 1 - 2^-24."""
    nu = np.zeros((3, 3, 2), np.float32)
    nc = np.zeros((3, 3, 2), np.float32)
    nu[1, 1] = (0.0, 1.0)
    nc[1, 1] = (2.0 ** -25, 0.0)
    ou, oc = oracle.point_wave_f32v(nu, nc, 0.25)
    U1 = Fraction(float(ou[0])) - Fraction(float(oc[0]))
    V1 = Fraction(float(ou[1])) - Fraction(float(oc[1]))
    assert V1 == 1 + Fraction(1, 2 ** 25)
    assert U1 == 1
    assert (float(ou[1]), float(oc[1])) == (1.0, -(2.0 ** -25))


def test_f32r_exact_when_fp32_is_exact():
    rng = np.random.default_rng(5)
    u0 = rng.integers(-8, 9, size=(1, 16, 16)).astype(np.float64)
    for n in (4, 8, 16, 0):
        got = oracle.advance_f32r(si.HEAT5, u0.astype(np.float32), [0.125], 6, n)
        assert np.array_equal(got.astype(np.float64), oracle.advance_f64(si.HEAT5, u0, [0.125], 6))


@pytest.mark.parametrize("pde,steps", [(si.HEAT5, 1500), (si.WAVE_LF, 600)])
def test_f32r_error_between_full_compensation_and_plain_fp32(pde, steps):
    """Dropping the compensation only where a value changes window loses part
    of its benefit: the error lies between that of the full compensated
    stepper and that of plain FP32, and deeper pyramids (larger tiles, fewer
    changes of window) keep more of it."""
    s0 = si.initial_state(pde, 256, 256, seed=0)
    p = si.default_params(pde)
    ref = oracle.advance_f64(pde, s0, p, steps)
    u, c = oracle.split_f32c(s0)
    ub, cb = oracle.advance_f32c(pde, u, c, p, steps)
    err_b = _norm_rel(ub.astype(np.float64) - cb.astype(np.float64), ref)
    u = oracle.split_f32r(pde, s0)
    errs = {n: _norm_rel(oracle.join_f32r(pde, oracle.advance_f32r(pde, u, p, steps, n)), ref)
            for n in (-1, 0, 16, 64)}
    assert errs[-1] < errs[64] < errs[16] < errs[0]
    assert err_b < errs[64] and errs[64] < 1e-6 and errs[-1] < 2 * err_b


def test_f32r_wave_long_run():
    """Over 10000 steps (256^2), the velocity form with every compensation
    kept stays within 2e-7 of FP64, which needs the velocity's compensation
    (without it the error exceeds 4e-7); confined to residencies at tile side
    64 it is still below the per-step method's plain FP32, which needs the
    new velocity's compensation in the displacement's increment."""
    pde, steps = si.WAVE_LF, 10000
    s0 = si.initial_state(pde, 256, 256, seed=0)
    p = si.default_params(pde)
    ref = oracle.advance_f64(pde, s0, p, steps)
    u = oracle.split_f32r(pde, s0)
    errs = {n: _norm_rel(oracle.join_f32r(pde, oracle.advance_f32r(pde, u, p, steps, n)), ref) for n in (-1, 0, 64)}
    assert errs[-1] < 2e-7
    assert errs[64] < errs[0]


def test_f32r_one_residency_is_the_compensated_stepper():
    """Tile side -1 keeps every compensation for the whole advance: for heat
    that is the FP32C stepper (compensation carried everywhere), bit for
    bit."""
    s0 = si.heat_field(64, 48, seed=6)
    p = si.default_params(si.HEAT5)
    u, c = oracle.split_f32c(s0)
    ref_u, _ = oracle.advance_f32c(si.HEAT5, u, np.zeros_like(c), p, 300)
    assert np.array_equal(oracle.advance_f32r(si.HEAT5, u, p, 300, -1), ref_u)


# ------------------------------------------------- stencils reaching two rings

def test_hash25_is_local_to_two_rings_and_position_sensitive():
    """One step of the 25-point hash changes exactly the 5x5 neighbourhood of
    a changed input (periodic wrap included); swapping two inputs of a
    neighbourhood, or changing the step index, changes the result."""
    nx, ny = 11, 9
    u = si.hash_field(nx, ny, seed=2)[0]
    base = oracle.advance_hash25(u, 1, k0=4)
    for (ci, cj) in [(0, 0), (10, 8), (5, 4)]:
        t = u.copy()
        t[cj, ci] += 1.0
        diff = oracle.advance_hash25(t, 1, k0=4) != base
        want = np.zeros_like(diff)
        for dj in range(-2, 3):
            for di in range(-2, 3):
                want[(cj + dj) % ny, (ci + di) % nx] = True
        assert np.array_equal(diff, want)
    w = u.copy()
    w[4, 3], w[4, 5] = u[4, 5], u[4, 3]
    assert oracle.advance_hash25(w, 1, k0=4)[4, 4] != base[4, 4]
    assert np.all(oracle.advance_hash25(u, 1, k0=5) != base)
    assert np.all(base < 2.0 ** 52) and np.all(base == np.floor(base))
    two = oracle.advance_hash25(u, 2, k0=4)
    assert np.array_equal(two, oracle.advance_hash25(base, 1, k0=5))


# ------------------------- rectangular tiles of any side (the level function)

@pytest.mark.parametrize("nx,ny,h,levels", [(11, 9, 2, 7), (13, 17, 3, 10), (10, 7, 2, 5), (9, 9, 4, 9),
                                            (20, 14, 3, 8), (12, 12, 3, 6)])
def test_rect_decomposition_equals_plain_stepping(nx, ny, h, levels):
    """Tiles of widths floor(L/t) and floor(L/t)+1 with t = floor(L/2h) on
    each axis (odd, uneven and single-tile axes included), alternating with
    the tiling whose edges are the tiles' midpoints: every half cycle lands
    on the plain result, the last one of reduced height included."""
    g = si.hash_field(nx, ny, seed=7)
    got = {}
    sm.swept2d_rect(sm.st_hash, g[0], h, levels, T0=3, after_half=lambda T, grid: got.__setitem__(T, grid))
    want = [3 + min(levels, k * h) for k in range(1, -(-levels // h) + 1)]
    assert sorted(got) == want
    for T, grid in got.items():
        ref = oracle.advance_f64(si.TEST_HASH, g, [], T - 3, t0=3)[0]
        assert np.array_equal(grid, ref)


def test_rect_decomposition_heat():
    g = si.heat_field(15, 13, seed=4)
    out = sm.swept2d_rect(sm.st_heat(si.HEAT_R), g[0], 3, 11)
    assert np.array_equal(out, oracle.advance_f64(si.HEAT5, g, [si.HEAT_R], 11)[0])


def test_rect_tiles_narrower_than_2H_break_the_order():
    """The bound w >= 2H is needed: on a tile of width 2H - 1 a point lies
    within l of both its edges at the top level, and the level function
    makes a bridge read a value of the other bridge of the same phase."""
    g = si.hash_field(10, 10, seed=1)
    ax = sm.Axis(10, (0, 5))  # widths 5 = 2H - 1 for H = 3
    with pytest.raises(sm.ModelError):
        sm.half_cycle_on(sm.st_hash, g[0], ax, ax, 0, 3)
    sm.half_cycle_on(sm.st_hash, g[0], ax, ax, 0, 2)  # 5 >= 2 * 2: fine


@pytest.mark.parametrize("wx,wy,H", [(7, 9, 3), (6, 11, 2), (8, 8, 4), (10, 5, 2)])
def test_rect_component_sizes(wx, wy, H):
    """Per tile of wx x wy and half cycle of H levels: the upward frustum
    computes sum (wx-2l)(wy-2l), the bridge across its east edge sum
    2l(wy-2l), the one across its south edge sum 2l(wx-2l), the downward
    pyramid at its south-east corner sum (2l)^2, l = 1..H; together wx wy H."""
    ax = sm.Axis(2 * wx, (0, wx))
    ay = sm.Axis(2 * wy, (0, wy))
    st = sm.Stats()
    sm.half_cycle_on(sm.st_hash, si.hash_field(2 * wx, 2 * wy)[0], ax, ay, 0, H, st)
    L = range(1, H + 1)
    assert st.computed.get(sm.UP, 0) == 4 * sum((wx - 2 * l) * (wy - 2 * l) for l in L)
    assert st.computed[sm.XB] == 4 * sum(2 * l * (wy - 2 * l) for l in L)
    assert st.computed[sm.YB] == 4 * sum(2 * l * (wx - 2 * l) for l in L)
    assert st.computed[sm.DOWN] == 4 * sum(4 * l * l for l in L)
    assert sum(st.computed.values()) == 4 * wx * wy * H


def test_rect_axis_and_midpoint_tiling():
    """For every axis length and h: floor(L/2h) tiles of two widths w, w+1
    (w >= 2h) in both tilings; each tile of one tiling holds exactly one
    edge of the other, at least h cells from either of its own edges (so a
    downward pyramid's 2h x 2h square lies inside one tile of the next
    tiling)."""
    for h in range(1, 9):
        for L in range(2 * h, 8 * h + 3):
            ax = sm.rect_axis(L, h)
            mx = sm.mid_axis(ax)
            for one, other in ((ax, mx), (mx, ax)):
                ws = one.widths()
                assert len(ws) == L // (2 * h) and sum(ws) == L
                assert min(ws) >= 2 * h and max(ws) - min(ws) <= 1
                for a, w in enumerate(ws):
                    inside = [(e - one.edges[a]) % L for e in other.edges if (e - one.edges[a]) % L < w]
                    assert len(inside) == 1
                    assert h <= inside[0] <= w - h
