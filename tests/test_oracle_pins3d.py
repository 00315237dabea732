"""Pins of the 3D oracle and of the 3D swept decomposition model (CPU).

The plain 3D stepper is pinned by closed forms (the discrete von Neumann
factor of the 7-point heat stencil, conservation, exact dyadic steps) and by
the locality and level seeding of the 27-point hash; planted mistakes in
either stencil fail these pins. The decomposition model (``oracle/swept_model3d.py``) must
reach plain stepping bit for bit on cube tilings of every even side that
divides the grid, for full and reduced half cycles and both tiling offsets,
and it must fail when the class groups run in another order or when a
component publishes a narrower band.
"""
import math

import numpy as np
import pytest

import oracle
import swept_inputs as si
from oracle import swept_model3d as m3

H7, HASH27 = si.HEAT7_3D, si.TEST_HASH27_3D


@pytest.mark.parametrize("shape,k,steps", [((8, 8, 8), (1, 2, 3), 7), ((6, 10, 12), (2, 0, 5), 4)])
def test_heat7_single_mode_von_neumann(shape, k, steps):
    nz, ny, nx = shape
    r = si.HEAT3D_R
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    th = [2 * math.pi * k[0] / nx, 2 * math.pi * k[1] / ny, 2 * math.pi * k[2] / nz]
    u0 = np.cos(th[0] * x + th[1] * y + th[2] * z)
    g = 1.0 + r * (2 * math.cos(th[0]) + 2 * math.cos(th[1]) + 2 * math.cos(th[2]) - 6.0)
    out = oracle.advance3d_f64(H7, u0, [r], steps)
    assert np.max(np.abs(out - g ** steps * u0)) < 1e-13


def test_heat7_mass_conserved_and_exact_on_dyadic_data():
    u0 = si.heat3d_field(12, 10, 8, seed=2)
    out = oracle.advance3d_f64(H7, u0, [si.HEAT3D_R], 40)
    assert abs(out.sum() - u0.sum()) < 1e-11
    # small integers with r = 1/8: every operation exact, so compare with
    # integer arithmetic scaled by 8 per step
    q = np.random.default_rng(1).integers(-8, 9, (4, 6, 6)).astype(np.float64)
    got = oracle.advance3d_f64(H7, q, [0.125], 1)
    lap = sum(np.roll(q, s, axis=a) for a in range(3) for s in (1, -1)) - 6 * q
    assert np.array_equal(got * 8, q * 8 + lap)


def test_hash27_is_local_to_the_neighbourhood():
    u0 = si.hash3d_field(11, 9, 7, seed=3)
    base = oracle.advance3d_f64(HASH27, u0, [], 2)
    v = u0.copy()
    v[3, 4, 5] += 1.0
    out = oracle.advance3d_f64(HASH27, v, [], 2)
    diff = np.argwhere(out != base)
    assert diff.min(axis=0).tolist() == [1, 2, 3] and diff.max(axis=0).tolist() == [5, 6, 7]
    assert len(diff) == 125


def test_hash27_is_seeded_with_the_sub_step_index():
    """A value computed at the wrong level must differ: the same
    neighbourhood hashed at sub-steps 0 and 1 gives different values."""
    u0 = si.hash3d_field(6, 5, 4, seed=8)
    a = oracle.advance3d_f64(HASH27, u0, [], 1, t0=0)
    b = oracle.advance3d_f64(HASH27, u0, [], 1, t0=1)
    assert np.all(a != b)
    # order-sensitive: exchanging two neighbours of a point changes its value
    w = u0.copy()
    w[2, 2, 2], w[2, 2, 3] = u0[2, 2, 3], u0[2, 2, 2]
    c = oracle.advance3d_f64(HASH27, w, [], 1, t0=0)
    assert c[2, 2, 2] != a[2, 2, 2] and c[2, 3, 3] != a[2, 3, 3]


@pytest.mark.parametrize("shape,n,steps", [((8, 8, 8), 4, 5), ((8, 12, 16), 4, 7), ((8, 8, 8), 8, 9),
                                          ((6, 6, 6), 2, 3), ((16, 8, 8), 8, 4), ((12, 12, 12), 6, 11),
                                          ((12, 12, 12), 6, 3)])
def test_model_equals_plain_stepping(shape, n, steps):
    h = si.hash3d_field(*shape[::-1], seed=4)
    assert np.array_equal(m3.swept3d(h, n, steps, m3.hash27), oracle.advance3d_f64(HASH27, h, [], steps))
    u = si.heat3d_field(*shape[::-1], seed=5)
    assert np.array_equal(m3.swept3d(u, n, steps, m3.heat7, [si.HEAT3D_R]),
                          oracle.advance3d_f64(H7, u, [si.HEAT3D_R], steps))


@pytest.mark.parametrize("groups", [((0,), (3, 5, 6), (1, 2, 4), (7,)), ((0, 1, 2, 4), (3, 5, 6), (7,)),
                                    ((0,), (1, 2, 4), (3, 5, 6, 7)), ((1, 2, 4), (0,), (3, 5, 6), (7,))])
def test_group_order_is_needed(groups):
    h = si.hash3d_field(16, 8, 8, seed=6)
    with pytest.raises(m3.OrderError):
        m3.swept3d(h, 8, 9, m3.hash27, groups=groups)


def test_two_wide_band_is_needed(monkeypatch):
    def narrow(shape, n, off, level):
        nz, ny, nx = shape
        out = np.zeros(shape, dtype=bool)
        for ax, L in ((2, nx), (1, ny), (0, nz)):
            d = m3._axis_geometry(L, n, off)[0]
            sl = [None, None, None]
            sl[ax] = slice(None)
            out |= (d == level)[tuple(sl)]
        return out
    monkeypatch.setattr(m3, "in_band", narrow)
    with pytest.raises(m3.OrderError):
        m3.swept3d(si.hash3d_field(16, 8, 8, seed=6), 8, 9, m3.hash27)


@pytest.mark.parametrize("n", [4, 8])
def test_component_volumes(n):
    h = n // 2
    shape = (n, n, 2 * n)
    counts = {}
    m3.swept3d(si.hash3d_field(2 * n, n, n, seed=7), n, h, m3.hash27, counts=counts)
    tiles = 2
    up = sum((n - 2 * l) ** 3 for l in range(1, h + 1))
    face = sum(2 * l * (n - 2 * l) ** 2 for l in range(1, h + 1))
    edge = sum((2 * l) ** 2 * (n - 2 * l) for l in range(1, h + 1))
    down = sum((2 * l) ** 3 for l in range(1, h + 1))
    assert counts == {0: tiles * up, 1: tiles * face, 2: tiles * face, 4: tiles * face, 3: tiles * edge,
                      5: tiles * edge, 6: tiles * edge, 7: tiles * down}
    assert up + 3 * face + 3 * edge + down == n ** 3 * h
