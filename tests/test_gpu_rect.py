"""GPU parity of the rectangular tiles (swept2d_set_rect) against the oracle.

Grids of odd, prime and uneven sides that no even square tile side divides,
tiles wider than 2h (frustums whose tops and bridge middles pass through the
state), single-tile axes, ragged step counts, split advances, graph replay,
every built-in scheme that runs them (FP64 and FP32C): bit for bit against
plain stepping in the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rect_run(pde, state, params, nsteps, hh, prec=sw.FP64, T=0, mode=sw.LAUNCH_DIRECT, splits=None):
    nvars, ny, nx = state.shape
    _say(si.PDE_NAMES[pde], f"{nx}x{ny}", "rect", hh, "steps", nsteps, "prec", prec, "T", T, "mode", mode)
    with sw.Swept2D(nx, ny, pde, params, prec=prec) as g:
        g.rect = hh
        assert g.rect == hh and g.tile == 0
        g.set_launch_mode(mode)
        if T:
            g.T = T
        if prec == sw.FP64:
            g.upload(state)
        else:
            g.upload_raw(state)
        for part in (splits or [nsteps]):
            g.advance(part)
        g.synchronize()
        return g.download_raw()


RECT_GRIDS = [(11, 9), (13, 17), (9, 9), (31, 29), (37, 64), (64, 37), (97, 89), (130, 67), (21, 21), (16, 16)]


@pytest.mark.parametrize("nx,ny", RECT_GRIDS)
def test_rect_hash_every_height_and_remainder(nx, ny):
    s0 = si.hash_field(nx, ny, seed=nx * 1000 + ny)
    for hh in sorted({1, 2, 3, 4, 5, 8, 16, min(nx, ny) // 2}):
        if 2 * hh > min(nx, ny) or hh > 32:
            continue
        for S in sorted({1, hh, hh + 1, 3 * hh + 2, 7 * hh}):
            ref = oracle.advance_f64(si.TEST_HASH, s0, [], S, t0=5)
            got = rect_run(si.TEST_HASH, s0, [], S, hh, T=5)
            assert np.array_equal(got, ref), (nx, ny, hh, S)


def test_rect_heat_and_wave_fp64():
    for pde, (nx, ny), hh, steps in [(si.HEAT5, (97, 89), 8, 1000), (si.HEAT5, (255, 129), 16, 300),
                                     (si.WAVE_LF, (67, 61), 6, 500), (si.WAVE_LF, (129, 257), 32, 200)]:
        s0 = si.initial_state(pde, nx, ny, seed=2)
        prm = si.default_params(pde)
        ref = oracle.advance_f64(pde, s0, prm, steps)
        got = rect_run(pde, s0, prm, steps, hh)
        assert np.array_equal(got, ref), (pde, nx, ny, hh)


def test_rect_euler_and_push5_fp64():
    s0 = si.euler_field(45, 39, seed=1)
    prm = si.default_params(si.EULER_RUS_RK2, s0)
    ref = oracle.advance_f64(si.EULER_RUS_RK2, s0, prm, 2 * 30)
    got = rect_run(si.EULER_RUS_RK2, s0, prm, 30, 4)
    assert np.array_equal(got, ref)
    s0 = si.push5_field(23, 19, seed=3)
    ref = oracle.advance_f64(si.TEST_PUSH5, s0, [], 2 * 13)
    got = rect_run(si.TEST_PUSH5, s0, [], 13, 3)
    assert np.array_equal(got, ref)


def test_rect_euler_wide_tiles_fp64():
    """Tiles 20 and more wide (window pitch 22 and up): the Euler column walk
    on its 8-wave workgroups."""
    s0 = si.euler_field(61, 43, seed=4)
    prm = si.default_params(si.EULER_RUS_RK2, s0)
    ref = oracle.advance_f64(si.EULER_RUS_RK2, s0, prm, 2 * 25)
    got = rect_run(si.EULER_RUS_RK2, s0, prm, 25, 10)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("pde,nx,ny,steps,hh", [
    (si.HEAT5, 61, 47, 400, 5),
    (si.WAVE_LF, 53, 71, 300, 7),
    (si.EULER_RUS_RK2, 33, 35, 20, 4),
    (si.EULER_RUS_RK2, 49, 45, 12, 11),
])
def test_rect_fp32c_bitwise_against_compensated_oracle(pde, nx, ny, steps, hh):
    s0 = si.initial_state(pde, nx, ny, seed=5)
    prm = si.default_params(pde, s0)
    sub = si.PDE_SHAPE[pde][1]
    u, c = oracle.split_f32c(s0)
    uo, co = oracle.advance_f32c(pde, u, c, prm, steps * sub)
    got = rect_run(pde, np.concatenate([u, c]).astype(np.float32), prm, steps, hh, prec=sw.FP32C)
    nv = s0.shape[0]
    assert np.array_equal(got[:nv], uo) and np.array_equal(got[nv:], co)


def test_rect_split_advances_and_graph_replay():
    s0 = si.hash_field(59, 43, seed=9)
    ref = oracle.advance_f64(si.TEST_HASH, s0, [], 53, t0=2)
    got = rect_run(si.TEST_HASH, s0, [], 53, 4, T=2, splits=[1, 7, 4, 41])
    assert np.array_equal(got, ref)
    got = rect_run(si.TEST_HASH, s0, [], 53, 4, T=2, mode=sw.LAUNCH_GRAPH, splits=[10, 10, 10, 10, 13])
    assert np.array_equal(got, ref)


def test_rect_selected_when_no_square_side_divides():
    """A grid of odd sides gets rectangular tiles by default and through
    set_tile(0); a square side selected afterwards leaves them."""
    nx, ny = 101, 77
    s0 = si.heat_field(nx, ny, seed=1)
    prm = si.default_params(si.HEAT5)
    ref = oracle.advance_f64(si.HEAT5, s0, prm, 257)
    with sw.Swept2D(nx, ny, si.HEAT5, prm) as g:
        assert g.tile == 0 and g.rect > 0
        _say("default rect", g.rect)
        g.upload(s0)
        g.advance(257)
        g.synchronize()
        assert np.array_equal(g.download_raw(), ref)
    with sw.Swept2D(64, 48, si.HEAT5, prm) as g:
        assert g.tile > 0 and g.rect == 0
        g.rect = 5
        assert g.tile == 0 and g.rect == 5
        g.tile = 16
        assert g.tile == 16 and g.rect == 0


def test_rect_errors():
    with sw.Swept2D(20, 20, si.HEAT5, [si.HEAT_R]) as g:
        with pytest.raises(sw.Swept2DError) as e:
            g.rect = 11
        assert e.value.code == sw.EINVAL
    with sw.Swept2D(20, 20, si.HEAT5, [si.HEAT_R], prec=sw.FP32R) as g:
        with pytest.raises(sw.Swept2DError) as e:
            g.rect = 3
        assert e.value.code == sw.EUNSUPPORTED


def test_rect_full_size_heat_odd_grid():
    """Heat on 1023 x 1021 (no even square side divides it) for 2000 steps at
    the default rectangular tiles, against the oracle."""
    nx, ny, steps = 1023, 1021, 2000
    s0 = si.heat_field(nx, ny, seed=0)
    prm = si.default_params(si.HEAT5)
    ref = oracle.advance_f64(si.HEAT5, s0, prm, steps)
    with sw.Swept2D(nx, ny, si.HEAT5, prm) as g:
        _say("full size rect", g.rect)
        assert g.rect > 0
        g.upload(s0)
        g.advance(steps)
        g.synchronize()
        assert np.array_equal(g.download_raw(), ref)
