"""GPU parity of the 3D swept rule (include/swept3d.h) against the 3D oracle,
bit for bit: the 27-point test hash (any misplaced neighbour or level changes
the result) at every even tile side that divides the grid, step counts that
end inside a half cycle, split advances and a nonzero starting sub-step; the
per-step method; 7-point heat at full size (128^3 at tile 16, 192^3 at tile
12); error codes.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu

HASH, HEAT = si.TEST_HASH27_3D, si.HEAT7_3D


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def run3(pde, state, params, steps, tile=0, method="swept", splits=None, T=0):
    nz, ny, nx = state.shape
    _say("3d", pde, f"{nx}x{ny}x{nz}", "tile", tile, "steps", steps, method, "splits", splits, "T", T)
    with sw.Swept3D(nx, ny, nz, pde, params, tile=tile) as g:
        if T:
            g.T = T
        g.upload(state)
        for part in (splits or [steps]):
            (g.advance if method == "swept" else g.plain_advance)(part)
        g.synchronize()
        return g.download(), g.tile


@pytest.mark.parametrize("shape,steps", [((16, 16, 16), 13), ((8, 12, 16), 7), ((24, 24, 24), 9), ((6, 6, 6), 5),
                                         ((18, 18, 36), 11)])
def test_hash27_every_tile_side(shape, steps):
    nz, ny, nx = shape
    s0 = si.hash3d_field(nx, ny, nz, seed=1)
    ref = oracle.advance3d_f64(HASH, s0, [], steps)
    sides = [n for n in range(2, 19, 2) if nx % n == 0 and ny % n == 0 and nz % n == 0]
    for n in sides:
        got, tile = run3(HASH, s0, [], steps, tile=n)
        assert tile == n and np.array_equal(got, ref), n
    got, _ = run3(HASH, s0, [], steps, method="plain")
    assert np.array_equal(got, ref)


def test_hash27_split_advances_and_start_step():
    s0 = si.hash3d_field(16, 16, 8, seed=2)
    ref = oracle.advance3d_f64(HASH, s0, [], 17, t0=5)
    got, _ = run3(HASH, s0, [], 17, tile=8, splits=[3, 1, 6, 7], T=5)
    assert np.array_equal(got, ref)
    got, _ = run3(HASH, s0, [], 17, tile=4, splits=[9, 8], T=5)
    assert np.array_equal(got, ref)


def test_heat7_default_tile_and_zero_steps():
    s0 = si.heat3d_field(32, 16, 24, seed=3)
    ref = oracle.advance3d_f64(HEAT, s0, [si.HEAT3D_R], 21)
    got, tile = run3(HEAT, s0, [si.HEAT3D_R], 21)
    assert tile == 8 and np.array_equal(got, ref)
    got, _ = run3(HEAT, s0, [si.HEAT3D_R], 0)
    assert np.array_equal(got, s0)


@pytest.mark.timeout(600)
def test_heat7_128_cubed_full_size():
    """128^3 at the default tile side (16), 200 steps, every point."""
    s0 = si.heat3d_field(128, 128, 128, seed=0)
    got, tile = run3(HEAT, s0, [si.HEAT3D_R], 200)
    ref = oracle.advance3d_f64(HEAT, s0, [si.HEAT3D_R], 200, threads=oracle.default_threads())
    assert tile == 16 and np.array_equal(got, ref)


@pytest.mark.timeout(600)
def test_heat7_192_cubed_default_tile_12():
    """192^3 at its default tile side (12, as the benchmark runs it), 64
    steps (eight half cycles, every downward pyramid but the last fused with
    the next upward pyramid), every point."""
    s0 = si.heat3d_field(192, 192, 192, seed=0)
    got, tile = run3(HEAT, s0, [si.HEAT3D_R], 64)
    ref = oracle.advance3d_f64(HEAT, s0, [si.HEAT3D_R], 64, threads=oracle.default_threads())
    assert tile == 12 and np.array_equal(got, ref)


def test_errors():
    with sw.Swept3D(12, 12, 12, HEAT, [si.HEAT3D_R]) as g:
        assert g.tile == 12
        for bad in (5, 8, 18, 20, 0):
            with pytest.raises(sw.Swept2DError):
                g.tile = bad
        assert g.tile == 12
    with pytest.raises(sw.Swept2DError):
        sw.Swept3D(12, 12, 12, 7)
    with sw.Swept3D(9, 9, 9, HASH) as g:
        assert g.tile == 0
        with pytest.raises(sw.Swept2DError):
            g.advance(1)
        g.plain_advance(1)
