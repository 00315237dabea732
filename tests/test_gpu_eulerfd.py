"""GPU parity of the paper's Euler discretisation (EULER_FD_RK4: skew-symmetric
central differences, four-stage Runge-Kutta as four sub-steps, 12 FP64 values
per point) against the oracle, bit for bit.

Square tiles of every side whose window fits the LDS, staged and unstaged
panels, step counts that end inside a half cycle, split advances that start
mid-step, graph replay, rectangular tiles on odd grids, per-step stepping, and
the paper's 1024 x 512 tunnel at full size in the benchmark's configuration.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu

EFD = si.EULER_FD_RK4


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def run(state, params, nsteps, tile=0, rect=0, method="swept", mode=sw.LAUNCH_DIRECT, staging=sw.STAGING_AUTO,
        splits=None):
    nvars, ny, nx = state.shape
    _say("euler_fd_rk4", f"{nx}x{ny}", "tile", tile, "rect", rect, "steps", nsteps, method, "mode", mode,
         "staging", staging, "splits", splits)
    with sw.Swept2D(nx, ny, EFD, params, tile=tile) as g:
        if rect:
            g.rect = rect
        g.set_launch_mode(mode)
        g.set_staging(staging)
        g.upload(state)
        for part in (splits or [nsteps]):
            (g.advance if method == "swept" else g.plain_advance)(part)
        g.synchronize()
        return g.download_raw(), g.tile, g.rect


def _field(nx, ny, seed):
    # a stronger pulse than the tunnel's (the small grids see few steps)
    return si.eulerfd_field(nx, ny, seed=seed, amp=0.2, width=3.0)


PRM = [1.4, 2e-4]


@pytest.mark.parametrize("nx,ny,steps", [(64, 32, 13), (48, 48, 7), (16, 16, 9)])
def test_eulerfd_square_tiles_bitwise(nx, ny, steps):
    s0 = _field(nx, ny, 1)
    ref = oracle.advance_f64(EFD, s0, PRM, 4 * steps)
    for n in (2, 4, 8, 16):
        if nx % n or ny % n:
            continue
        got, tile, _ = run(s0, PRM, steps, tile=n)
        assert tile == n and np.array_equal(got, ref), n
    got, _, _ = run(s0, PRM, steps, tile=8, staging=sw.STAGING_OFF)
    assert np.array_equal(got, ref)
    got, _, _ = run(s0, PRM, steps, method="plain")
    assert np.array_equal(got, ref)


def test_eulerfd_split_advances_and_graph_replay():
    s0 = _field(32, 32, 2)
    ref = oracle.advance_f64(EFD, s0, PRM, 4 * 11)
    got, _, _ = run(s0, PRM, 11, tile=8, splits=[3, 1, 5, 2])
    assert np.array_equal(got, ref)
    got, _, _ = run(s0, PRM, 11, tile=8, mode=sw.LAUNCH_GRAPH, splits=[4, 4, 3])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("nx,ny,hh,steps", [(45, 39, 3, 10), (37, 64, 4, 9), (21, 21, 2, 6), (45, 41, 10, 12)])
def test_eulerfd_rect_tiles_bitwise(nx, ny, hh, steps):
    s0 = _field(nx, ny, 3)
    ref = oracle.advance_f64(EFD, s0, PRM, 4 * steps)
    got, tile, rect = run(s0, PRM, steps, rect=hh)
    assert tile == 0 and rect == hh and np.array_equal(got, ref)


def test_eulerfd_uniform_free_stream_unchanged():
    c0 = np.sqrt(1.4 * si.EULERFD_P / si.EULERFD_RHO)
    s0 = si.eulerfd_state(si.eulerfd_conserved(*(np.full((32, 64), x) for x in (
        si.EULERFD_RHO, si.EULERFD_MACH * c0, 0.0, si.EULERFD_P))))
    got, _, _ = run(s0, si.default_params(EFD), 17, tile=16)
    assert np.array_equal(got, s0)


def test_eulerfd_has_no_fp32_forms():
    for prec in (sw.FP32C, sw.FP32R):
        with pytest.raises(sw.Swept2DError) as e:
            sw.Swept2D(64, 32, EFD, PRM, prec=prec)
        assert e.value.code == sw.EUNSUPPORTED


@pytest.mark.timeout(600)
def test_eulerfd_tunnel_1024x512_full_size_bitwise():
    """The paper's tunnel grid and time step in the benchmark's configuration
    (default tiling), 500 steps (2000 sub-steps), every output point."""
    s0 = si.initial_state(EFD, 1024, 512, seed=0)
    p = si.default_params(EFD)
    got, tile, rect = run(s0, p, 500)
    ref = oracle.advance_f64(EFD, s0, p, 4 * 500, threads=oracle.default_threads())
    assert np.array_equal(got, ref), (tile, rect)
    assert np.max(np.abs(got[0] - s0[0])) > 1e-6  # the pulse has moved
