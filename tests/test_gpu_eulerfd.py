"""GPU parity of the paper's Euler discretisation (EULER_FD_RK4: skew-symmetric
central differences, four-stage Runge-Kutta as four sub-steps, 12 values per
point) against the oracle, bit for bit, in FP64 and in compensated FP32.

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
        splits=None, prec=sw.FP64):
    """Advance `state` (FP64 slots, or for FP32C the raw u planes then c
    planes) and return the raw device state."""
    _, ny, nx = state.shape
    _say("euler_fd_rk4", f"{nx}x{ny}", "prec", prec, "tile", tile, "rect", rect, "steps", nsteps, method,
         "mode", mode, "staging", staging, "splits", splits)
    with sw.Swept2D(nx, ny, EFD, params, prec=prec, tile=tile) as g:
        if rect:
            g.rect = rect
        g.set_launch_mode(mode)
        g.set_staging(staging)
        if prec == sw.FP64:
            g.upload(state)
        else:
            g.upload_raw(state)
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


@pytest.mark.parametrize("staging", [sw.STAGING_ON, sw.STAGING_SINGLE_BRIDGES, sw.STAGING_OFF])
def test_eulerfd_every_staging_mode_bitwise(staging):
    """AUTO never stages this scheme at tile side 16 (a staged workgroup
    would be alone on its compute unit); the staged octahedra and bridges
    that STAGING_ON selects give the same bits, in FP64 and FP32C."""
    s0 = _field(64, 32, 8)
    ref = oracle.advance_f64(EFD, s0, PRM, 4 * 11)
    got, tile, _ = run(s0, PRM, 11, tile=16, staging=staging)
    assert tile == 16 and np.array_equal(got, ref)
    raw0, ref32 = _f32c(s0, PRM, 4 * 11)
    got, _, _ = run(raw0, PRM, 11, tile=16, staging=staging, prec=sw.FP32C)
    assert np.array_equal(got, ref32)


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


def test_eulerfd_has_no_fp32r_form():
    with pytest.raises(sw.Swept2DError) as e:
        sw.Swept2D(64, 32, EFD, PRM, prec=sw.FP32R)
    assert e.value.code == sw.EUNSUPPORTED


# ------------------------------------------------------ FP32 compensated

def _f32c(state64, params, nsub):
    """Raw FP32C start (u = fl32(x), c = 0) and the oracle's raw result."""
    u, c = oracle.split_f32c(state64)
    ru, rc = oracle.advance_f32c(EFD, u, c, params, nsub, threads=oracle.default_threads())
    return np.concatenate([u, c]), np.concatenate([ru, rc])


def test_eulerfd_fp32c_square_tiles_bitwise():
    s0 = _field(64, 32, 5)
    raw0, ref = _f32c(s0, PRM, 4 * 13)
    for n in (2, 4, 8, 16):
        got, tile, _ = run(raw0, PRM, 13, tile=n, prec=sw.FP32C)
        assert tile == n and np.array_equal(got, ref), n
    got, _, _ = run(raw0, PRM, 13, tile=8, staging=sw.STAGING_OFF, prec=sw.FP32C)
    assert np.array_equal(got, ref)
    got, _, _ = run(raw0, PRM, 13, method="plain", prec=sw.FP32C)
    assert np.array_equal(got, ref)
    assert np.any(got[12:16])  # the compensations carry information


def test_eulerfd_fp32c_split_advances_graph_and_rect_tiles():
    s0 = _field(32, 32, 6)
    raw0, ref = _f32c(s0, PRM, 4 * 11)
    got, _, _ = run(raw0, PRM, 11, tile=8, splits=[3, 1, 5, 2], prec=sw.FP32C)
    assert np.array_equal(got, ref)
    got, _, _ = run(raw0, PRM, 11, tile=8, mode=sw.LAUNCH_GRAPH, splits=[4, 4, 3], prec=sw.FP32C)
    assert np.array_equal(got, ref)
    for nx, ny, hh, steps in ((45, 39, 3, 10), (45, 41, 10, 12)):
        raw0, ref = _f32c(_field(nx, ny, 7), PRM, 4 * steps)
        got, tile, rect = run(raw0, PRM, steps, rect=hh, prec=sw.FP32C)
        assert tile == 0 and rect == hh and np.array_equal(got, ref), (nx, ny, hh)


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


@pytest.mark.timeout(600)
def test_eulerfd_tunnel_1024x512_fp32c_full_size():
    """The tunnel in compensated FP32 with the default tiling, 100 steps:
    bit for bit the oracle at every point, and within 1e-12 (normwise, both
    momenta against the momentum scale since v starts at zero) of the FP64
    stepper run from the same start; the oracle measures about 3e-14 there,
    plain FP32 about 5e-8."""
    s0 = si.initial_state(EFD, 1024, 512, seed=0)
    p = si.default_params(EFD)
    raw0, ref = _f32c(s0, p, 4 * 100)
    got, tile, rect = run(raw0, p, 100, prec=sw.FP32C)
    assert np.array_equal(got, ref), (tile, rect)
    r64, _, _ = run(raw0[:12].astype(np.float64), p, 100)
    wide = got[:12].astype(np.float64) - got[12:].astype(np.float64)
    mom = max(np.max(np.abs(r64[1])), np.max(np.abs(r64[2])))
    for k, scale in ((0, np.max(np.abs(r64[0]))), (1, mom), (2, mom), (3, np.max(np.abs(r64[3])))):
        assert np.max(np.abs(wide[k] - r64[k])) <= 1e-12 * scale, k
