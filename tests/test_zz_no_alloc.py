"""swept2d_advance_noalloc (panels in the library's static device array)
against swept2d_advance (panels allocated per handle), through the C ABI.

Two calls in a row share the static array, the second on a smaller grid; each
must equal the handle's advance of the same state bit for bit (and the oracle
where it is cheap). A grid whose panels exceed the array is rejected on the
host before any launch, leaving the state untouched.
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


def _handle_advance(pde, prec, params, s0, tile, T, nsteps):
    nvars, ny, nx = s0.shape
    with sw.Swept2D(nx, ny, pde, params, prec=prec, tile=tile) as g:
        g.T = T
        g.upload(s0)
        g.advance(nsteps)
        return g.download_raw()


def _noalloc_advance(pde, prec, params, s0, tile, T, nsteps, stream=None):
    import torch
    nvars, ny, nx = s0.shape
    with sw.Swept2D(nx, ny, pde, params, prec=prec) as g:
        g.upload(s0)
        raw = g.download_raw()          # the state in the precision's layout
    t = torch.from_numpy(raw).to("cuda:0")
    torch.cuda.synchronize()
    sw.swept2d_advance_noalloc(nx, ny, pde, prec, params, tile, t.data_ptr(), T, nsteps, stream)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_equals_handle_advance_two_calls():
    import torch
    # Call 1: the heat benchmark grid, FP64, tile side 64 (34.6 MB of panels),
    # a step count that ends in a reduced half cycle.
    s1 = si.heat_field(1024, 1024, seed=0)
    p1 = si.default_params(si.HEAT5)
    _say("noalloc heat 1024x1024 fp64 tile 64 steps 300")
    a = _noalloc_advance(si.HEAT5, sw.FP64, p1, s1, 64, 0, 300)
    b = _handle_advance(si.HEAT5, sw.FP64, p1, s1, 64, 0, 300)
    assert np.array_equal(a, b)
    # Call 2: a smaller grid, another scheme, a nonzero level, on a torch
    # side stream; the array still holds call 1's panels.
    s2 = si.hash_field(96, 64, seed=4)
    _say("noalloc hash 96x64 tile 16 T 5 steps 37")
    side = torch.cuda.Stream()
    a = _noalloc_advance(si.TEST_HASH, sw.FP64, [], s2, 16, 5, 37, stream=side.cuda_stream)
    b = _handle_advance(si.TEST_HASH, sw.FP64, [], s2, 16, 5, 37)
    assert np.array_equal(a, b)
    assert np.array_equal(a, oracle.advance_f64(si.TEST_HASH, s2, [], 37, t0=5))


def test_noalloc_fp32c_and_model_tile():
    s0 = si.wave_field(256, 128, seed=2, sigma=8.0)
    p = si.default_params(si.WAVE_LF)
    _say("noalloc wave 256x128 fp32c tile 32 steps 70")
    a = _noalloc_advance(si.WAVE_LF, sw.FP32C, p, s0, 32, 0, 70)
    b = _handle_advance(si.WAVE_LF, sw.FP32C, p, s0, 32, 0, 70)
    assert np.array_equal(a, b)
    _say("noalloc heat 128x128 fp64 model tile steps 45")
    s1 = si.heat_field(128, 128, seed=3)
    p1 = si.default_params(si.HEAT5)
    a = _noalloc_advance(si.HEAT5, sw.FP64, p1, s1, 0, 0, 45)
    assert np.array_equal(a[0], oracle.advance_f64(si.HEAT5, s1, p1, 45)[0])


def test_noalloc_euler_schemes_two_calls():
    """The column-walk schemes: the central-difference Euler scheme in FP64
    (12 values per point, four sub-steps), then a smaller Rusanov grid in
    FP32C on the same static array."""
    efd = si.EULER_FD_RK4
    s1 = si.eulerfd_field(256, 128, seed=6, amp=0.2, width=4.0)
    p1 = si.default_params(efd)
    _say("noalloc euler_fd 256x128 fp64 tile 16 steps 21")
    a = _noalloc_advance(efd, sw.FP64, p1, s1, 16, 0, 21)
    b = _handle_advance(efd, sw.FP64, p1, s1, 16, 0, 21)
    assert np.array_equal(a, b)
    assert np.array_equal(a, oracle.advance_f64(efd, s1, p1, 4 * 21))
    s2 = si.euler_field(64, 64, seed=7)
    p2 = si.default_params(si.EULER_RUS_RK2, s2)
    _say("noalloc euler_rus 64x64 fp32c tile 16 steps 13")
    a = _noalloc_advance(si.EULER_RUS_RK2, sw.FP32C, p2, s2, 16, 0, 13)
    b = _handle_advance(si.EULER_RUS_RK2, sw.FP32C, p2, s2, 16, 0, 13)
    assert np.array_equal(a, b)
    u, c = oracle.split_f32c(s2)
    assert np.array_equal(a, np.concatenate(oracle.advance_f32c(si.EULER_RUS_RK2, u, c, p2, 2 * 13)))


def test_noalloc_rejects_grids_beyond_the_static_array():
    import torch
    s0 = si.wave_field(2048, 2048, seed=0)
    t = torch.tensor(s0, device="cuda:0")
    before = t.clone()
    with pytest.raises(sw.Swept2DError) as e:
        sw.swept2d_advance_noalloc(2048, 2048, si.WAVE_LF, sw.FP64, si.default_params(si.WAVE_LF), 64,
                                   t.data_ptr(), 0, 10)
    assert e.value.code == sw.EINVAL and "static scratch" in str(e.value)
    with pytest.raises(sw.Swept2DError) as e:
        sw.swept2d_advance_noalloc(2048, 2048, si.WAVE_LF, sw.FP64, si.default_params(si.WAVE_LF), 48,
                                   t.data_ptr(), 0, 10)
    assert e.value.code == sw.EINVAL
    torch.cuda.synchronize()
    assert torch.equal(t, before)
