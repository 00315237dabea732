"""GPU parity: the HIP path (through the C ABI) against the oracle.

Bit-exact for every scheme in FP64 and for the FP32-compensated schemes
against the FP32-compensated oracle (both sides evaluate the same expressions
with contraction off). Cases span several tiles, ragged remainders (sub-step
counts that are not multiples of the half-cycle height), odd half heights,
single-tile grids and the degenerate tile side 2.
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


def gpu_run(pde, state, params, nsteps, tile=0, prec=sw.FP64, method="swept", T=0, mode=sw.LAUNCH_DIRECT,
            staging=sw.STAGING_AUTO):
    nvars, ny, nx = state.shape
    _say(si.PDE_NAMES[pde], f"{nx}x{ny}", "tile", tile, "steps", nsteps, "prec", prec, method, "T", T, "mode", mode,
         "staging", staging)
    with sw.Swept2D(nx, ny, pde, params, prec=prec, tile=tile) as g:
        g.set_launch_mode(mode)
        g.set_staging(staging)
        if T:
            g.T = T
        if prec == sw.FP64:
            g.upload(state)
        else:
            g.upload_raw(state)
        (g.advance if method == "swept" else g.plain_advance)(nsteps)
        g.synchronize()
        return g.download_raw()


def tiles_of(nx, ny, limit=64):
    return [n for n in range(2, min(nx, ny, limit) + 1, 2) if nx % n == 0 and ny % n == 0]


# ------------------------------------------------------------ hash stencil

HASH_GRIDS = [(8, 8), (16, 16), (24, 16), (12, 12), (32, 32), (18, 12), (64, 32)]


@pytest.mark.parametrize("staging", [sw.STAGING_AUTO, sw.STAGING_OFF, sw.STAGING_SINGLE_BRIDGES, sw.STAGING_ON])
@pytest.mark.parametrize("nx,ny", HASH_GRIDS)
def test_hash_every_tile_and_remainder(nx, ny, staging):
    s0 = si.hash_field(nx, ny, seed=nx * 100 + ny)
    for n in tiles_of(nx, ny):
        h = n // 2
        counts = sorted({1, 2, max(1, h - 1), h, h + 1, n, n + 1, 3 * h, 3 * n + 1})
        for S in counts:
            ref = oracle.advance_f64(si.TEST_HASH, s0, [], S, t0=5)
            got = gpu_run(si.TEST_HASH, s0, [], S, tile=n, T=5, staging=staging)
            assert np.array_equal(got, ref), (nx, ny, n, S)


def test_hash_large_tiles_both_paths():
    """Tile sides 64 and 96 (panel runs longer than one wave) on several tiles,
    staged and fetched, bridges paired and single."""
    for (nx, ny, n) in [(128, 64, 64), (192, 96, 96)]:
        s0 = si.hash_field(nx, ny, seed=n)
        for S in (n // 2 + 3, 2 * n + 1):
            ref = oracle.advance_f64(si.TEST_HASH, s0, [], S, t0=1)
            for staging in (sw.STAGING_AUTO, sw.STAGING_OFF, sw.STAGING_SINGLE_BRIDGES, sw.STAGING_ON):
                got = gpu_run(si.TEST_HASH, s0, [], S, tile=n, T=1, staging=staging)
                assert np.array_equal(got, ref), (nx, ny, n, S, staging)


@pytest.mark.parametrize("nx,ny", [(16, 16), (24, 16), (66, 34), (15, 9), (130, 3), (2, 2)])
def test_hash_plain(nx, ny):
    s0 = si.hash_field(nx, ny, seed=3)
    for S in (1, 2, 7):
        ref = oracle.advance_f64(si.TEST_HASH, s0, [], S, t0=2)
        assert np.array_equal(gpu_run(si.TEST_HASH, s0, [], S, method="plain", T=2), ref)


def test_incr_every_value_is_at_its_level():
    s0 = si.incr_field(48, 32)
    for n in (4, 8, 16):
        for S in (5, 8, 13):
            got = gpu_run(si.TEST_INCR, s0, [], S, tile=n)
            assert np.all(got == 1.0 + S), (n, S)


def test_zero_steps_is_identity():
    s0 = si.hash_field(16, 16, seed=9)
    assert np.array_equal(gpu_run(si.TEST_HASH, s0, [], 0, tile=8), s0)


# ------------------------------------------------------------------- heat

def test_heat_64x64_1000_steps_every_tile():
    """The 64x64 heat workload: swept with every tile side, and the per-step
    kernel, equal the oracle bit for bit."""
    s0 = si.heat_field(64, 64, seed=0)
    p = si.default_params(si.HEAT5)
    ref = oracle.advance_f64(si.HEAT5, s0, p, 1000)
    for n in (2, 4, 8, 16, 32, 64):
        assert np.array_equal(gpu_run(si.HEAT5, s0, p, 1000, tile=n), ref), n
        assert np.array_equal(gpu_run(si.HEAT5, s0, p, 1000, tile=n, staging=sw.STAGING_OFF), ref), n
        assert np.array_equal(gpu_run(si.HEAT5, s0, p, 1000, tile=n, staging=sw.STAGING_SINGLE_BRIDGES), ref), n
        assert np.array_equal(gpu_run(si.HEAT5, s0, p, 1000, tile=n, staging=sw.STAGING_ON), ref), n
    assert np.array_equal(gpu_run(si.HEAT5, s0, p, 1000, method="plain"), ref)


def test_heat_ragged_grid_and_counts():
    s0 = si.heat_field(96, 80, seed=1)
    p = si.default_params(si.HEAT5)
    for S in (37, 101):
        ref = oracle.advance_f64(si.HEAT5, s0, p, S)
        for n in (4, 8, 16):
            assert np.array_equal(gpu_run(si.HEAT5, s0, p, S, tile=n), ref), (n, S)


def test_heat_split_advances_and_repeat():
    s0 = si.heat_field(128, 64, seed=2)
    p = si.default_params(si.HEAT5)
    ref = oracle.advance_f64(si.HEAT5, s0, p, 77)
    with sw.Swept2D(128, 64, si.HEAT5, p, tile=32) as g:
        for _ in range(2):
            g.upload(s0)
            g.T = 0
            g.advance(13)
            g.advance(40)
            g.plain_advance(3)
            g.advance(21)
            assert g.T == 77
            assert np.array_equal(g.download(), ref)


def test_graph_replay_matches_direct():
    """Graph mode replays one captured graph per step count at any level;
    every replay, with eager work and host synchronisation in between, must
    equal the direct launches."""
    s0 = si.heat_field(64, 64, seed=4)
    p = si.default_params(si.HEAT5)
    with sw.Swept2D(64, 64, si.HEAT5, p, tile=16) as g:
        g.upload(s0)
        g.set_launch_mode(sw.LAUNCH_GRAPH)
        cur = s0
        for rep in range(4):
            g.advance(24)
            g.synchronize()
            cur = oracle.advance_f64(si.HEAT5, cur, p, 24)
            assert np.array_equal(g.download(), cur), rep
            g.plain_advance(5)
            g.synchronize()
            cur = oracle.advance_f64(si.HEAT5, cur, p, 5)
            assert np.array_equal(g.download(), cur), rep
    hs = si.hash_field(32, 32, seed=4)
    with sw.Swept2D(32, 32, si.TEST_HASH, [], tile=8) as g:
        g.upload(hs)
        g.set_launch_mode(sw.LAUNCH_GRAPH)
        for rep in range(3):
            g.advance(11)
            g.synchronize()
            hs = oracle.advance_f64(si.TEST_HASH, hs, [], 11, t0=11 * rep)
            assert np.array_equal(g.download(), hs), rep


def test_torch_bound_state():
    import torch
    s0 = si.heat_field(64, 32, seed=5)
    p = si.default_params(si.HEAT5)
    ref = oracle.advance_f64(si.HEAT5, s0, p, 50)
    t = torch.tensor(s0, device="cuda:0")
    with sw.Swept2D(64, 32, si.HEAT5, p, tile=16) as g:
        g.bind_tensor(t)
        g.advance(50)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), ref)
        g.plain_advance(1)
        g.synchronize()
        assert np.array_equal(t.cpu().numpy(), oracle.advance_f64(si.HEAT5, ref, p, 1))
        g.unbind()


def test_torch_default_stream_ordering():
    """Bound to torch's default stream (the HIP null stream), launches are
    ordered with torch work on it: a copy queued just before an advance is
    seen by it, and a read queued just after sees its result, with only
    stream-level synchronisation. A long torch product ahead of the copy
    keeps the stream busy, so a launch on an unordered stream would run
    before the copy lands."""
    import torch
    nx, ny = 256, 128
    s0 = si.heat_field(nx, ny, seed=6)
    p = si.default_params(si.HEAT5)
    src = torch.tensor(s0, device="cuda:0")
    a = torch.randn(4096, 4096, device="cuda:0")
    for launch_mode in (sw.LAUNCH_DIRECT, sw.LAUNCH_GRAPH):
        t = torch.zeros_like(src)
        with sw.Swept2D(nx, ny, si.HEAT5, p, tile=32) as g:
            g.set_launch_mode(launch_mode)
            g.bind_tensor(t)
            stream = torch.cuda.current_stream()
            assert stream.cuda_stream == 0
            for _ in range(3):
                a = a @ a / 64.0
            t.copy_(src)
            g.advance(40)
            out = t.clone()
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), oracle.advance_f64(si.HEAT5, s0, p, 40)), launch_mode
            g.unbind()


# ------------------------------------------------------------ other schemes

def test_wave_bitwise():
    s0 = si.wave_field(128, 64, seed=0, sigma=6.0)
    p = si.default_params(si.WAVE_LF)
    ref = oracle.advance_f64(si.WAVE_LF, s0, p, 300)
    for n in (8, 16, 32, 64):
        assert np.array_equal(gpu_run(si.WAVE_LF, s0, p, 300, tile=n), ref), n
    assert np.array_equal(gpu_run(si.WAVE_LF, s0, p, 300, method="plain"), ref)


def test_push5_equals_wide_stencil_path():
    s0 = si.push5_field(48, 32, seed=1)
    for n in (4, 8, 16):
        for steps in (1, 3, 8):
            ref = oracle.advance_f64(si.TEST_PUSH5, s0, [], 2 * steps)
            assert np.array_equal(gpu_run(si.TEST_PUSH5, s0, [], steps, tile=n), ref), (n, steps)
    ref = oracle.advance_f64(si.TEST_PUSH5, s0, [], 6)
    assert np.array_equal(gpu_run(si.TEST_PUSH5, s0, [], 3, method="plain"), ref)


def test_euler_bitwise():
    """Correctly rounded FP64 division and square root on both sides make the
    Rusanov update bit-exact."""
    s0 = si.euler_field(64, 64, seed=0)
    p = si.default_params(si.EULER_RUS_RK2, s0)
    ref = oracle.advance_f64(si.EULER_RUS_RK2, s0, p, 2 * 50)
    for n in (8, 16, 32):
        assert np.array_equal(gpu_run(si.EULER_RUS_RK2, s0, p, 50, tile=n), ref), n
    assert np.array_equal(gpu_run(si.EULER_RUS_RK2, s0, p, 50, tile=16, staging=sw.STAGING_OFF), ref)
    assert np.array_equal(gpu_run(si.EULER_RUS_RK2, s0, p, 50, method="plain"), ref)


def test_handles_on_concurrent_threads():
    """Handles are independent: eight host threads, each creating, advancing
    and reading back its own handle (heat, wave and both Euler schemes, FP64
    and FP32C, square and rectangular tiles) at the same time, each get the
    oracle's bits. The binding releases the interpreter lock in every
    library call, so the calls overlap."""
    import threading
    cases = [(si.HEAT5, 64, 64, 40, sw.FP64, 0), (si.WAVE_LF, 64, 32, 30, sw.FP64, 0),
             (si.EULER_RUS_RK2, 32, 32, 10, sw.FP64, 0), (si.EULER_FD_RK4, 32, 32, 6, sw.FP64, 0),
             (si.HEAT5, 45, 39, 25, sw.FP64, 3), (si.HEAT5, 64, 64, 40, sw.FP32C, 0),
             (si.EULER_FD_RK4, 48, 32, 5, sw.FP32C, 0), (si.WAVE_LF, 64, 64, 30, sw.FP32C, 0)]
    refs, inputs, params = [], [], []
    for pde, nx, ny, steps, prec, _ in cases:
        s0 = si.initial_state(pde, nx, ny, seed=11)
        p = si.default_params(pde, s0)
        params.append(p)
        m = si.PDE_SHAPE[pde][1]
        if prec == sw.FP64:
            inputs.append(s0)
            refs.append(oracle.advance_f64(pde, s0, p, m * steps))
        else:
            u, c = oracle.split_f32c(s0)
            inputs.append(np.concatenate([u, c]))
            refs.append(np.concatenate(oracle.advance_f32c(pde, u, c, p, m * steps)))
    results, errors = [None] * len(cases), []
    start = threading.Barrier(len(cases))

    def work(i):
        pde, nx, ny, steps, prec, rect = cases[i]
        try:
            start.wait()
            with sw.Swept2D(nx, ny, pde, params[i], prec=prec) as g:
                if rect:
                    g.rect = rect
                if prec == sw.FP64:
                    g.upload(inputs[i])
                else:
                    g.upload_raw(inputs[i])
                for part in (steps // 2, steps - steps // 2):
                    g.advance(part)
                g.synchronize()
                results[i] = g.download_raw()
        except Exception as e:  # reported below, with the case
            errors.append((i, repr(e)))

    _say("threads", len(cases))
    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i, (got, ref) in enumerate(zip(results, refs)):
        assert np.array_equal(got, ref), cases[i]


@pytest.mark.parametrize("staging", [sw.STAGING_ON, sw.STAGING_SINGLE_BRIDGES])
def test_euler_staged_paths_bitwise(staging):
    """The staged octahedra and bridges of the column walk (STAGING_ON
    stages whatever fits beside the window) in FP64 and FP32C."""
    s0 = si.euler_field(64, 64, seed=2)
    p = si.default_params(si.EULER_RUS_RK2, s0)
    ref = oracle.advance_f64(si.EULER_RUS_RK2, s0, p, 2 * 20)
    u, c = oracle.split_f32c(s0)
    ru, rc = oracle.advance_f32c(si.EULER_RUS_RK2, u, c, p, 2 * 20)
    for n in (8, 16, 32):
        assert np.array_equal(gpu_run(si.EULER_RUS_RK2, s0, p, 20, tile=n, staging=staging), ref), n
        got = gpu_run(si.EULER_RUS_RK2, np.concatenate([u, c]), p, 20, tile=n, prec=sw.FP32C, staging=staging)
        assert np.array_equal(got, np.concatenate([ru, rc])), n


# ------------------------------------------------------ FP32 compensated

@pytest.mark.parametrize("pde,nx,ny,steps,tiles", [
    (si.HEAT5, 64, 64, 300, (8, 32, 64)),
    (si.WAVE_LF, 64, 32, 200, (8, 16, 32)),
    (si.HEAT5, 128, 128, 150, (64,)),
    (si.WAVE_LF, 128, 128, 150, (16, 32, 64)),
    (si.EULER_RUS_RK2, 32, 32, 20, (8, 16, 32)),
])
def test_fp32c_bitwise_against_compensated_oracle(pde, nx, ny, steps, tiles):
    s0 = si.initial_state(pde, nx, ny, seed=3)
    p = si.default_params(pde, s0)
    u, c = oracle.split_f32c(s0)
    m = si.PDE_SHAPE[pde][1]
    ru, rc = oracle.advance_f32c(pde, u, c, p, m * steps)
    raw0 = np.concatenate([u, c])
    for n in tiles:
        got = gpu_run(pde, raw0, p, steps, tile=n, prec=sw.FP32C)
        assert np.array_equal(got[: s0.shape[0]], ru), n
        assert np.array_equal(got[s0.shape[0]:], rc), n
    got = gpu_run(pde, raw0, p, steps, prec=sw.FP32C, method="plain")
    assert np.array_equal(got, np.concatenate([ru, rc]))


# ------------------------------- FP32 with the compensation in a residency

STAGINGS = (sw.STAGING_AUTO, sw.STAGING_OFF, sw.STAGING_SINGLE_BRIDGES, sw.STAGING_ON)


@pytest.mark.parametrize("pde,nx,ny,steps,tiles", [
    (si.HEAT5, 64, 64, 300, (8, 16, 32, 64)),
    (si.WAVE_LF, 128, 64, 150, (8, 16, 32, 64)),
    (si.HEAT5, 96, 80, 37, (4, 8, 16)),
    (si.WAVE_LF, 36, 24, 29, (4, 6, 12)),
])
def test_fp32r_bitwise_against_residency_oracle(pde, nx, ny, steps, tiles):
    """Only u in the state and the panels, the compensations in the LDS
    windows: bit for bit the oracle that keeps a compensation exactly while
    one pyramid, bridge or octahedron computes the point, for every tile side
    and staging mode; the per-step method keeps none."""
    s0 = si.initial_state(pde, nx, ny, seed=4)
    p = si.default_params(pde)
    u0 = oracle.split_f32r(pde, s0)
    for n in tiles:
        ref = oracle.advance_f32r(pde, u0, p, steps, n)
        for staging in STAGINGS:
            got = gpu_run(pde, u0, p, steps, tile=n, prec=sw.FP32R, staging=staging)
            assert np.array_equal(got, ref), (n, staging)
    got = gpu_run(pde, u0, p, steps, prec=sw.FP32R, method="plain")
    assert np.array_equal(got, oracle.advance_f32r(pde, u0, p, steps, 0))


def test_fp32r_split_advances_restart_residencies():
    """Each advance starts from a state of values only, so an advance split
    in two equals two oracle advances."""
    s0 = si.heat_field(128, 64, seed=2)
    p = si.default_params(si.HEAT5)
    u = s0.astype(np.float32)
    with sw.Swept2D(128, 64, si.HEAT5, p, prec=sw.FP32R, tile=32) as g:
        g.upload_raw(u)
        g.advance(13)
        g.advance(40)
        got = g.download_raw()
    ref = oracle.advance_f32r(si.HEAT5, oracle.advance_f32r(si.HEAT5, u, p, 13, 32), p, 40, 32)
    assert np.array_equal(got, ref)
    assert not np.array_equal(got, oracle.advance_f32r(si.HEAT5, u, p, 53, 32))


# ------------------------------------------------------------------ errors

def test_error_codes():
    with sw.Swept2D(64, 48, si.HEAT5, [0.2]) as g:
        with pytest.raises(sw.Swept2DError) as e:
            g.tile = 20
        assert e.value.code == sw.EINVAL
        with pytest.raises(sw.Swept2DError):
            g.tile = 7
        with pytest.raises(sw.Swept2DError):
            g.advance(-1)
        with pytest.raises(sw.Swept2DError):
            sw.swept2d_set_params(g.h, [])
        with pytest.raises(sw.Swept2DError) as e:
            sw.swept2d_set_substep_counter(g.h, -2)
        assert e.value.code == sw.EINVAL
    with sw.Swept2D(16, 16, si.TEST_HASH, []) as g:
        with pytest.raises(sw.Swept2DError) as e:
            sw.swept2d_set_precision(g.h, sw.FP32C)
        assert e.value.code == sw.EUNSUPPORTED
