"""Full-size parity: the workloads at the sizes and step counts the
benchmark runs, in its launch configuration (default tile side, staged
panels, direct launches), against the oracle on every output point.

FP64: bit for bit (contraction off on both sides). FP32C and FP32R: the
normwise relative error against the FP64 oracle, max|x - x_ref| / max|x_ref|
per variable, must stay within 1e-6; both are also bitwise against their
FP32 oracles where those oracle runs are short enough.
"""
import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu

_ref_cache = {}


def _oracle64(key, pde, state, params, nsub):
    if key not in _ref_cache:
        _ref_cache[key] = oracle.advance_f64(pde, state, params, nsub, threads=oracle.default_threads())
    return _ref_cache[key]


def _normwise(x, ref):
    out = []
    for v in range(ref.shape[0]):
        out.append(float(np.abs(x[v] - ref[v]).max() / np.abs(ref[v]).max()))
    return max(out)


def _swept(pde, params, s0, steps, prec=sw.FP64):
    nvars, ny, nx = s0.shape
    with sw.Swept2D(nx, ny, pde, params, prec=prec) as g:
        g.upload(s0)
        g.advance(steps)
        return g.download(), g.tile


@pytest.mark.timeout(900)
def test_heat_1024_20000_steps_fp64_bitwise():
    s0 = si.heat_field(1024, 1024, seed=0)
    p = si.default_params(si.HEAT5)
    got, tile = _swept(si.HEAT5, p, s0, 20000)
    assert tile == 64
    ref = _oracle64("heat1024", si.HEAT5, s0, p, 20000)
    assert np.array_equal(got, ref)


@pytest.mark.timeout(900)
def test_heat_8192_fp64_bitwise():
    """The benchmark's grid beyond the Infinity Cache (512 MB of state; two
    64-tile workgroups per compute unit): 64 steps (two half cycles: the
    first pyramids, bridges, octahedra, bridges and the last downward
    pyramids) swept against the oracle at every point, and the benchmark's
    64 + 256 steps swept against the per-step kernel."""
    s0 = si.heat_field(8192, 8192, seed=0)
    p = si.default_params(si.HEAT5)
    got, tile = _swept(si.HEAT5, p, s0, 64)
    assert tile == 64
    ref = oracle.advance_f64(si.HEAT5, s0, p, 64, threads=oracle.default_threads())
    assert np.array_equal(got, ref)
    del got, ref
    res = {}
    for method in ("swept", "plain"):
        with sw.Swept2D(8192, 8192, si.HEAT5, p) as g:
            g.upload(s0)
            (g.advance if method == "swept" else g.plain_advance)(64)
            (g.advance if method == "swept" else g.plain_advance)(256)
            res[method] = g.download()
    assert np.array_equal(res["swept"], res["plain"])


@pytest.mark.timeout(900)
def test_heat_1024_20000_steps_fp32c_error():
    s0 = si.heat_field(1024, 1024, seed=0)
    p = si.default_params(si.HEAT5)
    got, _ = _swept(si.HEAT5, p, s0, 20000, prec=sw.FP32C)
    ref = _oracle64("heat1024", si.HEAT5, s0, p, 20000)
    err = _normwise(got, ref)
    print(f"heat 1024^2 FP32C after 20000 steps: normwise relative error {err:.3e}")
    assert err <= 1e-6


def test_heat_1024_fp32c_bitwise_against_compensated_oracle():
    s0 = si.heat_field(1024, 1024, seed=0)
    p = si.default_params(si.HEAT5)
    got, _ = _swept(si.HEAT5, p, s0, 2000, prec=sw.FP32C)
    u, c = oracle.split_f32c(s0)
    u, c = oracle.advance_f32c(si.HEAT5, u, c, p, 2000, threads=oracle.default_threads())
    assert np.array_equal(got, u.astype(np.float64) - c.astype(np.float64))


@pytest.mark.timeout(900)
def test_heat_1024_20000_steps_fp32r_error_and_bitwise():
    """FP32 values only in HBM (the compensations stay in the LDS windows):
    within 1e-6 of the FP64 oracle after the full 20000 steps, and bit for
    bit the residency oracle over the first 2000."""
    s0 = si.heat_field(1024, 1024, seed=0)
    p = si.default_params(si.HEAT5)
    got, tile = _swept(si.HEAT5, p, s0, 20000, prec=sw.FP32R)
    assert tile == 64
    ref = _oracle64("heat1024", si.HEAT5, s0, p, 20000)
    err = _normwise(got, ref)
    print(f"heat 1024^2 FP32R after 20000 steps: normwise relative error {err:.3e}")
    assert err <= 1e-6
    got2, _ = _swept(si.HEAT5, p, s0, 2000, prec=sw.FP32R)
    u = oracle.advance_f32r(si.HEAT5, s0.astype(np.float32), p, 2000, 64, threads=oracle.default_threads())
    assert np.array_equal(got2, u.astype(np.float64))


WAVE_STEPS = 10000


@pytest.mark.timeout(900)
def test_wave_2048_10000_steps_fp64_bitwise():
    s0 = si.wave_field(2048, 2048, seed=0)
    p = si.default_params(si.WAVE_LF)
    got, tile = _swept(si.WAVE_LF, p, s0, WAVE_STEPS)
    assert tile == 64
    ref = _oracle64("wave2048", si.WAVE_LF, s0, p, WAVE_STEPS)
    assert np.array_equal(got, ref), tile


@pytest.mark.timeout(900)
def test_wave_2048_10000_steps_fp32c_error():
    s0 = si.wave_field(2048, 2048, seed=0)
    p = si.default_params(si.WAVE_LF)
    got32, _ = _swept(si.WAVE_LF, p, s0, WAVE_STEPS, prec=sw.FP32C)
    ref = _oracle64("wave2048", si.WAVE_LF, s0, p, WAVE_STEPS)
    err = _normwise(got32, ref)
    print(f"wave 2048^2 FP32C after {WAVE_STEPS} steps: normwise relative error {err:.3e}")
    assert err <= 1e-6


@pytest.mark.timeout(900)
def test_wave_2048_10000_steps_fp32r_error_and_bitwise():
    """FP32 values only in HBM, the wave in velocity form: within 1e-6 of the
    FP64 oracle after the full 10000 steps at the benchmark's tile side, and
    bit for bit the residency oracle over the first 100."""
    s0 = si.wave_field(2048, 2048, seed=0)
    p = si.default_params(si.WAVE_LF)
    got, tile = _swept(si.WAVE_LF, p, s0, WAVE_STEPS, prec=sw.FP32R)
    assert tile == 64
    ref = _oracle64("wave2048", si.WAVE_LF, s0, p, WAVE_STEPS)
    err = _normwise(got, ref)
    print(f"wave 2048^2 FP32R after {WAVE_STEPS} steps: normwise relative error {err:.3e}")
    assert err <= 1e-6
    got2, _ = _swept(si.WAVE_LF, p, s0, 100, prec=sw.FP32R)
    u = oracle.advance_f32r(si.WAVE_LF, oracle.split_f32r(si.WAVE_LF, s0), p, 100, 64,
                            threads=oracle.default_threads())
    assert np.array_equal(got2, oracle.join_f32r(si.WAVE_LF, u))


@pytest.mark.timeout(900)
def test_wave_2048_fp32c_bitwise_against_compensated_oracle():
    """The benchmark's wave path (tile side 64, 1024 tiles) in FP32C, bit for
    bit against the FP32C oracle."""
    s0 = si.wave_field(2048, 2048, seed=0)
    p = si.default_params(si.WAVE_LF)
    got, tile = _swept(si.WAVE_LF, p, s0, 1000, prec=sw.FP32C)
    assert tile == 64
    u, c = oracle.split_f32c(s0)
    u, c = oracle.advance_f32c(si.WAVE_LF, u, c, p, 1000, threads=oracle.default_threads())
    assert np.array_equal(got, u.astype(np.float64) - c.astype(np.float64))


@pytest.mark.timeout(900)
def test_euler_512_5000_steps_fp64_bitwise_and_fp32c_error():
    s0 = si.euler_field(512, 512, seed=0)
    p = si.default_params(si.EULER_RUS_RK2, s0)
    got, tile = _swept(si.EULER_RUS_RK2, p, s0, 5000)
    ref = _oracle64("euler512", si.EULER_RUS_RK2, s0, p, 10000)
    assert np.array_equal(got, ref), tile
    got32, _ = _swept(si.EULER_RUS_RK2, p, s0, 5000, prec=sw.FP32C)
    err = _normwise(got32[:4], ref[:4])
    print(f"euler 512^2 FP32C after 5000 steps: normwise relative error {err:.3e}")
    assert err <= 1e-6
