"""Batch API on the GPU: many grids in one persistent, graph-captured kernel.

Each grid of a batch must give exactly what the oracle gives for that grid
alone (bitwise: hash, heat, wave in FP64; FP32C against the FP32C oracle),
whatever tile side each grid runs with, per-step grids included, across
split advances and graph replays. The failure path (a dependency wait that
hits its limit) is forced from the host with a zero wait limit.
"""
import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu

# The batched persistent kernel's first device runs hung: its work loop, as
# compiled, sent lanes 1..63 of every wave back to the item barrier without
# lane 0 (the ticket taker), so a workgroup repeated one item forever. The
# loop now has one thread-0 region per round and a scalar exit (checked in
# the generated code), but the fixed kernel has not run on a device yet and
# the library refuses to launch it (EUNSUPPORTED). These tests run it; they
# stay skipped until it is verified.
KERNEL_PENDING = pytest.mark.skip(reason="batched persistent kernel disabled pending device verification "
                                         "after a hang in its work loop (fixed, not yet run)")


def _params(pde):
    return list(si.default_params(pde))


def _oracle(spec, state, steps, t0=0):
    prec = spec.get("prec", sw.FP64)
    if prec == sw.FP64:
        return oracle.advance_f64(spec["pde"], state, _params(spec["pde"]), steps, t0=t0,
                                  threads=oracle.default_threads())
    u, c = oracle.split_f32c(state)
    u, c = oracle.advance_f32c(spec["pde"], u, c, _params(spec["pde"]), steps, t0=t0,
                               threads=oracle.default_threads())
    return u.astype(np.float64) - c.astype(np.float64)


def _make(specs):
    grids = [dict(nx=s["nx"], ny=s["ny"], pde=s["pde"], prec=s.get("prec", sw.FP64), params=_params(s["pde"]))
             for s in specs]
    return sw.Swept2DBatch(grids)


def _inits(specs):
    return [si.initial_state(s["pde"], s["nx"], s["ny"], seed=s.get("seed", i)) for i, s in enumerate(specs)]


MIXED = [
    dict(nx=64, ny=64, pde=si.TEST_HASH),
    dict(nx=96, ny=48, pde=si.TEST_HASH),
    dict(nx=67, ny=45, pde=si.TEST_HASH),          # no even side divides: per-step
    dict(nx=100, ny=36, pde=si.HEAT5),
    dict(nx=128, ny=64, pde=si.HEAT5),
    dict(nx=80, ny=48, pde=si.WAVE_LF),
    dict(nx=64, ny=96, pde=si.HEAT5, prec=sw.FP32C),
    dict(nx=48, ny=80, pde=si.WAVE_LF, prec=sw.FP32C),
    dict(nx=32, ny=32, pde=si.HEAT5),
]


@KERNEL_PENDING
def test_mixed_batch_matches_oracle_per_grid():
    specs = MIXED
    inits = _inits(specs)
    with _make(specs) as b:
        assert b.tile(2) == 0  # 67 x 45: per-step
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        steps = 70
        b.advance(steps)
        b.synchronize()
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            got = b.download(i)
            ref = _oracle(spec, s0, steps)
            assert np.array_equal(got, ref), (i, spec, b.tile(i), np.abs(got - ref).max())
            assert b.T(i) == steps


@KERNEL_PENDING
@pytest.mark.parametrize("tiles", [
    [64, 48, -1, 4, 32, 16, 32, 16, 32],
    [32, 16, -1, 2, 64, 8, 16, 8, 16],
    [-1, -1, -1, -1, -1, -1, -1, -1, -1],
])
def test_explicit_tiles_and_per_step(tiles):
    specs = MIXED
    inits = _inits(specs)
    with _make(specs) as b:
        for i, n in enumerate(tiles):
            b.set_tile(i, n)
            assert b.tile(i) == (0 if n < 0 else n)
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(37)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 37)), (i, tiles[i])


@KERNEL_PENDING
def test_split_advances_and_graph_replay():
    specs = MIXED[:6]
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        for k in (13, 13, 13, 40, 1):  # the 13-step graph replays three times
            b.advance(k)
        total = 13 * 3 + 40 + 1
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, total)), i
            assert b.T(i) == total


@KERNEL_PENDING
def test_batch_equals_single_handles():
    """Each grid of a batch gives the bits of a single handle with the same
    tile side."""
    specs = [dict(nx=128, ny=128, pde=si.HEAT5), dict(nx=96, ny=64, pde=si.WAVE_LF, prec=sw.FP32C),
             dict(nx=64, ny=64, pde=si.HEAT5, prec=sw.FP32C)]
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(100)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            g = sw.Swept2D(spec["nx"], spec["ny"], spec["pde"], _params(spec["pde"]),
                           prec=spec.get("prec", sw.FP64), tile=b.tile(i))
            g.upload(s0)
            g.advance(100)
            assert np.array_equal(b.download(i), g.download()), i
            g.close()


@KERNEL_PENDING
def test_measured_autotune_keeps_results():
    specs = MIXED[:5]
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.autotune(sw.TUNE_MEASURE)
        for i, spec in enumerate(specs):
            n = b.tile(i)
            assert n == 0 or (spec["nx"] % n == 0 and spec["ny"] % n == 0 and n % 2 == 0), (i, n)
            # tuning leaves the states alone
            assert np.array_equal(b.download(i), inits[i] if spec.get("prec", sw.FP64) == sw.FP64
                                  else _oracle(spec, inits[i], 0))
        b.advance(45)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 45)), i


@KERNEL_PENDING
def test_uneven_batch_sampled_against_oracle():
    """The uneven 256-grid workload (sides multiples of 16 in 64..512, heat or
    wave, FP64 or FP32C) for a few half cycles, sampled grids against the
    oracle."""
    specs = si.batch_specs(256, seed=0)
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        steps = 48
        b.advance(steps)
        b.synchronize()
        rng = np.random.default_rng(7)
        for i in rng.choice(len(specs), size=6, replace=False):
            ref = _oracle(specs[i], inits[i], steps)
            assert np.array_equal(b.download(int(i)), ref), (int(i), specs[i], b.tile(int(i)))


@KERNEL_PENDING
def test_any_sides_batch():
    """Sides drawn from every integer: most grids fall back to the per-step
    method, the rest run swept; all exact."""
    specs = si.batch_specs(12, seed=3, lo=20, hi=90, quantum=1)
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(21)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 21)), (i, spec, b.tile(i))


@KERNEL_PENDING
def test_wait_limit_abort_is_reported_and_recoverable():
    specs = [dict(nx=256, ny=256, pde=si.TEST_HASH)]
    inits = _inits(specs)
    with _make(specs) as b:
        b.set_tile(0, 16)
        b.upload(0, inits[0])
        b.set_wait_limit(0)
        b.advance(64)
        with pytest.raises(sw.Swept2DError) as ei:
            b.synchronize()
        assert ei.value.code == sw.EABORTED
        b.set_wait_limit(2_000_000)
        b.upload(0, inits[0])
        t0 = b.T(0)
        b.advance(20)
        assert np.array_equal(b.download(0), _oracle(specs[0], inits[0], 20, t0=t0))


def test_batch_argument_errors():
    with pytest.raises(sw.Swept2DError):
        sw.swept2d_batch_create([64], [64], [si.EULER_RUS_RK2], [sw.FP64])
    with pytest.raises(sw.Swept2DError):
        sw.swept2d_batch_create([2], [64], [si.HEAT5], [sw.FP64], [[0.2]], 1)
    with _make([dict(nx=64, ny=48, pde=si.HEAT5)]) as b:
        with pytest.raises(sw.Swept2DError):
            b.set_tile(0, 32)  # does not divide 48
        with pytest.raises(sw.Swept2DError):
            b.advance(-1)
        with pytest.raises(sw.Swept2DError) as ei:
            b.advance(1)  # the persistent kernel is not launched
        assert ei.value.code == sw.EUNSUPPORTED
        with pytest.raises(sw.Swept2DError):
            b.set_tile(5, 16)
