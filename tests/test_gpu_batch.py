"""Batch API on the GPU: many grids advanced together from one captured graph.

Each grid of a batch must give exactly what the oracle gives for that grid
alone (bitwise: hash, heat, wave in FP64; FP32C against the FP32C oracle),
whatever tile side (and hence launch class) each grid runs with, per-step
and rectangular-tile grids included, across split advances, graph replays and advances longer
than one graph. Every case runs in the phased mode (slots of launches, no
workgroup waits for another); the same cases in the persistent mode are
kept, skipped (see PERSISTENT_OFF).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu

# The persistent batch kernel hung on the device twice (its work loop, as
# compiled, sent lanes 1..63 of a wave back to the item barrier without lane
# 0, the ticket taker; a first fix did not cure it). It is not built into the
# library (advance returns EUNSUPPORTED in that mode); its cases stay here,
# skipped.
PERSISTENT_OFF = pytest.mark.skip(reason="persistent batch kernel hung on the device twice; not built, "
                                         "its mode returns EUNSUPPORTED")
MODES = [pytest.param(sw.BATCH_PHASED, id="phased"),
         pytest.param(sw.BATCH_PERSISTENT, id="persistent", marks=PERSISTENT_OFF)]


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


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


def _make(specs, mode=sw.BATCH_PHASED):
    grids = [dict(nx=s["nx"], ny=s["ny"], pde=s["pde"], prec=s.get("prec", sw.FP64), params=_params(s["pde"]))
             for s in specs]
    b = sw.Swept2DBatch(grids)
    b.set_mode(mode)
    return b


def _inits(specs):
    return [si.initial_state(s["pde"], s["nx"], s["ny"], seed=s.get("seed", i)) for i, s in enumerate(specs)]


MIXED = [
    dict(nx=64, ny=64, pde=si.TEST_HASH),
    dict(nx=96, ny=48, pde=si.TEST_HASH),
    dict(nx=67, ny=45, pde=si.TEST_HASH),          # no even side divides: rectangular tiles
    dict(nx=100, ny=36, pde=si.HEAT5),
    dict(nx=128, ny=64, pde=si.HEAT5),
    dict(nx=80, ny=48, pde=si.WAVE_LF),
    dict(nx=64, ny=96, pde=si.HEAT5, prec=sw.FP32C),
    dict(nx=48, ny=80, pde=si.WAVE_LF, prec=sw.FP32C),
    dict(nx=32, ny=32, pde=si.HEAT5),
]


@pytest.mark.parametrize("mode", MODES)
def test_mixed_batch_matches_oracle_per_grid(mode):
    specs = MIXED
    inits = _inits(specs)
    _say("mixed batch", len(specs), "grids, 70 steps, mode", mode)
    with _make(specs, mode) as b:
        assert b.tile(2) == 0 and b.rect(2) > 0  # 67 x 45: no even side divides, rectangular tiles
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


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("tiles", [
    [64, 48, -1, 4, 32, 16, 32, 16, 32],
    [32, 16, -1, 2, 64, 8, 16, 8, 16],
    [-1, -1, -1, -1, -1, -1, -1, -1, -1],
])
def test_explicit_tiles_and_per_step(tiles, mode):
    specs = MIXED
    inits = _inits(specs)
    _say("explicit tiles", tiles, "mode", mode)
    with _make(specs, mode) as b:
        for i, n in enumerate(tiles):
            b.set_tile(i, n)
            assert b.tile(i) == (0 if n < 0 else n)
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(37)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 37)), (i, tiles[i])


@pytest.mark.parametrize("mode", MODES)
def test_split_advances_and_graph_replay(mode):
    specs = MIXED[:6]
    inits = _inits(specs)
    _say("split advances 13,13,13,40,1 mode", mode)
    with _make(specs, mode) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        for k in (13, 13, 13, 40, 1):  # the 13-step graph replays three times
            b.advance(k)
        total = 13 * 3 + 40 + 1
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, total)), i
            assert b.T(i) == total


@pytest.mark.parametrize("mode", MODES)
def test_batch_equals_single_handles(mode):
    """Each grid of a batch gives the bits of a single handle with the same
    tile side."""
    specs = [dict(nx=128, ny=128, pde=si.HEAT5), dict(nx=96, ny=64, pde=si.WAVE_LF, prec=sw.FP32C),
             dict(nx=64, ny=64, pde=si.HEAT5, prec=sw.FP32C)]
    inits = _inits(specs)
    _say("batch vs single handles, mode", mode)
    with _make(specs, mode) as b:
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


@pytest.mark.parametrize("mode", MODES)
def test_measured_autotune_keeps_results(mode):
    specs = MIXED[:5]
    inits = _inits(specs)
    _say("measured autotune, mode", mode)
    with _make(specs, mode) as b:
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


@pytest.mark.parametrize("mode", MODES)
def test_uneven_batch_sampled_against_oracle(mode):
    """The uneven 256-grid workload (sides multiples of 16 in 64..512, heat or
    wave, FP64 or FP32C) for a few half cycles, sampled grids against the
    oracle."""
    specs = si.batch_specs(256, seed=0)
    inits = _inits(specs)
    _say("uneven 256-grid batch, 48 steps, mode", mode)
    with _make(specs, mode) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        steps = 48
        b.advance(steps)
        b.synchronize()
        rng = np.random.default_rng(7)
        for i in rng.choice(len(specs), size=6, replace=False):
            ref = _oracle(specs[i], inits[i], steps)
            assert np.array_equal(b.download(int(i)), ref), (int(i), specs[i], b.tile(int(i)))


@pytest.mark.timeout(900)
def test_literal_batch_50000_steps_sampled_against_oracle():
    """The 256-grid workload with sides drawn from every integer in 64..512
    (heat or wave, FP64 or FP32C) advanced its full 50000 steps in phased
    launches: every grid runs swept (square tiles where an even side divides
    both sides, rectangular tiles elsewhere); the three smallest grids of
    each kind equal the oracle bit for bit."""
    specs = si.batch_specs(256, seed=0, quantum=1)
    inits = _inits(specs)
    steps = 50000
    _say("literal 256-grid batch, 50000 steps")
    with _make(specs, sw.BATCH_PHASED) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(steps)
        b.synchronize()
        by_size = sorted(range(len(specs)), key=lambda i: specs[i]["nx"] * specs[i]["ny"])
        assert all(b.tile(i) > 0 or b.rect(i) > 0 for i in by_size)
        square = [i for i in by_size if b.tile(i) > 0][:3]
        rect = [i for i in by_size if b.rect(i) > 0][:3]
        assert len(square) == 3 and len(rect) == 3
        for i in square + rect:
            _say("grid", i, specs[i], "tile", b.tile(i), "rect", b.rect(i))
            ref = _oracle(specs[i], inits[i], steps)
            assert np.array_equal(b.download(i), ref), (i, specs[i], b.tile(i), b.rect(i))


RECT_MIXED = [
    dict(nx=67, ny=45, pde=si.TEST_HASH),
    dict(nx=101, ny=77, pde=si.HEAT5),
    dict(nx=97, ny=131, pde=si.WAVE_LF),
    dict(nx=83, ny=64, pde=si.HEAT5, prec=sw.FP32C),
    dict(nx=71, ny=59, pde=si.WAVE_LF, prec=sw.FP32C),
    dict(nx=64, ny=64, pde=si.TEST_HASH),
    dict(nx=96, ny=48, pde=si.HEAT5),
]


@pytest.mark.parametrize("heights", [[5, 8, 16, 12, 9, 7, 0], [2, 3, 24, 4, 6, 16, 11], [0, 0, 0, 0, 0, 0, 0]])
def test_rect_grids_in_batch(heights):
    """Rectangular tiles inside a batch (0: the model's choice), next to
    square tiles, through split advances and an advance longer than one
    graph: every grid bit for bit the oracle."""
    specs = RECT_MIXED
    inits = _inits(specs)
    _say("rect batch heights", heights)
    with _make(specs) as b:
        for i, hh in enumerate(heights):
            if hh:
                b.set_rect(i, hh)
                assert b.rect(i) == hh and b.tile(i) == 0
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        for k in (29, 29, 3, 1100):
            b.advance(k)
        total = 29 + 29 + 3 + 1100
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, total)), (i, spec, b.tile(i), b.rect(i))


def test_rect_batch_equals_single_handles():
    specs = [dict(nx=101, ny=77, pde=si.HEAT5), dict(nx=97, ny=61, pde=si.WAVE_LF, prec=sw.FP32C)]
    inits = _inits(specs)
    with _make(specs) as b:
        for i, s0 in enumerate(inits):
            b.set_rect(i, 8 + 4 * i)
            b.upload(i, s0)
        b.advance(100)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            g = sw.Swept2D(spec["nx"], spec["ny"], spec["pde"], _params(spec["pde"]), prec=spec.get("prec", sw.FP64))
            g.rect = b.rect(i)
            g.upload(s0)
            g.advance(100)
            assert np.array_equal(b.download(i), g.download()), i
            g.close()


@pytest.mark.parametrize("mode", MODES)
def test_any_sides_batch(mode):
    """Sides drawn from every integer: grids no even side divides run
    rectangular tiles, the rest square tiles; all exact."""
    specs = si.batch_specs(12, seed=3, lo=20, hi=90, quantum=1)
    inits = _inits(specs)
    _say("any-sides batch, mode", mode)
    with _make(specs, mode) as b:
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(21)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 21)), (i, spec, b.tile(i))


@PERSISTENT_OFF
def test_wait_limit_abort_is_reported_and_recoverable():
    specs = [dict(nx=256, ny=256, pde=si.TEST_HASH)]
    inits = _inits(specs)
    with _make(specs, sw.BATCH_PERSISTENT) as b:
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
        with pytest.raises(sw.Swept2DError):
            b.set_tile(5, 16)
        with pytest.raises(sw.Swept2DError):
            b.set_mode(7)
        b.set_mode(sw.BATCH_PERSISTENT)
        assert b.mode == sw.BATCH_PERSISTENT
        with pytest.raises(sw.Swept2DError) as ei:
            b.advance(1)  # the persistent kernel is not built
        assert ei.value.code == sw.EUNSUPPORTED
        b.set_mode(sw.BATCH_PHASED)
        with pytest.raises(sw.Swept2DError):
            b.launches(0)
        with pytest.raises(sw.Swept2DError):
            b.launches(1025)


def test_long_advance_replays_chunks():
    """An advance longer than one graph (1024 steps) replays the chunk graph
    and then a graph for the rest; one grid per launch class."""
    specs = [dict(nx=128, ny=64, pde=si.HEAT5), dict(nx=64, ny=32, pde=si.TEST_HASH),
             dict(nx=48, ny=48, pde=si.WAVE_LF), dict(nx=32, ny=32, pde=si.HEAT5, prec=sw.FP32C),
             dict(nx=27, ny=20, pde=si.TEST_HASH)]
    tiles = [64, 32, 24, 16, -1]
    inits = _inits(specs)
    _say("long advance 2100 steps, tiles", tiles)
    with _make(specs) as b:
        for i, n in enumerate(tiles):
            b.set_tile(i, n)
        for i, s0 in enumerate(inits):
            b.upload(i, s0)
        b.advance(2100)
        for i, (spec, s0) in enumerate(zip(specs, inits)):
            assert np.array_equal(b.download(i), _oracle(spec, s0, 2100)), (i, tiles[i])
            assert b.T(i) == 2100 * (2 if spec["pde"] == si.TEST_PUSH5 else 1)


def test_slot_layout_launch_count():
    """Phased schedule: the grid with the most phases sets the slot count; a
    slot holds one launch per launch class present in it."""
    specs = [dict(nx=128, ny=128, pde=si.HEAT5), dict(nx=64, ny=64, pde=si.HEAT5)]
    with _make(specs) as b:
        b.set_tile(0, 64)   # 16 steps: 1 + 2 * 1 phases (h = 32, one reduced half cycle)
        b.set_tile(1, 16)   # h = 8: 1 + 2 * 2 = 5 phases
        # 5 slots; grid 0's 3 phases sit in slots 0, 1, 3 next to grid 1's.
        assert b.launches(16) == 5 + 3
        b.set_tile(0, 16)   # both in the one-wave class: one launch per slot
        assert b.launches(16) == 5
