"""User schemes and stencils reaching two rings (Sec. 2; Sec. 6), on the GPU.

* TEST_HASH25: a 25-point stencil (offsets |di|, |dj| <= 2) split
  automatically into two nearest-neighbour sub-steps, bit for bit the
  oracle's direct application of the stencil, for several tile sides,
  staging modes, step counts and the per-step method.
* A user scheme compiled outside the library against
  include/swept2d_scheme.hpp (tests/plugin/paper_eq1_scheme.hip): the
  paper's Eq. (1) written as the wide stencil, registered with
  swept2d_register_scheme, initialised by its device Init; bit for bit the
  oracle's explicit sub-steps of Eq. (2)-(3) at every sub-step.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_1602_07558_amd as sw
import swept_inputs as si

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("nx,ny", [(64, 48), (24, 40)])
def test_hash25_two_ring_stencil_split_bitwise(nx, ny):
    s0 = si.hash25_field(nx, ny, seed=nx + ny)
    tiles = [n for n in (4, 8, 16) if nx % n == 0 and ny % n == 0]
    for steps in (1, 3, 8, 13):
        ref = oracle.advance_hash25(s0[0], steps, k0=2)
        for n in tiles:
            for staging in (sw.STAGING_AUTO, sw.STAGING_OFF, sw.STAGING_ON):
                _say("hash25", nx, ny, "tile", n, "steps", steps, "staging", staging)
                with sw.Swept2D(nx, ny, si.TEST_HASH25, [], tile=n) as g:
                    g.set_staging(staging)
                    g.T = 4
                    g.upload(s0)
                    g.advance(steps)
                    got = g.download()
                assert np.array_equal(got[0], ref), (n, steps, staging)
                assert not np.any(got[1:])
        with sw.Swept2D(nx, ny, si.TEST_HASH25, []) as g:
            g.T = 4
            g.upload(s0)
            g.plain_advance(steps)
            assert np.array_equal(g.download()[0], ref)


@pytest.fixture(scope="module")
def eq1_pde():
    sw.load_library()
    plug = ctypes.CDLL(sw._build.PLUGIN_LIB)
    plug.paper_eq1_register.restype = ctypes.c_int
    pde = plug.paper_eq1_register()
    assert pde >= sw.USER_PDE_BASE, sw.swept2d_last_error()
    return pde, plug


def test_user_scheme_init_and_paper_eq1_bitwise(eq1_pde):
    pde, _ = eq1_pde
    nx, ny = 96, 64
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    init = np.zeros((5, ny, nx))
    init[0] = (i * 7 + j * 13) % 17 - 8
    for n in (8, 16, 32):
        for steps in (1, 5, 12):
            _say("paper eq1 plugin tile", n, "steps", steps)
            with sw.Swept2D(nx, ny, pde, shape=(5, 2), tile=n) as g:
                g.init_state()
                assert np.array_equal(g.download(), init)
                g.advance(steps)
                got = g.download()
            assert np.array_equal(got, oracle.advance_f64(si.TEST_PUSH5, init, [], 2 * steps)), (n, steps)
    with sw.Swept2D(nx, ny, pde, shape=(5, 2)) as g:
        g.init_state()
        g.advance(3)
        g.plain_advance(2)
        g.advance(4)
        assert g.T == 18
        assert np.array_equal(g.download(), oracle.advance_f64(si.TEST_PUSH5, init, [], 18))


def test_user_scheme_errors(eq1_pde):
    pde, _ = eq1_pde
    with pytest.raises(sw.Swept2DError):
        sw.Swept2D(32, 32, pde, shape=(4, 2))          # wrong nvars
    with sw.Swept2D(32, 32, pde, shape=(5, 2)) as g:
        with pytest.raises(sw.Swept2DError) as e:
            sw.swept2d_set_precision(g.h, sw.FP32C)
        assert e.value.code == sw.EUNSUPPORTED
    with sw.Swept2D(32, 32, si.HEAT5, [0.2]) as g:
        with pytest.raises(sw.Swept2DError) as e:
            g.init_state()
        assert e.value.code == sw.EUNSUPPORTED
