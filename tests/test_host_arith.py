"""Host-side checks of integer facts the stage kernels rely on (no GPU): the
float row index of the point-per-thread pass, and the rectangular tilings the
library cuts (a host-only build of its tiling code against the oracle model).

The point-per-thread level pass (tile sides 16 and 32) maps thread index k
to row k // w and column k % w of a w-wide rectangle through one binary32
product, (k + 1/2) * rcp(w), truncated, where rcp(w) is the hardware
reciprocal (within one ulp of 1/w). The exact quotient (k + 1/2) / w is at
least 1/(2w) away from an integer, so an error of a few ulps keeps the
truncation exact; this checks every k < 4096 and w <= 64 (a tile holds at
most 64 x 64 points) with the reciprocal rounded to nearest and one ulp off
either way, the product rounded to nearest as on the device.
"""
import numpy as np


def test_float_row_index_equals_integer_division():
    k = np.arange(4096, dtype=np.int64)
    kf = k.astype(np.float32) + np.float32(0.5)
    for w in range(1, 65):
        near = np.float32(1.0) / np.float32(w)
        for inv in (near, np.nextafter(near, np.float32(0)), np.nextafter(near, np.float32(1))):
            row = (kf * inv).astype(np.int64)
            assert np.array_equal(row, k // w), (w, inv)
            col = k - row * w
            assert col.min() >= 0 and col.max() < w


def test_float_row_index_margin():
    # The distance of (k + 1/2) / w to the nearest integer, against the
    # product's worst error (a reciprocal one ulp off, then the product's
    # rounding, for values below 4096), leaves a wide margin at every size.
    k = np.arange(4096, dtype=np.float64)
    worst_err = 4096.0 * 3 * 2.0 ** -24
    for w in range(1, 65):
        q = (k + 0.5) / w
        margin = np.min(np.abs(q - np.rint(q)))
        assert margin >= 0.5 / w - 1e-12
        assert margin > 10 * worst_err


# ------------------------------------------------ rectangular tilings (host)
#
# The library cuts an axis of length L into floor(L / 2h) tiles for a half
# cycle of height h and alternates that tiling with the one whose edges are
# its midpoints. A host-only build of its tiling functions prints every span
# for L <= 160; the spans must be the oracle model's tilings exactly.

import os
import subprocess

import pytest

from oracle import swept_model as sm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def library_spans(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("host") / "rect_axis_dump")
    subprocess.run(["/opt/rocm/bin/hipcc", "--cuda-host-only", "-x", "hip", "-O1", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host", "rect_axis_dump.cpp"),
                    "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe, "160"], check=True, capture_output=True, text=True).stdout
    spans = {}
    for line in out.splitlines():
        L, h, par, t, *sw = map(int, line.split())
        assert len(sw) == 2 * t
        spans[(L, h, par)] = [(sw[2 * i], sw[2 * i + 1]) for i in range(t)]
    return spans


def test_library_rect_tilings_equal_the_model(library_spans):
    n = 0
    for (L, h, par), spans in library_spans.items():
        ax = sm.rect_axis(L, h)
        if par:
            ax = sm.mid_axis(ax)
        want = sorted(zip(ax.edges, ax.widths()))
        got = sorted((s % L, w) for s, w in spans)
        assert got == want, (L, h, par)
        # tiles in order, each starting where the one before ends
        for (s, w), (s2, _) in zip(spans, spans[1:]):
            assert s + w == s2, (L, h, par)
        assert min(w for _, w in spans) >= 2 * h and max(w for _, w in spans) - min(w for _, w in spans) <= 1
        n += 1
    assert n == sum(2 * (L // 2) for L in range(2, 161))
