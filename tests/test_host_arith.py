"""Host-side checks of integer facts the stage kernels rely on (no GPU).

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
