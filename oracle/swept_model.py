"""The paper's swept-rule components executed literally, in pure Python.

TEST INFRASTRUCTURE ONLY (part of the oracle; the GPU library neither imports
nor shares any of it).

This model runs Algorithms 1-5 of Sec. 3-4 in the paper's own order and
notation on a small doubly periodic grid split into P_x by P_y square tiles of
side n, one simulated process per tile, and records what each component
computes and exchanges. It pins the readings of the printed index ranges
against the plain stepper (``oracle.advance_f64``): with the readings below,
every half cycle must land exactly on the plain result.

Notation kept from the paper: 1-based indices, first index i (x, west to
east), second index j (y; j = 1 is the north row of a tile), internal arrays
``U`` and ``D`` of (n+2) x (n+2) entries indexed 0..n+1, ``a:b`` ranges
inclusive. Level k of a component is its k-th time level counted from the
component's first level 0; it is global level T0 + k of the half cycle that
starts at T0, and the stencil list is indexed by the global sub-step.

Readings of the printed algorithms (all checked by the tests against the
plain stepper):

* Alg. 2 and 3, compute loop: the bound printed as n/2-k+1 is read as n/2+k+1
  (the bridge computes a band 2k+2 wide at level k+1, which is what the
  placed panels and the worked example of Sec. 3.2 require).
* Alg. 3, outputs: the i-ranges printed for N^k and S^k are exchanged:
  N^k = D[n/2-k-1 : n/2+k, k+1 : k+2], S^k = D[n/2-k+1 : n/2+k+2, n-k-1 : n-k].
  With these, Alg. 4 places every value where it belongs (each of the four
  bridge panels carries one 2x2 corner of the ring, a pinwheel).
* Alg. 4: the loop over k runs 0..n/2-1 (levels 1..n/2 are computed; the
  printed upper bound n/2 would place panels that do not exist).
* Sec. 3.1: the upward pyramid computes levels 1..n/2-1; its tip, a 2x2
  square, is at level n/2-1.
* The stencil operation applied when level k+1 is produced is the one of the
  global sub-step T0 + k.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------- stencils
# Each stencil maps (global sub-step index, 3x3 neighbourhood nb[di+1][dj+1])
# to the new value. These are the same definitions as the C oracle's
# (Python floats are IEEE binary64 with round-to-nearest-even).


def st_heat(r: float):
    def f(T, nb):
        u = nb[1][1]
        t1 = nb[0][1] + nb[2][1]
        t2 = nb[1][0] + nb[1][2]
        lap = (t1 + t2) - 4.0 * u
        return u + r * lap
    return f


_M64 = (1 << 64) - 1


def st_hash(T, nb):
    h = (0x9E3779B97F4A7C15 ^ int(T)) & _M64
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            h ^= int(nb[di + 1][dj + 1])
            h = (h * 0xFF51AFD7ED558CCD) & _M64
            h ^= h >> 32
    return float(h >> 12)


def st_incr(T, nb):
    u = nb[1][1]
    same = all(nb[a][b] == u for a in range(3) for b in range(3))
    return u + 1.0 if same else float("nan")


# --------------------------------------------------------------- components

# Switches that restore the ranges exactly as printed, so the tests can show
# that the printed forms do not reproduce plain stepping (and the readings do).
LITERAL_BRIDGE_LOOP = False   # Alg. 2/3 compute bound n/2-k+1 as printed
LITERAL_LAT_OUTPUTS = False   # Alg. 3 N^k / S^k i-ranges as printed

def _nbhd(D, i, j):
    return [[D[i + di][j + dj] for dj in (-1, 0, 1)] for di in (-1, 0, 1)]


def _get(D, i0, i1, j0, j1):
    """D[i0:i1, j0:j1] with inclusive bounds, as an array indexed [i-i0][j-j0]."""
    return np.array([[D[i][j] for j in range(j0, j1 + 1)] for i in range(i0, i1 + 1)], dtype=np.float64)


def _put(D, i0, i1, j0, j1, P):
    assert P.shape == (i1 - i0 + 1, j1 - j0 + 1), (P.shape, i0, i1, j0, j1)
    for i in range(i0, i1 + 1):
        for j in range(j0, j1 + 1):
            D[i][j] = P[i - i0][j - j0]


@dataclass
class Stats:
    computed: dict = field(default_factory=dict)   # component name -> points computed
    panel_sizes: dict = field(default_factory=dict)  # (component, side) -> list of per-level sizes
    exchanges: int = 0

    def add(self, name, count):
        self.computed[name] = self.computed.get(name, 0) + count


def _new(n):
    return np.full((n + 2, n + 2), np.nan, dtype=np.float64)


def upward_pyramid(St, B, T0, stats=None):
    """Algorithm 1. B is n x n (indexed [i-1][j-1]); returns panels N, S, W, E
    as lists over levels k = 0..n/2-1."""
    n = B.shape[0]
    h = n // 2
    U, D = _new(n), _new(n)
    _put(D, 1, n, 1, n, B)
    N, S, W, E = [], [], [], []
    count = 0
    for k in range(h):
        N.append(_get(D, k + 1, n - k, k + 1, k + 2))
        S.append(_get(D, k + 1, n - k, n - k - 1, n - k))
        W.append(_get(D, k + 1, k + 2, k + 1, n - k))
        E.append(_get(D, n - k - 1, n - k, k + 1, n - k))
        for i in range(2 + k, n - k):
            for j in range(2 + k, n - k):
                U[i][j] = St(T0 + k, _nbhd(D, i, j))
                count += 1
        U, D = D, U
    if stats is not None:
        stats.add("up", count)
        stats.panel_sizes[("up", "N")] = [p.size for p in N]
    return N, S, W, E


def longitudinal_bridge(St, N, S, n, T0, stats=None):
    """Algorithm 2: the bridge between a tile (its south panel passed as N)
    and the tile south of it (its north panel passed as S)."""
    h = n // 2
    U, D = _new(n), _new(n)
    Wo, Eo = [], []
    count = 0
    for k in range(h):
        _put(D, k + 1, n - k, h - k - 1, h - k, N[k])
        _put(D, k + 1, n - k, h + k + 1, h + k + 2, S[k])
        Wo.append(_get(D, k + 1, k + 2, h - k + 1, h + k + 2))
        Eo.append(_get(D, n - k - 1, n - k, h - k - 1, h + k))
        for i in range(2 + k, n - k):
            jhi = (h - k + 1) if LITERAL_BRIDGE_LOOP else (h + k + 1)   # reading: n/2+k+1
            for j in range(h - k, jhi + 1):
                U[i][j] = St(T0 + k, _nbhd(D, i, j))
                count += 1
        U, D = D, U
    if stats is not None:
        stats.add("long", count)
        stats.panel_sizes[("long", "W")] = [p.size for p in Wo]
    return Wo, Eo


def latitudinal_bridge(St, W, E, n, T0, stats=None):
    """Algorithm 3: the bridge between a tile (its east panel passed as W) and
    the tile east of it (its west panel passed as E)."""
    h = n // 2
    U, D = _new(n), _new(n)
    No, So = [], []
    count = 0
    for k in range(h):
        _put(D, h - k - 1, h - k, k + 1, n - k, W[k])
        _put(D, h + k + 1, h + k + 2, k + 1, n - k, E[k])
        if LITERAL_LAT_OUTPUTS:
            No.append(_get(D, h - k + 1, h + k + 2, k + 1, k + 2))
            So.append(_get(D, h - k - 1, h + k, n - k - 1, n - k))
        else:                                                       # reading: i-ranges exchanged
            No.append(_get(D, h - k - 1, h + k, k + 1, k + 2))
            So.append(_get(D, h - k + 1, h + k + 2, n - k - 1, n - k))
        ihi = (h - k + 1) if LITERAL_BRIDGE_LOOP else (h + k + 1)       # reading: n/2+k+1
        for i in range(h - k, ihi + 1):
            for j in range(2 + k, n - k):
                U[i][j] = St(T0 + k, _nbhd(D, i, j))
                count += 1
        U, D = D, U
    if stats is not None:
        stats.add("lat", count)
        stats.panel_sizes[("lat", "N")] = [p.size for p in No]
    return No, So


def downward_pyramid(St, N, S, W, E, n, T0, stats=None):
    """Algorithm 4: fill the gap between four bridge panels; returns the n x n
    tile at level n/2 (indexed [i-1][j-1])."""
    h = n // 2
    U, D = _new(n), _new(n)
    count = 0
    for k in range(h):                                   # reading: k = 0..n/2-1
        _put(D, h - k - 1, h - k, h - k - 1, h + k, W[k])
        _put(D, h + k + 1, h + k + 2, h - k + 1, h + k + 2, E[k])
        _put(D, h - k + 1, h + k + 2, h - k - 1, h - k, N[k])
        _put(D, h - k - 1, h + k, h + k + 1, h + k + 2, S[k])
        for i in range(h - k, h + k + 2):
            for j in range(h - k, h + k + 2):
                U[i][j] = St(T0 + k, _nbhd(D, i, j))
                count += 1
        U, D = D, U
    if stats is not None:
        stats.add("down", count)
    return _get(D, 1, n, 1, n)


# ------------------------------------------------------------------- driver

def swept2d(St, grid: np.ndarray, n: int, cycles: int, T0: int = 0, stats: Stats | None = None,
            after_half=None) -> np.ndarray:
    """Algorithm 5 on a doubly periodic grid ``grid[j][i]`` (shape ny x nx)
    split into (nx/n) x (ny/n) tiles, one simulated process per tile.

    ``after_half(level, global_grid)`` is called after every half cycle with
    the grid reassembled in global coordinates."""
    ny, nx = grid.shape
    assert n % 2 == 0 and n >= 2 and nx % n == 0 and ny % n == 0
    h = n // 2
    px, py = nx // n, ny // n
    ranks = [(a, b) for b in range(py) for a in range(px)]

    def north(r):
        return (r[0], (r[1] - 1) % py)

    def south(r):
        return (r[0], (r[1] + 1) % py)

    def west(r):
        return ((r[0] - 1) % px, r[1])

    def east(r):
        return ((r[0] + 1) % px, r[1])

    # B[r][i-1][j-1]; process (a, b) starts with the tile whose north-west
    # point is global (a n, b n).
    B = {r: grid[r[1] * n:(r[1] + 1) * n, r[0] * n:(r[0] + 1) * n].T.copy() for r in ranks}
    shift = 0   # 0: tiles at (a n, b n); h: tiles at (a n + h, b n + h)
    T = T0

    def assemble():
        g = np.empty_like(grid)
        for (a, b) in ranks:
            x0, y0 = a * n + shift, b * n + shift
            for i in range(n):
                for j in range(n):
                    g[(y0 + j) % ny, (x0 + i) % nx] = B[(a, b)][i][j]
        return g

    for _ in range(cycles):
        for half in (0, 1):
            P = {r: upward_pyramid(St, B[r], T, stats) for r in ranks}     # (N, S, W, E)
            if stats is not None:
                stats.exchanges += 1
            WD, ED, ND, SD = {}, {}, {}, {}
            for r in ranks:
                if half == 0:
                    # N_U, W_U travel north and west: a process receives the
                    # north panel of its south neighbour and the west panel of
                    # its east neighbour, and builds the bridges on its south
                    # and east edges.
                    WD[r], ED[r] = longitudinal_bridge(St, P[r][1], P[south(r)][0], n, T, stats)
                    ND[r], SD[r] = latitudinal_bridge(St, P[r][3], P[east(r)][2], n, T, stats)
                else:
                    # S_U, E_U travel south and east: bridges on the north and
                    # west edges.
                    WD[r], ED[r] = longitudinal_bridge(St, P[north(r)][1], P[r][0], n, T, stats)
                    ND[r], SD[r] = latitudinal_bridge(St, P[west(r)][3], P[r][2], n, T, stats)
            if stats is not None:
                stats.exchanges += 1
            newB = {}
            for r in ranks:
                if half == 0:
                    # DownwardPyramid(St, S_D, N_D<-P_S, E_D, W_D<-P_E) fills the
                    # gap at the south-east corner.
                    newB[r] = downward_pyramid(St, SD[r], ND[south(r)], ED[r], WD[east(r)], n, T, stats)
                else:
                    # DownwardPyramid(St, S_D<-P_N, N_D, E_D<-P_W, W_D) fills
                    # the gap at the north-west corner.
                    newB[r] = downward_pyramid(St, SD[north(r)], ND[r], ED[west(r)], WD[r], n, T, stats)
            B = newB
            shift = h if half == 0 else 0
            T += h
            if after_half is not None:
                after_half(T, assemble())
    return assemble()
