"""The swept rule's space-time decomposition, executed on small grids in
pure Python.

TEST INFRASTRUCTURE ONLY (part of the oracle; the GPU library neither imports
nor shares any of it).

What it models (Sec. 3-4). One half cycle advances a doubly periodic grid by
H <= h = n/2 levels above a tiling of n x n squares. The half cycle's
space-time is split into components by a level function of each point's
distances dx, dy to the nearest edge of its tile (0 on the tile's outer
ring): level l in 1..H of the point belongs to

  the upward pyramid of its tile                if dx >= l and dy >= l,
  the bridge across the nearest x-edge          if dx <  l and dy >= l,
  the bridge across the nearest y-edge          if dx >= l and dy <  l,
  the downward pyramid at the nearest corner    if dx <  l and dy <  l,

and level 0 of every point to the upward pyramid of its tile (the values it
starts from). Components run phase by phase: all upward pyramids, then all
bridges, then all downward pyramids (Alg. 5's two exchanges per half cycle
sit between the phases). A component computes its points level by level, and
a point at level l reads its 3x3 neighbourhood at level l - 1 from its own
component or from a component of an earlier phase; anything else is an
error (ModelError). The next half cycle shifts the tiling by h in x and y.

The same level function partitions a half cycle of H levels over any
tiling of the periodic axes into rectangles whose sides are at least 2H
(a tile wider than 2H gives a frustum instead of a pyramid: its level-H top
is not empty). ``rect_axis`` splits an axis of any length L into
floor(L / 2h) tiles whose widths differ by at most one, and ``mid_axis``
gives the tiling whose edges lie at the tiles' midpoints; the two
alternate between half cycles (``swept2d_rect``). Every tile of either
contains exactly one edge of the other at a distance of at least h from
its own edges, which is what lets a downward pyramid continue as the next
half cycle's upward one.

So the model checks that the partition covers every point and level once,
that its dependencies respect the phase order, and that the result equals
plain stepping; it also counts each component's points and the values that
cross between components (the panels).

The paper prints the bridges' compute loop with the bound n/2 - k + 1 (a
band two points wide at every level). As a level function that is: the
bridge computes level l of a point only when it lies on the near side of
the edge at a distance dx of l - 1 or l - 2. ``LITERAL_BRIDGE_BAND`` switches
the model to that predicate, which leaves points uncomputed; the reading
used instead (and by the GPU library) is the band of all points with
dx < l on both sides, 2l wide, the only one consistent with the panels the
bridges receive and with the point counts of Sec. 3.2.
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


# ---------------------------------------------------------------- partition

LITERAL_BRIDGE_BAND = False

UP, XB, YB, DOWN = "up", "xbridge", "ybridge", "down"
PHASE = {UP: 0, XB: 1, YB: 1, DOWN: 2}


class ModelError(RuntimeError):
    pass


def edge_distance(t: int, n: int) -> int:
    """Distance of tile-local coordinate t (0..n-1) to the nearer tile edge."""
    return min(t, n - 1 - t)


@dataclass(frozen=True)
class Axis:
    """The tiles of one periodic axis of length L: tile a covers the cells
    edges[a] .. edges[a+1] - 1, the last one wrapping round to edges[0]."""
    L: int
    edges: tuple

    def widths(self) -> list:
        t = len(self.edges)
        return [(self.edges[(a + 1) % t] - self.edges[a]) % self.L or self.L for a in range(t)]

    def locate(self, x: int):
        """(tile, tile-local coordinate, tile width) of cell x."""
        for a, w in enumerate(self.widths()):
            lx = (x - self.edges[a]) % self.L
            if lx < w:
                return a, lx, w
        raise AssertionError("axis tiles do not cover the axis")


def uniform_axis(L: int, n: int, off: int) -> Axis:
    assert L % n == 0
    return Axis(L, tuple(sorted((off + k * n) % L for k in range(L // n))))


def rect_axis(L: int, h: int) -> Axis:
    """floor(L / 2h) tiles of widths floor(L/t) or floor(L/t) + 1 (the wider
    ones first), starting at cell 0."""
    t = L // (2 * h)
    assert t >= 1, "the axis is shorter than 2h"
    edges, e = [], 0
    for a in range(t):
        edges.append(e)
        e += L // t + (1 if a < L % t else 0)
    assert e == L
    return Axis(L, tuple(edges))


def mid_axis(ax: Axis) -> Axis:
    """The tiling whose edges are the midpoints edges[a] + floor(w_a / 2)."""
    return Axis(ax.L, tuple(sorted((e + w // 2) % ax.L for e, w in zip(ax.edges, ax.widths()))))


def component_at(x: int, y: int, l: int, ax: Axis, ay: Axis):
    """Component holding level l of point (x, y) in a half cycle on the
    tiling ax x ay, as (kind, id); None only under the printed bridge band."""
    a, lx, wx = ax.locate(x)
    b, ly, wy = ay.locate(y)
    dx, dy = edge_distance(lx, wx), edge_distance(ly, wy)
    ntx, nty = len(ax.edges), len(ay.edges)
    # the edge (and corner) nearest to the point, named by the tile to its
    # west (x-edges) or north (y-edges)
    ea = a if lx >= wx // 2 else (a - 1) % ntx
    eb = b if ly >= wy // 2 else (b - 1) % nty
    if l == 0 or (dx >= l and dy >= l):
        return (UP, (a, b))
    if LITERAL_BRIDGE_BAND:
        # printed loop: a two-point band on the west (x-bridge) / north
        # (y-bridge) side of the edge only
        if dy >= l and lx >= wx // 2 and dx in (l - 1, l - 2):
            return (XB, (ea, b))
        if dx >= l and ly >= wy // 2 and dy in (l - 1, l - 2):
            return (YB, (a, eb))
        if dx < l and dy < l:
            return (DOWN, (ea, eb))
        return None
    if dx < l and dy >= l:
        return (XB, (ea, b))
    if dx >= l and dy < l:
        return (YB, (a, eb))
    return (DOWN, (ea, eb))


def component(x: int, y: int, l: int, n: int, off: int, nx: int, ny: int):
    """component_at on the tiling of n x n squares offset by off in x and y."""
    return component_at(x, y, l, uniform_axis(nx, n, off), uniform_axis(ny, n, off))


@dataclass
class Stats:
    computed: dict = field(default_factory=dict)   # kind -> points computed
    # (producer kind, consumer kind, level) -> values read across components
    crossing: dict = field(default_factory=dict)
    # (tile, level) -> set of points of an upward pyramid's level read by others
    up_sent: dict = field(default_factory=dict)
    exchanges: int = 0

    def add(self, kind, count=1):
        self.computed[kind] = self.computed.get(kind, 0) + count


def half_cycle(St, grid: np.ndarray, n: int, off: int, T0: int, H: int, stats: Stats | None = None) -> np.ndarray:
    """Advance grid[y][x] (at level T0) by H <= n/2 levels on the tiling of
    side n and offset off, component by component; returns level T0 + H."""
    ny, nx = grid.shape
    assert n % 2 == 0 and n >= 2 and nx % n == 0 and ny % n == 0 and 0 < H <= n // 2
    return half_cycle_on(St, grid, uniform_axis(nx, n, off), uniform_axis(ny, n, off), T0, H, stats)


def half_cycle_on(St, grid: np.ndarray, ax: Axis, ay: Axis, T0: int, H: int,
                  stats: Stats | None = None) -> np.ndarray:
    """Advance grid[y][x] (at level T0) by H levels on the tiling ax x ay,
    component by component; returns level T0 + H."""
    ny, nx = grid.shape
    assert ax.L == nx and ay.L == ny and H > 0
    owner = {}
    members = {}
    for l in range(H + 1):
        for y in range(ny):
            for x in range(nx):
                c = component_at(x, y, l, ax, ay)
                if c is None:
                    if l == H:
                        raise ModelError(f"level {T0 + l} of point ({x}, {y}) belongs to no component")
                    continue
                owner[(x, y, l)] = c
                if l > 0:
                    members.setdefault(c, []).append((l, x, y))
    value = {(x, y, 0): float(grid[y, x]) for y in range(ny) for x in range(nx)}
    for phase in (0, 1, 2):
        for c in sorted(k for k in members if PHASE[k[0]] == phase):
            for (l, x, y) in sorted(members[c]):
                nb = [[None] * 3 for _ in range(3)]
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        q = ((x + di) % nx, (y + dj) % ny, l - 1)
                        src = owner.get(q)
                        if src is None or q not in value:
                            raise ModelError(f"{c} needs level {T0 + l - 1} of {q[:2]}, which nothing computed")
                        if src != c:
                            if PHASE[src[0]] >= phase:
                                raise ModelError(f"{c} needs {q} from {src}, which does not run before it")
                            if stats is not None:
                                key = (src[0], c[0], l - 1)
                                stats.crossing.setdefault(key, set()).add((c, q))
                                if src[0] == UP:
                                    stats.up_sent.setdefault((src[1], l - 1), set()).add(q[:2])
                        nb[di + 1][dj + 1] = value[q]
                value[(x, y, l)] = St(T0 + l - 1, nb)
                if stats is not None:
                    stats.add(c[0])
        if stats is not None and phase < 2:
            stats.exchanges += 1
    out = np.empty_like(grid)
    for y in range(ny):
        for x in range(nx):
            if (x, y, H) not in value:
                raise ModelError(f"level {T0 + H} of ({x}, {y}) was never computed")
            out[y, x] = value[(x, y, H)]
    return out


def swept2d(St, grid: np.ndarray, n: int, cycles: int, T0: int = 0, stats: Stats | None = None,
            after_half=None) -> np.ndarray:
    """Full cycles (two half cycles each, the tiling shifted by n/2 in x and y
    between them) on grid[y][x]; after_half(level, grid) is called after every
    half cycle."""
    h = n // 2
    off = 0
    T = T0
    g = np.array(grid, dtype=np.float64)
    for _ in range(2 * cycles):
        g = half_cycle(St, g, n, off, T, h, stats)
        T += h
        off = h - off
        if after_half is not None:
            after_half(T, g.copy())
    return g


def swept2d_rect(St, grid: np.ndarray, h: int, levels: int, T0: int = 0, stats: Stats | None = None,
                 after_half=None) -> np.ndarray:
    """Advance grid[y][x] by `levels` levels in half cycles of h levels (the
    last one shorter when h does not divide `levels`), alternating the
    tiling rect_axis(nx, h) x rect_axis(ny, h) and its midpoint tiling."""
    ny, nx = grid.shape
    tilings = [(rect_axis(nx, h), rect_axis(ny, h))]
    tilings.append((mid_axis(tilings[0][0]), mid_axis(tilings[0][1])))
    g = np.array(grid, dtype=np.float64)
    T, k = T0, 0
    while T < T0 + levels:
        H = min(h, T0 + levels - T)
        ax, ay = tilings[k % 2]
        g = half_cycle_on(St, g, ax, ay, T, H, stats)
        T += H
        k += 1
        if after_half is not None:
            after_half(T, g.copy())
    return g
