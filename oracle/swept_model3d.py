"""The swept rule in three dimensions, executed component by component.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): it pins the
geometry that the 3D stage kernels follow and is never called by them.

The paper develops the rule in 2D (Sec. 3-4) and motivates it with 3D grids
(Sec. 1). Its level function carries over: a cube tile of side n = 2h, a
point at distance d_x, d_y, d_z from the nearest tile faces (d = min(t,
n - 1 - t), t the point's position in its tile). At level l of a half cycle
the point belongs to the component class given by which of d_x, d_y, d_z are
below l: none (the upward pyramid U), one (a face bridge B_x, B_y, B_z), two
(an edge bridge B_xy, B_xz, B_yz) or all three (the downward pyramid D).
Along an axis where its d is at least l a component shrinks by one cell per
level (a "shrinking" axis); along the others it grows around a tile face.
The half cycle runs the classes in four groups, U, then the face bridges,
then the edge bridges, then D; the components of one group are independent.
Tilings alternate between offset 0 and h on all three axes (Sec. 4).

Every read of a point at level l - 1 must come from the reading component's
own level l - 1 or from a component of an earlier group, and in the latter
case it must lie in the producer's published band: the two cells at either
end of the producer's region along each of its shrinking axes (the 3D form of
the two-wide panels of Sec. 3). The model checks both for every read, so the
group order and the band rule are pinned together with the result.
"""
from __future__ import annotations

import numpy as np

GROUPS = ((0,), (1, 2, 4), (3, 5, 6), (7,))  # class = bit x | bit y << 1 | bit z << 2 of "d < l"


def _axis_geometry(L: int, n: int, off: int):
    """Per coordinate: d (distance to the nearest face in its tile), the tile
    index, and the face index it is nearest to (faces numbered by the tile
    they start)."""
    h = n // 2
    x = np.arange(L)
    t = (x - off) % n
    tile = ((x - off) // n) % (L // n)
    d = np.minimum(t, n - 1 - t)
    face = np.where(t < h, tile, (tile + 1) % (L // n))
    return d, tile, face


def classify(shape, n: int, off: int, level: int):
    """Class (0..7) and component id of every point at `level`."""
    nz, ny, nx = shape
    gx, gy, gz = (_axis_geometry(L, n, off) for L in (nx, ny, nz))
    dx, dy, dz = gx[0][None, None, :], gy[0][None, :, None], gz[0][:, None, None]
    cls = (dx < level).astype(np.int64) | ((dy < level).astype(np.int64) << 1) | ((dz < level).astype(np.int64) << 2)
    # along a growing axis the component is identified by its face, along a
    # shrinking axis by its tile
    ix = np.where(dx < level, gx[2][None, None, :], gx[1][None, None, :])
    iy = np.where(dy < level, gy[2][None, :, None], gy[1][None, :, None])
    iz = np.where(dz < level, gz[2][:, None, None], gz[1][:, None, None])
    tx, ty, tz = nx // n, ny // n, nz // n
    comp = ((cls * tz + iz) * ty + iy) * tx + ix
    return np.broadcast_to(cls, shape).copy(), comp


def in_band(shape, n: int, off: int, level: int):
    """Whether each point of its component's region at `level` lies in that
    region's published band: within two cells of either end along one of the
    component's shrinking axes."""
    nz, ny, nx = shape
    out = np.zeros(shape, dtype=bool)
    for ax, L in ((2, nx), (1, ny), (0, nz)):
        d = _axis_geometry(L, n, off)[0]
        # shrinking along this axis: d >= level; the region spans d in
        # [level, h - 1] mirrored, so its two end cells have d = level, level + 1
        band = (d >= level) & (d <= level + 1)
        sl = [None, None, None]
        sl[ax] = slice(None)
        out |= band[tuple(sl)]
    return out


def _neighbours(a: np.ndarray):
    """The 27 shifted copies of a, neighbour k = 9(dz+1) + 3(dy+1) + (dx+1)
    at index k (periodic)."""
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out.append(np.roll(a, (-dz, -dy, -dx), axis=(0, 1, 2)))
    return out


def heat7(T, nb, params):
    u = nb[13]
    t = ((nb[12] + nb[14]) + (nb[10] + nb[16])) + (nb[4] + nb[22])
    lap = t - 6.0 * u
    return u + params[0] * lap


def hash27(T, nb, params):
    with np.errstate(over="ignore", invalid="ignore"):
        h = np.full(nb[0].shape, np.uint64(0x94D049BB133111EB) ^ np.uint64(T), dtype=np.uint64)
        for k in range(27):
            h ^= nb[k].astype(np.uint64)
            h *= np.uint64(0xFF51AFD7ED558CCD)
            h ^= h >> np.uint64(32)
    return (h >> np.uint64(12)).astype(np.float64)


class OrderError(AssertionError):
    pass


def swept3d(u0: np.ndarray, n: int, nsub: int, step, params=(), t0: int = 0, groups=GROUPS, half0: int = 0,
            counts: dict | None = None) -> np.ndarray:
    """Advance u0 ([nz][ny][nx]) by nsub sub-steps with the 3D swept rule on
    cube tiles of side n (dividing every side), checking every read."""
    shape = u0.shape
    if n < 2 or n % 2 or any(L % n for L in shape):
        raise ValueError("tile side must be even and divide every side")
    h = n // 2
    cur = np.asarray(u0, dtype=np.float64).copy()
    done, half, T = 0, half0, t0
    while done < nsub:
        H = min(h, nsub - done)
        off = 0 if half % 2 == 0 else h
        vals = [cur] + [np.full(shape, np.nan) for _ in range(H)]
        avail = [np.ones(shape, dtype=bool)] + [np.zeros(shape, dtype=bool) for _ in range(H)]
        band = [np.ones(shape, dtype=bool)] + [in_band(shape, n, off, l) for l in range(1, H + 1)]
        meta = [None] + [classify(shape, n, off, l) for l in range(1, H + 1)]
        for group in groups:
            before = [a.copy() for a in avail]
            for l in range(1, H + 1):
                cls, comp = meta[l]
                mine = np.isin(cls, group)
                if not mine.any():
                    continue
                # reads at level l - 1: produced by an earlier group inside
                # the producer's band, or by the same component
                prev_ok = before[l - 1] & band[l - 1]
                prev_comp = meta[l - 1][1] if l > 1 else np.full(shape, -1)
                prev_same_group = np.isin(meta[l - 1][0], group) if l > 1 else np.zeros(shape, dtype=bool)
                ok_sh = _neighbours(prev_ok)
                comp_sh = _neighbours(np.where(prev_same_group, prev_comp, -1))
                for k in range(27):
                    good = ok_sh[k] | (comp_sh[k] == comp)
                    if not np.all(good[mine]):
                        raise OrderError(f"level {l}: a read of group {group} is not available (offset {k})")
                new = step(T + l - 1, _neighbours(vals[l - 1]), params)
                vals[l][mine] = new[mine]
                avail[l] |= mine
                if counts is not None:
                    for c in group:
                        counts[c] = counts.get(c, 0) + int(np.count_nonzero(cls == c))
        if not avail[H].all():
            raise OrderError("a point was not reached at the half cycle's last level")
        cur = vals[H]
        done += H
        half += 1
        T += H
    return cur
