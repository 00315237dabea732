/*
 * swept3d — the swept rule of space-time decomposition in three dimensions
 * on one GPU (MI355X, gfx950).
 *
 * The paper develops the rule in 2D (Sec. 3-4) and motivates it with 3D
 * grids that are small in space and long in time (Sec. 1). Here its level
 * function is carried to cube tiles of side n = 2h on a triply periodic grid
 * (Sec. 2, assumption 1): at level l of a half cycle a point belongs to the
 * upward pyramid of its tile, to a face bridge, to an edge bridge or to a
 * downward pyramid, by which of its three distances to the nearest tile
 * faces are below l. Each half cycle runs four stages in that order, each
 * one launch over all its components (the downward pyramids go on as the
 * next half cycle's upward pyramids, octahedra as in 2D, when another full
 * half cycle follows); a component computes its levels in
 * the LDS of one workgroup and exchanges only the two-wide bands at the ends
 * of its shrinking axes, level by level, through device memory. Tilings
 * alternate between offset 0 and h on every axis (Sec. 4). Every space-time
 * point is computed once, from its full 3x3x3 neighbourhood one level below
 * (Sec. 2, assumption 2), so results equal plain step-by-step stepping bit
 * for bit.
 *
 * Layout: one FP64 value per point, state[z][y][x], x fastest. All calls
 * return 0 (or a documented non-negative value) on success and a negative
 * SWEPT2D_E* code on failure; the message of the last failure is
 * swept2d_last_error() (swept2d.h). A handle is used by one host thread at a
 * time.
 */
#ifndef SWEPT3D_H
#define SWEPT3D_H

#ifdef __cplusplus
extern "C" {
#endif

/* Schemes (one value per point, one sub-step per step):
 *   HEAT7        7-point heat, t = ((u_W + u_E) + (u_N + u_S)) + (u_B + u_F),
 *                u' = u + r (t - 6u), B / F the z - 1 / z + 1 neighbours;
 *                params {r}
 *   TEST_HASH27  order-sensitive 64-bit mix of the 27 neighbours (index
 *                9 (dz + 1) + 3 (dy + 1) + (dx + 1)) seeded with the sub-step
 *                index; values are integers below 2^52 */
#define SWEPT3D_HEAT7 1
#define SWEPT3D_TEST_HASH27 100

typedef struct swept3d swept3d;

/* Create a grid of nx * ny * nz points (each at least 2) for scheme `pde`
 * on the current device, with the state at zero, sub-step counter 0 and the
 * default tile side (the first of 12, 14, 16, 10, 18, 8, 6, 4, 2 that
 * divides nx, ny and nz and whose two-buffer window fits the workgroup LDS;
 * 0 if none, and then only swept3d_plain_advance runs). Allocates three state
 * buffers (the advance rotates over them) and, at the first advance, two
 * band buffers of (n/2 - 1) levels each. NULL on error. */
swept3d *swept3d_create(int nx, int ny, int nz, int pde);

/* Wait for the handle's work, free its device memory and stream, and the
 * handle. NULL is ignored. */
void swept3d_destroy(swept3d *h);

/* Parameters of the scheme (HEAT7: {r}, 1 value; TEST_HASH27: none), copied
 * from the caller's array. EINVAL for a null handle or fewer values than
 * the scheme needs. */
int swept3d_set_params(swept3d *h, const double *params, int nparams);

/* Cube tile side n: even, at least 2, dividing nx, ny and nz, with
 * 2 (n + 2)^3 doubles of window within the workgroup LDS (n <= 18 in the
 * 160 KB of gfx950). EINVAL otherwise, leaving the side unchanged. */
int swept3d_set_tile(swept3d *h, int n);

/* The current tile side (0: no side divides the grid), or EINVAL for a null
 * handle. */
int swept3d_get_tile(const swept3d *h);

/* Host <-> device copies of the state (nz * ny * nx doubles, [z][y][x],
 * host memory owned by the caller). Synchronous: they wait for the handle's
 * earlier work. EINVAL for null arguments, EHIP on a copy failure. */
int swept3d_upload(swept3d *h, const double *host);
int swept3d_download(swept3d *h, double *host);

/* Advance nsteps steps (nsteps >= 0) with the swept rule (Sec. 3-4, the
 * level function on cube tiles): half cycles of h = n/2 levels, the last one
 * reduced to the remaining count, tilings alternating between offsets 0 and
 * h. Asynchronous on the handle's stream; the first call allocates the band
 * buffers (ENOMEM if they do not fit). EINVAL for a negative count or when
 * no tile side divides the grid. The results equal swept3d_plain_advance's
 * bit for bit. */
int swept3d_advance(swept3d *h, long long nsteps);

/* Advance nsteps steps with one launch per step (the comparison method;
 * Sec. 2's plain stepping). Asynchronous; EINVAL for a negative count. */
int swept3d_plain_advance(swept3d *h, long long nsteps);

/* Wait for the handle's work; EHIP reports a failure of earlier kernels. */
int swept3d_synchronize(swept3d *h);

/* Global sub-step counter (the stencil's sub-step index). set_step fixes it
 * (>= 0), e.g. to resume from a checkpoint. */
long long swept3d_get_step(const swept3d *h);
int swept3d_set_step(swept3d *h, long long T);

#ifdef __cplusplus
}
#endif

#endif
