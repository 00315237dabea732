/*
 * swept2d.h - C ABI of the MI355X (gfx950) swept-rule stencil library.
 *
 * The library advances explicit two-dimensional stencil schemes on a doubly
 * periodic, logically Cartesian grid (Sec. 2, assumption 1). Every sub-step
 * computes each point from its 3x3 neighbourhood one level below (Sec. 2,
 * assumption 2); a scheme may take several sub-steps per time step (Sec. 2,
 * Eq. (1)-(3)). The library runs such schemes two ways:
 *
 *   swept2d_advance        the swept rule of space-time decomposition
 *                          (Sec. 3-4, Algorithms 1-5): square tiles of side n
 *                          build upward pyramids, then the latitudinal and
 *                          longitudinal bridges, then downward pyramids, n/2
 *                          levels per half cycle, exchanging only the
 *                          pyramids' and bridges' triangular sides (panels).
 *                          On one GPU a panel exchange is an HBM round trip
 *                          between kernels instead of a network message.
 *   swept2d_plain_advance  the classical per-step method: one kernel launch
 *                          per sub-step (the "latency barrier" of Sec. 5).
 *
 * Both compute exactly the same values: the swept rule does no redundant work
 * and gives every point its complete 3x3 neighbourhood from the level below
 * (abstract; Sec. 4).
 *
 * Conventions for every call:
 *   - Return 0 on success or a negative SWEPT2D_E* code. The thread-local
 *     message of the last failure is available from swept2d_last_error().
 *   - Calls that launch GPU work are asynchronous on the handle's stream.
 *     A kernel fault is reported by swept2d_synchronize, swept2d_download or
 *     the next call that checks the stream.
 *   - No C++ exception crosses this interface.
 *   - A handle is not thread safe: one thread at a time per handle.
 *     Different handles may be created and used from different threads at
 *     once; the first handle on each device sets that device's kernel
 *     limits once, under a lock.
 *
 * State layout (device and host): structure of arrays [nvars][ny][nx], x
 * fastest, row j = 0 is the north edge. The paper's point (i, j) is
 * state[v][j][i].
 */
#ifndef SWEPT2D_H
#define SWEPT2D_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define SWEPT2D_OK 0
#define SWEPT2D_EINVAL (-1)       /* bad argument: sizes, ids, tile, null handle */
#define SWEPT2D_EHIP (-2)         /* HIP runtime error; message carries hipGetErrorString */
#define SWEPT2D_ENOMEM (-3)       /* device allocation failed */
#define SWEPT2D_EUNSUPPORTED (-4) /* valid request the library does not provide */
#define SWEPT2D_EABORTED (-5)     /* a persistent batch kernel stopped: a dependency wait hit its limit */

/* ------------------------------------------------------------- scheme ids
 * Built-in per-point sub-step operations (the paper's timestep(i, p)
 * callback of Sec. 6, compiled in). nvars / substeps each must take:
 *   HEAT5          1 / 1  u' = u + r lap(u), 5-point Laplacian; params {r}
 *   WAVE_LF        2 / 1  leapfrog, (u, u_prev) -> ((2u - u_prev) + C2 lap(u), u);
 *                         params {C2}
 *   EULER_RUS_RK2  8 / 2  compressible Euler, first-order finite volumes with
 *                         the Rusanov flux, two-stage SSP Runge-Kutta; slots
 *                         0..3 conserved (rho, rho u, rho v, E), 4..7 the
 *                         stage; params {gamma, dt/h}
 *   EULER_FD_RK4  12 / 4 compressible Euler in the discretisation of Sec. 8:
 *                         conservative skew-symmetric central differences
 *                         (face flux (m_L + m_R)(phi_L + phi_R) / 4 for phi
 *                         in {1, u, v, H}, pressure (p_L + p_R) / 2) and
 *                         the classical four-stage Runge-Kutta method, one
 *                         stage per sub-step; slots 0..3 conserved, 4..7
 *                         the stage value (equal to 0..3 at full steps),
 *                         8..11 the stage-derivative sum (zero at full
 *                         steps); params {gamma, dt/h}. FP64 and FP32C.
 *   TEST_HASH      1 / 1  order-sensitive 64-bit mix of the 9 neighbours and
 *                         the sub-step index (values: integers < 2^52)
 *   TEST_INCR      1 / 1  u' = u + 1 if all 9 neighbours equal u, else NaN
 *                         (the worked example of Sec. 3.1)
 *   TEST_PUSH5     5 / 2  Eq. (2) then Eq. (3): the 2-ring stencil of Eq. (1)
 *                         decomposed into nearest-neighbour sub-steps
 *   TEST_HASH25    9 / 2  a stencil reaching two rings (an order-sensitive
 *                         mix of the 25 values at offsets |di|, |dj| <= 2 and
 *                         the step index) split automatically into two
 *                         nearest-neighbour sub-steps (Sec. 2): slot 0 holds
 *                         the value, slots 1..8 the values pushed by the
 *                         first sub-step (zero at full steps)
 * User schemes registered with swept2d_register_scheme get ids from
 * SWEPT2D_USER_PDE_BASE on. */
#define SWEPT2D_HEAT5 1
#define SWEPT2D_WAVE_LF 2
#define SWEPT2D_EULER_RUS_RK2 3
#define SWEPT2D_EULER_FD_RK4 4
#define SWEPT2D_TEST_HASH 100
#define SWEPT2D_TEST_INCR 101
#define SWEPT2D_TEST_PUSH5 102
#define SWEPT2D_TEST_HASH25 103
#define SWEPT2D_USER_PDE_BASE 1000

/* ------------------------------------------------------------- precisions
 * FP64:  one double per value.
 * FP32C: FP32 value u plus an FP32 compensation c per value (the pair stands
 *        for u - c). Heat and wave compensate the time update (Kahan); the
 *        Euler schemes widen every value to the FP64 u - c, apply the FP64
 *        sub-step and split each result t into u = fl32(t), c = fl32(u - t).
 *        Available for HEAT5, WAVE_LF, EULER_RUS_RK2 and EULER_FD_RK4.
 *        Device layout: nvars u-planes then nvars c-planes,
 *        each [ny][nx] float. Swept and per-step results are identical.
 * FP32R: FP32 values u only in the state and the panels (half the bytes of
 *        FP32C); the compensations of the same updates live only in a
 *        workgroup's LDS window while it computes a point's successive
 *        levels, and start at zero whenever a value arrives from the state
 *        or a panel. Results therefore depend on the method and tile side:
 *        swept2d_plain_advance keeps no compensation (plain FP32), the swept
 *        advance keeps it within each pyramid, bridge and octahedron.
 *        Available for HEAT5 and WAVE_LF. Device layout: nvars planes,
 *        each [ny][nx] float; the wave runs in velocity form, its planes
 *        holding u^n and v = u^n - u^(n-1) (swept2d_upload and
 *        swept2d_download convert from and to the (u^n, u^(n-1)) slots of
 *        the other precisions: v = fl32(u^n - u^(n-1)) in, u^n - v out). */
#define SWEPT2D_FP64 0
#define SWEPT2D_FP32C 1
#define SWEPT2D_FP32R 2

/* ---------------------------------------------------------- launch modes
 * DIRECT: every kernel is launched with hipLaunchKernel.
 * GRAPH:  the launch sequence of an advance is captured once into a HIP
 *         graph (per distinct step count) and replayed. */
#define SWEPT2D_LAUNCH_DIRECT 0
#define SWEPT2D_LAUNCH_GRAPH 1

/* ------------------------------------------------------- panel staging
 * AUTO: a bridge or downward-pyramid workgroup copies all the panel levels it
 *       consumes into LDS when it starts, if they fit beside its window.
 * OFF:  every workgroup fetches each level's panels one level ahead. */
#define SWEPT2D_STAGING_AUTO 0
#define SWEPT2D_STAGING_OFF 1
#define SWEPT2D_STAGING_SINGLE_BRIDGES 2
#define SWEPT2D_STAGING_ON 3

typedef struct swept2d swept2d; /* opaque, owned by the library */

/* Create a handle for an nx by ny periodic grid (Sec. 2) with nvars values
 * per point and `substeps` sub-steps per time step, for scheme `pde`.
 * Uses the current HIP device and a stream of its own (created with
 * hipStreamNonBlocking); allocates and zeroes a library-owned FP64 state.
 * The tile side starts at the size the built-in tuner picks
 * (swept2d_set_tile(h, 0)).
 * Returns NULL on error (bad sizes, nvars/substeps not matching pde, nx or ny
 * below 2, no device, out of memory); see swept2d_last_error(). */
swept2d *swept2d_create(int nx, int ny, int nvars, int pde, int substeps);

/* Free all library-owned device memory, graphs and events. A bound state
 * (swept2d_bind) belongs to the caller and is not freed. Waits for the
 * handle's stream first. NULL is accepted and ignored. */
void swept2d_destroy(swept2d *h);

/* Set the scheme's physical parameters (see the scheme list). np must be at
 * least the number the scheme uses; p is copied. EINVAL otherwise. */
int swept2d_set_params(swept2d *h, const double *p, int np);

/* Select FP64, FP32C or FP32R. Reallocates a library-owned state (zeroed);
 * fails with EINVAL while a caller buffer is bound, EUNSUPPORTED for schemes
 * without that form. */
int swept2d_set_precision(swept2d *h, int prec);

/* Tile side n of the swept decomposition (Sec. 3: square subdomains of side
 * n; a half cycle advances n/2 levels). n must be even, at least 2, divide nx
 * and ny, and fit the tile's working set in one workgroup's LDS. n = 0 lets
 * the built-in tuner choose (cost model of Sec. 5, Eq. (4)-(5), constrained
 * by LDS size and compute-unit count), falling back to rectangular tiles
 * (swept2d_set_rect) when no square side is usable. EINVAL if n is not
 * usable. Selecting a square side leaves rectangular tiles. */
int swept2d_set_tile(swept2d *h, int n);

/* Current tile side (0 while rectangular tiles are selected). */
int swept2d_get_tile(const swept2d *h);

/* Rectangular tiles (the level function of Sec. 3 generalised: it
 * partitions a half cycle of H levels over any tiling into rectangles whose
 * sides are all at least 2H, so grids of any side, odd or prime, run the
 * swept rule). hh >= 1 is the half-cycle height: each axis of length L is cut
 * into floor(L / 2hh) tiles of widths floor(L / t) and floor(L / t) + 1
 * (tiles wider than 2hh are frustums, whose flat tops and bridge middles
 * pass through the state between half cycles), alternating between half
 * cycles with the tiling whose edges are those tiles' midpoints. Results
 * are those of plain stepping, bit for bit, as for square tiles. hh = 0
 * returns to square tiles (the tuner's side). EINVAL if nx or ny is below
 * 2 hh or a tile's window (2 (widest + 2)^2 values per value slot) exceeds
 * the workgroup LDS; EUNSUPPORTED for FP32R and registered user schemes.
 * swept2d_create and swept2d_set_tile(h, 0) select rectangular tiles of the
 * cost model's height when no even square side divides nx and ny. */
int swept2d_set_rect(swept2d *h, int hh);

/* Half-cycle height of the rectangular tiles in use, 0 for square tiles. */
int swept2d_get_rect(const swept2d *h);

/* Stream selector for swept2d_bind: the HIP null stream (hipStream_t 0,
 * which is torch's default stream on ROCm). NULL itself selects the
 * library's own stream. */
#define SWEPT2D_NULL_STREAM ((void *)(~(size_t)0))

/* Use a caller-owned device buffer as the state and a caller stream for all
 * launches. dev_state must hold swept2d_state_bytes(h) bytes in the layout
 * of the handle's precision and stay valid until the handle is destroyed or
 * rebound. hip_stream is a hipStream_t, SWEPT2D_NULL_STREAM for the null
 * stream, or NULL for the library's own stream (created with
 * hipStreamNonBlocking, so it is not ordered with the null stream). Graphs
 * of SWEPT2D_LAUNCH_GRAPH are captured on the library's own stream and
 * launched on the bound one. Passing dev_state = NULL returns to a
 * library-owned state (zeroed). Waits for the previous stream first. */
int swept2d_bind(swept2d *h, void *dev_state, void *hip_stream);

/* Bytes of the device state: nvars*nx*ny*8 for FP64 and FP32C (4-byte u and
 * 4-byte c per value), nvars*nx*ny*4 for FP32R. */
size_t swept2d_state_bytes(const swept2d *h);

/* Copy a host FP64 state [nvars][ny][nx] in (synchronous). FP32C stores
 * u = (float)x and c = 0, FP32R u = (float)x (the wave's second plane as
 * v = (float)(x0 - x1), its velocity form). */
int swept2d_upload(swept2d *h, const double *host);

/* Copy the state out as FP64 [nvars][ny][nx] (synchronous; waits for the
 * stream). FP32C returns (double)u - (double)c, FP32R (double)u (the wave's
 * second slot as (double)u - (double)v). */
int swept2d_download(swept2d *h, double *host);

/* Copy the raw device state (swept2d_state_bytes bytes, precision layout)
 * in or out (synchronous). */
int swept2d_upload_raw(swept2d *h, const void *host);
int swept2d_download_raw(swept2d *h, void *host);

/* Advance nsteps full time steps (nsteps * substeps sub-steps) with the
 * swept rule (Algorithm 5): an initial upward pyramid per tile, then for
 * every half cycle the bridges and the downward pyramid fused with the next
 * upward pyramid (an octahedron), the tiling shifting by n/2 in x and y each
 * half cycle; a remainder shorter than n/2 sub-steps is run as a half cycle
 * of reduced height. On return (after the stream completes) the state holds
 * every point at one level, in global coordinates. Results are bitwise equal
 * to swept2d_plain_advance. nsteps = 0 is a no-op; EINVAL if negative. */
int swept2d_advance(swept2d *h, long long nsteps);

/* Advance nsteps full time steps with one kernel launch per sub-step, the
 * classical per-step method (Sec. 5; the comparison baseline of Sec. 7-8). */
int swept2d_plain_advance(swept2d *h, long long nsteps);

/* Wait for the handle's stream; reports a pending kernel fault as EHIP. */
int swept2d_synchronize(swept2d *h);

/* ---------------------------------------------- advance without allocation
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * swept advance as swept2d_advance (same kernels, schedule and bits) on a
 * caller state, without a handle. Its panels live in one static device
 * array of SWEPT2D_NOALLOC_SCRATCH_BYTES, which every GPU the library runs
 * on holds from library load until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call.
 *
 *   nx, ny, nvars, pde, substeps  as swept2d_create
 *   prec          SWEPT2D_FP64, SWEPT2D_FP32C or SWEPT2D_FP32R (state layout
 *                 as a handle's)
 *   params, np    as swept2d_set_params
 *   tile          tile side as swept2d_set_tile; 0 lets the cost model pick
 *   dev_state     caller device buffer [nvars][ny][nx] in the precision's
 *                 layout, advanced in place (borrowed for the call's work)
 *   T             the state's level in sub-steps (a multiple of substeps);
 *                 the operation applied at level T is sub-step T mod substeps
 *   nsteps        full steps to advance (0: only validation)
 *   hip_stream    a hipStream_t, or NULL / SWEPT2D_NULL_STREAM for the null
 *                 stream; the call is asynchronous on it
 *
 * EINVAL for bad arguments and when the panels of the grid at that tile
 * side exceed the static array (1024 x 1024 heat at tile side 64 needs
 * 34.6 MB in FP64 and in FP32C); EHIP if the array's device address cannot
 * be looked up. Every call on a GPU shares that GPU's array and leaves its
 * last contents in it (every panel value an advance reads, it first writes,
 * so nothing needs clearing): calls that overlap on one GPU, on different
 * streams or from different threads, race and give undefined results. */
#define SWEPT2D_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int swept2d_advance_noalloc(int nx, int ny, int nvars, int pde, int substeps, int prec, const double *params,
                            int np, int tile, void *dev_state, long long T, long long nsteps, void *hip_stream);

/* Global sub-step counter T: the level of the state, counted in sub-steps
 * since creation (or since the last swept2d_set_substep_counter). The
 * scheme applied at level T is sub-step T mod substeps, so checkpoint and
 * resume save and restore T with the state. set: EINVAL if T < 0 or not a
 * multiple of substeps. */
long long swept2d_substep_counter(const swept2d *h);
int swept2d_set_substep_counter(swept2d *h, long long T);

/* Launch mode (SWEPT2D_LAUNCH_DIRECT or SWEPT2D_LAUNCH_GRAPH). */
int swept2d_set_launch_mode(swept2d *h, int mode);

/* Panel staging mode: whether a component copies all its panel inputs into
 * LDS at its start (staged) or fetches each level's inputs from HBM a few
 * levels before it places them. At tile sides 32 and 64 a tile's two
 * bridges run in one workgroup where both fit its LDS. SWEPT2D_STAGING_AUTO
 * stages an octahedron only where its workgroup has too few waves to keep
 * each wave's ring runs precomputed, and fetches the bridges' inputs (at
 * tile side 32 it runs the bridges as SWEPT2D_STAGING_SINGLE_BRIDGES does);
 * SWEPT2D_STAGING_ON stages every component whose inputs fit the LDS;
 * SWEPT2D_STAGING_OFF stages nothing; SWEPT2D_STAGING_SINGLE_BRIDGES is AUTO
 * with one staged workgroup per bridge. The one-wave groups (tile sides up
 * to 22 of the light schemes) always stage. All modes give identical
 * results. */
int swept2d_set_staging(swept2d *h, int mode);

/* Per-kernel timing. While on, every kernel the handle launches is bracketed
 * by HIP events on the handle's stream. get writes up to cap records of
 * {kind, launches, total_ms, work_points} (4 doubles each, kind: 0 plain,
 * 1 upward pyramid, 2 bridges, 3 octahedron / downward pyramid) and returns
 * the number of records; it synchronizes the stream. Turning timing on
 * clears the records. work_points counts the space-time points the kernels
 * of that kind computed. */
int swept2d_set_timing(swept2d *h, int on);
int swept2d_get_timing(swept2d *h, double *out, int cap);

/* ------------------------------------------------------------ user schemes
 * The paper's interface (Sec. 6): a scheme is an initialisation function
 * Init(i, j, p) and a time-stepping function timestep(k, p) of a point's
 * 9-point neighbourhood. Here both are device functions of a C++ struct
 * compiled by the user in a HIP source against include/swept2d_scheme.hpp,
 * which turns the struct into this table of launchers of the library's stage
 * kernels instantiated for it (stencils reaching two rings go through the
 * automatic split into nearest-neighbour sub-steps there). The launchers
 * take the library's internal descriptors (tile geometry, panel pointers,
 * parameters) by pointer, with the layout of that header; they return a
 * hipError_t value. */
#define SWEPT2D_SCHEME_ABI 1
typedef struct swept2d_scheme_ops {
  int abi;                 /* SWEPT2D_SCHEME_ABI */
  int nvars, substeps;     /* as swept2d_create takes them */
  int nparams;             /* parameters swept2d_set_params must supply (at most 4) */
  int nv, nw, vbytes;      /* values per point in the state, in the LDS window; bytes per value */
  int (*up)(const void *geo, int H, void *state, const void *panels, const void *params, void *stream);
  int (*bridge)(const void *geo, int H, int staged, int pair_ok, void *state, const void *panels,
                const void *params, void *stream);
  int (*oct)(const void *geo, int Hd, int Hu, int staged, void *state, const void *panels, const void *params,
             void *stream);
  int (*plain)(int nx, int ny, long long T, const long long *tbase, const void *in, void *out, const void *params,
               void *stream);
  int (*lds)(size_t bytes);     /* raise the stage kernels' dynamic LDS limit */
  int (*fetch_ahead)(int n);    /* octahedra of tile side n fetch ring runs ahead (1) or stage them (0) */
  int (*init)(int nx, int ny, void *state, const void *params, void *stream); /* Init on every point, or NULL */
} swept2d_scheme_ops;

/* Register a user scheme; ops is copied. Returns its pde id (from
 * SWEPT2D_USER_PDE_BASE, for swept2d_create with ops->nvars and
 * ops->substeps; FP64 precision only; not in batches), or EINVAL for a wrong
 * ABI version, inconsistent sizes or a missing launcher, EUNSUPPORTED when
 * 32 schemes are registered already. Uses the current device. */
int swept2d_register_scheme(const swept2d_scheme_ops *ops);

/* Set every point of the state with the scheme's Init (asynchronous on the
 * handle's stream; the level counter is left as it is). EUNSUPPORTED for
 * schemes without one (the built-in schemes' fields come from the host). */
int swept2d_init_state(swept2d *h);

/* Message of the last failed call on this thread ("" if none). */
const char *swept2d_last_error(void);

/* ------------------------------------------------------------------ batch
 * Many independent small grids advanced together, each by the swept rule
 * with its own tile side (Sec. 3-4; the tile side trades the exchange count
 * against pyramid depth as in Sec. 5, Eq. (4)), or by the per-step method
 * when no even side divides its grid. A grid's work is a chain of phases
 * (its upward pyramid, then bridges and octahedra alternating; one phase per
 * sub-step for the per-step method), each phase a set of independent work
 * items (one per tile, tile edge or block).
 *
 * SWEPT2D_BATCH_PHASED (default): the phases of all grids are spread over
 * one common sequence of slots, each grid's phases in order; a slot is one
 * kernel launch per launch class (workgroup size and stage code), one
 * workgroup per item; the launch boundaries order the phases and no
 * workgroup waits for another. An advance of up to 1024 steps is one
 * captured HIP graph (longer advances replay it).
 * SWEPT2D_BATCH_PERSISTENT: one persistent kernel whose workgroups take
 * items from a device queue and wait on per-grid completion counters; only
 * in libraries built with SWEPT2D_BUILD_PERSISTENT_BATCH defined (advance returns
 * EUNSUPPORTED otherwise).
 *
 * Grids: HEAT5 and WAVE_LF in FP64 or FP32C, TEST_HASH in FP64 (other
 * schemes return EUNSUPPORTED). Each grid keeps its own state, layout and
 * conversions as a single handle with the same pde and precision, and its
 * own sub-step counter; results equal a single handle's bit for bit. */
typedef struct swept2d_batch swept2d_batch;

#define SWEPT2D_TUNE_MODEL 0   /* tile sides from the cost model */
#define SWEPT2D_TUNE_MEASURE 1 /* tile sides from timed trial runs */

/* count grids; grid i is nx[i] x ny[i] (3..65536 per side, any shape), pde
 * pde[i] with its nvars and substeps, precision prec[i], parameters
 * params[i * params_stride ...] (as swept2d_set_params; params may be NULL
 * when no grid takes any). States start at zero, tile sides from the model.
 * NULL on error (see swept2d_last_error). */
swept2d_batch *swept2d_batch_create(int count, const int *nx, const int *ny, const int *pde, const int *prec,
                                    const double *params, int params_stride);
/* Waits for pending work, frees every device buffer of the batch. */
void swept2d_batch_destroy(swept2d_batch *b);
int swept2d_batch_count(const swept2d_batch *b);

/* Tile side of grid idx: n > 0 an even side dividing both grid sides (EINVAL
 * otherwise), 0 the model's choice (a square side, rectangular tiles when no
 * square side is usable, or the per-step method), negative the per-step
 * method. get returns the side, 0 for rectangular tiles or the per-step
 * method, or EINVAL. */
int swept2d_batch_set_tile(swept2d_batch *b, int idx, int n);
int swept2d_batch_get_tile(const swept2d_batch *b, int idx);

/* Rectangular tiles of half-cycle height hh (1..64) for grid idx, as
 * swept2d_set_rect for a handle; EINVAL if a side is below 2 hh or the
 * window exceeds the LDS. get returns the height, 0 when the grid runs
 * square tiles or the per-step method, or EINVAL. */
int swept2d_batch_set_rect(swept2d_batch *b, int idx, int hh);
int swept2d_batch_get_rect(const swept2d_batch *b, int idx);

/* Choose every grid's tiling: SWEPT2D_TUNE_MODEL from the cost model,
 * SWEPT2D_TUNE_MEASURE by timing each distinct grid (shape, pde, precision,
 * parameters) alone on a copy of its state at every usable square side up
 * to 64 and rectangular height 8, 12, .., 32, and keeping the fastest per
 * sub-step. Grid states are not changed. */
int swept2d_batch_autotune(swept2d_batch *b, int mode);

/* State of grid idx from / to the host, FP64 [nvars][ny][nx] (converted as
 * swept2d_upload / swept2d_download). download waits for the batch and
 * reports EABORTED if its last advance stopped. */
int swept2d_batch_upload(swept2d_batch *b, int idx, const double *host);
int swept2d_batch_download(swept2d_batch *b, int idx, double *host);

/* Advance every grid by nsteps full steps: one graph launch (asynchronous).
 * EINVAL if nsteps < 0; 0 is a no-op. */
int swept2d_batch_advance(swept2d_batch *b, long long nsteps);

/* Wait for the batch; EABORTED if a persistent kernel stopped on its wait
 * limit (grid states are then undefined), EHIP on a kernel fault. */
int swept2d_batch_synchronize(swept2d_batch *b);

/* Sub-steps grid idx has advanced, or EINVAL. */
long long swept2d_batch_substep_counter(const swept2d_batch *b, int idx);

#define SWEPT2D_BATCH_PHASED 0
#define SWEPT2D_BATCH_PERSISTENT 1
/* Select how advances run (see above); EINVAL for an unknown mode. get
 * returns the mode or EINVAL. */
int swept2d_batch_set_mode(swept2d_batch *b, int mode);
int swept2d_batch_get_mode(const swept2d_batch *b);

/* Kernel launches one advance of nsteps (1..1024) makes in the current mode
 * (builds and keeps its graph), or a negative error code. */
int swept2d_batch_launches(swept2d_batch *b, long long nsteps);

/* Persistent mode: longest time, in microseconds, a work item waits for its
 * dependency before the kernel stops with EABORTED (default 2 s). 0 stops at
 * the first wait that is not already satisfied. No effect on phased
 * advances, which never wait. */
int swept2d_batch_set_wait_limit(swept2d_batch *b, long long microseconds);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT2D_H */
