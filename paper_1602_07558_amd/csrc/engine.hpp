// Launch descriptors shared by the kernels (stages.hpp, swept2d_kernels.hip)
// and the host planners (swept2d_api.cpp, swept2d_batch.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/swept2d.h"
#include "schemes.hpp"

namespace swept {

// Thread layout of a stage kernel instantiation (WC: compile-time window
// pitch, 66 for tile side 64, 34 for 32, 18 for 16, 0 for any other side).
//  - Schemes with at most 16 bytes of state per point ("light") run 16 waves
//    at tile side 64, one wave at 16 and for other sides up to 22 (set by the
//    launcher), 4 waves otherwise; the Euler schemes 8 waves. A level is a short chain of
//    dependent LDS and arithmetic latencies ended by a barrier, so many waves
//    with few rows each hide it best (4 waves with 16 rows each measured
//    twice as slow at tile side 64).
//  - Light schemes at a fixed pitch use column ownership: thread t owns
//    window column 1 + t mod N and the R rows from 1 + R (t div N) at every
//    level, N = WC - 2, R = N^2 / NT. Otherwise a level is split into 2x2
//    quads handed out round robin.
//  - NTo overrides the workgroup size (the batched persistent kernel runs
//    every stage with one size).
// Schemes whose levels run as a column walk (S::WALK, the Euler schemes).
template <class S, class = void>
struct walks : std::false_type {};
template <class S>
struct walks<S, std::void_t<decltype(S::WALK)>> : std::bool_constant<S::WALK> {};

template <class S, int WC, int NTo = 0>
struct Lay {
  static constexpr bool light = S::NW * (int)sizeof(typename S::V) <= 16;
  static constexpr int N = WC ? WC - 2 : 0;
  static constexpr int NT =
      NTo ? NTo : (!light ? 512 : (WC == 66 ? 1024 : (WC == 18 ? 64 : 256)));
  static constexpr int NW = NT / 64;
  static constexpr bool cols = light && WC != 0 && (N * N) % NT == 0;
  static constexpr int R = cols ? N * N / NT : 0;
};

// Geometry of one half cycle of the swept decomposition.
//
// Tiles are n x n squares, n = 2h, whose north-west points sit at
// (off + a n, off + b n) modulo (nx, ny), a < ntx = nx/n, b < nty = ny/n; off is
// 0 or h and alternates between half cycles (Sec. 4: each half cycle shifts
// the arrangement by half a tile). Level l of the half cycle is global
// sub-step level T0 + l.
//
// Within a half cycle of height H (H = h for a full one, H < h only for the
// last, reduced one), with dx, dy the distance of a point to the nearest
// tile edge in x and y (0 on the outermost ring of the tile), level l in
// 1..H of the point is computed by
//   the upward pyramid          if dx >= l and dy >= l,
//   the bridge across an x-edge if dx <  l and dy >= l  (x-bridge),
//   the bridge across a y-edge  if dx >= l and dy <  l  (y-bridge),
//   the downward pyramid        if dx <  l and dy <  l.
// For H = h this is the paper's decomposition (Sec. 3): the upward pyramid
// of Alg. 1 holds levels 0..h-1, the bridges of Alg. 2-3 levels 1..h-1, the
// downward pyramid of Alg. 4 levels 1..h and ends as the full tile centred on
// the corner. The x-bridge is Alg. 3's latitudinal bridge (it joins a tile to
// its east neighbour), the y-bridge Alg. 2's longitudinal bridge.
struct Geo {
  int nx, ny;      // grid
  int n, h;        // tile side, h = n/2
  int ntx, nty;    // tiles in x and y
  int off;         // tiling offset (x and y)
  int W;           // LDS window side n + 2
  long long T0;    // level at the start of the half cycle, relative to *tbase
  const long long* tbase;  // device-resident level base (graph replay), or null
};

// Panels exchanged through HBM (the triangular sides of Sec. 3).
// Every panel is stored compactly, level after level, each level as
// [value v][k][t] with k = 0 the row or column nearer the edge the panel
// faces and t running along that edge over the level's valid range only:
//  up: upward-pyramid strip of one side (ends N, S, W, E) of a tile: the two
//      outermost rows / columns of the level-l square, t = 0 .. n-2l-1 for
//      tile-local positions l .. n-1-l.
//  xb: x-bridge over the east edge of tile (a, b), ends N, S: two rows of the
//      bridge's level-l band plus the 2x2 pyramid corners beside it,
//      2l+4 long, t = 0 at x = edge - l - 2.
//  yb: y-bridge over the south edge of tile (a, b), ends W, E: two columns of
//      the band, 2l long, t = 0 at y = edge - l.
// The downward pyramid at the south-east corner of tile (a, b) reads the
// S end of xb(a, b), the N end of xb(a, b+1), the E end of yb(a, b) and the
// W end of yb(a+1, b): the ring two wide around its level-l square, corners
// included (they arrive with the x-bridges).
struct PanelPtrs {
  void* up;
  void* xb;
  void* yb;
};

// Values of one end of a panel over levels 0..L-1, per value slot and k
// (multiply by 2 * nv for values).
__host__ __device__ inline int up_levels_len(int n, int L) { return L * (n - L + 1); }
__host__ __device__ inline int xb_levels_len(int L) { return L * (L + 3); }
__host__ __device__ inline int yb_levels_len(int L) { return L * (L - 1); }

inline size_t up_panel_values(int ntiles, int n, int nv) {
  return (size_t)ntiles * 4 * 2 * nv * up_levels_len(n, n / 2);
}
inline size_t xb_panel_values(int ntiles, int n, int nv) { return (size_t)ntiles * 2 * 2 * nv * xb_levels_len(n / 2); }
inline size_t yb_panel_values(int ntiles, int n, int nv) { return (size_t)ntiles * 2 * 2 * nv * yb_levels_len(n / 2); }

enum Scheme : int {
  kHeat64 = 0,
  kWave64,
  kEuler64,
  kHash64,
  kIncr64,
  kPush5,
  kHeat32C,
  kWave32C,
  kEuler32C,
  kHeat32R,
  kWave32R,
  kHash25x2,
  kEulerFD64,
  kEulerFD32C,
  kNumSchemes
};

// Rectangular tiles of any side (the level function above partitions a half
// cycle of H levels over any tiling whose tile sides are all at least 2H).
// An axis of length L >= 2h is cut into t = floor(L / 2h) tiles: tiling 0
// has tile i at start i*base + min(i, rem), width base + (i < rem ? 1 : 0)
// (base = floor(L / t), rem = L mod t), so widths differ by at most one and
// are at least 2h. Tiling 1 has its edges at tiling 0's midpoints, tile i
// starting at start0(i) + floor(width0(i) / 2); its widths are again base or
// base + 1. The two alternate between half cycles: every tile of one holds
// exactly one edge (corner) of the other at least h cells from its own
// edges, so a downward pyramid's 2h x 2h square at a corner of one tiling
// lies inside a tile of the next, and the stage that finishes the downward
// pyramid continues as that tile's upward frustum. A tile wider than 2H
// leaves regions that no downward pyramid covers at level H (the frustum's
// flat top, the bridges' middles); their stages write them to the state,
// and the next half cycle's frustum reads them back from there.
struct RAxis {
  int L;     // cells
  int t;     // tiles
  int base;  // floor(L / t)
  int rem;   // L mod t: the first rem tiles of tiling 0 are one wider
};

__host__ __device__ inline int rect_width0(const RAxis& a, int i) { return a.base + (i < a.rem ? 1 : 0); }
__host__ __device__ inline int rect_start0(const RAxis& a, int i) { return i * a.base + (i < a.rem ? i : a.rem); }
// Start (0 <= s < L) and width of tile i of tiling par.
__host__ __device__ inline void rect_span(const RAxis& a, int par, int i, int& s, int& w) {
  const int s0 = rect_start0(a, i), w0 = rect_width0(a, i);
  if (par == 0) {
    s = s0;
    w = w0;
    return;
  }
  const int j = (i + 1 == a.t) ? 0 : i + 1;
  const int s1 = rect_start0(a, j) + rect_width0(a, j) / 2 + (j == 0 ? a.L : 0);
  s = s0 + w0 / 2;
  w = s1 - s;
}

constexpr int kRectThreads = 256;  // workgroup size of the rectangular-tile stages

struct RGeo {
  RAxis ax, ay;
  int h;        // half-cycle height the tiles are cut for (every side >= 2h)
  int P;        // LDS window pitch and rows: widest tile + 2
  int urow;     // values per row of an upward-frustum panel level: widest tile
  long long T0;            // level at the start of the half cycle, relative to *tbase
  const long long* tbase;  // device-resident level base (graph replay), or null
};

// Light schemes (at most 16 bytes per point in the window) run the column
// layout at the fixed pitches.
inline bool light_scheme(int nw, int vbytes) { return nw * vbytes <= 16; }

inline RAxis rect_axis(int L, int h) {
  RAxis a{};
  a.L = L;
  a.t = L / (2 * h);
  a.base = a.t > 0 ? L / a.t : 0;
  a.rem = a.t > 0 ? L % a.t : 0;
  return a;
}
inline int rect_widest(const RAxis& a) { return a.base + (a.rem ? 1 : 0); }
// Geometry for an nx x ny grid at half-cycle height h (tiles: 0 if an axis
// is shorter than 2h). A light scheme's window takes pitch 34 or 66 when
// every tile is at most 32 or 64 wide (the fixed-pitch level code).
inline RGeo rect_geo(int nx, int ny, int h, bool light) {
  RGeo g{};
  g.h = h;
  g.ax = rect_axis(nx, h);
  g.ay = rect_axis(ny, h);
  g.urow = rect_widest(g.ax) > rect_widest(g.ay) ? rect_widest(g.ax) : rect_widest(g.ay);
  g.P = light && g.urow <= 32 ? 34 : (light && g.urow <= 64 ? 66 : g.urow + 2);
  return g;
}
inline int rect_tiles(const RGeo& g) { return g.ax.t * g.ay.t; }
// Panel values (the same three buffers as the square tiles'): per tile and
// level, an upward-frustum end holds 2 rows of urow values per value slot,
// an x-bridge end 2 rows of 2h + 4 (its band and the frustum corners beside
// it), a y-bridge end 2 rows of 2h; levels 0..h-1.
inline size_t rect_up_values(const RGeo& g, int nv) { return (size_t)rect_tiles(g) * 4 * g.h * 2 * nv * g.urow; }
inline size_t rect_xb_values(const RGeo& g, int nv) {
  return (size_t)rect_tiles(g) * 2 * g.h * 2 * nv * (2 * g.h + 4);
}
inline size_t rect_yb_values(const RGeo& g, int nv) { return (size_t)rect_tiles(g) * 2 * g.h * 2 * nv * (2 * g.h); }

// User schemes (swept2d_register_scheme) take scheme ids kNumSchemes + k;
// their launchers are the registered table's.
constexpr int kMaxUserSchemes = 32;
const swept2d_scheme_ops* user_scheme(int k);  // k-th registered table, or null
int add_user_scheme(const swept2d_scheme_ops& ops);  // its index, or -1 when full

// Launch entry points (swept2d_kernels.hip dispatches them). Each returns the
// hipError_t of the launch.
//   up:     upward pyramid of every tile from the state (height H; emits
//           panels of levels 0..H-1; if H < h writes its level-H region to
//           the state).
//   bridge: x- and y-bridges of every edge (height H; same conventions);
//           with pair_ok, tile sides 32 and 64 run both bridges of a tile
//           in one workgroup where two fit its LDS.
//   oct:    downward pyramid of height Hd at every tile corner; if Hd == h
//           and Hu > 0 it continues in LDS as the upward pyramid of the
//           shifted tile (an octahedron) of height Hu; the last stage of an
//           advance writes its region at the final level to the state.
//   plain:  one sub-step of every point, in -> out.
// `staged`: the kernel copies all panel inputs of the component into LDS at
// its start (one memory latency); otherwise it fetches each level's inputs
// one level ahead into registers.
hipError_t launch_up(int scheme, const Geo& g, int H, void* state, PanelPtrs p, const SchemeParams& sp,
                     hipStream_t s);
hipError_t launch_bridge(int scheme, const Geo& g, int H, bool staged, bool pair_ok, void* state, PanelPtrs p,
                         const SchemeParams& sp, hipStream_t s);
// Whether the octahedron of tile side n fetches its ring runs from HBM a few
// levels ahead with precomputed per-wave terms (then staging gains nothing).
bool oct_fetch_ahead(int scheme, int n);
hipError_t launch_oct(int scheme, const Geo& g, int Hd, int Hu, bool staged, void* state, PanelPtrs p,
                      const SchemeParams& sp, hipStream_t s);
hipError_t launch_plain(int scheme, int nx, int ny, long long T, const long long* tbase, const void* in, void* out,
                        const SchemeParams& sp, hipStream_t s);
// Rectangular tiles (RGeo): one workgroup per tile of tiling upar runs the
// downward pyramid of height Hd at the corner of tiling 1 - upar inside it
// (none if Hd == 0), loads the rest of the tile from the state, and
// continues as the tile's upward frustum of height Hu (Hu == 0: it writes
// the downward pyramid's square to the state instead); the frustum writes
// its panels and its level-Hu top. rect_bridge runs the x- and y-bridges of
// every edge of tiling par (2 t_x t_y workgroups), each writing its panels
// and its level-H band. Built-in schemes with nw == nv only (hipErrorNotSupported
// otherwise).
hipError_t launch_rect_oct(int scheme, const RGeo& g, int upar, int Hd, int Hu, void* state, PanelPtrs p,
                           const SchemeParams& sp, hipStream_t s);
hipError_t launch_rect_bridge(int scheme, const RGeo& g, int par, int H, void* state, PanelPtrs p,
                              const SchemeParams& sp, hipStream_t s);
// Device-side helpers that are safe inside a captured graph: copy `bytes`
// (a multiple of 8) and set the level base.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_set_base(long long* tbase, long long value, hipStream_t s);

// Static facts about a scheme.
struct SchemeInfo {
  int nv;          // values per point in the state and the panels
  int nw;          // values per point in the LDS window (nv plus window-only values)
  int nvar;        // the scheme's nvars
  int sub;         // sub-steps per step
  int vbytes;      // bytes per value
};
SchemeInfo scheme_info(int scheme);

// LDS bytes of the stage kernels for tile side n: a double-buffered
// (n+2)^2 window per window value, plus the staged panel inputs.
inline size_t window_lds_bytes(const SchemeInfo& si, int n) {
  return (size_t)2 * (size_t)(n + 2) * (size_t)(n + 2) * (size_t)si.nw * (size_t)si.vbytes;
}
inline size_t oct_stage_bytes(const SchemeInfo& si, int n) {
  const int h = n / 2;
  return (size_t)2 * 2 * si.nv * (size_t)(xb_levels_len(h) + yb_levels_len(h)) * si.vbytes;
}
inline size_t bridge_stage_bytes(const SchemeInfo& si, int n) {
  return (size_t)2 * 2 * si.nv * (size_t)up_levels_len(n, n / 2) * si.vbytes;
}
// LDS of a rectangular-tile stage: a double-buffered P x P window per value.
inline size_t rect_lds_bytes(const SchemeInfo& si, const RGeo& g) {
  return (size_t)2 * (size_t)g.P * (size_t)g.P * (size_t)si.nw * (size_t)si.vbytes;
}
// Largest panel run per level is n + 2 values; the per-level fetch path holds
// two per lane.
inline bool tile_fits_fetch(int n) { return n + 2 <= 128; }

// Raise the dynamic LDS limit of every stage kernel to `bytes` (once).
hipError_t configure_lds(size_t bytes);

// ------------------------------------------------------------------ batch
//
// A batch advances many independent grids. A grid's work is a sequence of
// phases: phase 0 is its upward pyramid, odd phases its bridges (2 items per
// tile), even phases its octahedra (1 item per tile); a per-step grid has
// one phase per sub-step (one item per 64 x 64 block) plus, after an odd
// count, a copy back. Phase p of a grid may start once its phase p - 1 has
// completed.
//
// Phased launches (the default): the phases of all grids are laid out on a
// common sequence of slots (grid g's phase j in slot floor(j L / P_g), L the
// largest phase count, so every grid's phases are spread evenly and keep
// their order). A slot is one kernel launch per launch class (workgroup size
// and window pitch), each workgroup running one item of one grid; kernel
// boundaries order the slots, so no workgroup ever waits for another. All
// launches of an advance are one captured HIP graph.
//
// Persistent (compiled only with SWEPT2D_BUILD_PERSISTENT_BATCH): one kernel whose
// workgroups take items from a device counter and wait on per-grid
// completion counters.
constexpr int kBatchThreads = 1024;
constexpr int kBatchBlock = 64;  // side of a per-step block

enum BatchKind : int { kBatchSwept = 0, kBatchPlain = 1, kBatchRect = 2 };

// Launch classes of the phased batch: the stage code of tile side 64 on 16
// waves, of tile side 32 on 4 waves, of tile side 16 on one wave, of any
// other side on 4 waves, of other sides up to 22 on one wave, and of
// rectangular tiles at window pitch 66 (16 waves), 34 (4 waves) or a
// run-time pitch (4 waves); per-step grids run in the 4-wave generic class.
// One-wave items always stage their panel inputs.
enum BatchClass : int {
  kClass66 = 0,
  kClass34,
  kClass18,
  kClassGen256,
  kClassGen64,
  kClassRect66,
  kClassRect34,
  kClassRect0,
  kNumBatchClasses
};
// Window-pitch template argument of a batch launch class that marks the
// rectangular-tile stage code: -66, -34, or -1 for the run-time pitch.
constexpr int rect_marker(int pitch) { return pitch == 66 || pitch == 34 ? -pitch : -1; }
inline int batch_class_of(int n, int rect_h = 0, int rect_pitch = 0) {
  if (rect_h > 0) return rect_pitch == 66 ? kClassRect66 : (rect_pitch == 34 ? kClassRect34 : kClassRect0);
  if (n == 64) return kClass66;
  if (n == 32) return kClass34;
  if (n == 16) return kClass18;
  if (n != 0 && n <= 22) return kClassGen64;
  return kClassGen256;
}
inline int batch_class_threads(int c) {
  return (c == kClass66 || c == kClassRect66) ? 1024 : ((c == kClassGen64 || c == kClass18) ? 64 : 256);
}

struct BatchGrid {
  Geo g0;          // off 0, T0 = the grid's level at the start of an advance
  RGeo rg;         // rectangular tiles (kind kBatchRect; its T0 unused)
  int scheme;      // Scheme (light schemes only)
  int kind;        // BatchKind
  int wc;          // window pitch of the stage code: 66, 34 or 0
  int staged_oct, staged_bridge;
  int units;       // tiles, or per-step blocks
  void* state;
  void* state2;    // second buffer of a per-step grid
  PanelPtrs pp;
  SchemeParams sp;
};

// Per-grid split of one advance of S sub-steps (h = n/2, or the height of
// the rectangular tiles): q full half cycles and a reduced one of height r,
// or S per-step phases.
struct BatchPlan {
  long long S;
  long long q;
  int r;
  int nphases;
};

// One launch of a slot: workgroup b runs item b - cum[j] of phase phase[j]
// of grid grid[j], j the last entry with cum[j] <= b (cum[0] = 0, cum[n] =
// the launch's workgroup count).
struct PhaseLaunch {
  const BatchGrid* grids;
  const BatchPlan* plans;
  const int* grid;
  const int* phase;
  const int* cum;
  int n;
};

hipError_t launch_batch_phase(int cls, const PhaseLaunch& L, int blocks, size_t lds, hipStream_t st);
hipError_t batch_phase_resident(int cls, size_t lds, int* out);
// grids[i].g0.T0 += plans[i].S for every grid.
hipError_t launch_batch_bump(BatchGrid* grids, const BatchPlan* plans, int ngrids, hipStream_t st);
bool batch_scheme_supported(int scheme);

#ifdef SWEPT2D_BUILD_PERSISTENT_BATCH
// Items are numbered phase by phase; within a phase, grid by grid in `order`
// (grids with more phases first, so the grids active in phase p are a
// prefix of `order`). Workgroups take items in that order from one counter,
// and an item of phase p waits until its grid has completed every item of
// phases < p; a wait longer than `wait_ticks` sets `error` and every
// workgroup stops.
struct BatchSched {
  long long total;
  int nphases;
  int ngrids;
  const long long* phase_base;  // nphases + 1 ticket offsets
  const int* phase_active;      // grids active in each phase
  const int* order;
  const long long* cum1;        // per-grid item prefix over `order`, phases 0 and even
  const long long* cum2;        // same, odd phases
  BatchGrid* grids;
  const BatchPlan* plans;
  unsigned* done;               // items completed per grid
  unsigned long long* head;     // next ticket
  int* error;
  long long wait_ticks;         // longest dependency wait, in 100 MHz ticks
};

hipError_t launch_batch(const BatchSched& s, int blocks, size_t lds, hipStream_t st);
// done[] = 0 and *head = 0 (a kernel, so it may sit in a captured graph).
hipError_t launch_batch_reset(unsigned* done, int ngrids, unsigned long long* head, hipStream_t st);
// Resident workgroups of the persistent kernel per compute unit at `lds` bytes.
hipError_t batch_blocks_per_cu(size_t lds, int* out);
#endif

// Launchers of one scheme's stage kernels (defined in stages.hpp, explicitly
// instantiated once per scheme in its own translation unit).
template <class S>
struct Stages {
  static SchemeInfo info();
  static hipError_t up(const Geo& g, int H, void* state, PanelPtrs p, const SchemeParams& sp, hipStream_t s);
  static hipError_t bridge(const Geo& g, int H, bool staged, bool pair_ok, void* state, PanelPtrs p,
                           const SchemeParams& sp, hipStream_t s);
  static hipError_t oct(const Geo& g, int Hd, int Hu, bool staged, void* state, PanelPtrs p, const SchemeParams& sp,
                        hipStream_t s);
  static hipError_t plain(int nx, int ny, long long T, const long long* tbase, const void* in, void* out,
                          const SchemeParams& sp, hipStream_t s);
  static hipError_t lds(size_t bytes);
  static bool fetch_ahead(int n);
  static hipError_t rect_oct(const RGeo& g, int upar, int Hd, int Hu, void* state, PanelPtrs p,
                             const SchemeParams& sp, hipStream_t s);
  static hipError_t rect_bridge(const RGeo& g, int par, int H, void* state, PanelPtrs p, const SchemeParams& sp,
                                hipStream_t s);
};

// Kernel of one batch launch class (window pitch WC, NT threads).
template <int WC, int NT>
struct BatchPhase {
  static hipError_t launch(const PhaseLaunch& L, int blocks, size_t lds, hipStream_t st);
  static hipError_t lds(int bytes);
  // Workgroups resident per compute unit at `lds` bytes of dynamic LDS.
  static hipError_t resident(size_t lds, int* out);
};

// Host helpers shared by the host files (swept2d_api.cpp).
int set_error(int code, const char* fmt, ...);  // message kept per thread
size_t device_lds_limit();
int device_setup(int* device_out);
int scheme_for(int pde, int prec);
int pde_param_count(int pde);
int pde_var_count(int pde);
int pde_substep_count(int pde);

}  // namespace swept
