// Host side of the swept2d C ABI: validation, device memory, the half-cycle
// schedule of the swept rule (Algorithm 5), the per-step baseline, HIP graph
// replay, per-kernel timing and the tile-size tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/swept2d.h"
#include "engine.hpp"

using namespace swept;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hipfail(hipError_t e, const char* what) {
  return fail(SWEPT2D_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hipfail(e_, what); \
  } while (0)

enum Kind { kKindPlain = 0, kKindUp = 1, kKindBridge = 2, kKindOct = 3, kNumKinds = 4 };

struct TimedLaunch {
  int kind;
  double work;
  hipEvent_t a, b;
};

const swept2d_scheme_ops* user_pde(int pde) {
  return pde >= SWEPT2D_USER_PDE_BASE ? user_scheme(pde - SWEPT2D_USER_PDE_BASE) : nullptr;
}

int pde_nvars(int pde) {
  if (const swept2d_scheme_ops* u = user_pde(pde)) return u->nvars;
  switch (pde) {
    case SWEPT2D_HEAT5: return 1;
    case SWEPT2D_WAVE_LF: return 2;
    case SWEPT2D_EULER_RUS_RK2: return 8;
    case SWEPT2D_EULER_FD_RK4: return 12;
    case SWEPT2D_TEST_HASH: return 1;
    case SWEPT2D_TEST_INCR: return 1;
    case SWEPT2D_TEST_PUSH5: return 5;
    case SWEPT2D_TEST_HASH25: return Hash25x2::NVAR;
    default: return -1;
  }
}

int pde_substeps(int pde) {
  if (const swept2d_scheme_ops* u = user_pde(pde)) return u->substeps;
  switch (pde) {
    case SWEPT2D_EULER_RUS_RK2:
    case SWEPT2D_TEST_PUSH5:
    case SWEPT2D_TEST_HASH25: return 2;
    case SWEPT2D_EULER_FD_RK4: return 4;
    default: return pde_nvars(pde) > 0 ? 1 : -1;
  }
}

int pde_nparams(int pde) {
  if (const swept2d_scheme_ops* u = user_pde(pde)) return u->nparams;
  switch (pde) {
    case SWEPT2D_HEAT5: return 1;
    case SWEPT2D_WAVE_LF: return 1;
    case SWEPT2D_EULER_RUS_RK2: return 2;
    case SWEPT2D_EULER_FD_RK4: return 2;
    default: return 0;
  }
}

int scheme_of(int pde, int prec) {
  if (prec == SWEPT2D_FP64) {
    switch (pde) {
      case SWEPT2D_HEAT5: return kHeat64;
      case SWEPT2D_WAVE_LF: return kWave64;
      case SWEPT2D_EULER_RUS_RK2: return kEuler64;
      case SWEPT2D_EULER_FD_RK4: return kEulerFD64;
      case SWEPT2D_TEST_HASH: return kHash64;
      case SWEPT2D_TEST_INCR: return kIncr64;
      case SWEPT2D_TEST_PUSH5: return kPush5;
      case SWEPT2D_TEST_HASH25: return kHash25x2;
    }
    if (pde >= SWEPT2D_USER_PDE_BASE && user_pde(pde)) return kNumSchemes + (pde - SWEPT2D_USER_PDE_BASE);
  } else if (prec == SWEPT2D_FP32C) {
    switch (pde) {
      case SWEPT2D_HEAT5: return kHeat32C;
      case SWEPT2D_WAVE_LF: return kWave32C;
      case SWEPT2D_EULER_RUS_RK2: return kEuler32C;
      case SWEPT2D_EULER_FD_RK4: return kEulerFD32C;
    }
  } else if (prec == SWEPT2D_FP32R) {
    switch (pde) {
      case SWEPT2D_HEAT5: return kHeat32R;
      case SWEPT2D_WAVE_LF: return kWave32R;
    }
  }
  return -1;
}

// Each device's kernels get their dynamic-LDS limit once, the first time a
// handle is made on it; handles may be created from several threads at
// once. g_lds_limit is the smallest per-workgroup LDS of the devices set up
// (one value on a node of one GPU model).
constexpr int kMaxSetupDevices = 64;
std::mutex g_setup_mu;
bool g_setup_done[kMaxSetupDevices] = {};
std::atomic<size_t> g_lds_limit{0};

int ensure_device_setup(int* device_out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxSetupDevices)
    return swept::set_error(SWEPT2D_EUNSUPPORTED, "device %d beyond the %d the library sets up", dev,
                            kMaxSetupDevices);
  std::lock_guard<std::mutex> lock(g_setup_mu);
  if (!g_setup_done[dev]) {
    int lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    HIP_TRY(configure_lds((size_t)lds), "hipFuncSetAttribute");  // on the current device
    for (int k = 0; const swept2d_scheme_ops* u = user_scheme(k); ++k)
      HIP_TRY(static_cast<hipError_t>(u->lds((size_t)lds)), "scheme LDS limit");
    const size_t cur = g_lds_limit.load();
    if (cur == 0 || (size_t)lds < cur) g_lds_limit.store((size_t)lds);
    g_setup_done[dev] = true;
  }
  *device_out = dev;
  return 0;
}

// Registers a user scheme: its kernels' LDS limit is set on every device
// set up so far (devices set up later take it from the table), and it joins
// the table under the same lock, so no device misses it. Returns its index,
// or a negative error code.
int register_user_scheme(const swept2d_scheme_ops& ops) {
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_setup_mu);
  int rc = 0;
  for (int d = 0; d < kMaxSetupDevices && rc == 0; ++d) {
    if (!g_setup_done[d]) continue;
    hipError_t e = hipSetDevice(d);
    if (e == hipSuccess) e = static_cast<hipError_t>(ops.lds(g_lds_limit));
    if (e != hipSuccess) rc = hipfail(e, "scheme LDS limit");
  }
  const hipError_t back = hipSetDevice(cur);
  if (rc) return rc;
  if (back != hipSuccess) return hipfail(back, "hipSetDevice");
  const int k = add_user_scheme(ops);
  if (k < 0) return swept::set_error(SWEPT2D_EUNSUPPORTED, "%d user schemes are registered already", kMaxUserSchemes);
  return k;
}

}  // namespace

namespace swept {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
size_t device_lds_limit() { return g_lds_limit; }
int device_setup(int* device_out) { return ensure_device_setup(device_out); }
int scheme_for(int pde, int prec) { return scheme_of(pde, prec); }
int pde_param_count(int pde) { return pde_nparams(pde); }
int pde_var_count(int pde) { return pde_nvars(pde); }
int pde_substep_count(int pde) { return pde_substeps(pde); }
}  // namespace swept

struct swept2d {
  int nx = 0, ny = 0, nvars = 0, pde = 0, substeps = 0, prec = SWEPT2D_FP64;
  int scheme = 0;
  SchemeInfo si{};
  SchemeParams sp{};
  int device = 0;
  int cu_count = 0;
  int n = 0;  // tile side
  void* state = nullptr;
  bool owns_state = true;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  void* scratch = nullptr;  // second state buffer of the per-step method
  void* up = nullptr;
  void* xb = nullptr;
  void* yb = nullptr;
  size_t panel_tile = 0;    // tile side the panels are sized for
  int rect_h = 0;           // half-cycle height of rectangular tiles (0: square tiles of side n)
  int panel_rect = 0;       // rectangular-tile height the panels are sized for
  long long T = 0;          // global sub-step counter
  long long* d_tbase = nullptr;  // device copy of the level base for graph replay
  int launch_mode = SWEPT2D_LAUNCH_DIRECT;
  int staging = SWEPT2D_STAGING_AUTO;
  std::map<std::pair<int, long long>, hipGraphExec_t> graphs;  // (method, substeps) -> replayable graph
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
};

namespace {

size_t state_bytes_of(const swept2d* h) {
  return (size_t)h->nx * h->ny * h->si.nv * h->si.vbytes;
}

void drop_graphs(swept2d* h) {
  for (auto& kv : h->graphs) hipGraphExecDestroy(kv.second);
  h->graphs.clear();
}

int alloc_state(swept2d* h) {
  if (h->owns_state && h->state) hipFree(h->state);
  h->state = nullptr;
  h->owns_state = true;
  const size_t bytes = state_bytes_of(h);
  if (hipMalloc(&h->state, bytes) != hipSuccess) {
    hipGetLastError();
    h->state = nullptr;
    return fail(SWEPT2D_ENOMEM, "cannot allocate %zu bytes of state", bytes);
  }
  HIP_TRY(hipMemsetAsync(h->state, 0, bytes, h->stream), "hipMemsetAsync");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (h->scratch) hipFree(h->scratch);
  h->scratch = nullptr;
  drop_graphs(h);
  return 0;
}

int ensure_scratch(swept2d* h) {
  if (h->scratch) return 0;
  const size_t bytes = state_bytes_of(h);
  if (hipMalloc(&h->scratch, bytes) != hipSuccess) {
    hipGetLastError();
    h->scratch = nullptr;
    return fail(SWEPT2D_ENOMEM, "cannot allocate %zu bytes of per-step scratch", bytes);
  }
  return 0;
}

void free_panels(swept2d* h) {
  if (h->up) hipFree(h->up);
  if (h->xb) hipFree(h->xb);
  if (h->yb) hipFree(h->yb);
  h->up = h->xb = h->yb = nullptr;
  h->panel_tile = 0;
  h->panel_rect = 0;
}

int ensure_panels(swept2d* h) {
  if (h->up && (h->rect_h ? h->panel_rect == h->rect_h : (h->panel_rect == 0 && h->panel_tile == (size_t)h->n)))
    return 0;
  free_panels(h);
  const size_t vb = h->si.vbytes;
  size_t ub, xbb, ybb;
  if (h->rect_h) {
    const RGeo g = rect_geo(h->nx, h->ny, h->rect_h, light_scheme(h->si.nw, h->si.vbytes));
    ub = rect_up_values(g, h->si.nv) * vb;
    xbb = rect_xb_values(g, h->si.nv) * vb;
    ybb = rect_yb_values(g, h->si.nv) * vb;
  } else {
    const int ntiles = (h->nx / h->n) * (h->ny / h->n);
    ub = up_panel_values(ntiles, h->n, h->si.nv) * vb;
    xbb = xb_panel_values(ntiles, h->n, h->si.nv) * vb;
    ybb = yb_panel_values(ntiles, h->n, h->si.nv) * vb;
  }
  ub = std::max<size_t>(8, ub);
  xbb = std::max<size_t>(8, xbb);
  ybb = std::max<size_t>(8, ybb);
  if (hipMalloc(&h->up, ub) != hipSuccess || hipMalloc(&h->xb, xbb) != hipSuccess ||
      hipMalloc(&h->yb, ybb) != hipSuccess) {
    hipGetLastError();
    free_panels(h);
    return fail(SWEPT2D_ENOMEM, "cannot allocate panels (%zu + %zu + %zu bytes)", ub, xbb, ybb);
  }
  if (h->rect_h)
    h->panel_rect = h->rect_h;
  else
    h->panel_tile = (size_t)h->n;
  drop_graphs(h);
  return 0;
}

// Why rectangular tiles of half-cycle height hh cannot serve the handle, or
// nullptr.
const char* rect_problem(const swept2d* h, int hh) {
  if (hh < 1) return "half-cycle height must be at least 1";
  if (h->nx < 2 * hh || h->ny < 2 * hh) return "nx and ny must be at least twice the half-cycle height";
  if (user_scheme(h->scheme - kNumSchemes)) return "registered user schemes run square tiles only";
  if (h->si.nw != h->si.nv) return "FP32R runs square tiles only";
  if (rect_lds_bytes(h->si, rect_geo(h->nx, h->ny, hh, light_scheme(h->si.nw, h->si.vbytes))) > g_lds_limit) return "tile window exceeds the workgroup LDS";
  return nullptr;
}

// Why a tile side is not usable, or nullptr.
const char* tile_problem(const swept2d* h, int n) {
  if (n < 2 || (n & 1)) return "tile side must be even and at least 2";
  if (h->nx % n || h->ny % n) return "tile side must divide nx and ny";
  if (window_lds_bytes(h->si, n) > g_lds_limit) return "tile working set exceeds the workgroup LDS";
  if (!tile_fits_fetch(n)) return "tile side above 126";
  return nullptr;
}

// Staging policy (one-wave groups stage whatever is asked). ON stages every
// component whose inputs fit the LDS; AUTO stages an octahedron only when it
// cannot fetch its ring runs ahead with precomputed per-wave terms and
// staging does not leave it alone on its compute unit, and no bridge (their fetch path runs three levels ahead); SINGLE_BRIDGES is AUTO
// with one staged workgroup per bridge; OFF stages nothing.
bool oct_staged(const swept2d* h) {
  if (h->staging == SWEPT2D_STAGING_OFF) return false;
  const size_t win = window_lds_bytes(h->si, h->n), st = win + oct_stage_bytes(h->si, h->n);
  if (st > g_lds_limit) return false;
  if (h->staging == SWEPT2D_STAGING_ON) return true;
  // AUTO does not stage where the staged workgroup would be alone on its
  // compute unit and the unstaged one would not (12-value Euler at tile side
  // 16: 2.73e9 point-steps/s staged, against 3.31e9 unstaged with two
  // workgroups per CU).
  if (g_lds_limit / st < 2 && g_lds_limit / win >= 2) return false;
  return !oct_fetch_ahead(h->scheme, h->n);
}

// At tile side 32, AUTO runs the bridges as SINGLE_BRIDGES does: one staged
// workgroup per bridge measured as fast as the pairs for heat and wave in
// FP64, Euler and wave FP32C, and faster for heat FP32C (7.1 against 7.6 ms
// per 2048 steps of 1024^2).
bool auto_single_bridges(const swept2d* h) { return h->staging == SWEPT2D_STAGING_AUTO && h->n == 32; }

bool bridge_staged(const swept2d* h) {
  if (h->staging == SWEPT2D_STAGING_OFF) return false;
  if (h->staging == SWEPT2D_STAGING_AUTO && !auto_single_bridges(h)) return false;
  return window_lds_bytes(h->si, h->n) + bridge_stage_bytes(h->si, h->n) <= g_lds_limit;
}

// Relative cost of one point sub-step of a scheme (heat FP64 = 1), for the
// tuner's cost model.
double scheme_cost(int scheme) {
  switch (scheme) {
    case kWave64: return 1.4;
    case kEuler64: return 30.0;
    case kEulerFD64: return 60.0;
    case kHash64: return 3.0;
    case kPush5: return 2.5;
    case kHeat32C: return 1.5;
    case kWave32C: return 2.2;
    case kHeat32R: return 1.5;
    case kWave32R: return 2.2;
    case kEuler32C: return 36.0;
    case kEulerFD32C: return 66.0;
    default: return 1.0;
  }
}

// Tile-size choice from the swept rule's cost model (Sec. 5, Eq. (4)): the
// time per sub-step is [2 tau + (half-cycle work) + (n/2) beta] / (n/2), where
// tau is the cost of one exchange (on one GPU, a kernel boundary), the work
// of a half cycle is n^2 * n/2 point updates per tile spread over the compute
// units (ceil(tiles / CUs) tiles in sequence per CU), and beta is the cost of
// one level's workgroup barrier, paid once per resident wave of tiles. The
// constants are rough gfx950 figures; the model only ranks tile sides.
int model_tile(const swept2d* h) {
  const double tau = 3.0e-6;
  const double s_cu = 0.17e-9 * scheme_cost(h->scheme);
  const double beta = 0.1e-6;
  int best = 0;
  double best_cost = 1e300;
  for (int n = 2; n <= std::min(h->nx, h->ny); n += 2) {
    if (tile_problem(h, n)) continue;
    const double tiles = (double)(h->nx / n) * (h->ny / n);
    const double per_cu = std::max(1.0, std::floor((double)g_lds_limit / (double)window_lds_bytes(h->si, n)));
    const double seq = std::ceil(tiles / h->cu_count);
    const double resident = std::ceil(tiles / (h->cu_count * std::min(per_cu, 8.0)));
    const double half = 2.0 * tau + seq * n * (double)n * (n / 2) * s_cu + resident * (n / 2) * beta;
    const double cost = half / (n / 2);
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best = n;
    }
  }
  return best;
}

// Half-cycle height of rectangular tiles by the same model: a tile of about
// (nx / t_x) x (ny / t_y) points, its levels computed one point per thread
// (weighted 2x against the square tiles' code).
int model_rect(const swept2d* h) {
  const double tau = 3.0e-6;
  const double s_cu = 2.0 * 0.17e-9 * scheme_cost(h->scheme);
  const double beta = 0.1e-6;
  int best = 0;
  double best_cost = 1e300;
  for (int hh = 1; hh <= std::min(64, std::min(h->nx, h->ny) / 2); ++hh) {
    if (rect_problem(h, hh)) continue;
    const RGeo g = rect_geo(h->nx, h->ny, hh, light_scheme(h->si.nw, h->si.vbytes));
    const double tiles = (double)rect_tiles(g);
    const double per_cu = std::max(1.0, std::floor((double)g_lds_limit / (double)rect_lds_bytes(h->si, g)));
    const double seq = std::ceil(tiles / h->cu_count);
    const double resident = std::ceil(tiles / (h->cu_count * std::min(per_cu, 8.0)));
    const double pts = (double)h->nx * h->ny / tiles;
    const double half = 2.0 * tau + seq * pts * hh * s_cu + resident * 2 * hh * beta;
    const double cost = half / hh;
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best = hh;
    }
  }
  return best;
}

hipEvent_t next_event(swept2d* h) {
  if (h->event_next == h->event_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->event_pool.push_back(e);
  }
  return h->event_pool[h->event_next++];
}

// Points each kernel kind computes (the space-time volume of its component).
double up_points(int n, int H) {
  double s = 0;
  for (int l = 1; l <= std::min(H, n / 2 - 1); ++l) s += (double)(n - 2 * l) * (n - 2 * l);
  return s;
}
double bridge_points(int n, int H) {
  double s = 0;
  for (int l = 1; l <= std::min(H, n / 2 - 1); ++l) s += 2.0 * l * (n - 2 * l);
  return 2.0 * s;  // x- and y-bridge per tile
}
double down_points(int Hd) {
  double s = 0;
  for (int l = 1; l <= Hd; ++l) s += 4.0 * l * l;
  return s;
}

struct Launcher {
  swept2d* h;
  bool timed;
  template <class F>
  int run(int kind, double work, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
      a = next_event(h);
      b = next_event(h);
      if (!a || !b) return fail(SWEPT2D_EHIP, "cannot create timing events");
      HIP_TRY(hipEventRecord(a, h->stream), "hipEventRecord");
    }
    hipError_t e = f();
    if (e != hipSuccess) return hipfail(e, "kernel launch");
    if (timed) {
      HIP_TRY(hipEventRecord(b, h->stream), "hipEventRecord");
      h->timed.push_back(TimedLaunch{kind, work, a, b});
    }
    return 0;
  }
};

// Enqueue the swept schedule for S sub-steps starting at level T.
int enqueue_swept(swept2d* h, long long S, long long T, const long long* tbase, bool timed) {
  const int n = h->n, hh = n / 2;
  Geo g{};
  g.nx = h->nx;
  g.ny = h->ny;
  g.n = n;
  g.h = hh;
  g.ntx = h->nx / n;
  g.nty = h->ny / n;
  g.off = 0;
  g.W = n + 2;
  g.T0 = T;
  g.tbase = tbase;
  const double ntiles = (double)g.ntx * g.nty;
  PanelPtrs pp{h->up, h->xb, h->yb};
  Launcher L{h, timed};
  const int sc = h->scheme;
  const bool so = oct_staged(h), sb = bridge_staged(h);
  const bool pairs = h->staging != SWEPT2D_STAGING_SINGLE_BRIDGES && !auto_single_bridges(h);
  const long long q = S / hh;
  const int r = (int)(S % hh);
  int rc;
  if (q == 0) {
    // A single reduced half cycle of height r.
    rc = L.run(kKindUp, ntiles * up_points(n, r), [&] { return launch_up(sc, g, r, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    rc = L.run(kKindBridge, ntiles * bridge_points(n, r),
               [&] { return launch_bridge(sc, g, r, sb, pairs, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    return L.run(kKindOct, ntiles * down_points(r),
                 [&] { return launch_oct(sc, g, r, 0, so, h->state, pp, h->sp, h->stream); });
  }
  rc = L.run(kKindUp, ntiles * up_points(n, hh), [&] { return launch_up(sc, g, hh, h->state, pp, h->sp, h->stream); });
  if (rc) return rc;
  for (long long c = 0; c < q; ++c) {
    rc = L.run(kKindBridge, ntiles * bridge_points(n, hh),
               [&] { return launch_bridge(sc, g, hh, sb, pairs, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    const bool last = (c == q - 1);
    const int Hu = last ? r : hh;
    rc = L.run(kKindOct, ntiles * (down_points(hh) + up_points(n, Hu)),
               [&] { return launch_oct(sc, g, hh, Hu, so, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    g.off = (g.off == 0) ? hh : 0;
    g.T0 += hh;
  }
  if (r > 0) {
    rc = L.run(kKindBridge, ntiles * bridge_points(n, r),
               [&] { return launch_bridge(sc, g, r, sb, pairs, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    rc = L.run(kKindOct, ntiles * down_points(r), [&] { return launch_oct(sc, g, r, 0, so, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
  }
  return 0;
}

// Points computed per half cycle of height H on rectangular tiles, by the
// frustums, the bridges and the downward pyramids (sums over the tiles of
// the per-tile volumes).
double rect_up_points(const RGeo& g, int H) {
  double s = 0;
  for (int l = 1; l <= H; ++l) s += (double)(g.ax.L - 2 * l * g.ax.t) * (g.ay.L - 2 * l * g.ay.t);
  return s;
}
double rect_bridge_points(const RGeo& g, int H) {
  double s = 0;
  for (int l = 1; l <= H; ++l)
    s += 2.0 * l * ((double)g.ax.t * (g.ay.L - 2 * l * g.ay.t) + (double)g.ay.t * (g.ax.L - 2 * l * g.ax.t));
  return s;
}
double rect_down_points(const RGeo& g, int H) { return (double)rect_tiles(g) * down_points(H); }

// Enqueue the swept schedule on rectangular tiles for S sub-steps from level
// T: the first frustums, then per half cycle the bridges and the stage that
// finishes the downward pyramids and starts the next frustums (the last one
// writes its squares to the state). Tilings 0 and 1 alternate.
int enqueue_rect(swept2d* h, long long S, long long T, const long long* tbase, bool timed) {
  RGeo g = rect_geo(h->nx, h->ny, h->rect_h, light_scheme(h->si.nw, h->si.vbytes));
  g.T0 = T;
  g.tbase = tbase;
  const int hh = g.h, sc = h->scheme;
  PanelPtrs pp{h->up, h->xb, h->yb};
  Launcher L{h, timed};
  const long long q = S / hh;
  const int r = (int)(S % hh);
  const long long nh = q + (r > 0 ? 1 : 0);
  auto height = [&](long long c) { return c < q ? hh : r; };
  int rc = L.run(kKindUp, rect_up_points(g, height(0)), [&] {
    return launch_rect_oct(sc, g, 0, 0, height(0), h->state, pp, h->sp, h->stream);
  });
  if (rc) return rc;
  int par = 0;
  for (long long c = 0; c < nh; ++c) {
    const int Hc = height(c), Hn = c + 1 < nh ? height(c + 1) : 0;
    rc = L.run(kKindBridge, rect_bridge_points(g, Hc),
               [&] { return launch_rect_bridge(sc, g, par, Hc, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    rc = L.run(kKindOct, rect_down_points(g, Hc) + rect_up_points(g, Hn),
               [&] { return launch_rect_oct(sc, g, 1 - par, Hc, Hn, h->state, pp, h->sp, h->stream); });
    if (rc) return rc;
    par ^= 1;
    g.T0 += Hc;
  }
  return 0;
}

// Enqueue S per-step launches starting at level T; the last one writes the
// state buffer.
int enqueue_plain(swept2d* h, long long S, long long T, const long long* tbase, bool timed) {
  Launcher L{h, timed};
  const double pts = (double)h->nx * h->ny;
  void* bufs[2] = {h->state, h->scratch};
  int src;
  if (S & 1) {
    // odd count: start from a copy so the final write lands in the state
    HIP_TRY(launch_copy(h->scratch, h->state, state_bytes_of(h), h->stream), "copy kernel");
    src = 1;
  } else {
    src = 0;
  }
  for (long long s = 0; s < S; ++s) {
    const void* in = bufs[src];
    void* out = bufs[src ^ 1];
    const long long Ts = T + s;
    int rc = L.run(kKindPlain, pts,
                   [&] { return launch_plain(h->scheme, h->nx, h->ny, Ts, tbase, in, out, h->sp, h->stream); });
    if (rc) return rc;
    src ^= 1;
  }
  return 0;
}

int run_method(swept2d* h, int method, long long nsteps) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (nsteps < 0) return fail(SWEPT2D_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return 0;
  if (nsteps > (1LL << 40)) return fail(SWEPT2D_EINVAL, "nsteps too large");
  const long long S = nsteps * h->substeps;
  int rc;
  if (method == 0) {
    if (h->rect_h) {
      if (const char* why = rect_problem(h, h->rect_h))
        return fail(h->si.nw != h->si.nv || user_scheme(h->scheme - kNumSchemes) ? SWEPT2D_EUNSUPPORTED
                                                                                 : SWEPT2D_EINVAL,
                    "rectangular tiles %d: %s", h->rect_h, why);
    } else if (const char* why = tile_problem(h, h->n)) {
      return fail(SWEPT2D_EINVAL, "tile %d: %s", h->n, why);
    }
    if ((rc = ensure_panels(h))) return rc;
  } else {
    if ((rc = ensure_scratch(h))) return rc;
  }
  const bool use_graph = (h->launch_mode == SWEPT2D_LAUNCH_GRAPH) && !h->timing;
  if (!use_graph) {
    rc = method == 0 ? (h->rect_h ? enqueue_rect(h, S, h->T, nullptr, h->timing)
                                  : enqueue_swept(h, S, h->T, nullptr, h->timing))
                     : enqueue_plain(h, S, h->T, nullptr, h->timing);
    if (rc) return rc;
    h->T += S;
    return 0;
  }
  // Graph mode: kernels take their level relative to a device-resident base,
  // so one captured graph per (method, sub-step count) replays at any level.
  if (!h->d_tbase) {
    if (hipMalloc(&h->d_tbase, sizeof(long long)) != hipSuccess) {
      hipGetLastError();
      h->d_tbase = nullptr;
      return fail(SWEPT2D_ENOMEM, "cannot allocate the level base");
    }
  }
  hipGraphExec_t exec = nullptr;
  auto it = h->graphs.find({method, S});
  if (it != h->graphs.end()) exec = it->second;
  if (!exec) {
    // The null stream cannot be captured: record the launches on the
    // library's own stream (capture executes nothing) and launch the graph
    // on the bound stream.
    const hipStream_t run_stream = h->stream;
    const hipStream_t cap = run_stream ? run_stream : h->own_stream;
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    h->stream = cap;
    rc = method == 0 ? (h->rect_h ? enqueue_rect(h, S, 0, h->d_tbase, false) : enqueue_swept(h, S, 0, h->d_tbase, false))
                     : enqueue_plain(h, S, 0, h->d_tbase, false);
    h->stream = run_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    if (rc) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hipfail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hipfail(e, "hipGraphInstantiate");
    h->graphs[{method, S}] = exec;
  }
  HIP_TRY(launch_set_base(h->d_tbase, h->T, h->stream), "level base kernel");
  HIP_TRY(hipGraphLaunch(exec, h->stream), "hipGraphLaunch");
  h->T += S;
  return 0;
}

}  // namespace

namespace swept {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The swept advance of swept2d_advance_noalloc (its contract is in
// swept2d.h): validated like a handle's calls, panels carved from the
// caller's scratch at 256-byte boundaries, the same kernels and schedule on
// `stream` with direct launches. Uses no device allocation: the handle below
// lives on the host stack and only names the buffers.
int noalloc_advance(int nx, int ny, int nvars, int pde, int substeps, int prec, const double* params, int np,
                    int tile, void* dev_state, long long T, long long nsteps, hipStream_t stream, void* scratch,
                    size_t scratch_bytes) {
  g_err.clear();
  if (pde_nvars(pde) < 0) return fail(SWEPT2D_EINVAL, "unknown pde id %d", pde);
  if (nvars != pde_nvars(pde) || substeps != pde_substeps(pde))
    return fail(SWEPT2D_EINVAL, "pde %d takes nvars=%d substeps=%d (got %d, %d)", pde, pde_nvars(pde),
                pde_substeps(pde), nvars, substeps);
  if (nx < 2 || ny < 2 || nx > (1 << 16) || ny > (1 << 16))
    return fail(SWEPT2D_EINVAL, "grid %d x %d out of range (2..65536 per side)", nx, ny);
  const int need = pde_nparams(pde);
  if (np < need || np > 4 || (need > 0 && !params)) return fail(SWEPT2D_EINVAL, "pde %d takes %d parameters", pde, need);
  if (prec != SWEPT2D_FP64 && prec != SWEPT2D_FP32C && prec != SWEPT2D_FP32R)
    return fail(SWEPT2D_EINVAL, "unknown precision %d", prec);
  const int sc = scheme_of(pde, prec);
  if (sc < 0) return fail(SWEPT2D_EUNSUPPORTED, "pde %d has no form in precision %d", pde, prec);
  if (!dev_state) return fail(SWEPT2D_EINVAL, "null state");
  if (nsteps < 0 || nsteps > (1LL << 40)) return fail(SWEPT2D_EINVAL, "nsteps out of range");
  if (T < 0 || T % substeps) return fail(SWEPT2D_EINVAL, "level must be >= 0 and a multiple of substeps");
  int dev = 0;
  if (int rc = ensure_device_setup(&dev)) return rc;
  swept2d h;
  h.nx = nx;
  h.ny = ny;
  h.nvars = nvars;
  h.pde = pde;
  h.substeps = substeps;
  h.prec = prec;
  h.scheme = sc;
  h.si = scheme_info(sc);
  for (int i = 0; i < 4; ++i) h.sp.p[i] = (i < np) ? params[i] : 0.0;
  h.device = dev;
  hipDeviceGetAttribute(&h.cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (h.cu_count <= 0) h.cu_count = 256;
  h.n = tile ? tile : model_tile(&h);
  if (h.n == 0) return fail(SWEPT2D_EINVAL, "no usable tile side for %d x %d", nx, ny);
  if (const char* why = tile_problem(&h, h.n)) return fail(SWEPT2D_EINVAL, "tile %d: %s", h.n, why);
  const int ntiles = (nx / h.n) * (ny / h.n);
  const size_t vb = h.si.vbytes;
  const size_t ub = align_up(up_panel_values(ntiles, h.n, h.si.nv) * vb, 256);
  const size_t xbb = align_up(xb_panel_values(ntiles, h.n, h.si.nv) * vb, 256);
  const size_t ybb = align_up(yb_panel_values(ntiles, h.n, h.si.nv) * vb, 256);
  if (ub + xbb + ybb > scratch_bytes)
    return fail(SWEPT2D_EINVAL, "%d x %d at tile side %d needs %zu bytes of panels; the static scratch holds %zu", nx,
                ny, h.n, ub + xbb + ybb, scratch_bytes);
  if (nsteps == 0) return 0;
  h.state = dev_state;
  h.owns_state = false;
  h.stream = stream;
  h.up = scratch;
  h.xb = static_cast<char*>(scratch) + ub;
  h.yb = static_cast<char*>(scratch) + ub + xbb;
  h.panel_tile = (size_t)h.n;
  h.staging = SWEPT2D_STAGING_AUTO;
  return enqueue_swept(&h, nsteps * substeps, T, nullptr, false);
}

}  // namespace swept

extern "C" {

const char* swept2d_last_error(void) { return g_err.c_str(); }

swept2d* swept2d_create(int nx, int ny, int nvars, int pde, int substeps) {
  g_err.clear();
  if (pde_nvars(pde) < 0) {
    fail(SWEPT2D_EINVAL, "unknown pde id %d", pde);
    return nullptr;
  }
  if (nvars != pde_nvars(pde) || substeps != pde_substeps(pde)) {
    fail(SWEPT2D_EINVAL, "pde %d takes nvars=%d substeps=%d (got %d, %d)", pde, pde_nvars(pde), pde_substeps(pde),
         nvars, substeps);
    return nullptr;
  }
  if (nx < 2 || ny < 2 || nx > (1 << 16) || ny > (1 << 16)) {
    fail(SWEPT2D_EINVAL, "grid %d x %d out of range (2..65536 per side)", nx, ny);
    return nullptr;
  }
  int dev = 0;
  if (ensure_device_setup(&dev)) return nullptr;
  swept2d* h = new (std::nothrow) swept2d();
  if (!h) {
    fail(SWEPT2D_ENOMEM, "out of host memory");
    return nullptr;
  }
  h->nx = nx;
  h->ny = ny;
  h->nvars = nvars;
  h->pde = pde;
  h->substeps = substeps;
  h->prec = SWEPT2D_FP64;
  h->scheme = scheme_of(pde, SWEPT2D_FP64);
  h->si = scheme_info(h->scheme);
  h->device = dev;
  hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (h->cu_count <= 0) h->cu_count = 256;
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess) {
    hipGetLastError();
    fail(SWEPT2D_EHIP, "cannot create a stream");
    delete h;
    return nullptr;
  }
  h->stream = h->own_stream;
  if (alloc_state(h)) {
    hipStreamDestroy(h->own_stream);
    delete h;
    return nullptr;
  }
  h->n = model_tile(h);
  if (h->n == 0) h->rect_h = model_rect(h);
  return h;
}

void swept2d_destroy(swept2d* h) {
  if (!h) return;
  hipStreamSynchronize(h->stream);
  if (h->own_stream && h->own_stream != h->stream) hipStreamSynchronize(h->own_stream);
  drop_graphs(h);
  free_panels(h);
  if (h->scratch) hipFree(h->scratch);
  if (h->owns_state && h->state) hipFree(h->state);
  if (h->d_tbase) hipFree(h->d_tbase);
  for (hipEvent_t e : h->event_pool) hipEventDestroy(e);
  if (h->own_stream) hipStreamDestroy(h->own_stream);
  delete h;
}

int swept2d_set_params(swept2d* h, const double* p, int np) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  const int need = pde_nparams(h->pde);
  if (np < need || np > 4 || (need > 0 && !p)) return fail(SWEPT2D_EINVAL, "pde %d takes %d parameters", h->pde, need);
  for (int i = 0; i < 4; ++i) h->sp.p[i] = (i < np) ? p[i] : 0.0;
  drop_graphs(h);
  return 0;
}

int swept2d_set_precision(swept2d* h, int prec) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (prec != SWEPT2D_FP64 && prec != SWEPT2D_FP32C && prec != SWEPT2D_FP32R)
    return fail(SWEPT2D_EINVAL, "unknown precision %d", prec);
  const int sc = scheme_of(h->pde, prec);
  if (sc < 0) return fail(SWEPT2D_EUNSUPPORTED, "pde %d has no form in precision %d", h->pde, prec);
  if (!h->owns_state) return fail(SWEPT2D_EINVAL, "unbind the caller buffer before changing precision");
  if (prec == h->prec) return 0;
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->prec = prec;
  h->scheme = sc;
  h->si = scheme_info(sc);
  free_panels(h);
  int rc = alloc_state(h);
  if (rc) return rc;
  if (!h->rect_h && tile_problem(h, h->n)) h->n = model_tile(h);
  if (!h->rect_h && h->n == 0) h->rect_h = model_rect(h);
  return 0;
}

int swept2d_set_tile(swept2d* h, int n) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (n == 0) {
    n = model_tile(h);
    if (n == 0) {
      const int hh = model_rect(h);
      if (hh == 0) return fail(SWEPT2D_EINVAL, "no usable tile for %d x %d", h->nx, h->ny);
      return swept2d_set_rect(h, hh);
    }
  }
  if (const char* why = tile_problem(h, n)) return fail(SWEPT2D_EINVAL, "tile %d: %s", n, why);
  if (n != h->n || h->rect_h) {
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    free_panels(h);
    drop_graphs(h);
  }
  h->n = n;
  h->rect_h = 0;
  return 0;
}

int swept2d_get_tile(const swept2d* h) { return h ? (h->rect_h ? 0 : h->n) : SWEPT2D_EINVAL; }

int swept2d_set_rect(swept2d* h, int hh) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (hh < 0) return fail(SWEPT2D_EINVAL, "half-cycle height must be >= 0");
  if (hh == 0) {
    if (!h->rect_h) return 0;
    const int n = tile_problem(h, h->n) ? model_tile(h) : h->n;
    if (n == 0) return fail(SWEPT2D_EINVAL, "no usable square tile side for %d x %d", h->nx, h->ny);
    return swept2d_set_tile(h, n);
  }
  if (const char* why = rect_problem(h, hh))
    return fail(h->si.nw != h->si.nv || user_scheme(h->scheme - kNumSchemes) ? SWEPT2D_EUNSUPPORTED : SWEPT2D_EINVAL,
                "rectangular tiles %d: %s", hh, why);
  if (hh != h->rect_h) {
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    free_panels(h);
    drop_graphs(h);
  }
  h->rect_h = hh;
  return 0;
}

int swept2d_get_rect(const swept2d* h) { return h ? h->rect_h : SWEPT2D_EINVAL; }

int swept2d_bind(swept2d* h, void* dev_state, void* hip_stream) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  drop_graphs(h);
  if (hip_stream == SWEPT2D_NULL_STREAM)
    h->stream = nullptr;
  else
    h->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : h->own_stream;
  if (dev_state) {
    if (h->owns_state && h->state) hipFree(h->state);
    h->state = dev_state;
    h->owns_state = false;
    if (h->scratch) {
      hipFree(h->scratch);
      h->scratch = nullptr;
    }
    return 0;
  }
  if (!h->owns_state) {
    h->state = nullptr;
    return alloc_state(h);
  }
  return 0;
}

size_t swept2d_state_bytes(const swept2d* h) { return h ? state_bytes_of(h) : 0; }

int swept2d_upload_raw(swept2d* h, const void* host) {
  if (!h || !host) return fail(SWEPT2D_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(h->state, host, state_bytes_of(h), hipMemcpyHostToDevice), "hipMemcpy");
  return 0;
}

int swept2d_download_raw(swept2d* h, void* host) {
  if (!h || !host) return fail(SWEPT2D_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(host, h->state, state_bytes_of(h), hipMemcpyDeviceToHost), "hipMemcpy");
  return 0;
}

int swept2d_upload(swept2d* h, const double* host) {
  if (!h || !host) return fail(SWEPT2D_EINVAL, "null argument");
  if (h->prec == SWEPT2D_FP64) return swept2d_upload_raw(h, host);
  const size_t cnt = (size_t)h->nx * h->ny * h->nvars;
  // FP32C: u then zero compensations; FP32R: u only (the wave as u and
  // v = fl32(u^n - u^(n-1)))
  std::vector<float> buf(h->prec == SWEPT2D_FP32C ? 2 * cnt : cnt, 0.0f);
  for (size_t i = 0; i < cnt; ++i) buf[i] = (float)host[i];
  if (h->scheme == kWave32R) {
    const size_t plane = (size_t)h->nx * h->ny;
    for (size_t i = 0; i < plane; ++i) buf[plane + i] = (float)(host[i] - host[plane + i]);
  }
  return swept2d_upload_raw(h, buf.data());
}

int swept2d_download(swept2d* h, double* host) {
  if (!h || !host) return fail(SWEPT2D_EINVAL, "null argument");
  if (h->prec == SWEPT2D_FP64) return swept2d_download_raw(h, host);
  const size_t cnt = (size_t)h->nx * h->ny * h->nvars;
  const bool comp = h->prec == SWEPT2D_FP32C;
  std::vector<float> buf(comp ? 2 * cnt : cnt);
  int rc = swept2d_download_raw(h, buf.data());
  if (rc) return rc;
  for (size_t i = 0; i < cnt; ++i) host[i] = comp ? (double)buf[i] - (double)buf[cnt + i] : (double)buf[i];
  if (h->scheme == kWave32R) {
    const size_t plane = (size_t)h->nx * h->ny;
    for (size_t i = 0; i < plane; ++i) host[plane + i] = (double)buf[i] - (double)buf[plane + i];
  }
  return 0;
}

int swept2d_register_scheme(const swept2d_scheme_ops* ops) {
  g_err.clear();
  if (!ops) return fail(SWEPT2D_EINVAL, "null scheme table");
  if (ops->abi != SWEPT2D_SCHEME_ABI) return fail(SWEPT2D_EINVAL, "scheme table ABI %d, library %d", ops->abi,
                                                 SWEPT2D_SCHEME_ABI);
  if (ops->nvars < 1 || ops->substeps < 1 || ops->nparams < 0 || ops->nparams > 4 || ops->nv != ops->nvars ||
      ops->nw < ops->nv || (ops->vbytes != 4 && ops->vbytes != 8))
    return fail(SWEPT2D_EINVAL, "inconsistent scheme sizes");
  if (!ops->up || !ops->bridge || !ops->oct || !ops->plain || !ops->lds || !ops->fetch_ahead)
    return fail(SWEPT2D_EINVAL, "scheme table lacks a launcher");
  int dev = 0;
  if (int rc = ensure_device_setup(&dev)) return rc;
  const int k = register_user_scheme(*ops);
  if (k < 0) return k;
  return SWEPT2D_USER_PDE_BASE + k;
}

int swept2d_init_state(swept2d* h) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  const swept2d_scheme_ops* u = user_pde(h->pde);
  if (!u || !u->init) return fail(SWEPT2D_EUNSUPPORTED, "pde %d has no device initialisation", h->pde);
  HIP_TRY(static_cast<hipError_t>(u->init(h->nx, h->ny, h->state, &h->sp, h->stream)), "init launch");
  return 0;
}

int swept2d_advance(swept2d* h, long long nsteps) { return run_method(h, 0, nsteps); }

int swept2d_plain_advance(swept2d* h, long long nsteps) { return run_method(h, 1, nsteps); }

int swept2d_synchronize(swept2d* h) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(h->stream), "kernel execution");
  return 0;
}

long long swept2d_substep_counter(const swept2d* h) { return h ? h->T : (long long)SWEPT2D_EINVAL; }

int swept2d_set_substep_counter(swept2d* h, long long T) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (T < 0 || T % h->substeps) return fail(SWEPT2D_EINVAL, "counter must be >= 0 and a multiple of substeps");
  h->T = T;
  return 0;
}

int swept2d_set_launch_mode(swept2d* h, int mode) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (mode != SWEPT2D_LAUNCH_DIRECT && mode != SWEPT2D_LAUNCH_GRAPH) return fail(SWEPT2D_EINVAL, "unknown mode");
  h->launch_mode = mode;
  return 0;
}

int swept2d_set_staging(swept2d* h, int mode) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  if (mode != SWEPT2D_STAGING_AUTO && mode != SWEPT2D_STAGING_OFF && mode != SWEPT2D_STAGING_SINGLE_BRIDGES &&
      mode != SWEPT2D_STAGING_ON)
    return fail(SWEPT2D_EINVAL, "unknown staging mode");
  if (mode != h->staging) drop_graphs(h);
  h->staging = mode;
  return 0;
}

int swept2d_set_timing(swept2d* h, int on) {
  if (!h) return fail(SWEPT2D_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  h->timing = on != 0;
  h->timed.clear();
  h->event_next = 0;
  return 0;
}

int swept2d_get_timing(swept2d* h, double* out, int cap) {
  if (!h || (cap > 0 && !out)) return fail(SWEPT2D_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  double launches[kNumKinds] = {0}, ms[kNumKinds] = {0}, work[kNumKinds] = {0};
  for (const TimedLaunch& t : h->timed) {
    float e = 0;
    HIP_TRY(hipEventElapsedTime(&e, t.a, t.b), "hipEventElapsedTime");
    launches[t.kind] += 1;
    ms[t.kind] += e;
    work[t.kind] += t.work;
  }
  int k = 0;
  for (int kind = 0; kind < kNumKinds; ++kind) {
    if (launches[kind] == 0) continue;
    if (k < cap) {
      out[4 * k + 0] = kind;
      out[4 * k + 1] = launches[kind];
      out[4 * k + 2] = ms[kind];
      out[4 * k + 3] = work[kind];
    }
    ++k;
  }
  return std::min(k, std::max(cap, 0));
}

}  // extern "C"
