// Host side of the batch API: many independent grids (the swept rule per
// grid, or the per-step method for a grid no even tile side divides), their
// phases laid out on slots of launches replayed from a captured HIP graph,
// and the per-grid tile-side tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/swept2d.h"
#include "engine.hpp"

using namespace swept;

namespace {

int hip_error(hipError_t e, const char* what) {
  return set_error(SWEPT2D_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define BHIP(call, what)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_error(e_, what);      \
  } while (0)

// Tile sides with compile-time window pitch; other sides run the generic
// stage code.
int pitch_of(int n) { return n == 64 ? 66 : (n == 32 ? 34 : (n == 16 ? 18 : 0)); }

struct HostGrid {
  int nx = 0, ny = 0, pde = 0, prec = 0, scheme = 0, substeps = 1;
  SchemeInfo si{};
  SchemeParams sp{};
  int n = 0;   // square tile side; 0 = rectangular tiles or the per-step method
  int rh = 0;  // half-cycle height of rectangular tiles (n == 0); 0 with n == 0: per-step
  void* state = nullptr;
  void* state2 = nullptr;
  void* up = nullptr;
  void* xb = nullptr;
  void* yb = nullptr;
  long long T = 0;
};

struct Plan {
  BatchPlan* d_plans = nullptr;
  int* d_egrid = nullptr;   // phased: entries (grid, phase) of every launch
  int* d_ephase = nullptr;
  int* d_cum = nullptr;     // phased: per launch, its entries' workgroup offsets
  long long* d_phase_base = nullptr;  // persistent schedule
  int* d_active = nullptr;
  int* d_order = nullptr;
  long long* d_cum1 = nullptr;
  long long* d_cum2 = nullptr;
  hipGraphExec_t exec = nullptr;
  int launches = 0;
  std::vector<long long> S;  // per grid
};

// Longest advance one graph covers; longer advances replay it.
constexpr long long kChunkSteps = 1024;

}  // namespace

struct swept2d_batch {
  int count = 0;
  int device = 0;
  int cu_count = 256;
  hipStream_t stream = nullptr;
  std::vector<HostGrid> grids;
  BatchGrid* d_grids = nullptr;
  unsigned* d_done = nullptr;
  unsigned long long* d_head = nullptr;
  int* d_error = nullptr;
  long long wait_us = 2000000;  // longest dependency wait of the persistent kernel
  int mode = SWEPT2D_BATCH_PHASED;
  bool dirty = true;  // device descriptors out of date
  std::map<long long, Plan> plans;
};

namespace {

size_t state_bytes(const HostGrid& g) { return (size_t)g.nx * g.ny * g.si.nv * g.si.vbytes; }

// How a grid advances: square tiles of side n, rectangular tiles of
// half-cycle height rh, or (both 0) the per-step method.
struct Tiling {
  int n = 0, rh = 0;
};
bool swept(const HostGrid& g) { return g.n > 0 || g.rh > 0; }
int half_of(const HostGrid& g) { return g.n > 0 ? g.n / 2 : g.rh; }
RGeo rect_of(const HostGrid& g) { return rect_geo(g.nx, g.ny, g.rh, light_scheme(g.si.nw, g.si.vbytes)); }
int class_of(const HostGrid& g) { return batch_class_of(g.n, g.rh, g.rh > 0 ? rect_of(g).P : 0); }

// Staging as the single-grid AUTO policy: an octahedron stages its ring runs
// only when its workgroup has too few waves to keep each wave's runs
// precomputed for the fetch path (a wave would hold more than two of the
// 8 NV units); bridges fetch (one-wave classes stage everything).
size_t stage_lds(const HostGrid& g, bool* staged_oct, bool* staged_bridge) {
  *staged_oct = *staged_bridge = false;
  if (g.rh > 0) return rect_lds_bytes(g.si, rect_of(g));
  if (g.n == 0) return 0;
  const size_t lim = device_lds_limit();
  const size_t win = window_lds_bytes(g.si, g.n);
  const int waves = batch_class_threads(batch_class_of(g.n)) / 64;
  const bool fetch_ahead = (8 * g.si.nv + waves - 1) / waves <= 2;
  *staged_oct = !fetch_ahead && win + oct_stage_bytes(g.si, g.n) <= lim;
  *staged_bridge = false;
  return std::max(win + (*staged_oct ? oct_stage_bytes(g.si, g.n) : 0),
                  win + (*staged_bridge ? bridge_stage_bytes(g.si, g.n) : 0));
}

// LDS of one item of phase p of grid g.
size_t entry_lds(const HostGrid& g, int p) {
  if (g.rh > 0) return rect_lds_bytes(g.si, rect_of(g));
  if (g.n == 0) return 0;
  bool so = false, sb = false;
  stage_lds(g, &so, &sb);
  if (batch_class_threads(batch_class_of(g.n)) == 64) so = sb = true;  // the kernel stages them
  const size_t win = window_lds_bytes(g.si, g.n);
  if (p == 0) return win;
  if (p & 1) return win + (sb ? bridge_stage_bytes(g.si, g.n) : 0);
  return win + (so ? oct_stage_bytes(g.si, g.n) : 0);
}

// Why tile side n cannot serve grid g in a batch, or nullptr.
const char* batch_tile_problem(const HostGrid& g, int n) {
  if (n == 0) return nullptr;  // per-step
  if (n < 2 || (n & 1)) return "tile side must be even and at least 2";
  if (g.nx % n || g.ny % n) return "tile side must divide nx and ny";
  if (n + 2 > 128) return "tile side above 126";
  if (window_lds_bytes(g.si, n) > device_lds_limit()) return "tile working set exceeds the workgroup LDS";
  // One-wave items (sides up to 22) always stage their panel inputs.
  if (batch_class_threads(batch_class_of(n)) == 64 &&
      window_lds_bytes(g.si, n) + std::max(oct_stage_bytes(g.si, n), bridge_stage_bytes(g.si, n)) > device_lds_limit())
    return "tile working set exceeds the workgroup LDS";
  return nullptr;
}

// Why rectangular tiles of half-cycle height rh cannot serve grid g in a
// batch, or nullptr.
const char* batch_rect_problem(const HostGrid& g, int rh) {
  if (rh < 1 || rh > 64) return "half-cycle height must be 1..64";
  if (g.nx < 2 * rh || g.ny < 2 * rh) return "grid sides must be at least twice the half-cycle height";
  if (g.si.nw != g.si.nv) return "FP32R runs square tiles only";
  if (rect_lds_bytes(g.si, rect_geo(g.nx, g.ny, rh, light_scheme(g.si.nw, g.si.vbytes))) > device_lds_limit()) return "tile window exceeds the workgroup LDS";
  return nullptr;
}

// Model ranking of tile sides for one grid of a batch. Per half cycle
// (h = n/2 sub-steps) a grid runs one bridge and one octahedron phase, each
// a fixed cost tau (a launch) plus one workgroup barrier lambda per level
// (h levels for the bridge, 2h for the octahedron), times the rounds of
// items it needs when its items outnumber the workgroups resident on `cus`
// compute units (residency from the item's LDS and its launch class's
// workgroup size). Cost per sub-step, in the spirit of Sec. 5, Eq. (4):
// [2 tau + 3 h lambda] * rounds / h. The per-step method competes at one
// launch per sub-step, tau times its rounds of 64 x 64 blocks: a grid whose
// only usable sides are small (a half cycle of a few levels) runs per step.
Tiling model_tiling(const HostGrid& g, int cus) {
  const double tau = 6.0e-6, lambda = 0.75e-6;
  const size_t lim = std::max<size_t>(device_lds_limit(), 1);
  const double blocks = (double)((g.nx + kBatchBlock - 1) / kBatchBlock) * ((g.ny + kBatchBlock - 1) / kBatchBlock);
  const double plain_per_cu = 2048.0 / batch_class_threads(kClassGen256);
  Tiling best;
  double best_cost = tau * std::ceil(blocks / (plain_per_cu * std::max(cus, 1)));
  auto consider = [&](Tiling t, int h, double tiles, size_t lds, int threads, double weight) {
    const double per_cu = std::max(1.0, std::min((double)(lim / std::max<size_t>(lds, 1)), 2048.0 / threads));
    const double rounds = std::ceil(2.0 * tiles / (per_cu * std::max(cus, 1)));
    const double cost = weight * (2.0 * tau + 3.0 * h * lambda * threads / 1024.0) * rounds / h;
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best = t;
    }
  };
  for (int n = 4; n <= 64; n += 2) {
    if (batch_tile_problem(g, n)) continue;
    HostGrid t = g;
    t.n = n;
    t.rh = 0;
    bool so, sb;
    // Generic stage code (window pitch known only at run time). In a batch
    // the tile-16 grids set the number of phases, so a larger generic side
    // gains no latency there and costs throughput: measured on the uneven
    // 256-grid workload, side 16 beat the generic sides 34-60 that a factor
    // of 1.25 chose.
    consider(Tiling{n, 0}, n / 2, (double)(g.nx / n) * (g.ny / n), stage_lds(t, &so, &sb),
             batch_class_threads(batch_class_of(n)), pitch_of(n) == 0 ? 2.0 : 1.0);
  }
  // Rectangular tiles (one point per thread, run-time pitch: weighted as the
  // generic square code), for grids no usable square side divides.
  if (best.n == 0) {
    for (int rh = 2; rh <= 32; ++rh) {
      if (batch_rect_problem(g, rh)) continue;
      const RGeo r = rect_geo(g.nx, g.ny, rh, light_scheme(g.si.nw, g.si.vbytes));
      const int cls = batch_class_of(0, rh, r.P);
      consider(Tiling{0, rh}, rh, (double)rect_tiles(r), rect_lds_bytes(g.si, r), batch_class_threads(cls),
               cls == kClassRect0 ? 2.0 : 1.0);
    }
  }
  return best;
}

void free_panels(HostGrid& g) {
  if (g.up) hipFree(g.up);
  if (g.xb) hipFree(g.xb);
  if (g.yb) hipFree(g.yb);
  if (g.state2) hipFree(g.state2);
  g.up = g.xb = g.yb = g.state2 = nullptr;
}

int alloc_work(HostGrid& g) {
  free_panels(g);
  if (g.rh > 0) {
    const RGeo r = rect_of(g);
    const size_t vb = g.si.vbytes;
    const size_t ub = std::max<size_t>(8, rect_up_values(r, g.si.nv) * vb);
    const size_t xbb = std::max<size_t>(8, rect_xb_values(r, g.si.nv) * vb);
    const size_t ybb = std::max<size_t>(8, rect_yb_values(r, g.si.nv) * vb);
    if (hipMalloc(&g.up, ub) != hipSuccess || hipMalloc(&g.xb, xbb) != hipSuccess ||
        hipMalloc(&g.yb, ybb) != hipSuccess) {
      hipGetLastError();
      free_panels(g);
      return set_error(SWEPT2D_ENOMEM, "cannot allocate panels");
    }
    return 0;
  }
  if (g.n == 0) {
    if (hipMalloc(&g.state2, state_bytes(g)) != hipSuccess) {
      hipGetLastError();
      g.state2 = nullptr;
      return set_error(SWEPT2D_ENOMEM, "cannot allocate a per-step buffer of %zu bytes", state_bytes(g));
    }
    return 0;
  }
  const int ntiles = (g.nx / g.n) * (g.ny / g.n);
  const size_t vb = g.si.vbytes;
  const size_t ub = std::max<size_t>(8, up_panel_values(ntiles, g.n, g.si.nv) * vb);
  const size_t xbb = std::max<size_t>(8, xb_panel_values(ntiles, g.n, g.si.nv) * vb);
  const size_t ybb = std::max<size_t>(8, yb_panel_values(ntiles, g.n, g.si.nv) * vb);
  if (hipMalloc(&g.up, ub) != hipSuccess || hipMalloc(&g.xb, xbb) != hipSuccess ||
      hipMalloc(&g.yb, ybb) != hipSuccess) {
    hipGetLastError();
    free_panels(g);
    return set_error(SWEPT2D_ENOMEM, "cannot allocate panels");
  }
  return 0;
}

void drop_plans(swept2d_batch* b) {
  for (auto& kv : b->plans) {
    Plan& p = kv.second;
    if (p.exec) hipGraphExecDestroy(p.exec);
    hipFree(p.d_plans);
    hipFree(p.d_egrid);
    hipFree(p.d_ephase);
    hipFree(p.d_cum);
    hipFree(p.d_phase_base);
    hipFree(p.d_active);
    hipFree(p.d_order);
    hipFree(p.d_cum1);
    hipFree(p.d_cum2);
  }
  b->plans.clear();
}

int units_of(const HostGrid& g) {
  if (g.rh > 0) return rect_tiles(rect_of(g));
  if (g.n == 0) return ((g.nx + kBatchBlock - 1) / kBatchBlock) * ((g.ny + kBatchBlock - 1) / kBatchBlock);
  return (g.nx / g.n) * (g.ny / g.n);
}

BatchPlan plan_of(const HostGrid& g, long long S) {
  BatchPlan p{};
  p.S = S;
  if (S == 0) return p;
  if (!swept(g)) {
    p.nphases = (int)(S + (S & 1));
    return p;
  }
  const int h = half_of(g);
  p.q = S / h;
  p.r = (int)(S % h);
  p.nphases = (int)(p.q == 0 ? 3 : 1 + 2 * (p.q + (p.r > 0 ? 1 : 0)));
  return p;
}

int upload_descriptors(swept2d_batch* b, size_t* lds_out) {
  std::vector<BatchGrid> d(b->count);
  size_t lds = 0;
  for (int i = 0; i < b->count; ++i) {
    const HostGrid& g = b->grids[i];
    BatchGrid& x = d[i];
    x.g0.nx = g.nx;
    x.g0.ny = g.ny;
    x.g0.n = g.n;
    x.g0.h = g.n / 2;
    x.g0.ntx = g.n ? g.nx / g.n : 0;
    x.g0.nty = g.n ? g.ny / g.n : 0;
    x.g0.off = 0;
    x.g0.W = g.n + 2;
    x.g0.T0 = g.T;
    x.g0.tbase = nullptr;
    x.rg = g.rh > 0 ? rect_of(g) : RGeo{};
    x.scheme = g.scheme;
    x.kind = g.rh > 0 ? kBatchRect : (g.n ? kBatchSwept : kBatchPlain);
    x.wc = pitch_of(g.n);
    bool so = false, sb = false;
    lds = std::max(lds, stage_lds(g, &so, &sb));
    x.staged_oct = so;
    x.staged_bridge = sb;
    x.units = units_of(g);
    x.state = g.state;
    x.state2 = g.state2;
    x.pp = PanelPtrs{g.up, g.xb, g.yb};
    x.sp = g.sp;
  }
  BHIP(hipMemcpy(b->d_grids, d.data(), sizeof(BatchGrid) * b->count, hipMemcpyHostToDevice), "hipMemcpy");
  *lds_out = lds;
  b->dirty = false;
  return 0;
}

template <class T>
int upload_array(T** dst, const std::vector<T>& v) {
  const size_t bytes = std::max<size_t>(sizeof(T), v.size() * sizeof(T));
  if (hipMalloc(dst, bytes) != hipSuccess) {
    hipGetLastError();
    *dst = nullptr;
    return set_error(SWEPT2D_ENOMEM, "cannot allocate %zu bytes of batch schedule", bytes);
  }
  if (!v.empty()) BHIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return 0;
}

// Workgroups of phase p of a grid (the device decode's item count).
int phase_items(const HostGrid& g, int p) {
  const int u = units_of(g);
  if (!swept(g)) return u;
  return (p & 1) ? 2 * u : u;
}

int capture_graph(swept2d_batch* b, Plan& pl, const std::function<hipError_t()>& body) {
  BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  hipError_t e1 = body();
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &graph);
  hipError_t first = e1 != hipSuccess ? e1 : e;
  if (first == hipSuccess) first = hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0);
  if (graph) hipGraphDestroy(graph);
  if (first != hipSuccess) return hip_error(first, "batch graph capture");
  return 0;
}

// Phased schedule: grid g's phase j goes to slot floor(j L / P_g) (strictly
// increasing in j since P_g <= L); a slot is one or two launches per launch
// class holding that class's entries. A slot's entries are independent (one
// phase each of distinct grids), so they may be split between launches: a
// launch's LDS is its largest entry's, and items of a small footprint (a
// one-variable scheme) sharing a launch with large ones (two variables)
// would run at the residency of the large. Entries sorted by LDS are cut
// where the estimated rounds of items on the compute units, plus about one
// round per launch for its fill and drain, are fewest.
int plan_phased(swept2d_batch* b, const std::vector<BatchPlan>& plans, Plan& pl) {
  const int G = b->count;
  int L = 0;
  for (int i = 0; i < G; ++i) L = std::max(L, plans[i].nphases);
  std::vector<std::vector<std::pair<int, int>>> slot(L);
  for (int i = 0; i < G; ++i) {
    const int P = plans[i].nphases;
    for (int j = 0; j < P; ++j) slot[(size_t)((long long)j * L / P)].push_back({i, j});
  }
  struct Rec {
    int cls, first, count, cumoff, blocks;
    size_t lds;
  };
  struct Ent {
    int grid, phase;
    long long items;
    size_t lds;
  };
  std::map<std::pair<int, size_t>, int> resident_cache;
  auto resident = [&](int cls, size_t lds, int* out) -> int {
    auto it = resident_cache.find({cls, lds});
    if (it == resident_cache.end()) {
      int r = 0;
      BHIP(batch_phase_resident(cls, lds, &r), "hipOccupancyMaxActiveBlocksPerMultiprocessor");
      it = resident_cache.emplace(std::make_pair(cls, lds), std::max(r, 1)).first;
    }
    *out = it->second;
    return 0;
  };
  const double cus = std::max(b->cu_count, 1);
  std::vector<int> egrid, ephase, cum;
  std::vector<Rec> recs;
  int rc;
  for (int sidx = 0; sidx < L; ++sidx) {
    for (int cls = 0; cls < kNumBatchClasses; ++cls) {
      std::vector<Ent> es;
      for (const auto& e : slot[sidx]) {
        const HostGrid& g = b->grids[e.first];
        if (class_of(g) != cls) continue;
        es.push_back({e.first, e.second, phase_items(g, e.second), entry_lds(g, e.second)});
      }
      if (es.empty()) continue;
      std::stable_sort(es.begin(), es.end(), [](const Ent& a, const Ent& c) { return a.lds < c.lds; });
      const size_t m = es.size();
      std::vector<long long> pre(m + 1, 0);
      for (size_t i = 0; i < m; ++i) pre[i + 1] = pre[i] + es[i].items;
      // Cost of entries [i, j) as one launch, in rounds.
      auto cost = [&](size_t i, size_t j, double* out) -> int {
        int r = 1;
        if ((rc = resident(cls, es[j - 1].lds, &r))) return rc;
        *out = (double)(pre[j] - pre[i]) / (r * cus) + 1.0;
        return 0;
      };
      size_t cut = m;
      double best = 0.0;
      if ((rc = cost(0, m, &best))) return rc;
      for (size_t k = 1; k < m; ++k) {
        if (es[k].lds == es[k - 1].lds) continue;
        double c0 = 0.0, c1 = 0.0;
        if ((rc = cost(0, k, &c0)) || (rc = cost(k, m, &c1))) return rc;
        if (c0 + c1 < best * (1.0 - 1e-9)) best = c0 + c1, cut = k;
      }
      for (size_t lo = 0; lo < m; lo = cut, cut = m) {
        Rec r{cls, (int)egrid.size(), 0, (int)cum.size(), 0, 0};
        long long tot = 0;
        cum.push_back(0);
        for (size_t i = lo; i < cut; ++i) {
          egrid.push_back(es[i].grid);
          ephase.push_back(es[i].phase);
          tot += es[i].items;
          if (tot >= (1LL << 31)) return set_error(SWEPT2D_EINVAL, "batch launch exceeds 2^31 workgroups");
          cum.push_back((int)tot);
          r.lds = std::max(r.lds, es[i].lds);
          ++r.count;
        }
        r.blocks = (int)tot;
        recs.push_back(r);
      }
    }
  }
  if ((rc = upload_array(&pl.d_egrid, egrid)) || (rc = upload_array(&pl.d_ephase, ephase)) ||
      (rc = upload_array(&pl.d_cum, cum)))
    return rc;
  pl.launches = (int)recs.size();
  return capture_graph(b, pl, [&]() -> hipError_t {
    for (const Rec& r : recs) {
      PhaseLaunch l{b->d_grids, pl.d_plans, pl.d_egrid + r.first, pl.d_ephase + r.first, pl.d_cum + r.cumoff,
                    r.count};
      hipError_t e = launch_batch_phase(r.cls, l, r.blocks, r.lds, b->stream);
      if (e != hipSuccess) return e;
    }
    return launch_batch_bump(b->d_grids, pl.d_plans, G, b->stream);
  });
}

#ifdef SWEPT2D_BUILD_PERSISTENT_BATCH
int plan_persistent(swept2d_batch* b, const std::vector<BatchPlan>& plans, Plan& pl) {
  const int G = b->count;
  std::vector<int> order(G);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return plans[a].nphases > plans[c].nphases; });
  const int P = G ? plans[order[0]].nphases : 0;
  std::vector<long long> cum1(G + 1, 0), cum2(G + 1, 0);
  for (int j = 0; j < G; ++j) {
    const HostGrid& g = b->grids[order[j]];
    const long long u = units_of(g);
    cum1[j + 1] = cum1[j] + u;
    cum2[j + 1] = cum2[j] + (swept(g) ? 2 * u : u);
  }
  std::vector<int> active(std::max(P, 1), 0);
  std::vector<long long> base(P + 1, 0);
  {
    int a = G;
    for (int p = 0; p < P; ++p) {
      while (a > 0 && plans[order[a - 1]].nphases <= p) --a;
      active[p] = a;
      base[p + 1] = base[p] + ((p & 1) ? cum2[a] : cum1[a]);
    }
  }
  const long long total = base[P];
  int rc;
  if ((rc = upload_array(&pl.d_phase_base, base)) || (rc = upload_array(&pl.d_active, active)) ||
      (rc = upload_array(&pl.d_order, order)) || (rc = upload_array(&pl.d_cum1, cum1)) ||
      (rc = upload_array(&pl.d_cum2, cum2)))
    return rc;
  size_t lds = 0;
  for (const HostGrid& g : b->grids) {
    bool so, sb;
    lds = std::max(lds, stage_lds(g, &so, &sb));
  }
  int per_cu = 0;
  BHIP(batch_blocks_per_cu(lds, &per_cu), "batch kernel occupancy");
  if (per_cu < 1) return set_error(SWEPT2D_EUNSUPPORTED, "batch kernel does not fit a compute unit (%zu B LDS)", lds);
  const long long blocks = std::max(1LL, std::min<long long>(total, (long long)b->cu_count * per_cu));
  BatchSched s{};
  s.total = total;
  s.nphases = P;
  s.ngrids = G;
  s.phase_base = pl.d_phase_base;
  s.phase_active = pl.d_active;
  s.order = pl.d_order;
  s.cum1 = pl.d_cum1;
  s.cum2 = pl.d_cum2;
  s.grids = b->d_grids;
  s.plans = pl.d_plans;
  s.done = b->d_done;
  s.head = b->d_head;
  s.error = b->d_error;
  s.wait_ticks = b->wait_us * 100;  // the wait clock runs at 100 MHz
  pl.launches = 1;
  return capture_graph(b, pl, [&]() -> hipError_t {
    hipError_t e = launch_batch_reset(b->d_done, G, b->d_head, b->stream);
    if (e == hipSuccess && total > 0) e = launch_batch(s, (int)blocks, lds, b->stream);
    if (e == hipSuccess) e = launch_batch_bump(b->d_grids, pl.d_plans, G, b->stream);
    return e;
  });
}
#endif

// Build (or find) the schedule and graph of an advance by nsteps.
int plan_for(swept2d_batch* b, long long nsteps, Plan** out) {
  auto it = b->plans.find(nsteps);
  if (it != b->plans.end()) {
    *out = &it->second;
    return 0;
  }
  const int G = b->count;
  std::vector<BatchPlan> plans(G);
  Plan pl;
  pl.S.resize(G);
  for (int i = 0; i < G; ++i) {
    pl.S[i] = nsteps * b->grids[i].substeps;
    plans[i] = plan_of(b->grids[i], pl.S[i]);
  }
  int rc = upload_array(&pl.d_plans, plans);
  if (rc == 0) {
#ifdef SWEPT2D_BUILD_PERSISTENT_BATCH
    rc = b->mode == SWEPT2D_BATCH_PERSISTENT ? plan_persistent(b, plans, pl) : plan_phased(b, plans, pl);
#else
    rc = plan_phased(b, plans, pl);
#endif
  }
  b->plans[nsteps] = pl;  // freed by drop_plans
  if (rc) {
    drop_plans(b);
    return rc;
  }
  *out = &b->plans[nsteps];
  return 0;
}

int check_idx(const swept2d_batch* b, int idx) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (idx < 0 || idx >= b->count) return set_error(SWEPT2D_EINVAL, "grid index %d out of range", idx);
  return 0;
}

int sync_and_check(swept2d_batch* b) {
  BHIP(hipStreamSynchronize(b->stream), "batch kernel execution");
  int err = 0;
  BHIP(hipMemcpy(&err, b->d_error, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy");
  if (err) {
    const int zero = 0;
    BHIP(hipMemcpy(b->d_error, &zero, sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
    // The grids' levels are unknown after an abort: descriptors are rebuilt
    // from the host counters on the next advance.
    b->dirty = true;
    return set_error(SWEPT2D_EABORTED, "batch kernel stopped: a dependency wait exceeded its limit");
  }
  return 0;
}

int set_tiling_impl(swept2d_batch* b, int idx, Tiling t) {
  HostGrid& g = b->grids[idx];
  if (t.n > 0)
    if (const char* why = batch_tile_problem(g, t.n)) return set_error(SWEPT2D_EINVAL, "tile %d: %s", t.n, why);
  if (t.rh > 0)
    if (const char* why = batch_rect_problem(g, t.rh))
      return set_error(g.si.nw != g.si.nv ? SWEPT2D_EUNSUPPORTED : SWEPT2D_EINVAL, "rectangular tiles %d: %s", t.rh, why);
  if (t.n == g.n && t.rh == g.rh && ((t.n || t.rh) ? g.up != nullptr : g.state2 != nullptr)) return 0;
  BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  g.n = t.n;
  g.rh = t.n > 0 ? 0 : t.rh;
  int rc = alloc_work(g);
  if (rc) return rc;
  drop_plans(b);
  b->dirty = true;
  return 0;
}

int set_tile_impl(swept2d_batch* b, int idx, int n) { return set_tiling_impl(b, idx, Tiling{n, 0}); }

}  // namespace

extern "C" {

swept2d_batch* swept2d_batch_create(int count, const int* nx, const int* ny, const int* pde, const int* prec,
                                    const double* params, int params_stride) {
  if (count < 1 || count > (1 << 20) || !nx || !ny || !pde || !prec) {
    set_error(SWEPT2D_EINVAL, "batch needs count >= 1 and nx, ny, pde, prec arrays");
    return nullptr;
  }
  for (int i = 0; i < count; ++i) {
    const int sc = scheme_for(pde[i], prec[i]);
    if (pde_var_count(pde[i]) < 0 || (prec[i] != SWEPT2D_FP64 && prec[i] != SWEPT2D_FP32C)) {
      set_error(SWEPT2D_EINVAL, "grid %d: unknown pde %d or precision %d", i, pde[i], prec[i]);
      return nullptr;
    }
    if (sc < 0 || !batch_scheme_supported(sc)) {
      set_error(SWEPT2D_EUNSUPPORTED, "grid %d: pde %d precision %d is not available in a batch", i, pde[i], prec[i]);
      return nullptr;
    }
    if (nx[i] < 3 || ny[i] < 3 || nx[i] > (1 << 16) || ny[i] > (1 << 16)) {
      set_error(SWEPT2D_EINVAL, "grid %d: %d x %d out of range (3..65536 per side)", i, nx[i], ny[i]);
      return nullptr;
    }
    const int np = pde_param_count(pde[i]);
    if (np > 0 && (!params || params_stride < np)) {
      set_error(SWEPT2D_EINVAL, "grid %d: pde %d takes %d parameters (stride %d)", i, pde[i], np, params_stride);
      return nullptr;
    }
  }
  int dev = 0;
  if (device_setup(&dev)) return nullptr;
  swept2d_batch* b = new (std::nothrow) swept2d_batch();
  if (!b) {
    set_error(SWEPT2D_ENOMEM, "out of host memory");
    return nullptr;
  }
  b->count = count;
  b->device = dev;
  hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (b->cu_count <= 0) b->cu_count = 256;
  auto bail = [&](int code, const char* what) -> swept2d_batch* {
    if (code == SWEPT2D_ENOMEM) set_error(code, "%s", what);
    swept2d_batch_destroy(b);
    return nullptr;
  };
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    hipGetLastError();
    b->stream = nullptr;
    set_error(SWEPT2D_EHIP, "cannot create a stream");
    return bail(0, "");
  }
  b->grids.resize(count);
  for (int i = 0; i < count; ++i) {
    HostGrid& g = b->grids[i];
    g.nx = nx[i];
    g.ny = ny[i];
    g.pde = pde[i];
    g.prec = prec[i];
    g.scheme = scheme_for(pde[i], prec[i]);
    g.si = scheme_info(g.scheme);
    g.substeps = pde_substep_count(pde[i]);
    const int np = pde_param_count(pde[i]);
    for (int k = 0; k < np; ++k) g.sp.p[k] = params[(size_t)i * params_stride + k];
    if (hipMalloc(&g.state, state_bytes(g)) != hipSuccess) {
      hipGetLastError();
      g.state = nullptr;
      return bail(SWEPT2D_ENOMEM, "cannot allocate grid state");
    }
    if (hipMemset(g.state, 0, state_bytes(g)) != hipSuccess) {
      set_error(SWEPT2D_EHIP, "hipMemset failed");
      return bail(0, "");
    }
  }
  if (hipMalloc(&b->d_grids, sizeof(BatchGrid) * count) != hipSuccess ||
      hipMalloc(&b->d_done, sizeof(unsigned) * count) != hipSuccess ||
      hipMalloc(&b->d_head, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&b->d_error, sizeof(int)) != hipSuccess) {
    hipGetLastError();
    return bail(SWEPT2D_ENOMEM, "cannot allocate batch descriptors");
  }
  if (hipMemset(b->d_error, 0, sizeof(int)) != hipSuccess) {
    set_error(SWEPT2D_EHIP, "hipMemset failed");
    return bail(0, "");
  }
  // Initial tilings from the model.
  for (int i = 0; i < count; ++i) {
    if (set_tiling_impl(b, i, model_tiling(b->grids[i], b->cu_count))) return bail(0, "");
  }
  return b;
}

void swept2d_batch_destroy(swept2d_batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  drop_plans(b);
  for (HostGrid& g : b->grids) {
    free_panels(g);
    if (g.state) hipFree(g.state);
  }
  if (b->d_grids) hipFree(b->d_grids);
  if (b->d_done) hipFree(b->d_done);
  if (b->d_head) hipFree(b->d_head);
  if (b->d_error) hipFree(b->d_error);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

int swept2d_batch_count(const swept2d_batch* b) { return b ? b->count : SWEPT2D_EINVAL; }

int swept2d_batch_set_tile(swept2d_batch* b, int idx, int n) {
  int rc = check_idx(b, idx);
  if (rc) return rc;
  if (n < 0) return set_tile_impl(b, idx, 0);
  if (n == 0) return set_tiling_impl(b, idx, model_tiling(b->grids[idx], b->cu_count));
  return set_tile_impl(b, idx, n);
}

int swept2d_batch_get_tile(const swept2d_batch* b, int idx) {
  if (!b || idx < 0 || idx >= b->count) return SWEPT2D_EINVAL;
  return b->grids[idx].n;
}

int swept2d_batch_set_rect(swept2d_batch* b, int idx, int hh) {
  int rc = check_idx(b, idx);
  if (rc) return rc;
  if (hh < 1) return set_error(SWEPT2D_EINVAL, "half-cycle height must be at least 1");
  return set_tiling_impl(b, idx, Tiling{0, hh});
}

int swept2d_batch_get_rect(const swept2d_batch* b, int idx) {
  if (!b || idx < 0 || idx >= b->count) return SWEPT2D_EINVAL;
  return b->grids[idx].rh;
}

int swept2d_batch_upload(swept2d_batch* b, int idx, const double* host) {
  int rc = check_idx(b, idx);
  if (rc) return rc;
  if (!host) return set_error(SWEPT2D_EINVAL, "null host buffer");
  HostGrid& g = b->grids[idx];
  BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  const size_t cnt = (size_t)g.nx * g.ny * g.si.nvar;
  if (g.prec == SWEPT2D_FP64) {
    BHIP(hipMemcpy(g.state, host, state_bytes(g), hipMemcpyHostToDevice), "hipMemcpy");
    return 0;
  }
  std::vector<float> buf(2 * cnt, 0.0f);
  for (size_t i = 0; i < cnt; ++i) buf[i] = (float)host[i];
  BHIP(hipMemcpy(g.state, buf.data(), state_bytes(g), hipMemcpyHostToDevice), "hipMemcpy");
  return 0;
}

int swept2d_batch_download(swept2d_batch* b, int idx, double* host) {
  int rc = check_idx(b, idx);
  if (rc) return rc;
  if (!host) return set_error(SWEPT2D_EINVAL, "null host buffer");
  if ((rc = sync_and_check(b))) return rc;
  HostGrid& g = b->grids[idx];
  const size_t cnt = (size_t)g.nx * g.ny * g.si.nvar;
  if (g.prec == SWEPT2D_FP64) {
    BHIP(hipMemcpy(host, g.state, state_bytes(g), hipMemcpyDeviceToHost), "hipMemcpy");
    return 0;
  }
  std::vector<float> buf(2 * cnt);
  BHIP(hipMemcpy(buf.data(), g.state, state_bytes(g), hipMemcpyDeviceToHost), "hipMemcpy");
  for (size_t i = 0; i < cnt; ++i) host[i] = (double)buf[i] - (double)buf[cnt + i];
  return 0;
}

int swept2d_batch_advance(swept2d_batch* b, long long nsteps) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (nsteps < 0) return set_error(SWEPT2D_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return 0;
  if (nsteps > (1LL << 30)) return set_error(SWEPT2D_EINVAL, "nsteps too large");
#ifndef SWEPT2D_BUILD_PERSISTENT_BATCH
  if (b->mode == SWEPT2D_BATCH_PERSISTENT)
    return set_error(SWEPT2D_EUNSUPPORTED,
                     "the persistent batch kernel is not built (it hung on the device in an earlier form; "
                     "the phased launches are the supported mode)");
#endif
  int rc;
  if (b->dirty) {
    BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    size_t lds = 0;
    if ((rc = upload_descriptors(b, &lds))) return rc;
  }
  // Advances longer than one chunk replay the chunk's graph, then one graph
  // for the rest (every grid's chain restarts with an upward pyramid at a
  // chunk boundary; results are the same bits).
  const long long chunk = std::min(nsteps, kChunkSteps);
  const long long reps = nsteps / chunk, rest = nsteps % chunk;
  Plan* pl = nullptr;
  if ((rc = plan_for(b, chunk, &pl))) return rc;
  for (long long k = 0; k < reps; ++k) {
    BHIP(hipGraphLaunch(pl->exec, b->stream), "hipGraphLaunch");
    for (int i = 0; i < b->count; ++i) b->grids[i].T += pl->S[i];
  }
  if (rest) {
    if ((rc = plan_for(b, rest, &pl))) return rc;
    BHIP(hipGraphLaunch(pl->exec, b->stream), "hipGraphLaunch");
    for (int i = 0; i < b->count; ++i) b->grids[i].T += pl->S[i];
  }
  return 0;
}

int swept2d_batch_set_mode(swept2d_batch* b, int mode) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (mode != SWEPT2D_BATCH_PHASED && mode != SWEPT2D_BATCH_PERSISTENT)
    return set_error(SWEPT2D_EINVAL, "unknown batch mode %d", mode);
  if (mode == b->mode) return 0;
  BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  b->mode = mode;
  drop_plans(b);
  return 0;
}

int swept2d_batch_get_mode(const swept2d_batch* b) { return b ? b->mode : SWEPT2D_EINVAL; }

int swept2d_batch_launches(swept2d_batch* b, long long nsteps) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (nsteps < 1 || nsteps > kChunkSteps) return set_error(SWEPT2D_EINVAL, "nsteps must be in 1..%lld", kChunkSteps);
  int rc;
  if (b->dirty) {
    BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    size_t lds = 0;
    if ((rc = upload_descriptors(b, &lds))) return rc;
  }
  Plan* pl = nullptr;
  if ((rc = plan_for(b, nsteps, &pl))) return rc;
  return pl->launches;
}

int swept2d_batch_synchronize(swept2d_batch* b) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  return sync_and_check(b);
}

long long swept2d_batch_substep_counter(const swept2d_batch* b, int idx) {
  if (!b || idx < 0 || idx >= b->count) return SWEPT2D_EINVAL;
  return b->grids[idx].T;
}

int swept2d_batch_set_wait_limit(swept2d_batch* b, long long microseconds) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (microseconds < 0 || microseconds > (1LL << 40)) return set_error(SWEPT2D_EINVAL, "wait limit out of range");
  BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  b->wait_us = microseconds;
  drop_plans(b);
  return 0;
}

int swept2d_batch_autotune(swept2d_batch* b, int mode) {
  if (!b) return set_error(SWEPT2D_EINVAL, "null batch");
  if (mode != SWEPT2D_TUNE_MODEL && mode != SWEPT2D_TUNE_MEASURE) return set_error(SWEPT2D_EINVAL, "unknown mode");
  int rc;
  if (mode == SWEPT2D_TUNE_MODEL) {
    for (int i = 0; i < b->count; ++i)
      if ((rc = set_tiling_impl(b, i, model_tiling(b->grids[i], b->cu_count)))) return rc;
    return 0;
  }
  // Measured: run each grid alone, on a copy of its state, for a few
  // half cycles at every usable square side (up to 64) and rectangular
  // height (8 to 32 in steps of 4), and keep the fastest per sub-step.
  // Grids of one shape, scheme and parameters share a result.
  BHIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  std::map<std::vector<double>, Tiling> seen;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP(hipEventCreate(&e0), "hipEventCreate");
  BHIP(hipEventCreate(&e1), "hipEventCreate");
  rc = 0;
  for (int i = 0; i < b->count && rc == 0; ++i) {
    const HostGrid& g = b->grids[i];
    std::vector<double> key = {(double)g.nx, (double)g.ny, (double)g.pde, (double)g.prec,
                               g.sp.p[0], g.sp.p[1], g.sp.p[2], g.sp.p[3]};
    auto it = seen.find(key);
    if (it != seen.end()) {
      rc = set_tiling_impl(b, i, it->second);
      continue;
    }
    const double par[4] = {g.sp.p[0], g.sp.p[1], g.sp.p[2], g.sp.p[3]};
    swept2d_batch* t = swept2d_batch_create(1, &g.nx, &g.ny, &g.pde, &g.prec, par, 4);
    if (!t) {
      rc = SWEPT2D_EHIP;
      break;
    }
    t->mode = b->mode;
    if (hipMemcpy(t->grids[0].state, g.state, state_bytes(g), hipMemcpyDeviceToDevice) != hipSuccess) {
      swept2d_batch_destroy(t);
      rc = set_error(SWEPT2D_EHIP, "hipMemcpy");
      break;
    }
    Tiling best{g.n, g.rh};
    double best_t = 1e300;
    std::vector<Tiling> cands;
    for (int n = 64; n >= 4; n -= 2)
      if (!batch_tile_problem(g, n)) cands.push_back(Tiling{n, 0});
    for (int rh = 32; rh >= 8; rh -= 4)
      if (!batch_rect_problem(g, rh)) cands.push_back(Tiling{0, rh});
    for (const Tiling& c : cands) {
      if ((rc = set_tiling_impl(t, 0, c))) break;
      const int hh = c.n > 0 ? c.n / 2 : c.rh;
      const long long steps = std::max(2LL * hh, 64LL);
      if ((rc = swept2d_batch_advance(t, steps)) || (rc = swept2d_batch_synchronize(t))) break;
      if (hipEventRecord(e0, t->stream) != hipSuccess) { rc = set_error(SWEPT2D_EHIP, "hipEventRecord"); break; }
      if ((rc = swept2d_batch_advance(t, steps))) break;
      if (hipEventRecord(e1, t->stream) != hipSuccess) { rc = set_error(SWEPT2D_EHIP, "hipEventRecord"); break; }
      if ((rc = swept2d_batch_synchronize(t))) break;
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = set_error(SWEPT2D_EHIP, "hipEventElapsedTime"); break; }
      const double per = ms / (double)steps;
      if (per < best_t) {
        best_t = per;
        best = c;
      }
    }
    swept2d_batch_destroy(t);
    if (rc) break;
    seen[key] = best;
    rc = set_tiling_impl(b, i, best);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
