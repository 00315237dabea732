// The swept rule in 3D on cube tiles (the level function of the 2D rule,
// Sec. 3-4, carried to three axes): stage kernels, the per-step kernel and
// the C ABI of include/swept3d.h.
//
// Geometry. Tiles of side n = 2h start at off + i n on every axis (off = 0
// or h, alternating between half cycles, Sec. 4). A point at distance d to
// the nearest tile face along an axis (d = min(t, n - 1 - t), t its
// position in the tile) is, at level l of a half cycle, on a growing axis of
// its component if d < l and on a shrinking axis otherwise; its component
// class is the set of growing axes: none (upward pyramid), one (face
// bridge), two (edge bridge) or three (downward pyramid). A component's
// region at level l is, along a shrinking axis of its tile [T, T + n),
// [T + l, T + n - l), and along a growing axis around its face F,
// [F - l, F + l). The half cycle runs the classes in four launches (no
// growing axis, one, two, three): every value a component reads from
// another one at level l - 1 was computed by an earlier launch, and lies in
// the two cells at either end of the producer's region along one of the
// producer's shrinking axes, which is what each component publishes per
// level (the 3D form of the two-wide panels of Sec. 3).
//
// Exchange. The published bands of level l (1 <= l < H) go to a band buffer
// indexed by level and global point; level 0 is the state the half cycle
// starts from and level H is written to the other state buffer. The band
// buffer is dense (one slot per point and level) but only band points are
// written and read, so the traffic is that of the bands.
//
// A component runs in one workgroup with a double-buffered window of
// (n + 2)^3 values in LDS: per axis the tile and one cell each side
// (shrinking) or the face's 2h cells and one each side (growing). Per level
// it loads its ring (the points of its next region's neighbourhood it did
// not compute itself) from the level below, publishes the previous level's
// bands, computes its region from the window (one point per thread) and
// moves on; the two buffers alternate by level parity.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "engine.hpp"
#include "swept2d.h"
#include "swept3d.h"

#pragma clang fp contract(off)

namespace {

struct G3 {
  int nx, ny, nz;
  int n, h, off;
  int tx, ty, tz;
  int H;
  long long T0;  // level l applies sub-step T0 + l - 1
  double r;
  int Hn;        // downward pyramids: height of the next half cycle's upward pyramid to continue with (0: none)
};

__device__ __forceinline__ void axis_range(bool grow, int l, int n, int h, int& a, int& b) {
  if (grow) {
    a = h + 1 - l;
    b = h + 1 + l;
  } else {
    a = l + 1;
    b = n + 1 - l;
  }
}

// A window coordinate's global position lies in [-L, 2L) (the window starts
// at most h + 1 before the grid and ends at most h + 1 past it, n = 2h <= L).
__device__ __forceinline__ int wrap3(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// q = a d + b, 0 <= b < d, for q < 2^24: the float reciprocal gives a within
// one, which the correction fixes.
__device__ __forceinline__ void divmod3(int q, int d, float inv, int& a, int& b) {
  a = (int)((float)q * inv);
  b = q - a * d;
  if (b < 0) {
    a -= 1;
    b += d;
  } else if (b >= d) {
    a += 1;
    b -= d;
  }
}

// The points of a product of per-axis position sets: along each axis either
// the range [p0, p0 + cnt) or four positions p0, p0 + 1, p2, p2 + 1.
struct AxisSet {
  int cnt;
  bool range;
  int p0, p2;
  __device__ int at(int i) const { return (range || i < 2) ? p0 + i : p2 + (i - 2); }
};
__device__ __forceinline__ AxisSet aset_range(int a, int b) { return AxisSet{b > a ? b - a : 0, true, a, 0}; }
// The two cells at either end of [a, b) (all of it when it is at most four
// wide): a shrinking axis's band positions.
__device__ __forceinline__ AxisSet aset_ends(int a, int b) {
  return b - a <= 4 ? aset_range(a, b) : AxisSet{4, false, a, b - 2};
}
// Ring positions of a growing axis at level l: the expanded range [a - 1,
// b + 1) without the previous level's [a + 1, b - 1).
__device__ __forceinline__ AxisSet aset_ring(int a, int b) { return AxisSet{4, false, a - 1, b - 1}; }

// Calls f(x, y, z) for every point of sx * sy * sz, NT threads in turn.
template <int NT, class F>
__device__ __forceinline__ void for_points(const AxisSet& sx, const AxisSet& sy, const AxisSet& sz, F&& f) {
  const int nxy = sx.cnt * sy.cnt, tot = nxy * sz.cnt;
  if (tot <= 0) return;
  const float ixy = 1.0f / (float)nxy, ix = 1.0f / (float)sx.cnt;
  for (int k = (int)threadIdx.x; k < tot; k += NT) {
    int z, r, y, x;
    divmod3(k, nxy, ixy, z, r);
    divmod3(r, sx.cnt, ix, y, x);
    f(sx.at(x), sy.at(y), sz.at(z));
  }
}

// 7-point heat and the 27-point hash; nb(q) is neighbour q =
// 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
template <class NB>
__device__ __forceinline__ double heat7(const NB& nb, double r) {
  const double u = nb(13);
  const double t = ((nb(12) + nb(14)) + (nb(10) + nb(16))) + (nb(4) + nb(22));
  const double lap = t - 6.0 * u;
  return u + r * lap;
}

template <class NB>
__device__ __forceinline__ double hash27(long long T, const NB& nb) {
  uint64_t m = 0x94D049BB133111EBull ^ (uint64_t)T;
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    m ^= (uint64_t)nb(q);
    m *= 0xFF51AFD7ED558CCDull;
    m ^= m >> 32;
  }
  return (double)(m >> 12);
}

template <int PDE, class NB>
__device__ __forceinline__ double apply(long long T, const NB& nb, double r) {
  if constexpr (PDE == SWEPT3D_HEAT7)
    return heat7(nb, r);
  else
    return hash27(T, nb);
}

// One component of launch `group` (0: upward pyramids, 1: face bridges,
// 2: edge bridges, 3: downward pyramids) per workgroup of NT threads. A
// downward pyramid that reaches the half cycle's last level h holds the whole
// tile centred on its corner: that is a tile of the next half cycle's tiling
// (shifted by h), whose window starts at the same cell, so with g.Hn > 0 the
// workgroup goes on as that tile's upward pyramid (an octahedron, as in
// 2D), publishing into the next half cycle's band buffer and output state.
template <int PDE, int NT>
__global__ __launch_bounds__(NT) void k3_stage(G3 g, int group, const double* __restrict__ in,
                                               double* __restrict__ out, double* __restrict__ bands,
                                               double* __restrict__ out_next, double* __restrict__ bands_next) {
  extern __shared__ double win[];
  const int n = g.n, h = g.h, W = n + 2, W3 = W * W * W;
  const int tiles = g.tx * g.ty * g.tz;
  int j = (int)blockIdx.x, cls;
  if (group == 0) {
    cls = 0;
  } else if (group == 3) {
    cls = 7;
  } else {
    const int b = j / tiles;
    j -= b * tiles;
    cls = group == 1 ? (1 << b) : (7 ^ (1 << b));
  }
  const int ix = j % g.tx, iy = (j / g.tx) % g.ty, iz = j / (g.tx * g.ty);
  // global coordinate of window cell 0 per axis
  const int bx = g.off + ix * n + ((cls & 1) ? -h - 1 : -1);
  const int by = g.off + iy * n + ((cls & 2) ? -h - 1 : -1);
  const int bz = g.off + iz * n + ((cls & 4) ? -h - 1 : -1);
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  auto gidx = [&](int x, int y, int z) {
    return ((size_t)wrap3(bz + z, g.nz) * g.ny + wrap3(by + y, g.ny)) * g.nx + wrap3(bx + x, g.nx);
  };
  auto widx = [&](int x, int y, int z) { return (z * W + y) * W + x; };

  // Levels 1..H of a component of class c whose level l lives in window
  // buffer (l + pb) & 1 (kept as an offset from the LDS array: a selected
  // pointer would be a generic one, and every window access a flat access).
  // With from_state, level 0 of the region's neighbourhood is loaded from
  // `src0`; otherwise the window already holds it.
  auto run = [&](int c, int H, long long T0, const double* src0, bool from_state, double* dst_out, double* bnd,
                 int pb) {
    auto grows = [&](int a) { return ((c >> a) & 1) != 0; };
    auto off = [&](int l) { return ((l + pb) & 1) * W3; };
    // publish level l: the bands of its shrinking axes to the band buffer
    // (l < H; each band point once: along the first shrinking axis where it
    // is in a band), or its whole region to the output state (l == H)
    auto publish = [&](int l) {
      int lo[3], hi[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) axis_range(grows(a), l, n, h, lo[a], hi[a]);
      const int src = off(l);
      if (l == H) {
        for_points<NT>(aset_range(lo[0], hi[0]), aset_range(lo[1], hi[1]), aset_range(lo[2], hi[2]),
                       [&](int x, int y, int z) { dst_out[gidx(x, y, z)] = win[src + widx(x, y, z)]; });
        return;
      }
      double* dst = bnd + (size_t)(l - 1) * N;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (grows(a)) continue;
        AxisSet s[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (b == a)
            s[b] = aset_ends(lo[b], hi[b]);
          else if (b < a && !grows(b))
            s[b] = aset_range(lo[b] + 2, hi[b] - 2);
          else
            s[b] = aset_range(lo[b], hi[b]);
        }
        for_points<NT>(s[0], s[1], s[2],
                       [&](int x, int y, int z) { dst[gidx(x, y, z)] = win[src + widx(x, y, z)]; });
      }
    };
    for (int l = 1; l <= H; ++l) {
      int lo[3], hi[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) axis_range(grows(a), l, n, h, lo[a], hi[a]);
      // the inputs at level l - 1 this component did not compute: at l = 1
      // the whole neighbourhood of its region, from the state; later only the
      // ring along its growing axes (each ring point once: along the first
      // growing axis where it is outside the previous level's region)
      const int dst = off(l - 1);
      if (l == 1) {
        if (from_state)
          for_points<NT>(aset_range(lo[0] - 1, hi[0] + 1), aset_range(lo[1] - 1, hi[1] + 1),
                         aset_range(lo[2] - 1, hi[2] + 1),
                         [&](int x, int y, int z) { win[dst + widx(x, y, z)] = src0[gidx(x, y, z)]; });
      } else {
        const double* src = bnd + (size_t)(l - 2) * N;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (!grows(a)) continue;
          AxisSet s[3];
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            if (b == a)
              s[b] = aset_ring(lo[b], hi[b]);
            else if (b < a && grows(b))
              s[b] = aset_range(lo[b] + 1, hi[b] - 1);
            else
              s[b] = aset_range(lo[b] - 1, hi[b] + 1);
          }
          for_points<NT>(s[0], s[1], s[2],
                         [&](int x, int y, int z) { win[dst + widx(x, y, z)] = src[gidx(x, y, z)]; });
        }
      }
      if (l >= 2) publish(l - 1);
      __syncthreads();
      const int I = off(l - 1), O = off(l);
      const long long T = T0 + l - 1;
      for_points<NT>(aset_range(lo[0], hi[0]), aset_range(lo[1], hi[1]), aset_range(lo[2], hi[2]),
                     [&](int x, int y, int z) {
                       const int cc = widx(x, y, z);
                       auto nb = [&](int q) {
                         return win[I + cc + ((q / 9 - 1) * W + ((q / 3) % 3 - 1)) * W + (q % 3 - 1)];
                       };
                       win[O + cc] = apply<PDE>(T, nb, g.r);
                     });
      __syncthreads();
    }
    publish(H);
  };

  run(cls, g.H, g.T0, in, true, out, bands, 0);
  if (group == 3 && g.Hn > 0) run(0, g.Hn, g.T0 + g.H, nullptr, false, out_next, bands_next, g.H);
}

// One step of every point, reading its neighbourhood with periodic wrap.
template <int PDE>
__global__ __launch_bounds__(256) void k3_plain(const double* __restrict__ in, double* __restrict__ out, int nx,
                                                int ny, int nz, long long T, double r) {
  const size_t N = (size_t)nx * ny * nz;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((size_t)nx * ny));
  int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  auto nb = [&](int q) { return in[((size_t)zs[q / 9] * ny + ys[(q / 3) % 3]) * nx + xs[q % 3]]; };
  out[p] = apply<PDE>(T, nb, r);
}

size_t window_bytes3(int n) { return (size_t)2 * (n + 2) * (n + 2) * (n + 2) * sizeof(double); }

// Workgroup size by tile side: 1024 threads from side 16 (one workgroup per
// CU; 192^3 heat 5.4e10 point-updates/s against 5.1e10 on 512), 512 at
// sides 12 and 14, 256 below.
constexpr int stage_threads(int n) { return n >= 16 ? 1024 : (n >= 12 ? 512 : 256); }

template <int PDE, int NT>
hipError_t stage_lds_one(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k3_stage<PDE, NT>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template <int PDE>
hipError_t stage_lds(size_t bytes) {
  hipError_t e = stage_lds_one<PDE, 256>(bytes);
  if (e == hipSuccess) e = stage_lds_one<PDE, 512>(bytes);
  return e != hipSuccess ? e : stage_lds_one<PDE, 1024>(bytes);
}

template <int PDE>
void launch_stage(int n, int blocks, size_t lds, hipStream_t st, const G3& g, int group, const double* in,
                  double* out, double* bands, double* out_next, double* bands_next) {
  if (stage_threads(n) == 1024)
    hipLaunchKernelGGL((k3_stage<PDE, 1024>), dim3(blocks), dim3(1024), lds, st, g, group, in, out, bands, out_next,
                       bands_next);
  else if (stage_threads(n) == 512)
    hipLaunchKernelGGL((k3_stage<PDE, 512>), dim3(blocks), dim3(512), lds, st, g, group, in, out, bands, out_next,
                       bands_next);
  else
    hipLaunchKernelGGL((k3_stage<PDE, 256>), dim3(blocks), dim3(256), lds, st, g, group, in, out, bands, out_next,
                       bands_next);
}

}  // namespace

struct swept3d {
  int nx = 0, ny = 0, nz = 0, pde = 0, n = 0;
  double r = 0.0;
  size_t N = 0;
  // three state buffers: a half cycle reads level 0 from one and writes its
  // last level to the next; the octahedra of its downward pyramids write the
  // next half cycle's upward pyramids' last level to the third
  double* state[3] = {nullptr, nullptr, nullptr};
  int cur = 0;
  double* bands[2] = {nullptr, nullptr};  // by half-cycle parity
  int band_levels = 0;
  hipStream_t stream = nullptr;
  long long T = 0, half = 0;
  size_t lds_limit = 0;
};

namespace {

using swept::set_error;

int hip3(hipError_t e, const char* what) {
  return set_error(SWEPT2D_EHIP, "%s: %s", what, hipGetErrorString(e));
}
#define HIP3(call, what)                   \
  do {                                     \
    hipError_t e_ = (call);                \
    if (e_ != hipSuccess) return hip3(e_, what); \
  } while (0)

const char* tile_problem3(const swept3d* h, int n) {
  if (n < 2 || (n & 1)) return "tile side must be even and at least 2";
  if (h->nx % n || h->ny % n || h->nz % n) return "tile side must divide nx, ny and nz";
  if (window_bytes3(n) > h->lds_limit) return "tile window exceeds the workgroup LDS";
  return nullptr;
}

int ensure_bands(swept3d* h, int levels) {
  if (levels <= h->band_levels) return 0;
  for (double*& b : h->bands) {
    if (b) hipFree(b);
    b = nullptr;
  }
  h->band_levels = 0;
  for (double*& b : h->bands)
    if (hipMalloc(&b, (size_t)levels * h->N * sizeof(double)) != hipSuccess)
      return set_error(SWEPT2D_ENOMEM, "cannot allocate %d band levels", levels);
  h->band_levels = levels;
  return 0;
}

// The stage kernels' dynamic LDS limit is raised once per device (the
// attribute is per device).
constexpr int kMaxDevices3 = 64;
std::mutex g_lds3_mu;
bool g_lds3_done[kMaxDevices3] = {};

}  // namespace

extern "C" {

swept3d* swept3d_create(int nx, int ny, int nz, int pde) {
  if (nx < 2 || ny < 2 || nz < 2) {
    set_error(SWEPT2D_EINVAL, "grid sides must be at least 2");
    return nullptr;
  }
  if (pde != SWEPT3D_HEAT7 && pde != SWEPT3D_TEST_HASH27) {
    set_error(SWEPT2D_EINVAL, "unknown 3D scheme %d", pde);
    return nullptr;
  }
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    set_error(SWEPT2D_EHIP, "no device");
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices3) {
    set_error(SWEPT2D_EUNSUPPORTED, "device index %d", dev);
    return nullptr;
  }
  {
    std::lock_guard<std::mutex> lock(g_lds3_mu);
    if (!g_lds3_done[dev]) {
      hipError_t e = stage_lds<SWEPT3D_HEAT7>((size_t)lds);
      if (e == hipSuccess) e = stage_lds<SWEPT3D_TEST_HASH27>((size_t)lds);
      if (e != hipSuccess) {
        hip3(e, "hipFuncSetAttribute");
        return nullptr;
      }
      g_lds3_done[dev] = true;
    }
  }
  swept3d* h = new swept3d();
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->pde = pde;
  h->N = (size_t)nx * ny * nz;
  h->lds_limit = (size_t)lds;
  // Default side by measured preference (7-point heat, point-updates/s):
  // 12 before 16 (192^3: 6.1e10 against 5.1e10; 96^3: 5.0e10 against
  // 4.5e10; a side-12 window leaves three workgroups per CU, side 16 one),
  // 16 before 8 (128^3: 5.5e10 against 4.0e10), small sides last.
  for (int n : {12, 14, 16, 10, 18, 8, 6, 4, 2})
    if (!tile_problem3(h, n)) {
      h->n = n;
      break;
    }
  const size_t bytes = h->N * sizeof(double);
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&h->state[0], bytes) != hipSuccess || hipMalloc(&h->state[1], bytes) != hipSuccess ||
      hipMalloc(&h->state[2], bytes) != hipSuccess) {
    set_error(SWEPT2D_ENOMEM, "cannot allocate %zu bytes of state", 3 * bytes);
    swept3d_destroy(h);
    return nullptr;
  }
  if (hipMemsetAsync(h->state[0], 0, bytes, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    set_error(SWEPT2D_EHIP, "cannot clear the state");
    swept3d_destroy(h);
    return nullptr;
  }
  return h;
}

void swept3d_destroy(swept3d* h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  for (double* p : h->state)
    if (p) hipFree(p);
  for (double* p : h->bands)
    if (p) hipFree(p);
  if (h->stream) hipStreamDestroy(h->stream);
  delete h;
}

int swept3d_set_params(swept3d* h, const double* params, int nparams) {
  if (!h) return set_error(SWEPT2D_EINVAL, "null handle");
  const int need = h->pde == SWEPT3D_HEAT7 ? 1 : 0;
  if (nparams < need || (need && !params)) return set_error(SWEPT2D_EINVAL, "scheme needs %d parameters", need);
  if (need) h->r = params[0];
  return 0;
}

int swept3d_set_tile(swept3d* h, int n) {
  if (!h) return set_error(SWEPT2D_EINVAL, "null handle");
  if (const char* why = tile_problem3(h, n)) return set_error(SWEPT2D_EINVAL, "tile side %d: %s", n, why);
  h->n = n;
  return 0;
}

int swept3d_get_tile(const swept3d* h) { return h ? h->n : set_error(SWEPT2D_EINVAL, "null handle"); }

int swept3d_upload(swept3d* h, const double* host) {
  if (!h || !host) return set_error(SWEPT2D_EINVAL, "null argument");
  HIP3(hipMemcpyAsync(h->state[h->cur], host, h->N * sizeof(double), hipMemcpyHostToDevice, h->stream),
       "hipMemcpyAsync");
  HIP3(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return 0;
}

int swept3d_download(swept3d* h, double* host) {
  if (!h || !host) return set_error(SWEPT2D_EINVAL, "null argument");
  HIP3(hipMemcpyAsync(host, h->state[h->cur], h->N * sizeof(double), hipMemcpyDeviceToHost, h->stream),
       "hipMemcpyAsync");
  HIP3(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return 0;
}

int swept3d_advance(swept3d* h, long long nsteps) {
  if (!h) return set_error(SWEPT2D_EINVAL, "null handle");
  if (nsteps < 0) return set_error(SWEPT2D_EINVAL, "negative step count");
  if (nsteps == 0) return 0;
  if (!h->n) return set_error(SWEPT2D_EINVAL, "no even tile side up to 16 divides %d x %d x %d", h->nx, h->ny, h->nz);
  const int hh = h->n / 2;
  if (hh > 1) {
    if (int rc = ensure_bands(h, hh - 1)) return rc;
  }
  const size_t lds = window_bytes3(h->n);
  const int tiles = (h->nx / h->n) * (h->ny / h->n) * (h->nz / h->n);
  // Half cycles: upward pyramids (only where the previous half cycle's
  // octahedra did not already compute them), face bridges, edge bridges,
  // downward pyramids, the last fused with the next half cycle's upward
  // pyramids when this half cycle is full and another follows.
  bool ups_done = false;
  for (long long done = 0; done < nsteps;) {
    G3 g;
    g.nx = h->nx;
    g.ny = h->ny;
    g.nz = h->nz;
    g.n = h->n;
    g.h = hh;
    g.off = (h->half & 1) ? hh : 0;
    g.tx = h->nx / h->n;
    g.ty = h->ny / h->n;
    g.tz = h->nz / h->n;
    g.H = (int)std::min<long long>(hh, nsteps - done);
    g.T0 = h->T;
    g.r = h->r;
    const long long rest = nsteps - done - g.H;
    g.Hn = (g.H == hh && rest > 0) ? (int)std::min<long long>(hh, rest) : 0;
    const double* in = h->state[h->cur];
    double* out = h->state[(h->cur + 1) % 3];
    double* out_next = h->state[(h->cur + 2) % 3];
    double* bands = h->bands[h->half & 1];
    double* bands_next = h->bands[(h->half + 1) & 1];
    for (int group = ups_done ? 1 : 0; group < 4; ++group) {
      const int blocks = (group == 1 || group == 2) ? 3 * tiles : tiles;
      if (h->pde == SWEPT3D_HEAT7)
        launch_stage<SWEPT3D_HEAT7>(h->n, blocks, lds, h->stream, g, group, in, out, bands, out_next, bands_next);
      else
        launch_stage<SWEPT3D_TEST_HASH27>(h->n, blocks, lds, h->stream, g, group, in, out, bands, out_next,
                                          bands_next);
      HIP3(hipGetLastError(), "stage launch");
    }
    ups_done = g.Hn > 0;
    h->cur = (h->cur + 1) % 3;
    h->half += 1;
    h->T += g.H;
    done += g.H;
  }
  return 0;
}

int swept3d_plain_advance(swept3d* h, long long nsteps) {
  if (!h) return set_error(SWEPT2D_EINVAL, "null handle");
  if (nsteps < 0) return set_error(SWEPT2D_EINVAL, "negative step count");
  const unsigned blocks = (unsigned)((h->N + 255) / 256);
  for (long long s = 0; s < nsteps; ++s) {
    const double* in = h->state[h->cur];
    double* out = h->state[(h->cur + 1) % 3];
    if (h->pde == SWEPT3D_HEAT7)
      hipLaunchKernelGGL(k3_plain<SWEPT3D_HEAT7>, dim3(blocks), dim3(256), 0, h->stream, in, out, h->nx, h->ny, h->nz,
                         h->T, h->r);
    else
      hipLaunchKernelGGL(k3_plain<SWEPT3D_TEST_HASH27>, dim3(blocks), dim3(256), 0, h->stream, in, out, h->nx, h->ny,
                         h->nz, h->T, h->r);
    HIP3(hipGetLastError(), "per-step launch");
    h->cur = (h->cur + 1) % 3;
    h->T += 1;
  }
  return 0;
}

int swept3d_synchronize(swept3d* h) {
  if (!h) return set_error(SWEPT2D_EINVAL, "null handle");
  HIP3(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  return 0;
}

long long swept3d_get_step(const swept3d* h) { return h ? h->T : set_error(SWEPT2D_EINVAL, "null handle"); }

int swept3d_set_step(swept3d* h, long long T) {
  if (!h || T < 0) return set_error(SWEPT2D_EINVAL, "null handle or negative step");
  h->T = T;
  return 0;
}

}  // extern "C"
