// Dispatch of the swept2d kernels by scheme and launch class, the small
// helper kernels (copy, level base, batch level bump) and the LDS limits.
// The stage kernels themselves are in stages.hpp, instantiated once per
// scheme (stages_scheme.hip) and per batch launch class (stages_batch.hip).
#include <algorithm>
#include <atomic>
#include <mutex>

#include "engine.hpp"

namespace swept {

extern template struct Stages<Heat64>;
extern template struct Stages<Wave64>;
extern template struct Stages<Euler64>;
extern template struct Stages<Hash64>;
extern template struct Stages<Incr64>;
extern template struct Stages<Push5>;
extern template struct Stages<Heat32C>;
extern template struct Stages<Wave32C>;
extern template struct Stages<Euler32C>;
extern template struct Stages<Heat32R>;
extern template struct Stages<Wave32R>;
extern template struct Stages<Hash25x2>;
extern template struct Stages<EulerFD64>;
extern template struct Stages<EulerFD32C>;
extern template struct BatchPhase<66, 1024>;
extern template struct BatchPhase<34, 256>;
extern template struct BatchPhase<18, 64>;
extern template struct BatchPhase<0, 256>;
extern template struct BatchPhase<0, 64>;
extern template struct BatchPhase<-66, 1024>;
extern template struct BatchPhase<-34, 256>;
extern template struct BatchPhase<-1, 256>;

namespace {

__global__ void k_copy8(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_set_base(long long* tbase, long long value) {
  if (threadIdx.x == 0) *tbase = value;
}

__global__ void k_batch_bump(BatchGrid* grids, const BatchPlan* plans, int ngrids) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ngrids) grids[i].g0.T0 += plans[i].S;
}

#define SWEPT_DISPATCH(FN, ...)                              \
  switch (scheme) {                                          \
    case kHeat64: return Stages<Heat64>::FN(__VA_ARGS__);     \
    case kWave64: return Stages<Wave64>::FN(__VA_ARGS__);     \
    case kEuler64: return Stages<Euler64>::FN(__VA_ARGS__);   \
    case kHash64: return Stages<Hash64>::FN(__VA_ARGS__);     \
    case kIncr64: return Stages<Incr64>::FN(__VA_ARGS__);     \
    case kPush5: return Stages<Push5>::FN(__VA_ARGS__);       \
    case kHeat32C: return Stages<Heat32C>::FN(__VA_ARGS__);   \
    case kWave32C: return Stages<Wave32C>::FN(__VA_ARGS__);   \
    case kEuler32C: return Stages<Euler32C>::FN(__VA_ARGS__); \
    case kHeat32R: return Stages<Heat32R>::FN(__VA_ARGS__);   \
    case kWave32R: return Stages<Wave32R>::FN(__VA_ARGS__);   \
    case kHash25x2: return Stages<Hash25x2>::FN(__VA_ARGS__); \
    case kEulerFD64: return Stages<EulerFD64>::FN(__VA_ARGS__); \
    case kEulerFD32C: return Stages<EulerFD32C>::FN(__VA_ARGS__); \
    default: break;                                          \
  }

std::mutex g_user_mu;
swept2d_scheme_ops g_user[kMaxUserSchemes];
std::atomic<int> g_user_count{0};

const swept2d_scheme_ops* user_of(int scheme) {
  const int k = scheme - kNumSchemes;
  return (k >= 0 && k < g_user_count.load()) ? &g_user[k] : nullptr;
}

hipError_t as_hip(int e) { return static_cast<hipError_t>(e); }

}  // namespace

const swept2d_scheme_ops* user_scheme(int k) {
  return (k >= 0 && k < g_user_count.load()) ? &g_user[k] : nullptr;
}

int add_user_scheme(const swept2d_scheme_ops& ops) {
  std::lock_guard<std::mutex> lock(g_user_mu);
  const int k = g_user_count.load();
  if (k >= kMaxUserSchemes) return -1;
  g_user[k] = ops;
  g_user_count.store(k + 1);
  return k;
}

SchemeInfo scheme_info(int scheme) {
  if (const swept2d_scheme_ops* u = user_of(scheme)) return SchemeInfo{u->nv, u->nw, u->nvars, u->substeps, u->vbytes};
  SWEPT_DISPATCH(info)
  return SchemeInfo{0, 0, 0, 0, 0};
}

hipError_t launch_up(int scheme, const Geo& g, int H, void* state, PanelPtrs p, const SchemeParams& sp,
                     hipStream_t s) {
  if (const swept2d_scheme_ops* u = user_of(scheme)) return as_hip(u->up(&g, H, state, &p, &sp, s));
  SWEPT_DISPATCH(up, g, H, state, p, sp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_bridge(int scheme, const Geo& g, int H, bool staged, bool pair_ok, void* state, PanelPtrs p,
                         const SchemeParams& sp, hipStream_t s) {
  if (const swept2d_scheme_ops* u = user_of(scheme))
    return as_hip(u->bridge(&g, H, staged ? 1 : 0, pair_ok ? 1 : 0, state, &p, &sp, s));
  SWEPT_DISPATCH(bridge, g, H, staged, pair_ok, state, p, sp, s)
  return hipErrorInvalidValue;
}

bool oct_fetch_ahead(int scheme, int n) {
  if (const swept2d_scheme_ops* u = user_of(scheme)) return u->fetch_ahead(n) != 0;
  SWEPT_DISPATCH(fetch_ahead, n)
  return false;
}

hipError_t launch_oct(int scheme, const Geo& g, int Hd, int Hu, bool staged, void* state, PanelPtrs p,
                      const SchemeParams& sp, hipStream_t s) {
  if (const swept2d_scheme_ops* u = user_of(scheme))
    return as_hip(u->oct(&g, Hd, Hu, staged ? 1 : 0, state, &p, &sp, s));
  SWEPT_DISPATCH(oct, g, Hd, Hu, staged, state, p, sp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_rect_oct(int scheme, const RGeo& g, int upar, int Hd, int Hu, void* state, PanelPtrs p,
                           const SchemeParams& sp, hipStream_t s) {
  if (user_of(scheme)) return hipErrorNotSupported;
  SWEPT_DISPATCH(rect_oct, g, upar, Hd, Hu, state, p, sp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_rect_bridge(int scheme, const RGeo& g, int par, int H, void* state, PanelPtrs p,
                              const SchemeParams& sp, hipStream_t s) {
  if (user_of(scheme)) return hipErrorNotSupported;
  SWEPT_DISPATCH(rect_bridge, g, par, H, state, p, sp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_plain(int scheme, int nx, int ny, long long T, const long long* tbase, const void* in, void* out,
                        const SchemeParams& sp, hipStream_t s) {
  if (const swept2d_scheme_ops* u = user_of(scheme)) return as_hip(u->plain(nx, ny, T, tbase, in, out, &sp, s));
  SWEPT_DISPATCH(plain, nx, ny, T, tbase, in, out, sp, s)
  return hipErrorInvalidValue;
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy8, dim3(blocks), dim3(256), 0, s, static_cast<uint64_t*>(dst),
                     static_cast<const uint64_t*>(src), n);
  return hipGetLastError();
}

hipError_t launch_set_base(long long* tbase, long long value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_base, dim3(1), dim3(64), 0, s, tbase, value);
  return hipGetLastError();
}

hipError_t configure_lds(size_t bytes) {
  for (int scheme = 0; scheme < kNumSchemes; ++scheme) {
    hipError_t e = [&]() -> hipError_t {
      SWEPT_DISPATCH(lds, bytes)
      return hipErrorInvalidValue;
    }();
    if (e != hipSuccess) return e;
  }
  const int b = (int)bytes;
  hipError_t e = BatchPhase<66, 1024>::lds(b);
  if (e == hipSuccess) e = BatchPhase<34, 256>::lds(b);
  if (e == hipSuccess) e = BatchPhase<18, 64>::lds(b);
  if (e == hipSuccess) e = BatchPhase<0, 256>::lds(b);
  if (e == hipSuccess) e = BatchPhase<0, 64>::lds(b);
  if (e == hipSuccess) e = BatchPhase<-66, 1024>::lds(b);
  if (e == hipSuccess) e = BatchPhase<-34, 256>::lds(b);
  if (e == hipSuccess) e = BatchPhase<-1, 256>::lds(b);
  return e;
}

hipError_t launch_batch_phase(int cls, const PhaseLaunch& L, int blocks, size_t lds, hipStream_t st) {
  switch (cls) {
    case kClass66: return BatchPhase<66, 1024>::launch(L, blocks, lds, st);
    case kClass34: return BatchPhase<34, 256>::launch(L, blocks, lds, st);
    case kClass18: return BatchPhase<18, 64>::launch(L, blocks, lds, st);
    case kClassGen256: return BatchPhase<0, 256>::launch(L, blocks, lds, st);
    case kClassGen64: return BatchPhase<0, 64>::launch(L, blocks, lds, st);
    case kClassRect66: return BatchPhase<-66, 1024>::launch(L, blocks, lds, st);
    case kClassRect34: return BatchPhase<-34, 256>::launch(L, blocks, lds, st);
    case kClassRect0: return BatchPhase<-1, 256>::launch(L, blocks, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batch_phase_resident(int cls, size_t lds, int* out) {
  switch (cls) {
    case kClass66: return BatchPhase<66, 1024>::resident(lds, out);
    case kClass34: return BatchPhase<34, 256>::resident(lds, out);
    case kClass18: return BatchPhase<18, 64>::resident(lds, out);
    case kClassGen256: return BatchPhase<0, 256>::resident(lds, out);
    case kClassGen64: return BatchPhase<0, 64>::resident(lds, out);
    case kClassRect66: return BatchPhase<-66, 1024>::resident(lds, out);
    case kClassRect34: return BatchPhase<-34, 256>::resident(lds, out);
    case kClassRect0: return BatchPhase<-1, 256>::resident(lds, out);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_bump(BatchGrid* grids, const BatchPlan* plans, int ngrids, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_bump, dim3((ngrids + 255) / 256), dim3(256), 0, st, grids, plans, ngrids);
  return hipGetLastError();
}

bool batch_scheme_supported(int scheme) {
  return scheme == kHeat64 || scheme == kWave64 || scheme == kHash64 || scheme == kHeat32C || scheme == kWave32C;
}

}  // namespace swept
