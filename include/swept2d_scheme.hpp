// swept2d_scheme.hpp - user schemes for the swept2d library (HIP C++).
//
// The paper's interface (Sec. 6) is two functions: an initialisation
// Init(i, j, p) that sets a point's variables from its global indices, and a
// time-stepping function timestep(k, p) that performs sub-step k on a point
// from its 9-point neighbourhood. Here a scheme is a struct with those two
// as device functions; compiled in the user's own HIP source with this
// header, it becomes a swept2d_scheme_ops table of launchers of the
// library's stage kernels instantiated for it, for swept2d_register_scheme.
//
//   struct MyScheme {
//     using V = double;                      // value type (double or float)
//     static constexpr int NV = 2, NW = 2;   // values per point (state = window)
//     static constexpr int NVAR = 2, SUB = 1;// nvars and sub-steps per step
//     static constexpr bool XY_SYM = false;  // see csrc/schemes.hpp
//     template <class NB>                    // timestep: nb(di, dj, v), |di|, |dj| <= 1
//     __device__ static void step(long long T, const NB& nb, V* out, const swept::SchemeParams& sp);
//     __device__ static void init(long long i, long long j, int nx, int ny, V* out,
//                                 const swept::SchemeParams& sp);  // Init (optional)
//   };
//   static swept2d_scheme_ops ops = swept2d_user::scheme_ops<MyScheme>();
//   int pde = swept2d_register_scheme(&ops);   // then swept2d_create(nx, ny, 2, pde, 1)
//
// A stencil that reads two rings (offsets |di|, |dj| <= 2) is written as a
// one-step struct with its offsets listed (NVAR, SUB = 1, NOFF, OFF, step on
// the far offsets; see Hash25 in csrc/schemes.hpp) and wrapped in
// swept::PushTwoRing<...>, which splits it into two nearest-neighbour
// sub-steps (Sec. 2, Eq. (1)-(3)) automatically.
//
// Every launcher returns a hipError_t value. The table refers to kernels of
// the translation unit that instantiates it, which must stay loaded while
// the library uses the scheme.
#pragma once

#include <type_traits>

#include "../paper_1602_07558_amd/csrc/stages.hpp"
#include "swept2d.h"

namespace swept2d_user {

template <class S, class = void>
struct has_init : std::false_type {};
template <class S>
struct has_init<S, std::void_t<decltype(&S::init)>> : std::true_type {};

// Init on every point: one thread per point, the NV values in the state's
// planes [v][ny][nx].
template <class S>
__global__ __launch_bounds__(256) void k_init(int nx, int ny, typename S::V* __restrict__ state,
                                              swept::SchemeParams sp) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long plane = (long long)nx * ny;
  if (p >= plane) return;
  const long long j = p / nx, i = p - j * nx;
  typename S::V out[S::NV];
  S::init(i, j, nx, ny, out, sp);
#pragma unroll
  for (int v = 0; v < S::NV; ++v) state[v * plane + p] = out[v];
}

template <class S>
swept2d_scheme_ops scheme_ops(int nparams = 0) {
  using swept::Geo;
  using swept::PanelPtrs;
  using swept::SchemeParams;
  using St = swept::Stages<S>;
  swept2d_scheme_ops o{};
  o.abi = SWEPT2D_SCHEME_ABI;
  o.nvars = S::NVAR;
  o.substeps = S::SUB;
  o.nparams = nparams;
  o.nv = S::NV;
  o.nw = S::NW;
  o.vbytes = (int)sizeof(typename S::V);
  o.up = [](const void* g, int H, void* state, const void* p, const void* sp, void* s) -> int {
    return St::up(*static_cast<const Geo*>(g), H, state, *static_cast<const PanelPtrs*>(p),
                  *static_cast<const SchemeParams*>(sp), static_cast<hipStream_t>(s));
  };
  o.bridge = [](const void* g, int H, int staged, int pair_ok, void* state, const void* p, const void* sp,
                void* s) -> int {
    return St::bridge(*static_cast<const Geo*>(g), H, staged != 0, pair_ok != 0, state,
                      *static_cast<const PanelPtrs*>(p), *static_cast<const SchemeParams*>(sp),
                      static_cast<hipStream_t>(s));
  };
  o.oct = [](const void* g, int Hd, int Hu, int staged, void* state, const void* p, const void* sp, void* s) -> int {
    return St::oct(*static_cast<const Geo*>(g), Hd, Hu, staged != 0, state, *static_cast<const PanelPtrs*>(p),
                   *static_cast<const SchemeParams*>(sp), static_cast<hipStream_t>(s));
  };
  o.plain = [](int nx, int ny, long long T, const long long* tbase, const void* in, void* out, const void* sp,
               void* s) -> int {
    return St::plain(nx, ny, T, tbase, in, out, *static_cast<const SchemeParams*>(sp), static_cast<hipStream_t>(s));
  };
  o.lds = [](size_t bytes) -> int { return St::lds(bytes); };
  o.fetch_ahead = [](int n) -> int { return St::fetch_ahead(n) ? 1 : 0; };
  if constexpr (has_init<S>::value) {
    o.init = [](int nx, int ny, void* state, const void* sp, void* s) -> int {
      const long long pts = (long long)nx * ny;
      hipLaunchKernelGGL(k_init<S>, dim3((unsigned)((pts + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(s),
                         nx, ny, static_cast<typename S::V*>(state), *static_cast<const SchemeParams*>(sp));
      return hipGetLastError();
    };
  }
  return o;
}

}  // namespace swept2d_user
