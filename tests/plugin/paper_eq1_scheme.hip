// A user scheme through swept2d_register_scheme: the paper's example of a
// stencil reaching two rings (Sec. 2, Eq. (1)), written as the wide stencil
// itself and split into nearest-neighbour sub-steps by the library's
// adapter, with an Init (Sec. 6) that sets each point from its indices.
// Built by the package's build step; the GPU tests register it and compare
// it with the oracle's explicit two sub-steps of Eq. (2)-(3).
#include "../../include/swept2d_scheme.hpp"

#pragma clang fp contract(off)

namespace {

// u' = u(i-2, j) + u(i+2, j) + u(i, j-2) + u(i, j+2) - 4 u(i, j)
struct Eq1Wide {
  using V = double;
  static constexpr int NVAR = 1, SUB = 1, NOFF = 5;
  static constexpr int OFF[5][2] = {{-2, 0}, {2, 0}, {0, -2}, {0, 2}, {0, 0}};
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const swept::SchemeParams&) {
    out[0] = nb(-2, 0, 0) + nb(2, 0, 0) + nb(0, -2, 0) + nb(0, 2, 0) - 4.0 * nb(0, 0, 0);
  }
};

struct Eq1 : swept::PushTwoRing<Eq1Wide> {
  // Init: small integers from the point's global indices, pushed slots zero.
  __device__ static void init(long long i, long long j, int, int, V* out, const swept::SchemeParams&) {
    out[0] = (double)((i * 7 + j * 13) % 17 - 8);
    for (int k = 1; k < NV; ++k) out[k] = 0.0;
  }
};

}  // namespace

extern "C" int paper_eq1_register(void) {
  static const swept2d_scheme_ops ops = swept2d_user::scheme_ops<Eq1>();
  return swept2d_register_scheme(&ops);
}

extern "C" int paper_eq1_slots(void) { return Eq1::NV; }
