// Per-point sub-step operations (the paper's timestep(i, p) callback of
// Sec. 6, compiled in) for the built-in schemes, on gfx950.
//
// Each scheme is a struct with
//   V        value type stored in the state, LDS and panels
//   NV       values per grid point in the state and the panels (FP32C
//            schemes: nvars u's then nvars c's)
//   NW       values per point in a workgroup's LDS window: NV, or more for
//            schemes with window-only values (the compensations of the FP32
//            schemes whose compensation stays within a residency), which
//            start at zero whenever a point's value arrives from the state or
//            a panel and never leave the window
//   NVAR     the scheme's nvars, SUB its sub-steps per time step
//   XY_SYM   step gives the same bits when x and y are exchanged (every
//            neighbour (di, dj) read as (dj, di)): true where the x terms
//            and the y terms enter only through one commutative sum, e.g.
//            (uW + uE) + (uN + uS)
//   step(T, nb, out, prm)
//            computes the point at level T+1 from its 3x3 neighbourhood at
//            level T (Sec. 2, assumption 2); nb(di, dj, v) returns value v of
//            the neighbour at offset (di, dj), dj = -1 being north. T is the
//            global sub-step index, so St_{T mod SUB} is applied.
//
// Every expression is evaluated exactly as written (the library is compiled
// with -ffp-contract=off): sums are left to right, and the compiler fuses no
// multiply-add. A step writes a fused multiply-add itself only where the
// product is exact (a scale by a power of two), so the one rounding of the
// fused form gives the same bits as the written product and sum.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace swept {

struct SchemeParams {
  double p[4];
};

// ------------------------------------------------------------------ FP64

// Heat, forward time centred space: u' = u + r lap(u), 5-point Laplacian
// lap = ((uW + uE) + (uN + uS)) - 4u.
struct Heat64 {
  using V = double;
  static constexpr int NV = 1, NW = 1, NVAR = 1, SUB = 1;
  static constexpr bool XY_SYM = true;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams& sp) {
    const double r = sp.p[0];
    const double u = nb(0, 0, 0);
    const double t1 = nb(-1, 0, 0) + nb(1, 0, 0);
    const double t2 = nb(0, -1, 0) + nb(0, 1, 0);
    // 4u is exact (a power-of-two scale), so the fused form rounds once at
    // the same exact value as the written difference (t1 + t2) - 4u.
    const double lap = __builtin_fma(-4.0, u, t1 + t2);
    out[0] = u + r * lap;
  }
};

// Wave equation, leapfrog with the previous level as a second variable:
// (u, q) -> ((2u - q) + C2 lap(u), u).
struct Wave64 {
  using V = double;
  static constexpr int NV = 2, NW = 2, NVAR = 2, SUB = 1;
  static constexpr bool XY_SYM = true;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams& sp) {
    const double c2 = sp.p[0];
    const double u = nb(0, 0, 0);
    const double q = nb(0, 0, 1);
    const double t1 = nb(-1, 0, 0) + nb(1, 0, 0);
    const double t2 = nb(0, -1, 0) + nb(0, 1, 0);
    // 4u and 2u are exact, so each fused form rounds once at the value of
    // the written difference: (t1 + t2) - 4u and 2u - q.
    const double lap = __builtin_fma(-4.0, u, t1 + t2);
    out[0] = __builtin_fma(2.0, u, -q) + c2 * lap;
    out[1] = u;
  }
};

// Test stencil: 64-bit mix, in row-major neighbour order (north-west first),
// of the nine neighbour values (integers < 2^52 held in doubles) seeded with
// the sub-step index; the top 52 bits are the new value.
struct Hash64 {
  using V = double;
  static constexpr int NV = 1, NW = 1, NVAR = 1, SUB = 1;
  static constexpr bool XY_SYM = false;
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams&) {
    uint64_t m = 0x9E3779B97F4A7C15ull ^ (uint64_t)T;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        m ^= (uint64_t)nb(di, dj, 0);
        m *= 0xFF51AFD7ED558CCDull;
        m ^= m >> 32;
      }
    out[0] = (double)(m >> 12);
  }
};

// Test stencil from the worked example of Sec. 3.1: increment by one; NaN
// when the nine neighbours are not all at the centre's value (level).
struct Incr64 {
  using V = double;
  static constexpr int NV = 1, NW = 1, NVAR = 1, SUB = 1;
  static constexpr bool XY_SYM = false;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams&) {
    const double u = nb(0, 0, 0);
    bool same = true;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) same = same && (nb(di, dj, 0) == u);
    out[0] = same ? u + 1.0 : __builtin_nan("");
  }
};

// Eq. (2)-(3): sub-step 0 pushes (u, u_W, u_E, u_N, u_S) into slots 0..4;
// sub-step 1 forms W.slot1 + E.slot2 + N.slot3 + S.slot4 - 4 C.slot0, which is
// the 2-ring stencil of Eq. (1), and clears slots 1..4.
struct Push5 {
  using V = double;
  static constexpr int NV = 5, NW = 5, NVAR = 5, SUB = 2;
  static constexpr bool XY_SYM = false;
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams&) {
    if ((T & 1) == 0) {
      out[0] = nb(0, 0, 0);
      out[1] = nb(-1, 0, 0);
      out[2] = nb(1, 0, 0);
      out[3] = nb(0, -1, 0);
      out[4] = nb(0, 1, 0);
    } else {
      const double s = nb(-1, 0, 1) + nb(1, 0, 2) + nb(0, -1, 3) + nb(0, 1, 4);
      out[0] = s - 4.0 * nb(0, 0, 0);
      out[1] = 0.0;
      out[2] = 0.0;
      out[3] = 0.0;
      out[4] = 0.0;
    }
  }
};

// Compressible Euler, first-order finite volumes, Rusanov flux.
// State U = (rho, mx, my, E); p = (gamma-1)(E - 0.5 (mx^2 + my^2)/rho),
// c = sqrt(gamma p / rho). Physical flux along x: (mx, mx u + p, my u, (E+p) u)
// with u = mx/rho; along y: (my, mx v, my v + p, (E+p) v) with v = my/rho.
// Face flux 0.5 (F(L) + F(R)) - 0.5 (a (R - L)), a = max(|u_L|+c_L, |u_R|+c_R),
// always taken with (left/north, right/south) argument order so neighbouring
// cells see identical bits.
namespace euler {

__device__ __forceinline__ void phys(const double* U, int d, double gamma, double* F, double& speed) {
  const double rho = U[0], mx = U[1], my = U[2], en = U[3];
  const double ke = 0.5 * ((mx * mx + my * my) / rho);
  const double p = (gamma - 1.0) * (en - ke);
  const double c = sqrt((gamma * p) / rho);
  if (d == 0) {
    const double un = mx / rho;
    F[0] = mx;
    F[1] = mx * un + p;
    F[2] = my * un;
    F[3] = (en + p) * un;
    speed = fabs(un) + c;
  } else {
    const double un = my / rho;
    F[0] = my;
    F[1] = mx * un;
    F[2] = my * un + p;
    F[3] = (en + p) * un;
    speed = fabs(un) + c;
  }
}

// Face flux from both sides' physical fluxes and signal speeds.
__device__ __forceinline__ void face(const double* FL, double aL, const double* L, const double* FR, double aR,
                                     const double* R, double* Fh) {
  const double a = fmax(aL, aR);
#pragma unroll
  for (int k = 0; k < 4; ++k) Fh[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * (a * (R[k] - L[k]));
}

__device__ __forceinline__ void rusanov(const double* L, const double* R, int d, double gamma, double* Fh) {
  double FL[4], FR[4], aL, aR;
  phys(L, d, gamma, FL, aL);
  phys(R, d, gamma, FR, aR);
  face(FL, aL, L, FR, aR, R, Fh);
}

// dt L(U) at the centre from the 5-point states W, E, N, S, C (4 values each).
__device__ __forceinline__ void increment(const double* W, const double* E, const double* N, const double* S,
                                          const double* C, double gamma, double dtoh, double* du) {
  double Fw[4], Fe[4], Gn[4], Gs[4];
  rusanov(W, C, 0, gamma, Fw);
  rusanov(C, E, 0, gamma, Fe);
  rusanov(N, C, 1, gamma, Gn);
  rusanov(C, S, 1, gamma, Gs);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double div = (Fe[k] - Fw[k]) + (Gs[k] - Gn[k]);
    du[k] = -(dtoh * div);
  }
}

// Column-walk hooks of the Rusanov schemes: a cell's face data along an
// axis is its state, its physical flux and its signal speed (9 doubles).
constexpr int kCellN = 9;
__device__ __forceinline__ void cells(const double* C, double gamma, double* cx, double* cy) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    cx[k] = C[k];
    cy[k] = C[k];
  }
  phys(C, 0, gamma, cx + 4, cx[8]);
  phys(C, 1, gamma, cy + 4, cy[8]);
}
__device__ __forceinline__ void cell_face(const double* cL, const double* cR, double* F) {
  face(cL + 4, cL[8], cL, cR + 4, cR[8], cR, F);
}

}  // namespace euler

// Two-stage SSP Runge-Kutta as two sub-steps; slots 0..3 = U^n, 4..7 = U*.
// sub-step 0: U* = U + dt L(U), U^n carried. sub-step 1:
// U' = 0.5 U + 0.5 (U* + dt L(U*)), written to both halves.
struct Euler64 {
  using V = double;
  static constexpr int NV = 8, NW = 8, NVAR = 8, SUB = 2;
  static constexpr bool XY_SYM = false;
  // Levels run by the column walk of the stage kernels, which computes each
  // cell's physical fluxes once and each face flux once; the same
  // expressions as step.
  static constexpr bool WALK = true;
  static constexpr int CN = euler::kCellN;
  __device__ __forceinline__ static int wstage(long long T) { return (T & 1) ? 4 : 0; }
  __device__ __forceinline__ static double wload(const V* p, int plane, int v) { return p[v * plane]; }
  __device__ __forceinline__ static void wcells(const double* C, const SchemeParams& sp, double* cx, double* cy) {
    euler::cells(C, sp.p[0], cx, cy);
  }
  __device__ __forceinline__ static void wface(const double* cL, const double* cR, int, const SchemeParams&,
                                               double* F) {
    euler::cell_face(cL, cR, F);
  }
  __device__ __forceinline__ static void finish(long long T, const V* own, int plane, const double* C,
                                                const double* div, const SchemeParams& sp, V* dst) {
    double du[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) du[k] = -(sp.p[1] * div[k]);
    if ((T & 1) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dst[k * plane] = own[k * plane];
        dst[(4 + k) * plane] = C[k] + du[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = 0.5 * own[k * plane] + 0.5 * (C[k] + du[k]);
        dst[k * plane] = v;
        dst[(4 + k) * plane] = v;
      }
    }
  }
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams& sp) {
    const double gamma = sp.p[0], dtoh = sp.p[1];
    // The stage's slots are picked by value: a slot index known only at run
    // time would put a caller's register neighbourhood on the stack.
    const bool odd = (T & 1) != 0;
    double W[4], E[4], N[4], S[4], C[4], du[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      W[k] = odd ? nb(-1, 0, 4 + k) : nb(-1, 0, k);
      E[k] = odd ? nb(1, 0, 4 + k) : nb(1, 0, k);
      N[k] = odd ? nb(0, -1, 4 + k) : nb(0, -1, k);
      S[k] = odd ? nb(0, 1, 4 + k) : nb(0, 1, k);
      C[k] = odd ? nb(0, 0, 4 + k) : nb(0, 0, k);
    }
    euler::increment(W, E, N, S, C, gamma, dtoh, du);
    if ((T & 1) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        out[k] = C[k];
        out[4 + k] = C[k] + du[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = 0.5 * nb(0, 0, k) + 0.5 * (C[k] + du[k]);
        out[k] = v;
        out[4 + k] = v;
      }
    }
  }
};

// Compressible Euler in the paper's discretisation (Sec. 8): conservative,
// skew-symmetric central differences and the classical four-stage
// Runge-Kutta method. The split form of a convective derivative d(m phi)
// (m the mass flux along the axis, phi in {1, u, v, H}, H = (E + p) / rho)
// is half of d(m phi) + m d(phi) + phi d(m); with central differences it
// equals the difference of the face fluxes (m_L + m_R)(phi_L + phi_R) / 4,
// and the pressure enters as (p_L + p_R) / 2 on the face. Faces are taken
// with (left/north, right/south) arguments.
namespace eulerfd {

struct Prim {
  double u, v, p, H;
};

// Primitives through one reciprocal of the density.
__device__ __forceinline__ Prim prim(const double* U, double gamma) {
  const double rho = U[0], mx = U[1], my = U[2], en = U[3];
  const double ri = 1.0 / rho;
  Prim q;
  q.u = mx * ri;
  q.v = my * ri;
  q.p = (gamma - 1.0) * (en - 0.5 * ((mx * mx + my * my) * ri));
  q.H = (en + q.p) * ri;
  return q;
}

// Face flux along d between L and R from their mass fluxes mL, mR along d
// and their primitives.
__device__ __forceinline__ void face(double mL, const Prim& L, double mR, const Prim& R, int d, double* F) {
  const double a = 0.25 * (mL + mR);
  const double pf = 0.5 * (L.p + R.p);
  F[0] = 2.0 * a;
  if (d == 0) {
    F[1] = a * (L.u + R.u) + pf;
    F[2] = a * (L.v + R.v);
  } else {
    F[1] = a * (L.u + R.u);
    F[2] = a * (L.v + R.v) + pf;
  }
  F[3] = a * (L.H + R.H);
}

}  // namespace eulerfd

// The four-stage Runge-Kutta step as four sub-steps. Slots 0..3 = U^n,
// 4..7 = the stage value Y the fluxes are taken from, 8..11 = the sum K of
// the stage derivatives so far, in units of -r with r = h div F(Y). Sub-step
// s: s = 0: K = -r, Y = U - (dt/2h) r; s = 1: K = K - 2r, Y = U - (dt/2h) r;
// s = 2: K = K - 2r, Y = U - (dt/h) r; s = 3: U = Y = U + (dt/6h)(K - r),
// K = 0. A state enters a step with Y = U and K = 0. Params {gamma, dt/h}.
struct EulerFD64 {
  using V = double;
  static constexpr int NV = 12, NW = 12, NVAR = 12, SUB = 4;
  static constexpr bool XY_SYM = false;
  // Column walk (as Euler64): a cell's face data along an axis is its mass
  // flux along that axis and its primitives (u, v, p, H), one set of
  // divisions per cell.
  static constexpr bool WALK = true;
  static constexpr int CN = 5;
  __device__ __forceinline__ static int wstage(long long) { return 4; }
  __device__ __forceinline__ static double wload(const V* p, int plane, int v) { return p[v * plane]; }
  __device__ __forceinline__ static void wcells(const double* C, const SchemeParams& sp, double* cx, double* cy) {
    const eulerfd::Prim q = eulerfd::prim(C, sp.p[0]);
    cx[0] = C[1];
    cy[0] = C[2];
    cx[1] = cy[1] = q.u;
    cx[2] = cy[2] = q.v;
    cx[3] = cy[3] = q.p;
    cx[4] = cy[4] = q.H;
  }
  __device__ __forceinline__ static void wface(const double* cL, const double* cR, int d, const SchemeParams&,
                                               double* F) {
    eulerfd::face(cL[0], eulerfd::Prim{cL[1], cL[2], cL[3], cL[4]}, cR[0], eulerfd::Prim{cR[1], cR[2], cR[3], cR[4]},
                  d, F);
  }
  __device__ __forceinline__ static void finish(long long T, const V* own, int plane, const double*,
                                                const double* div, const SchemeParams& sp, V* dst) {
    update(T, [&](int v) { return own[v * plane]; }, div, sp.p[1], dst, plane);
  }
  // Sub-step s of variable k: its new U, Y and K from its old U and K and r.
  __device__ __forceinline__ static void slot(int s, double U, double K, double r, double dth, double& nu,
                                              double& ny, double& nk) {
    if (s == 3) {
      const double v = U + (dth / 6.0) * (K - r);
      nu = v;
      ny = v;
      nk = 0.0;
    } else {
      nu = U;
      nk = s == 0 ? -r : K - 2.0 * r;
      ny = U - (s == 2 ? dth : 0.5 * dth) * r;
    }
  }
  // The point's new slots from its old ones and r. Each slot is stored once
  // at a fixed index (stores to different slots at the ends of per-sub-step
  // branches would be merged into one store at a computed index, which puts
  // a register array on the stack).
  template <class OLD>
  __device__ __forceinline__ static void update(long long T, const OLD& old, const double* r, double dth, V* out,
                                                int stride) {
    const int s = (int)(T & 3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double nu, ny, nk;
      slot(s, old(k), old(8 + k), r[k], dth, nu, ny, nk);
      out[k * stride] = nu;
      out[(4 + k) * stride] = ny;
      out[(8 + k) * stride] = nk;
    }
  }
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams& sp) {
    const double gamma = sp.p[0], dth = sp.p[1];
    double W[4], E[4], N[4], S[4], C[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      W[k] = nb(-1, 0, 4 + k);
      E[k] = nb(1, 0, 4 + k);
      N[k] = nb(0, -1, 4 + k);
      S[k] = nb(0, 1, 4 + k);
      C[k] = nb(0, 0, 4 + k);
    }
    double r[4];
    divergence(W, E, N, S, C, gamma, r);
    update(T, [&](int v) { return nb(0, 0, v); }, r, dth, out, 1);
  }
  // r = h div F from the stage values of the point (C) and its four
  // neighbours, x terms first.
  __device__ __forceinline__ static void divergence(const double* W, const double* E, const double* N,
                                                    const double* S, const double* C, double gamma, double* r) {
    const eulerfd::Prim pw = eulerfd::prim(W, gamma), pe = eulerfd::prim(E, gamma);
    const eulerfd::Prim pn = eulerfd::prim(N, gamma), ps = eulerfd::prim(S, gamma);
    const eulerfd::Prim pc = eulerfd::prim(C, gamma);
    double Fw[4], Fe[4], Gn[4], Gs[4];
    eulerfd::face(W[1], pw, C[1], pc, 0, Fw);
    eulerfd::face(C[1], pc, E[1], pe, 0, Fe);
    eulerfd::face(N[2], pn, C[2], pc, 1, Gn);
    eulerfd::face(C[2], pc, S[2], ps, 1, Gs);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (Fe[k] - Fw[k]) + (Gs[k] - Gn[k]);
  }
};

// ------------------------------------------- FP32 with compensated update
// Values u and compensations c; the pair stands for u - c. Heat and wave use
// Kahan's update for u += delta: y = delta - c, t = u + y, c' = (t - u) - y,
// u' = t; neighbour differences are taken against the centre first.

struct Heat32C {
  using V = float;
  static constexpr int NV = 2, NW = 2, NVAR = 1, SUB = 1;
  static constexpr bool XY_SYM = true;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams& sp) {
    const float r = (float)sp.p[0];
    const float u = nb(0, 0, 0);
    const float c = nb(0, 0, 1);
    const float lap = ((nb(-1, 0, 0) - u) + (nb(1, 0, 0) - u)) + ((nb(0, -1, 0) - u) + (nb(0, 1, 0) - u));
    const float y = r * lap - c;
    const float t = u + y;
    out[1] = (t - u) - y;
    out[0] = t;
  }
};

// Leapfrog as u' = u + v, v = ((u - q) - (c_u - c_q)) + C2 lap, with Kahan
// on u; q' = u and c_q' = c_u. Slots: u, q, c_u, c_q. lap is the Laplacian
// of the compensated values u - c_u: that of the u's (differences against
// the centre, exact for a smooth field) minus that of the c_u's (rounding
// errors in size, so their plain sum is accurate far below the unit of u).
// Leapfrog keeps every error of v in the displacement, so both corrections
// matter over long runs.
struct Wave32C {
  using V = float;
  static constexpr int NV = 4, NW = 4, NVAR = 2, SUB = 1;
  static constexpr bool XY_SYM = true;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams& sp) {
    const float c2 = (float)sp.p[0];
    const float u = nb(0, 0, 0);
    const float q = nb(0, 0, 1);
    const float cu = nb(0, 0, 2);
    const float cq = nb(0, 0, 3);
    const float lapu = ((nb(-1, 0, 0) - u) + (nb(1, 0, 0) - u)) + ((nb(0, -1, 0) - u) + (nb(0, 1, 0) - u));
    // 4 c_u is exact, so the fused form rounds once at the written difference.
    const float lapc = __builtin_fmaf(-4.0f, cu, (nb(-1, 0, 2) + nb(1, 0, 2)) + (nb(0, -1, 2) + nb(0, 1, 2)));
    const float lap = lapu - lapc;
    const float v = ((u - q) - (cu - cq)) + c2 * lap;
    const float y = v - cu;
    const float t = u + y;
    out[2] = (t - u) - y;
    out[0] = t;
    out[1] = u;
    out[3] = cu;
  }
};

// Euler with FP32 state: every input is widened to the FP64 value u - c,
// the FP64 update above is applied, and the FP64 result t is split into
// u = fl32(t), c = fl32(u - t). Slots 0..7 values, 8..15 compensations.
struct Euler32C {
  using V = float;
  static constexpr int NV = 16, NW = 16, NVAR = 8, SUB = 2;
  static constexpr bool XY_SYM = false;
  static constexpr bool WALK = true;  // as Euler64
  static constexpr int CN = euler::kCellN;
  __device__ __forceinline__ static int wstage(long long T) { return (T & 1) ? 4 : 0; }
  __device__ __forceinline__ static double wload(const V* p, int plane, int v) {
    return (double)p[v * plane] - (double)p[(8 + v) * plane];
  }
  __device__ __forceinline__ static void wcells(const double* C, const SchemeParams& sp, double* cx, double* cy) {
    euler::cells(C, sp.p[0], cx, cy);
  }
  __device__ __forceinline__ static void wface(const double* cL, const double* cR, int, const SchemeParams&,
                                               double* F) {
    euler::cell_face(cL, cR, F);
  }
  __device__ __forceinline__ static void finish(long long T, const V* own, int plane, const double* C,
                                                const double* div, const SchemeParams& sp, V* dst) {
    double du[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) du[k] = -(sp.p[1] * div[k]);
    if ((T & 1) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dst[k * plane] = own[k * plane];
        dst[(8 + k) * plane] = own[(8 + k) * plane];
        float u, c;
        split(C[k] + du[k], u, c);
        dst[(4 + k) * plane] = u;
        dst[(12 + k) * plane] = c;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = 0.5 * wload(own, plane, k) + 0.5 * (C[k] + du[k]);
        float u, c;
        split(v, u, c);
        dst[k * plane] = u;
        dst[(8 + k) * plane] = c;
        dst[(4 + k) * plane] = u;
        dst[(12 + k) * plane] = c;
      }
    }
  }
  template <class NB>
  __device__ __forceinline__ static double wide(const NB& nb, int di, int dj, int v) {
    return (double)nb(di, dj, v) - (double)nb(di, dj, 8 + v);
  }
  __device__ __forceinline__ static void split(double t, float& u, float& c) {
    const float hi = (float)t;
    u = hi;
    c = (float)((double)hi - t);
  }
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams& sp) {
    const double gamma = sp.p[0], dtoh = sp.p[1];
    const bool odd = (T & 1) != 0;  // slots picked by value, as Euler64
    double W[4], E[4], N[4], S[4], C[4], du[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      W[k] = odd ? wide(nb, -1, 0, 4 + k) : wide(nb, -1, 0, k);
      E[k] = odd ? wide(nb, 1, 0, 4 + k) : wide(nb, 1, 0, k);
      N[k] = odd ? wide(nb, 0, -1, 4 + k) : wide(nb, 0, -1, k);
      S[k] = odd ? wide(nb, 0, 1, 4 + k) : wide(nb, 0, 1, k);
      C[k] = odd ? wide(nb, 0, 0, 4 + k) : wide(nb, 0, 0, k);
    }
    euler::increment(W, E, N, S, C, gamma, dtoh, du);
    if ((T & 1) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        out[k] = nb(0, 0, k);
        out[8 + k] = nb(0, 0, 8 + k);
        split(C[k] + du[k], out[4 + k], out[12 + k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = 0.5 * wide(nb, 0, 0, k) + 0.5 * (C[k] + du[k]);
        split(v, out[k], out[8 + k]);
        out[4 + k] = out[k];
        out[12 + k] = out[8 + k];
      }
    }
  }
};

// The central-difference Euler scheme with FP32 state, as Euler32C: every
// slot widened to the FP64 value u - c, EulerFD64's sub-step applied, and
// each slot the sub-step changes split into u = fl32(t), c = fl32(u - t);
// the U slots that sub-steps 0..2 carry keep both halves as they are, and
// the last sub-step clears K in both. Slots 0..11 values, 12..23
// compensations.
struct EulerFD32C {
  using V = float;
  static constexpr int NV = 24, NW = 24, NVAR = 12, SUB = 4;
  static constexpr bool XY_SYM = false;
  static constexpr bool WALK = true;  // as EulerFD64, on the widened values
  static constexpr int CN = EulerFD64::CN;
  __device__ __forceinline__ static int wstage(long long T) { return EulerFD64::wstage(T); }
  __device__ __forceinline__ static double wload(const V* p, int plane, int v) {
    return (double)p[v * plane] - (double)p[(12 + v) * plane];
  }
  __device__ __forceinline__ static void wcells(const double* C, const SchemeParams& sp, double* cx, double* cy) {
    EulerFD64::wcells(C, sp, cx, cy);
  }
  __device__ __forceinline__ static void wface(const double* cL, const double* cR, int d, const SchemeParams& sp,
                                               double* F) {
    EulerFD64::wface(cL, cR, d, sp, F);
  }
  __device__ __forceinline__ static void finish(long long T, const V* own, int plane, const double*,
                                                const double* div, const SchemeParams& sp, V* dst) {
    update(T, [&](int v) { return own[v * plane]; }, div, sp.p[1], dst, plane);
  }
  // The point's new slots from its old halves (old(v), v < 24) and r: per
  // variable, the FP64 sub-step on the widened U and K, then the changed
  // slots split. One split serves U on the last sub-step and K before it.
  template <class OLD>
  __device__ __forceinline__ static void update(long long T, const OLD& old, const double* r, double dth, V* out,
                                                int stride) {
    const int s = (int)(T & 3);
    const bool last = s == 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float uu = old(k), uc = old(12 + k);
      double nu, ny, nk;
      EulerFD64::slot(s, (double)uu - (double)uc, (double)old(8 + k) - (double)old(20 + k), r[k], dth, nu, ny, nk);
      float a, b, yu, yc;
      split(last ? nu : nk, a, b);
      split(ny, yu, yc);
      out[k * stride] = last ? a : uu;
      out[(12 + k) * stride] = last ? b : uc;
      out[(8 + k) * stride] = last ? 0.0f : a;
      out[(20 + k) * stride] = last ? 0.0f : b;
      out[(4 + k) * stride] = yu;
      out[(16 + k) * stride] = yc;
    }
  }
  __device__ __forceinline__ static void split(double t, float& u, float& c) {
    const float hi = (float)t;
    u = hi;
    c = (float)((double)hi - t);
  }
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams& sp) {
    const double gamma = sp.p[0];
    double W[4], E[4], N[4], S[4], C[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      W[k] = wide(nb, -1, 0, 4 + k);
      E[k] = wide(nb, 1, 0, 4 + k);
      N[k] = wide(nb, 0, -1, 4 + k);
      S[k] = wide(nb, 0, 1, 4 + k);
      C[k] = wide(nb, 0, 0, 4 + k);
    }
    double r[4];
    EulerFD64::divergence(W, E, N, S, C, gamma, r);
    update(T, [&](int v) { return nb(0, 0, v); }, r, sp.p[1], out, 1);
  }
  template <class NB>
  __device__ __forceinline__ static double wide(const NB& nb, int di, int dj, int v) {
    return (double)nb(di, dj, v) - (double)nb(di, dj, 12 + v);
  }
};

// ------------------------------------------- stencils reaching two rings
//
// Sec. 2 asks a stencil that reads beyond its nearest neighbours to be split
// into sub-steps that each read only those, and shows the split for one
// example (Eq. (1) into Eq. (2)-(3)): the first sub-step pushes neighbour
// values into extra slots of every point, the second reads them one hop
// away. PushTwoRing<WS> does that split for any one-step scheme WS whose
// step reads offsets (di, dj) with |di|, |dj| <= 2 (the offsets it declares
// in OFF). Offset (di, dj) is reached as the hop (a, b) = (di / 2, dj / 2)
// (rounded toward zero) to a neighbour, then the value that neighbour pushed
// from its own offset (di - a, dj - b); both hops lie within one ring.
// Slots: for each of WS's variables, one per distinct pushed offset, the
// offset (0, 0) first, so slot v * P of a point at a full step holds
// variable v and the other slots are zero. Sub-step 0 pushes; sub-step 1
// evaluates WS's step on the pushed values (the same values in the same
// expression as a direct evaluation, so the same bits) and clears them.
namespace wide {
constexpr int hop1(int d) { return d / 2; }
constexpr int hop2(int d) { return d - d / 2; }
// Index of pushed offset (c, d) among WS's pushed offsets, or -1.
template <class WS>
constexpr int pushed_index(int c, int d) {
  int k = 1;  // (0, 0) is index 0
  if (c == 0 && d == 0) return 0;
  bool seen[9] = {};
  seen[4] = true;
  for (int i = 0; i < WS::NOFF; ++i) {
    const int pc = hop2(WS::OFF[i][0]), pd = hop2(WS::OFF[i][1]);
    const int key = 3 * (pd + 1) + (pc + 1);
    if (seen[key]) continue;
    seen[key] = true;
    if (pc == c && pd == d) return k;
    ++k;
  }
  return -1;
}
template <class WS>
constexpr int pushed_count() {
  bool seen[9] = {};
  seen[4] = true;
  int k = 1;
  for (int i = 0; i < WS::NOFF; ++i) {
    const int key = 3 * (hop2(WS::OFF[i][1]) + 1) + (hop2(WS::OFF[i][0]) + 1);
    if (!seen[key]) {
      seen[key] = true;
      ++k;
    }
  }
  return k;
}
}  // namespace wide

template <class WS>
struct PushTwoRing {
  using V = typename WS::V;
  static constexpr int P = wide::pushed_count<WS>();
  static constexpr int NV = WS::NVAR * P, NW = NV, NVAR = NV, SUB = 2;
  static constexpr bool XY_SYM = false;
  static_assert(WS::SUB == 1, "a one-step wide scheme");
  // The wide step's view of the pushed values: offset (di, dj), variable v.
  template <class NB>
  struct Far {
    const NB& nb;
    __device__ __forceinline__ V operator()(int di, int dj, int v) const {
      return nb(wide::hop1(di), wide::hop1(dj), v * P + wide::pushed_index<WS>(wide::hop2(di), wide::hop2(dj)));
    }
  };
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams& sp) {
    if ((T & 1) == 0) {
#pragma unroll
      for (int v = 0; v < WS::NVAR; ++v) {
        out[v * P] = nb(0, 0, v * P);
#pragma unroll
        for (int i = 0; i < WS::NOFF; ++i) {
          const int c = wide::hop2(WS::OFF[i][0]), d = wide::hop2(WS::OFF[i][1]);
          out[v * P + wide::pushed_index<WS>(c, d)] = nb(c, d, v * P);
        }
      }
    } else {
      V res[WS::NVAR];
      WS::step(T >> 1, Far<NB>{nb}, res, sp);
#pragma unroll
      for (int v = 0; v < WS::NVAR; ++v) {
        out[v * P] = res[v];
#pragma unroll
        for (int k = 1; k < P; ++k) out[v * P + k] = V(0);
      }
    }
  }
};

// Test stencil reaching two rings: a 64-bit mix, in row-major order (north
// west first), of the 25 values at offsets |di|, |dj| <= 2 (integers below
// 2^52 held in doubles), seeded with the step index; the top 52 bits are the
// new value.
struct Hash25 {
  using V = double;
  static constexpr int NVAR = 1, SUB = 1, NOFF = 25;
  static constexpr int OFF[25][2] = {{-2, -2}, {-1, -2}, {0, -2}, {1, -2}, {2, -2}, {-2, -1}, {-1, -1}, {0, -1}, {1, -1},
                                     {2, -1},  {-2, 0},  {-1, 0}, {0, 0},  {1, 0},  {2, 0},   {-2, 1},  {-1, 1}, {0, 1},
                                     {1, 1},   {2, 1},   {-2, 2}, {-1, 2}, {0, 2},  {1, 2},   {2, 2}};
  template <class NB>
  __device__ __forceinline__ static void step(long long T, const NB& nb, V* out, const SchemeParams&) {
    uint64_t m = 0xC2B2AE3D27D4EB4Full ^ (uint64_t)T;
#pragma unroll
    for (int dj = -2; dj <= 2; ++dj)
#pragma unroll
      for (int di = -2; di <= 2; ++di) {
        m ^= (uint64_t)nb(di, dj, 0);
        m *= 0xFF51AFD7ED558CCDull;
        m ^= m >> 32;
      }
    out[0] = (double)(m >> 12);
  }
};
using Hash25x2 = PushTwoRing<Hash25>;

// FP32 with the compensation kept only within a residency: the state and
// the panels hold the values u alone (half the bytes of FP32C); the
// compensations are window-only values, zero when a point's value arrives
// from the state or a panel, so a value keeps its compensation while one
// workgroup computes its successive levels and loses it when it moves on.
// The heat update is Heat32C's (slots as there, the compensation after the
// value); the wave runs in velocity form (below).
struct Heat32R : Heat32C {
  static constexpr int NV = 1, NW = 2;
};
// The wave in velocity form, v = u^n - u^(n-1): v' = v + C2 lap and
// u' = u + v', each a compensated sum (the pair tv, c_v' of the new
// velocity is u's increment, both compensations folded in first); slots u,
// v and the window-only c_u, c_v; lap as in Wave32C. Equal to leapfrog in
// exact arithmetic. The stored pair is (u, v): a compensation dropped when a
// value changes window perturbs u or v by half a unit of its own size,
// whereas in the (u, u_prev) form the rounding of the displacement would
// enter the velocity u - u_prev and be integrated.
struct Wave32R {
  using V = float;
  static constexpr int NV = 2, NW = 4, NVAR = 2, SUB = 1;
  static constexpr bool XY_SYM = true;
  template <class NB>
  __device__ __forceinline__ static void step(long long, const NB& nb, V* out, const SchemeParams& sp) {
    const float c2 = (float)sp.p[0];
    const float u = nb(0, 0, 0);
    const float v = nb(0, 0, 1);
    const float cu = nb(0, 0, 2);
    const float cv = nb(0, 0, 3);
    const float lapu = ((nb(-1, 0, 0) - u) + (nb(1, 0, 0) - u)) + ((nb(0, -1, 0) - u) + (nb(0, 1, 0) - u));
    const float lapc = __builtin_fmaf(-4.0f, cu, (nb(-1, 0, 2) + nb(1, 0, 2)) + (nb(0, -1, 2) + nb(0, 1, 2)));
    const float lap = lapu - lapc;
    const float yv = c2 * lap - cv;
    const float tv = v + yv;
    const float cv1 = (tv - v) - yv;
    const float y = tv - (cu + cv1);
    const float t = u + y;
    out[2] = (t - u) - y;
    out[0] = t;
    out[1] = tv;
    out[3] = cv1;
  }
};

}  // namespace swept
