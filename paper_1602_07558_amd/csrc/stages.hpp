// Device code of the swept-rule stages on gfx950 (CDNA4), included by the
// per-scheme and per-launch-class translation units (stages_scheme.hip,
// stages_batch.hip); each instantiates its launchers once.
//
// Stage kernels: one workgroup per tile (upward pyramid, octahedron) or tile
// edge (bridge; at tile sides 32 and 64 a tile's two bridges share one
// workgroup). A workgroup keeps its whole space-time component in LDS: a
// window of (n+2) x (n+2) points per value slot (the internal arrays U and D
// of Algorithms 1-4), double buffered by level. A level is one pass over
// that level's rectangle, followed by a workgroup barrier.
//
// At tile sides 16, 32 and 64 the window pitch is a compile-time constant
// and the light schemes use column ownership (a lane per window column, a
// few rows per thread, horizontal neighbours by DPP lane shifts); other
// sides and the Euler schemes split a level into 2x2 quads.
//
// Panels (Sec. 3) travel through HBM between kernel launches. A level's
// panel strip is the two-wide boundary band of its rectangle; with double
// buffering, the band of level l stays untouched in buffer l mod 2 for the
// rest of the component (later levels of that parity lie strictly inside it),
// so the strips of level l can be stored while level l+1 is computed: the
// panel stores of a kernel spread over its whole run rather than leaving in
// one burst at its end, when every workgroup would write at once. A consumer
// either copies all its panel levels into LDS at its start, with every load
// in flight at once (staged), or fetches each level into registers a few
// levels before it places it.
//
// The plain kernel advances every point by one sub-step, reading its 3x3
// neighbourhood from HBM (rows kept in registers as a thread walks down a
// column strip).
#pragma once
#include <algorithm>
#include <type_traits>

#include "engine.hpp"

#pragma clang fp contract(off)

namespace swept {

namespace {

// Neighbour access in an LDS window. TR: the window holds the point at
// (x, y) in row x, column y (transposed), so the same stencil code reads
// (di, dj) from row di, column dj.
template <class V, bool TR = false>
struct WinNb {
  const V* c;
  int pitch;
  int plane;
  __device__ __forceinline__ V operator()(int di, int dj, int v) const {
    return TR ? c[v * plane + di * pitch + dj] : c[v * plane + dj * pitch + di];
  }
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
// Thread and wave index within a group of kThreads threads (a power of
// two): the whole workgroup, or one half of a workgroup that runs two
// components side by side. The wave index is read back as a wave-uniform
// (scalar) value, so per-wave loops branch on scalars instead of masking
// lanes.
template <int kThreads>
__device__ __forceinline__ int ltid() {
  static_assert((kThreads & (kThreads - 1)) == 0, "group size must be a power of two");
  return (int)(threadIdx.x & (kThreads - 1));
}
template <int kThreads>
__device__ __forceinline__ int lwave() {
  return __builtin_amdgcn_readfirstlane((int)((threadIdx.x & (kThreads - 1)) >> 6));
}

// A (wave-uniform) level hidden from the optimiser. The prefetch loops
// fetch the first levels before their loop with every load issued
// unconditionally, as inside it; with a known small level the compiler would
// drop a load it proves unused, and the loads in flight would then differ
// between the paths into the loop, which makes it wait for all of them.
__device__ __forceinline__ int opaque_level(int l) {
  __asm__ volatile("" : "+v"(l));
  return __builtin_amdgcn_readfirstlane(l);
}

__device__ __forceinline__ int wrap(int x, int m) {
  if (x < 0) x += m;
  if (x >= m) x -= m;
  if (x >= m) x -= m;
  return x;
}

__device__ __forceinline__ long long level_base(const Geo& g) { return g.T0 + (g.tbase ? *g.tbase : 0LL); }

// q = a d + b for 0 <= q < 2^21: (q + 1/2) / d is at least 1/(2d) away from
// an integer, far more than the error of the float product below.
__device__ __forceinline__ void fdivmod(int q, int d, float invd, int& a, int& b) {
  a = (int)(((float)q + 0.5f) * invd);
  b = q - a * d;
}

// Start of one end of a tile's panel (values).
__device__ __forceinline__ size_t up_end(const Geo& g, int nv, int tile, int end) {
  return ((size_t)tile * 4 + end) * (size_t)(2 * nv * up_levels_len(g.n, g.h));
}
__device__ __forceinline__ size_t xb_end(const Geo& g, int nv, int tile, int end) {
  return ((size_t)tile * 2 + end) * (size_t)(2 * nv * xb_levels_len(g.h));
}
__device__ __forceinline__ size_t yb_end(const Geo& g, int nv, int tile, int end) {
  return ((size_t)tile * 2 + end) * (size_t)(2 * nv * yb_levels_len(g.h));
}

// Gather `total` values into LDS with up to kBatch loads in flight per
// thread. Within a batch the loads are unconditional (indices clamped into
// range) so they issue back to back; the batch stops at the first row of
// kThreads that lies wholly past the end (a uniform test), and only the LDS
// stores are guarded.
constexpr int kBatch = 16;
template <int kThreads, class V, class Src, class Dst>
__device__ __forceinline__ void gather(int total, Src src, Dst dst) {
  if (total <= 0) return;
  for (int base = 0; base < total; base += kBatch * kThreads) {
    V r[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      if (base + i * kThreads >= total) break;
      const int q = base + ltid<kThreads>() + i * kThreads;
      r[i] = src(q < total ? q : total - 1);
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      if (base + i * kThreads >= total) break;
      const int q = base + ltid<kThreads>() + i * kThreads;
      if (q < total) dst(q, r[i]);
    }
  }
}

// Copy up to four contiguous global runs, back to back, into LDS.
template <int kThreads, class V>
__device__ __forceinline__ void stage_runs(V* __restrict__ lds, const V* s0, int n0, const V* s1, int n1, const V* s2,
                                           int n2, const V* s3, int n3) {
  const int e1 = n0, e2 = n0 + n1, e3 = n0 + n1 + n2, total = e3 + n3;
  gather<kThreads, V>(
      total,
      [&](int q) -> V {
        const V* p = s0 + q;
        if (q >= e1) p = s1 + (q - e1);
        if (q >= e2) p = s2 + (q - e2);
        if (q >= e3) p = s3 + (q - e3);
        return *p;
      },
      [&](int q, V v) { lds[q] = v; });
}

// The same copy for NR runs of at most C kThreads elements each: every run
// is read from its own base, so a load costs an index clamp and its offset
// instead of a choice among the runs per element; all loads are issued
// before the first store. Runs past NR are ignored.
template <int kThreads, int C, int NR, class V>
__device__ __forceinline__ void stage_runs_fixed(V* __restrict__ lds, const V* s0, int n0, const V* s1, int n1,
                                                 const V* s2, int n2, const V* s3, int n3) {
  const V* src[4] = {s0, s1, s2, s3};
  const int cnt[4] = {n0, n1, n2, n3};
  const int t = ltid<kThreads>();
  V r[NR][C];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int last = cnt[k] > 0 ? cnt[k] - 1 : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int q = t + c * kThreads;
      r[k][c] = src[k][q < last ? q : last];
    }
  }
  int off = 0;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int q = t + c * kThreads;
      if (q < cnt[k]) lds[off + q] = r[k][c];
    }
    off += cnt[k];
  }
}

// Elements per thread of the longest of `runs` staged runs of `len` values
// at a compiled window pitch, or 0 where the fixed copy does not apply (run
// time pitch, or more than 192 bytes of loads in flight per thread).
template <class V, int kThreads>
constexpr int stage_fixed_count(int len, int runs) {
  const int c = (len + kThreads - 1) / kThreads;
  return (len > 0 && c * runs * (int)sizeof(V) <= 192) ? c : 0;
}

// ------------------------------------------------------------------ quads

// The four points of a quad: o[0] = (x, y), o[1] = (x+1, y), o[2] = (x, y+1),
// o[3] = (x+1, y+1).
template <class S>
struct Quad {
  typename S::V o[4][S::NW];
};

template <class S, int WC, bool TR>
__device__ __forceinline__ void quad_step(const typename S::V* __restrict__ in, int idx, int Wrt, long long T,
                                          const SchemeParams& sp, Quad<S>& q) {
  const int W = WC ? WC : Wrt, plane = W * W;
  using NB = WinNb<typename S::V, TR>;
  S::step(T, NB{in + idx, W, plane}, q.o[0], sp);
  S::step(T, NB{in + idx + 1, W, plane}, q.o[1], sp);
  S::step(T, NB{in + idx + W, W, plane}, q.o[2], sp);
  S::step(T, NB{in + idx + W + 1, W, plane}, q.o[3], sp);
}

template <class S, int WC>
__device__ __forceinline__ void quad_store(typename S::V* __restrict__ out, int idx, int Wrt, const Quad<S>& q) {
  const int W = WC ? WC : Wrt, plane = W * W;
#pragma unroll
  for (int v = 0; v < S::NW; ++v) {
    out[v * plane + idx] = q.o[0][v];
    out[v * plane + idx + 1] = q.o[1][v];
    out[v * plane + idx + W] = q.o[2][v];
    out[v * plane + idx + W + 1] = q.o[3][v];
  }
}

// One level, double buffered: every quad of the window rectangle
// [x0, x0+w) x [y0, y0+hg) gets sub-step T from `in` into `out`; thread t
// takes quads t, t + kThreads, ... in row-major quad order.
template <class S, int WC, int kThreads, bool TR>
__device__ __forceinline__ void compute_quads(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                              int Wrt, int x0, int y0, int w, int hg, long long T,
                                              const SchemeParams& sp) {
  const int W = WC ? WC : Wrt;
  const int bw = w >> 1, nq = bw * (hg >> 1);
  if (nq <= 0) return;
  const float inv = 1.0f / (float)bw;
  for (int q = ltid<kThreads>(); q < nq; q += kThreads) {
    int by, bx;
    fdivmod(q, bw, inv, by, bx);
    const int idx = (y0 + 2 * by) * W + x0 + 2 * bx;
    Quad<S> r;
    quad_step<S, WC, TR>(in, idx, W, T, sp, r);
    quad_store<S, WC>(out, idx, W, r);
  }
}

// Neighbour access in registers: rw[row][column][v] around the point (TR as
// for WinNb).
template <class V, int NV, bool TR = false>
struct RegNb {
  const V (*rw)[3][NV];
  __device__ __forceinline__ V operator()(int di, int dj, int v) const {
    return TR ? rw[di + 1][dj + 1][v] : rw[dj + 1][di + 1][v];
  }
};

// Value of the lane one below (SR: lane i receives lane i-1) or one above
// (lane i receives lane i+1) in the wave, by DPP wave shifts; the end lane
// of the wave receives 0 (bound_ctrl, so no old value is needed). 64-bit
// values move as two 32-bit halves.
template <bool SR>
__device__ __forceinline__ int dpp_shift(int x) {
  return __builtin_amdgcn_update_dpp(x, x, SR ? 0x138 : 0x130, 0xF, 0xF, true);
}
template <bool SR>
__device__ __forceinline__ float dpp_shift(float x) {
  return __builtin_bit_cast(float, dpp_shift<SR>(__builtin_bit_cast(int, x)));
}
template <bool SR>
__device__ __forceinline__ double dpp_shift(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)dpp_shift<SR>((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)dpp_shift<SR>((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One level at window pitch 66 (64 lanes on the 64 interior columns), as
// this wave runs it. A wave is one row of groups: the rectangle's rows, from
// its first, are cut into groups of four dealt to the waves in turn, so a
// level keeps ceil(hg / 4) waves busy whatever the rectangle's position in
// the window. With hg >= 4 the last group is moved up to end on the
// rectangle's last row, so every group is whole (rows it shares with the
// group before get the same values twice) and every row read lies in the
// window; a rectangle of fewer rows (one group from y0 on wave 0, rows
// tested) lies in the middle of the window at this pitch. A tall rectangle at
// most 30 columns wide (a bridge's band in its later levels) gives each half
// wave a row group of its own, lane i of a half on window column x0 - 1 + i
// (a half without a group repeats the last one). The plan is worked out
// before the barrier that precedes the level, so that after it only the row
// reads' addresses stand between the barrier and the LDS reads.
template <int NT>
struct ColsPlan {
  static constexpr int R = 4, NW = NT / 64, KG = (64 / R + NW - 1) / NW;  // groups per wave at most
  int off[KG];    // window offset of the first row read, (r0 - 1) W + column
  bool act[KG];   // the group exists (wave-uniform)
  bool store;     // this lane's column lies in the rectangle
  int nrows;      // rows stored per group: 4, or hg < 4
};

template <int WC, int NT>
__device__ __forceinline__ ColsPlan<NT> cols_plan(int x0, int y0, int w, int hg) {
  using P = ColsPlan<NT>;
  constexpr int R = P::R, NW = P::NW, W = WC;
  const int wave = lwave<NT>(), lane = lane_id();
  P p;
  if (w + 2 <= 32 && hg > R * NW) {
    const int half = lane >> 5, i = lane & 31, col = x0 - 1 + i;
    const int r0 = min(y0 + R * (2 * wave + half), y0 + hg - R);
#pragma unroll
    for (int k = 0; k < P::KG; ++k) {
      p.act[k] = k == 0 && 2 * R * wave < hg;  // a second pass would need hg > 8 NW rows
      p.off[k] = (r0 - 1) * W + col;
    }
    p.store = i >= 1 && i <= w;
    p.nrows = R;
  } else if (hg >= R) {
    const int col = 1 + lane;
#pragma unroll
    for (int k = 0; k < P::KG; ++k) {
      const int grp = wave + k * NW;
      p.act[k] = R * grp < hg;
      p.off[k] = (min(y0 + R * grp, y0 + hg - R) - 1) * W + col;
    }
    p.store = (unsigned)(col - x0) < (unsigned)w;
    p.nrows = R;
  } else {
    const int col = 1 + lane;
#pragma unroll
    for (int k = 0; k < P::KG; ++k) {
      p.act[k] = k == 0 && wave == 0;
      p.off[k] = (y0 - 1) * W + col;
    }
    p.store = (unsigned)(col - x0) < (unsigned)w;
    p.nrows = hg;
  }
  return p;
}

template <class S, int WC, int NT, bool TR, bool DPP>
__device__ __forceinline__ void cols_run(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                         const ColsPlan<NT>& p, long long T, const SchemeParams& sp) {
  using V = typename S::V;
  constexpr int NV = S::NW, W = WC, plane = W * W, R = ColsPlan<NT>::R;  // every window value
#pragma unroll
  for (int k = 0; k < ColsPlan<NT>::KG; ++k) {
    if (!p.act[k]) continue;
    // Rows r0-1 .. r0+R into registers, the side neighbours by DPP (or LDS
    // at EDGE levels), for every lane of the wave.
    const V* src = in + p.off[k];
    V nb[R + 2][3][NV];
#pragma unroll
    for (int j = 0; j < R + 2; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const V m = src[v * plane + j * W];
        nb[j][1][v] = m;
        if constexpr (DPP) {
          nb[j][0][v] = dpp_shift<true>(m);
          nb[j][2][v] = dpp_shift<false>(m);
        } else {
          nb[j][0][v] = src[v * plane + j * W - 1];
          nb[j][2][v] = src[v * plane + j * W + 1];
        }
      }
    if (p.store) {
      V* dst = out + p.off[k] + W;
      if (p.nrows == R) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          V o[NV];
          S::step(T, RegNb<V, NV, TR>{&nb[i]}, o, sp);
#pragma unroll
          for (int v = 0; v < NV; ++v) dst[v * plane + i * W] = o[v];
        }
      } else {
#pragma unroll
        for (int i = 0; i < R - 1; ++i) {
          if (i < p.nrows) {
            V o[NV];
            S::step(T, RegNb<V, NV, TR>{&nb[i]}, o, sp);
#pragma unroll
            for (int v = 0; v < NV; ++v) dst[v * plane + i * W] = o[v];
          }
        }
      }
    }
  }
}

// One level at tile sides 16 and 32 (a few waves), one rectangle point per
// thread: thread i of pass q takes point k = i + NT q of the rectangle in row
// order (row k / w, column k mod w) and reads its 3x3 neighbourhood from LDS.
// A level of w hg points takes ceil(w hg / NT) passes, where the column layout
// would take one pass over every row of the tile whatever the rectangle; the
// pyramids' and bridges' small levels fit one pass. The row index comes from a float
// product with the hardware reciprocal of w (within one ulp): for k < 4096
// and w <= 64, (k + 1/2) / w lies at least 1/(2w) from an integer, far
// beyond the product's error.
template <class S, int WC, int NT, bool TR>
__device__ __forceinline__ void compute_compact(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                                int x0, int y0, int w, int hg, long long T, const SchemeParams& sp) {
  using V = typename S::V;
  constexpr int NV = S::NW, W = WC, plane = W * W;  // every window value
  const int npts = w * hg;
  const float inv_w = __builtin_amdgcn_rcpf((float)(w > 0 ? w : 1));
  for (int base = 0; base < npts; base += NT) {
    const int k = base + ltid<NT>();
    if (k < npts) {
      const int dy = (int)(((float)k + 0.5f) * inv_w);
      const int o = (y0 + dy) * W + x0 + (k - dy * w);
      V nb[3][3][NV];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int v = 0; v < NV; ++v) nb[r][c][v] = in[v * plane + o + (r - 1) * W + (c - 1)];
      V res[NV];
      S::step(T, RegNb<V, NV, TR>{&nb[0]}, res, sp);
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v * plane + o] = res[v];
    }
  }
}

// One level with column ownership: the rows of the thread's column that lie
// in the rectangle [x0, x0+w) x [y0, y0+hg) get sub-step T from `in` into
// `out`. The thread first reads the R+2 rows of its column it needs (its own
// value per row) with every lane of the wave active, and takes the columns
// left and right of it from the neighbouring lanes by DPP (DPP) or from LDS
// (EDGE levels); then, under one column mask, it computes and stores the
// rows inside the rectangle. Lanes are consecutive window columns, N of them
// per row group, so every LDS access of a wave is one contiguous run. A row
// group's first and last lanes (window columns 1 and N) get no valid
// neighbour from a shift, so DPP levels must keep the rectangle within
// columns 2 .. N-1 (true for every level of every component except the
// downward pyramid's last, full-tile level).
template <class S, int WC, int NT, bool TR, bool DPP>
__device__ __forceinline__ void compute_cols(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                             int x0, int y0, int w, int hg, long long T, const SchemeParams& sp) {
  using V = typename S::V;
  constexpr int NV = S::NW, W = WC, plane = W * W, N = Lay<S, WC, NT>::N;  // every window value
  if constexpr (N == 64) {
    cols_run<S, WC, NT, TR, DPP>(in, out, cols_plan<WC, NT>(x0, y0, w, hg), T, sp);
  } else if constexpr (WC == 18 || WC == 34) {
    compute_compact<S, WC, NT, TR>(in, out, x0, y0, w, hg, T, sp);
  } else {
    constexpr int R = Lay<S, WC, NT>::R;
    const int t = ltid<NT>();
    const int c = 1 + t % N;
    const int r0 = 1 + R * (t / N);
    const bool rows_in = !(r0 + R <= y0 || r0 >= y0 + hg);
    if (!__builtin_amdgcn_ballot_w64(rows_in)) return;  // wave-uniform exit
    const V* src = in + (r0 - 1) * W + c;
    V nb[R + 2][3][NV];
#pragma unroll
    for (int j = 0; j < R + 2; ++j)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const V m = src[v * plane + j * W];
        nb[j][1][v] = m;
        if constexpr (DPP) {
          nb[j][0][v] = dpp_shift<true>(m);
          nb[j][2][v] = dpp_shift<false>(m);
        } else {
          nb[j][0][v] = src[v * plane + j * W - 1];
          nb[j][2][v] = src[v * plane + j * W + 1];
        }
      }
    if ((unsigned)(c - x0) >= (unsigned)w) return;
    V* dst = out + r0 * W + c;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if ((unsigned)(r0 + i - y0) < (unsigned)hg) {
        V o[NV];
        S::step(T, RegNb<V, NV, TR>{&nb[i]}, o, sp);
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v * plane + i * W] = o[v];
      }
    }
  }
}

// One level of a flux scheme (S::WALK: the Euler schemes) over the rectangle
// [x0, x0+w) x [y0, y0+hg) as a column walk. The rectangle is cut into
// segments of at most 30 columns (one or two chunks across) by kWalkRows
// rows; a segment runs on cw + 2 consecutive lanes of one wave (lane i on
// window column xa - 1 + i: the chunk's columns and one on each side; lanes
// past them repeat the last one), as many segments per wave as fit. Each
// lane walks its segment's rows with one row above and below it. Per row a
// lane computes its cell's face data along both axes once (S::wcells: what
// a face flux needs of one side, e.g. the pressure, velocities and sound
// speed, with their divisions and square root), takes the east lane's by a
// DPP lane shift, forms the face flux between them (S::wface), and passes it
// west by another shift (the shifts cross segments only at their side
// lanes, which store nothing); the face between consecutive rows is formed
// once as the walk reaches the lower row. Every face flux is the same
// expression on the same operands as in the per-point step (left/lower side
// first), and the flux difference is summed in the step's order, so the
// results are bit for bit the same. TR (transposed window, the x-bridge):
// window rows run along x, so the walk is the x axis and the lanes the y
// axis.
//
// A WALK scheme provides: CN (doubles of face data per cell and axis),
// wstage(T) (first slot of the four values the fluxes are taken from),
// wload(p, plane, v) (slot v at p as a double), wcells(C, sp, cx, cy) (the
// face data along x and y from those four values), wface(cL, cR, d, sp, F)
// (the flux through the face along d between cells L and R), and
// finish(T, own, plane, C, div, sp, dst) (the cell's new slots from its own
// old slots at `own`, its four flux values C and div = h times the
// divergence of the face fluxes, x terms first).
//
// Rows per segment: one. The levels are latency-bound, so independent lanes
// pay more than the flux work a lane repeats for the rows above and below
// it. Measured with 1, 2 and 4 rows: Rusanov Euler on 512^2 at tile side 32
// (one 8-wave workgroup per CU), full RK2 steps per second 1.27e10, 1.23e10,
// 9.6e9 (6 rows 7.6e9); the 12-value Euler on 1024 x 512 at tile side 16,
// full RK4 steps 3.32e9, 2.83e9, 1.20e9.
constexpr int kWalkRows = 1;
template <class S, int WC, int NT, bool TR>
__device__ __forceinline__ void flux_walk(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                          int Wrt, int x0, int y0, int w, int hg, long long T,
                                          const SchemeParams& sp) {
  constexpr int R = kWalkRows, NWv = NT / 64, CN = S::CN;
  const int W = WC ? WC : Wrt, plane = W * W;
  const int o = S::wstage(T);
  constexpr int dl = TR ? 1 : 0;  // axis along the lanes (window columns)
  constexpr int dw = TR ? 0 : 1;  // axis along the walk (window rows)
  if (w <= 0 || hg <= 0) return;
  const int nch = w + 2 <= 32 ? 1 : 2;          // chunks across
  const int cw = (w + nch - 1) / nch;            // columns per chunk (the last may have fewer)
  const int lps = cw + 2;                        // lanes per segment
  // A segment fits one wave for w <= 124. The walk schemes' windows (at
  // least 64 bytes per point, two buffers) bound their tiles to 33 columns
  // in the 160 KB of LDS, so this never returns.
  if (lps > 64) return;
  const int spw = 64 / lps;                      // segments per wave
  const int nseg = nch * ((hg + R - 1) / R);
  const int nunit = (nseg + spw - 1) / spw;
  const int lane = lane_id();
  int slot, li;
  fdivmod(lane, lps, __builtin_amdgcn_rcpf((float)lps), slot, li);
  for (int unit = lwave<NT>(); unit < nunit; unit += NWv) {
    const int sraw = unit * spw + slot;
    const bool real = slot < spw && sraw < nseg;
    const int seg = real ? sraw : unit * spw;    // idle lanes repeat a real segment and store nothing
    const int rs = seg / nch, ch = seg - rs * nch;
    const int xa = x0 + ch * cw;
    const int cwc = min(cw, x0 + w - xa);        // this chunk's columns
    const int col = xa - 1 + (li <= cwc + 1 ? li : cwc + 1);
    const bool store = real && li >= 1 && li <= cwc;
    const int ys = y0 + rs * R;
    const int ye = min(ys + R, y0 + hg);         // rows ys .. ye-1 are computed
    // Rows ys-1 .. ys+R (rows past ye repeat row ye and store nothing): all
    // rows' face data first, independent of one another, then the faces,
    // then the updates.
    double C[R + 2][4], cx[R + 2][CN], cy[R + 2][CN];
#pragma unroll
    for (int i = 0; i < R + 2; ++i) {
      const int r = min(ys - 1 + i, ye);
      const typename S::V* src = in + r * W + col;
#pragma unroll
      for (int k = 0; k < 4; ++k) C[i][k] = S::wload(src, plane, o + k);
      S::wcells(C[i], sp, cx[i], cy[i]);
    }
    auto& cl = TR ? cy : cx;  // face data along the lanes
    auto& cwk = TR ? cx : cy;  // face data along the walk
    double G[R + 1][4];  // G[i]: face between rows i and i+1 (walk axis)
#pragma unroll
    for (int i = 0; i < R + 1; ++i) S::wface(cwk[i], cwk[i + 1], dw, sp, G[i]);
#pragma unroll
    for (int i = 1; i <= R; ++i) {
      // faces along the lanes: with the east lane, then the west one's
      // passed over
      double ce[CN], FeL[4], FwL[4];
#pragma unroll
      for (int k = 0; k < CN; ++k) ce[k] = dpp_shift<false>(cl[i][k]);
      S::wface(cl[i], ce, dl, sp, FeL);
#pragma unroll
      for (int k = 0; k < 4; ++k) FwL[k] = dpp_shift<true>(FeL[k]);
      double div[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        div[k] = TR ? (G[i][k] - G[i - 1][k]) + (FeL[k] - FwL[k]) : (FeL[k] - FwL[k]) + (G[i][k] - G[i - 1][k]);
      const int r = ys - 1 + i;
      if (store && r < ye) {
        const int q = r * W + col;
        S::finish(T, in + q, plane, C[i], div, sp, out + q);
      }
    }
  }
}

// EDGE: the rectangle may touch window columns 1 or N (the downward
// pyramid's full-tile level); otherwise the column layout uses DPP shifts.
template <class S, int WC, int NT, bool TR = false, bool EDGE = false>
__device__ __forceinline__ void compute_level(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                              int Wrt, int x0, int y0, int w, int hg, long long T,
                                              const SchemeParams& sp) {
  if constexpr (walks<S>::value) {
    flux_walk<S, WC, NT, TR>(in, out, Wrt, x0, y0, w, hg, T, sp);
  } else if constexpr (Lay<S, WC, NT>::cols) {
    compute_cols<S, WC, NT, TR, !EDGE>(in, out, x0, y0, w, hg, T, sp);
  } else {
    compute_quads<S, WC, NT, TR>(in, out, Wrt, x0, y0, w, hg, T, sp);
  }
}

// A level's rectangle, planned ahead of its barrier where the layout allows
// (window pitch 66), and run after it.
template <class S, int WC, int NT, bool C66 = (WC == 66 && Lay<S, WC, NT>::cols)>
struct LevelPlan {
  int x0, y0, w, hg;
};
template <class S, int WC, int NT>
struct LevelPlan<S, WC, NT, true> {
  ColsPlan<NT> cp;
};

template <class S, int WC, int NT>
__device__ __forceinline__ LevelPlan<S, WC, NT> level_plan(int x0, int y0, int w, int hg) {
  if constexpr (WC == 66 && Lay<S, WC, NT>::cols)
    return LevelPlan<S, WC, NT>{cols_plan<WC, NT>(x0, y0, w, hg)};
  else
    return LevelPlan<S, WC, NT>{x0, y0, w, hg};
}

template <class S, int WC, int NT, bool TR = false>
__device__ __forceinline__ void level_run(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                          int Wrt, const LevelPlan<S, WC, NT>& p, long long T,
                                          const SchemeParams& sp) {
  if constexpr (WC == 66 && Lay<S, WC, NT>::cols)
    cols_run<S, WC, NT, TR, true>(in, out, p.cp, T, sp);
  else
    compute_level<S, WC, NT, TR>(in, out, Wrt, p.x0, p.y0, p.w, p.hg, T, sp);
}

// Window -> state for the rectangle [wx0, wx0+w) x [wy0, wy0+hg); the window
// origin is global (xw0, yw0). TR: the window is transposed.
template <class S, int kThreads, bool TR = false>
__device__ void write_rect(const typename S::V* __restrict__ win, typename S::V* __restrict__ state, const Geo& g,
                           int xw0, int yw0, int wx0, int wy0, int w, int hg) {
  const int npts = w * hg;
  if (npts <= 0) return;
  const int plane = g.W * g.W;
  const size_t gplane = (size_t)g.nx * g.ny;
  const float invw = 1.0f / (float)w;
  for (int p = ltid<kThreads>(); p < npts; p += kThreads) {
    int y, x;
    fdivmod(p, w, invw, y, x);
    const int wx = wx0 + x, wy = wy0 + y;
    const int gx = wrap(xw0 + wx, g.nx), gy = wrap(yw0 + wy, g.ny);
#pragma unroll
    for (int v = 0; v < S::NV; ++v)
      state[v * gplane + (size_t)gy * g.nx + gx] = win[v * plane + (TR ? wx * g.W + wy : wy * g.W + wx)];
  }
}

// Panel strips of one level on their way from LDS to HBM, read before a
// level's compute pass and stored after it, so that the stores of all
// levels spread over the kernel instead of leaving in one burst at its end
// (when every workgroup would write at once). Unit u = w + j kWaves with w
// counted from the last wave (the first to fall idle as a pyramid shrinks),
// lanes along the strip, P positions per lane.
template <class S, int kThreads, int P, int UNITS>
struct EmitSlot {
  static constexpr int J = (UNITS + kThreads / 64 - 1) / (kThreads / 64);
  typename S::V val[J][P];
  typename S::V* dst[J];
  int len[J];
};

// Schemes with few values per point read a level's panels before its
// compute pass (the LDS latency hides behind it); the others read them
// after it, which keeps the panel registers free during the compute.
template <class S>
constexpr bool emit_early() {
  return S::NV * (int)sizeof(typename S::V) <= 16;
}

template <class S, int kThreads, int P, int UNITS>
__device__ __forceinline__ void emit_write(const EmitSlot<S, kThreads, P, UNITS>& e) {
#pragma unroll
  for (int j = 0; j < EmitSlot<S, kThreads, P, UNITS>::J; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      if (t < e.len[j]) e.dst[j][t] = e.val[j][i];
    }
}

// Upward-pyramid panel strips of level l (Alg. 1): strip k of side `end`
// is the row (ends 0, 1) or column (ends 2, 3) at distance l + k from the
// tile edge, n - 2l long, read from the buffer where level l's band
// survives. A wave's units are fixed, so everything but the level is set up
// once: the strip's panel offset, 2 NV up_levels_len(n, l) + rem (n - 2l),
// is d0 + l d1 - 2 NV l^2, and its window start is s0 + l ds.
template <class S, int kThreads>
struct UpEmitPre {
  static constexpr int J = EmitSlot<S, kThreads, 1, 8 * S::NV>::J;
  typename S::V* base[J];  // panel of the unit's side and slot row, null: no unit
  int d1[J], s0[J], ds[J], stride[J];
};

template <class S, int kThreads>
__device__ __forceinline__ void up_emit_init(UpEmitPre<S, kThreads>& r, typename S::V* __restrict__ up,
                                             const Geo& g, int tile) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, per = 8 * NV;
  const int n = g.n, W = g.W, plane = W * W;
  const int w = kWaves - 1 - lwave<kThreads>();
#pragma unroll
  for (int j = 0; j < UpEmitPre<S, kThreads>::J; ++j) {
    const int u = w + j * kWaves;
    const int uu = u < per ? u : 0;
    const int end = uu / (2 * NV), rem = uu - end * 2 * NV, v = rem >> 1, k = rem & 1;
    r.base[j] = u < per ? up + up_end(g, NV, tile, end) + rem * n : nullptr;
    r.d1[j] = 2 * NV * (n + 1) - 2 * rem;
    if (end == 0) {  // row l+1+k from column l+1
      r.s0[j] = (1 + k) * W + 1, r.ds[j] = W + 1, r.stride[j] = 1;
    } else if (end == 1) {  // row n-l-k from column l+1
      r.s0[j] = (n - k) * W + 1, r.ds[j] = 1 - W, r.stride[j] = 1;
    } else if (end == 2) {  // column l+1+k from row l+1
      r.s0[j] = W + 1 + k, r.ds[j] = W + 1, r.stride[j] = W;
    } else {  // column n-l-k from row l+1
      r.s0[j] = W + n - k, r.ds[j] = W - 1, r.stride[j] = W;
    }
    r.s0[j] += v * plane;
  }
}

template <class S, int kThreads, int P>
__device__ __forceinline__ void up_strips_read(EmitSlot<S, kThreads, P, 8 * S::NV>& e, const UpEmitPre<S, kThreads>& r,
                                               const typename S::V* __restrict__ win, const Geo& g, int l) {
  constexpr int NV = S::NV;
  const int len = g.n - 2 * l;
#pragma unroll
  for (int j = 0; j < EmitSlot<S, kThreads, P, 8 * NV>::J; ++j) {
    e.len[j] = 0;
    if (r.base[j] == nullptr) continue;
    e.len[j] = len;
    e.dst[j] = r.base[j] + (l * r.d1[j] - 2 * NV * l * l);
    const typename S::V* src = win + r.s0[j] + l * r.ds[j];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      e.val[j][i] = src[(t < len ? t : 0) * r.stride[j]];
    }
  }
}

// The same strips with every term worked out at each level (groups of few
// waves, whose many units per wave would not fit precomputed in registers).
template <class S, int kThreads, int P>
__device__ __forceinline__ void up_strips_read_direct(EmitSlot<S, kThreads, P, 8 * S::NV>& e,
                                               const typename S::V* __restrict__ win, typename S::V* __restrict__ up,
                                               const Geo& g, int tile, int l) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, per = 8 * NV;
  const int n = g.n, W = g.W, plane = W * W, len = n - 2 * l;
  const int w = kWaves - 1 - lwave<kThreads>();
#pragma unroll
  for (int j = 0; j < EmitSlot<S, kThreads, P, per>::J; ++j) {
    const int u = w + j * kWaves;
    e.len[j] = 0;
    if (u >= per) continue;
    const int end = u / (2 * NV), rem = u - end * 2 * NV, v = rem >> 1, k = rem & 1;
    e.len[j] = len;
    e.dst[j] = up + up_end(g, NV, tile, end) + (size_t)2 * NV * up_levels_len(n, l) + (size_t)rem * len;
    int wx0, wy0, stride;  // window position of t = 0 and step along the strip
    if (end == 0) {
      wx0 = l + 1, wy0 = l + 1 + k, stride = 1;
    } else if (end == 1) {
      wx0 = l + 1, wy0 = n - l - k, stride = 1;
    } else if (end == 2) {
      wx0 = l + 1 + k, wy0 = l + 1, stride = W;
    } else {
      wx0 = n - l - k, wy0 = l + 1, stride = W;
    }
    const typename S::V* src = win + v * plane + wy0 * W + wx0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      e.val[j][i] = src[(t < len ? t : 0) * stride];
    }
  }
}

// Panel emission with several short runs side by side in one wave slot
// (tile side 16 on one wave): G runs of 64 / G lanes each, every term of a
// lane's element set up once. An element's panel address is
// base + l d1 +- 2 NV l^2 and its window index s0 + l ds; it exists at level
// l when c0 < 2l.
template <class S, int J>
struct EmitLanes {
  typename S::V val[J];
  typename S::V* dst[J];
  bool ok[J];
};

template <class S, int J>
__device__ __forceinline__ void emit_write(const EmitLanes<S, J>& e) {
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (e.ok[j]) *e.dst[j] = e.val[j];
}

template <class S, int kThreads, int G, int UNITS>
struct PackPre {
  static constexpr int kWaves = kThreads / 64, LG = 64 / G;
  static constexpr int J = ((UNITS + G - 1) / G + kWaves - 1) / kWaves;
  typename S::V* base[J];
  int d1[J], s0[J], ds[J], c0[J];
};

// Upward-pyramid strips (as up_strips_read), packed: element t of a strip
// exists while t < n - 2l, that is while c0 + 2l < 0 with c0 = t - n.
template <class S, int kThreads, int G>
__device__ __forceinline__ void up_pack_init(PackPre<S, kThreads, G, 8 * S::NV>& r, typename S::V* __restrict__ up,
                                             const Geo& g, int tile) {
  using R = PackPre<S, kThreads, G, 8 * S::NV>;
  constexpr int NV = S::NV;
  const int n = g.n, W = g.W, plane = W * W;
  const int sub = lane_id() / R::LG, t = lane_id() - sub * R::LG;
#pragma unroll
  for (int j = 0; j < R::J; ++j) {
    const int u = (lwave<kThreads>() + j * R::kWaves) * G + sub;
    const bool has = sub < G && u < 8 * NV;
    const int uu = has ? u : 0;
    const int end = uu / (2 * NV), rem = uu - end * 2 * NV, v = rem >> 1, k = rem & 1;
    r.base[j] = up + up_end(g, NV, tile, end) + rem * n + t;
    r.d1[j] = 2 * NV * (n + 1) - 2 * rem;
    int s0, ds, stride;
    if (end == 0) {
      s0 = (1 + k) * W + 1, ds = W + 1, stride = 1;
    } else if (end == 1) {
      s0 = (n - k) * W + 1, ds = 1 - W, stride = 1;
    } else if (end == 2) {
      s0 = W + 1 + k, ds = W + 1, stride = W;
    } else {
      s0 = W + n - k, ds = W - 1, stride = W;
    }
    r.s0[j] = v * plane + s0 + t * stride;
    r.ds[j] = ds;
    r.c0[j] = has ? t - n : 1 << 28;
  }
}

template <class S, int kThreads, int G>
__device__ __forceinline__ void up_pack_read(EmitLanes<S, PackPre<S, kThreads, G, 8 * S::NV>::J>& e,
                                             const PackPre<S, kThreads, G, 8 * S::NV>& r,
                                             const typename S::V* __restrict__ win, int l) {
  constexpr int NV = S::NV;
#pragma unroll
  for (int j = 0; j < PackPre<S, kThreads, G, 8 * S::NV>::J; ++j) {
    e.ok[j] = r.c0[j] + 2 * l < 0;
    e.val[j] = win[e.ok[j] ? r.s0[j] + l * r.ds[j] : 0];
    e.dst[j] = r.base[j] + (l * r.d1[j] - 2 * NV * l * l);
  }
}

// Bridge panels (as bridge_ends_read), packed: element t exists while
// t < len(l) = 2l + cz, stored as c0 = t - cz (exists when c0 < 2l).
template <class S, int kThreads, int G>
__device__ __forceinline__ void bridge_pack_init(PackPre<S, kThreads, G, 4 * S::NV>& r,
                                                 typename S::V* __restrict__ out, bool isx, const Geo& g, int e) {
  using R = PackPre<S, kThreads, G, 4 * S::NV>;
  constexpr int NV = S::NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W;
  const int sub = lane_id() / R::LG, t = lane_id() - sub * R::LG;
#pragma unroll
  for (int j = 0; j < R::J; ++j) {
    const int u = (lwave<kThreads>() + j * R::kWaves) * G + sub;
    const bool has = sub < G && u < 4 * NV;
    const int uu = has ? u : 0;
    const int end = uu / (2 * NV), rem = uu - end * 2 * NV, v = rem >> 1, k = rem & 1;
    r.base[j] = out + (isx ? xb_end(g, NV, e, end) + 4 * rem : yb_end(g, NV, e, end)) + t;
    r.d1[j] = isx ? 6 * NV + 2 * rem : 2 * rem - 2 * NV;
    r.s0[j] = v * plane + (isx ? h - 1 : h + 1) * W + (end ? n - k : 1 + k) + t * W;
    r.ds[j] = end ? -W - 1 : 1 - W;
    r.c0[j] = has ? t - (isx ? 4 : 0) : 1 << 28;
  }
}

template <class S, int kThreads, int G>
__device__ __forceinline__ void bridge_pack_read(EmitLanes<S, PackPre<S, kThreads, G, 4 * S::NV>::J>& e,
                                                 const PackPre<S, kThreads, G, 4 * S::NV>& r,
                                                 const typename S::V* __restrict__ win, int l) {
  constexpr int NV = S::NV;
#pragma unroll
  for (int j = 0; j < PackPre<S, kThreads, G, 4 * S::NV>::J; ++j) {
    e.ok[j] = r.c0[j] < 2 * l;
    e.val[j] = win[e.ok[j] ? r.s0[j] + l * r.ds[j] : 0];
    e.dst[j] = r.base[j] + (l * r.d1[j] + 2 * NV * l * l);
  }
}

// Levels 1..H of the upward pyramid of `tile` whose level 0 (the whole tile,
// window interior) is in buffer b0, then its panels of levels 0..H-1; when
// H < h (reduced last half cycle) it also writes the level-H square to the
// state.
template <class S, int WC, int NT>
__device__ void up_levels(typename S::V* buf0, typename S::V* buf1, int b0, const Geo& g, int tile, int x0, int y0,
                          long long T0, int H, typename S::V* state, typename S::V* up, const SchemeParams& sp) {
  const int n = g.n, h = g.h;
  const int top = H < h - 1 ? H : h - 1;
  // Strips are at most n long: one position per lane up to n = 64.
  constexpr int kP = (WC != 0 && WC <= 66) ? 1 : 2;
  // Groups of many waves hold each wave's few units precomputed; groups of
  // few waves work every term out per level.
  // At tile sides up to 32 on few waves, 64 / n strips share a wave slot.
  constexpr bool kPre = UpEmitPre<S, NT>::J <= 2;
  constexpr bool kPack = !kPre && WC != 0 && WC <= 34;
  constexpr int kG = kPack ? 64 / (WC > 2 ? WC - 2 : 1) : 1;
  using PK = PackPre<S, NT, kG, 8 * S::NV>;
  using E = std::conditional_t<kPack, EmitLanes<S, PK::J>, EmitSlot<S, NT, kP, 8 * S::NV>>;
  [[maybe_unused]] UpEmitPre<S, NT> ep;
  [[maybe_unused]] PK pk;
  if constexpr (kPre) up_emit_init<S, NT>(ep, up, g, tile);
  if constexpr (kPack) up_pack_init<S, NT, kG>(pk, up, g, tile);
  auto strips_read = [&](E& es, const typename S::V* win, int l) {
    if constexpr (kPre)
      up_strips_read<S, NT, kP>(es, ep, win, g, l);
    else if constexpr (kPack)
      up_pack_read<S, NT, kG>(es, pk, win, l);
    else
      up_strips_read_direct<S, NT, kP>(es, win, up, g, tile, l);
  };
  // Level l's pass also emits the panel strips of level l-1; the next
  // level's rectangle is planned before the barrier.
  auto plan = [&](int l) { return level_plan<S, WC, NT>(l + 1, l + 1, n - 2 * l, n - 2 * l); };
  auto pl = plan(1);
  for (int l = 1; l <= top; ++l) {
    typename S::V* cur = ((b0 + l) & 1) ? buf1 : buf0;
    const typename S::V* prv = ((b0 + l) & 1) ? buf0 : buf1;
    E es;
    if constexpr (emit_early<S>()) strips_read(es, prv, l - 1);
    level_run<S, WC, NT>(prv, cur, g.W, pl, T0 + l - 1, sp);
    if constexpr (!emit_early<S>()) strips_read(es, prv, l - 1);
    emit_write(es);
    pl = plan(l + 1);
    __syncthreads();
  }
  for (int l = top; l < H; ++l) {  // the last emitted level (level h-1 of a full half cycle)
    E es;
    strips_read(es, ((b0 + l) & 1) ? buf1 : buf0, l);
    emit_write(es);
  }
  if (H < h) {
    const typename S::V* fin = ((b0 + H) & 1) ? buf1 : buf0;
    write_rect<S, NT>(fin, state, g, x0 - 1, y0 - 1, H + 1, H + 1, n - 2 * H, n - 2 * H);
  }
}

// Per-level panel inputs held in registers: slot j of a wave covers G units
// (runs) side by side, 64 / G lanes each, with P positions per lane (runs
// are at most n + 2 <= 128 long); J slots are enough for the 8 NV units of a
// ring and the 4 NV of a bridge. The fetch path from HBM uses G = 1: unit
// u = wave + j * kWaves.
template <class S, int kThreads, int P = 2, int G = 1>
struct Fetch {
  static constexpr int J = ((8 * S::NV + G - 1) / G + kThreads / 64 - 1) / (kThreads / 64);
  typename S::V val[J][P];
  int dst[J][P];
};

// Window position of element t of ring band `band` (0 top, 1 bottom, 2 left,
// 3 right) at level l, row/column k; the downward pyramid's square at level
// l is [h+1-l, h+1+l)^2.
__device__ __forceinline__ void ring_pos(int h, int l, int band, int k, int t, int& wx, int& wy) {
  if (band == 0) {
    wx = h - l - 1 + t;
    wy = h - l - k;
  } else if (band == 1) {
    wx = h - l - 1 + t;
    wy = h + 1 + l + k;
  } else if (band == 2) {
    wx = h - l - k;
    wy = h + 1 - l + t;
  } else {
    wx = h + 1 + l + k;
    wy = h + 1 - l + t;
  }
}

// Window index (one value slot) of element t of bridge input strip `side`
// (0: tile A's facing strip, 1: tile B's) at level l, row/column k. Both
// bridges use the y-bridge's layout: strips are window rows; the x-bridge's
// window is the transposed one (row = x, column = y), where its facing
// columns become rows.
__device__ __forceinline__ int strip_idx(int W, int h, int l, int side, int k, int t) {
  const int across = side ? (h + 1 + l + k) : (h - l - k);
  return across * W + l + 1 + t;
}

template <class S, int kThreads, int P>
__device__ __forceinline__ void fetch_ring(Fetch<S, kThreads, P>& f, const Geo& g, int l, const typename S::V* __restrict__ xb,
                                           const typename S::V* __restrict__ yb, int eTop, int eBot, int eLeft,
                                           int eRight) {
  constexpr int kWaves = kThreads / 64;
  constexpr int NV = S::NV;
  const int h = g.h, W = g.W, plane = W * W;
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P>::J; ++j) {
    const int u = lwave<kThreads>() + j * kWaves;
#pragma unroll
    for (int i = 0; i < P; ++i) f.dst[j][i] = -1;
    if (u >= 8 * NV) continue;
    const int band = u / (2 * NV), rem = u - band * 2 * NV, v = rem >> 1, k = rem & 1;
    const bool horiz = band < 2;
    const int len = horiz ? 2 * l + 4 : 2 * l;
    const typename S::V* src;
    if (band == 0)
      src = xb + xb_end(g, NV, eTop, 1) + 2 * NV * xb_levels_len(l);
    else if (band == 1)
      src = xb + xb_end(g, NV, eBot, 0) + 2 * NV * xb_levels_len(l);
    else if (band == 2)
      src = yb + yb_end(g, NV, eLeft, 1) + 2 * NV * yb_levels_len(l);
    else
      src = yb + yb_end(g, NV, eRight, 0) + 2 * NV * yb_levels_len(l);
    src += rem * len;
    if (len == 0) continue;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      f.val[j][i] = src[t < len ? t : len - 1];
      int wx, wy;
      ring_pos(h, l, band, k, t, wx, wy);
      f.dst[j][i] = t < len ? v * plane + wy * W + wx : -1;
    }
  }
}

// The ring fetch path's per-wave terms, set up once for groups of many
// waves (as StripFetchPre): a unit's HBM run at level l starts at
// base + l d1 + 2 NV l^2 (2 NV levels_len(l) + rem len(l), with
// levels_len = l^2 + 3l and len = 2l + 4 across the tile, l^2 - l and 2l
// down it), and element t goes to window index a0 + l da.
template <class S, int kThreads, int P>
struct RingFetchPre {
  static constexpr int J = Fetch<S, kThreads, P>::J;
  const typename S::V* base[J];  // a valid address even for waves without a unit
  bool has[J];                   // the wave has a unit in this slot
  int d1[J], da[J], cz[J];       // cz = len(l) - 2l
  int a0[J][P];
  int a0x[J];                    // window index at level 0 of element 64 P + lane (runs past 64 P)
};

template <class S, int kThreads, int P>
__device__ __forceinline__ void ring_fetch_init(RingFetchPre<S, kThreads, P>& r, const Geo& g,
                                                const typename S::V* __restrict__ xb,
                                                const typename S::V* __restrict__ yb, int eTop, int eBot,
                                                int eLeft, int eRight) {
  constexpr int kWaves = kThreads / 64, NV = S::NV;
  const int h = g.h, W = g.W, plane = W * W;
  // Units go to the last waves first: small levels are computed by the
  // first waves, so the fetch and placement stay off their path.
  const int w = kWaves - 1 - lwave<kThreads>();
#pragma unroll
  for (int j = 0; j < RingFetchPre<S, kThreads, P>::J; ++j) {
    const int u = w + j * kWaves;
    const int uu = u < 8 * NV ? u : 0;
    const int band = uu / (2 * NV), rem = uu - band * 2 * NV, v = rem >> 1, k = rem & 1;
    const bool horiz = band < 2;
    const typename S::V* run = band == 0   ? xb + xb_end(g, NV, eTop, 1)
                               : band == 1 ? xb + xb_end(g, NV, eBot, 0)
                               : band == 2 ? yb + yb_end(g, NV, eLeft, 1)
                                           : yb + yb_end(g, NV, eRight, 0);
    r.has[j] = u < 8 * NV;
    r.base[j] = run + (horiz ? 4 * rem : 0);
    r.d1[j] = horiz ? 6 * NV + 2 * rem : 2 * rem - 2 * NV;
    r.cz[j] = horiz ? 4 : 0;
    r.da[j] = band == 0 || band == 2 ? -(W + 1) : (band == 1 ? W - 1 : 1 - W);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      int wx, wy;
      ring_pos(h, 0, band, k, lane_id() + 64 * i, wx, wy);
      r.a0[j][i] = v * plane + wy * W + wx;
    }
    int wx, wy;
    ring_pos(h, 0, band, k, lane_id() + 64 * P, wx, wy);
    r.a0x[j] = v * plane + wy * W + wx;
  }
}

// Elements 64 P + lane of the runs of level l, which fetch_ring_pre leaves
// out: at window pitch 66 only the 66-long runs across the tile at level
// h - 1 reach past 64. Loaded once, at the start.
template <class S, int kThreads, int P>
struct RingPast {
  typename S::V val[Fetch<S, kThreads, P>::J];
  int dst[Fetch<S, kThreads, P>::J];  // -1: nothing to place
};

template <class S, int kThreads, int P>
__device__ __forceinline__ void fetch_ring_past(RingPast<S, kThreads, P>& x, const RingFetchPre<S, kThreads, P>& r,
                                                int l) {
  constexpr int NV = S::NV;
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P>::J; ++j) {
    const int len = r.has[j] ? 2 * l + r.cz[j] : 0;
    const int t = lane_id() + 64 * P;
    const typename S::V* src = r.base[j] + (l * r.d1[j] + 2 * NV * l * l);
    x.val[j] = src[t < len ? t : 0];
    x.dst[j] = t < len ? r.a0x[j] + l * r.da[j] : -1;
  }
}

// Every wave issues its loads, clamped into the panel where it has no unit
// or the run is short, so the number of loads in flight is the same on
// every path and the wait before a slot's placement counts only the loads
// issued after it.
template <class S, int kThreads, int P>
__device__ __forceinline__ void fetch_ring_pre(Fetch<S, kThreads, P>& f, const RingFetchPre<S, kThreads, P>& r,
                                               int l) {
  constexpr int NV = S::NV;
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P>::J; ++j) {
    const int len = r.has[j] ? 2 * l + r.cz[j] : 0;
    const typename S::V* src = r.base[j] + (l * r.d1[j] + 2 * NV * l * l);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      f.val[j][i] = src[t < len ? t : 0];
      f.dst[j][i] = t < len ? r.a0[j][i] + l * r.da[j] : -1;
    }
  }
}

// Ring prefetch from the staged LDS runs into registers, placed after the
// level's compute pass so the LDS read latency hides behind it. Slot j of a
// wave holds units u = (wave + j kWaves) G + lane / (64 / G), each one
// (band, slot v, row k) run with its lanes along it (P positions per lane
// when G = 1). Everything that does not depend on the level is set up once
// per lane: the window index of element t is linear in the level
// (a0 + l da, from ring_pos), and its staged offset,
// run0 + 2 NV levels_len(l) + rem len(l) + t, is a0s + l bs + 2 NV l^2
// (levels_len(l) = l^2 + 3l and len = 2l + 4 across the tile, l^2 - l and 2l
// down it). Element t exists at level l when t - (len(l) - 2l) < 2l.
template <class S, int kThreads, int P, int G>
struct RingPre {
  static constexpr int J = Fetch<S, kThreads, P, G>::J;
  int a0[J][P];
  int a0s[J][P];  // G > 1
  int c0[J][P];   // G > 1: t - (len(l) - 2l); large for lanes without a unit
  int s0[J];      // G = 1 (one unit per wave slot): a0s - t
  int cz[J];      // G = 1: len(l) - 2l; large for waves without a unit
  int da[J];
  int bs[J];
};

template <class S, int kThreads, int P, int G>
__device__ __forceinline__ void ring_pre_init(RingPre<S, kThreads, P, G>& r, const Geo& g, int LxH, int LyH) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, LG = 64 / G;
  const int h = g.h, W = g.W, plane = W * W;
  const int sub = G > 1 ? lane_id() / LG : 0, t0 = lane_id() - sub * LG;
#pragma unroll
  for (int j = 0; j < RingPre<S, kThreads, P, G>::J; ++j) {
    const int u = (lwave<kThreads>() + j * kWaves) * G + sub;
    const bool has = sub < G && u < 8 * NV;
    const int uu = has ? u : 0;
    const int band = uu / (2 * NV), rem = uu - band * 2 * NV, v = rem >> 1, k = rem & 1;
    const bool horiz = band < 2;
    const int run0 = horiz ? band * LxH : 2 * LxH + (band - 2) * LyH;
    r.da[j] = band == 0 || band == 2 ? -(W + 1) : (band == 1 ? W - 1 : 1 - W);
    r.bs[j] = horiz ? 2 * rem + 6 * NV : 2 * rem - 2 * NV;
    r.s0[j] = run0 + (horiz ? 4 * rem : 0);
    r.cz[j] = has ? (horiz ? 4 : 0) : -(1 << 28);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = t0 + 64 * i;
      int wx, wy;
      ring_pos(h, 0, band, k, t, wx, wy);
      r.a0[j][i] = v * plane + wy * W + wx;
      if constexpr (G > 1) {
        r.a0s[j][i] = r.s0[j] + t;
        r.c0[j][i] = has ? t - (horiz ? 4 : 0) : (1 << 28);
      }
    }
  }
}

template <class S, int kThreads, int P, int G>
__device__ __forceinline__ void fetch_ring_stg(Fetch<S, kThreads, P, G>& f, const RingPre<S, kThreads, P, G>& r,
                                               const typename S::V* __restrict__ stg, int l) {
  constexpr int NV = S::NV;
  const int sq = 2 * NV * l * l;
#pragma unroll
  for (int j = 0; j < RingPre<S, kThreads, P, G>::J; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      // With one unit per slot the run's terms are wave-uniform (scalar).
      const int t = lane_id() + 64 * i;
      const bool ok = G == 1 ? t < 2 * l + r.cz[j] : r.c0[j][i] < 2 * l;
      const int off = G == 1 ? r.s0[j] + l * r.bs[j] + sq + t : r.a0s[j][i] + l * r.bs[j] + sq;
      f.val[j][i] = stg[ok ? off : 0];
      f.dst[j][i] = ok ? r.a0[j][i] + l * r.da[j] : -1;
    }
}

// Ring of level l straight from the staged LDS runs into the window, all
// threads over the flattened ring (16 (l+1) NV values: per slot and row k,
// the top and bottom bands of 2l+4 and the left and right bands of 2l).
template <class S, int kThreads>
__device__ __forceinline__ void place_ring_flat(const typename S::V* __restrict__ stg, typename S::V* __restrict__ win,
                                                const Geo& g, int l, int LxH, int LyH) {
  constexpr int NV = S::NV;
  const int h = g.h, W = g.W, plane = W * W;
  const int lh = 2 * l + 4, lv = 2 * l, A = 2 * NV * lh, B = 2 * NV * lv, total = 2 * A + 2 * B;
  const float ih = 1.0f / (float)lh, iv = lv ? 1.0f / (float)lv : 0.0f;
  for (int q = ltid<kThreads>(); q < total; q += kThreads) {
    int band, r;
    if (q < 2 * A) {
      band = q < A ? 0 : 1;
      r = q - band * A;
    } else {
      band = q - 2 * A < B ? 2 : 3;
      r = q - 2 * A - (band - 2) * B;
    }
    const bool horiz = band < 2;
    int rem, t;
    fdivmod(r, horiz ? lh : lv, horiz ? ih : iv, rem, t);
    const int base =
        horiz ? band * LxH + 2 * NV * xb_levels_len(l) : 2 * LxH + (band - 2) * LyH + 2 * NV * yb_levels_len(l);
    int wx, wy;
    ring_pos(h, l, band, rem & 1, t, wx, wy);
    win[(rem >> 1) * plane + wy * W + wx] = stg[base + r];
  }
}

// Bridge strips of level l straight from the staged LDS runs, all threads
// over the flattened strips (4 (n-2l) NV values).
template <class S, int kThreads>
__device__ __forceinline__ void place_strips_flat(const typename S::V* __restrict__ stg,
                                                  typename S::V* __restrict__ win, const Geo& g, int l, int LH) {
  constexpr int NV = S::NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W, len = n - 2 * l, A = 2 * NV * len;
  const float il = 1.0f / (float)len;
  for (int q = ltid<kThreads>(); q < 2 * A; q += kThreads) {
    const int side = q < A ? 0 : 1, r = q - side * A;
    int rem, t;
    fdivmod(r, len, il, rem, t);
    win[(rem >> 1) * plane + strip_idx(W, h, l, side, rem & 1, t)] =
        stg[side * LH + 2 * NV * up_levels_len(n, l) + r];
  }
}

template <class S, int kThreads, int P, int G>
__device__ __forceinline__ void place_fetched(const Fetch<S, kThreads, P, G>& f, typename S::V* __restrict__ win) {
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P, G>::J; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (f.dst[j][i] >= 0) win[f.dst[j][i]] = f.val[j][i];
}

template <class S, int kThreads, int P>
__device__ __forceinline__ void fetch_strips(Fetch<S, kThreads, P>& f, bool isx, const Geo& g, int l,
                                             const typename S::V* __restrict__ up, int tA, int tB) {
  constexpr int kWaves = kThreads / 64;
  constexpr int NV = S::NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W, len = n - 2 * l;
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P>::J; ++j) {
    const int u = lwave<kThreads>() + j * kWaves;
#pragma unroll
    for (int i = 0; i < P; ++i) f.dst[j][i] = -1;
    if (u >= 4 * NV) continue;
    const int side = u / (2 * NV), rem = u - side * 2 * NV, v = rem >> 1, k = rem & 1;
    const int end = isx ? (side ? 2 : 3) : (side ? 0 : 1);
    const typename S::V* src = up + up_end(g, NV, side ? tB : tA, end) + 2 * NV * up_levels_len(n, l) + rem * len;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      f.val[j][i] = src[t < len ? t : len - 1];
      f.dst[j][i] = t < len ? v * plane + strip_idx(W, h, l, side, k, t) : -1;
    }
  }
}

// The fetch path's per-wave terms, set up once for groups of many waves:
// a unit's HBM run starts at base + l d1 - 2 NV l^2 (its panel offset
// 2 NV up_levels_len(n, l) + rem (n - 2l) with the level-0 part in base),
// and element t goes to window index a0 + l da.
template <class S, int kThreads, int P>
struct StripFetchPre {
  static constexpr int J = Fetch<S, kThreads, P>::J;
  const typename S::V* base[J];  // a valid address even for waves without a unit
  bool has[J];                   // the wave has a unit in this slot
  int d1[J], da[J];
  int a0[J][P];
};

template <class S, int kThreads, int P>
__device__ __forceinline__ void strip_fetch_init(StripFetchPre<S, kThreads, P>& r, bool isx, const Geo& g,
                                                 const typename S::V* __restrict__ up, int tA, int tB) {
  constexpr int kWaves = kThreads / 64, NV = S::NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W;
  // First waves first: a bridge's last waves store its panels.
#pragma unroll
  for (int j = 0; j < StripFetchPre<S, kThreads, P>::J; ++j) {
    const int u = lwave<kThreads>() + j * kWaves;
    const int uu = u < 4 * NV ? u : 0;
    const int side = uu / (2 * NV), rem = uu - side * 2 * NV, v = rem >> 1, k = rem & 1;
    const int end = isx ? (side ? 2 : 3) : (side ? 0 : 1);
    r.has[j] = u < 4 * NV;
    r.base[j] = up + up_end(g, NV, side ? tB : tA, end) + rem * n;
    r.d1[j] = 2 * NV * (n + 1) - 2 * rem;
    r.da[j] = side ? W + 1 : 1 - W;
#pragma unroll
    for (int i = 0; i < P; ++i) r.a0[j][i] = v * plane + strip_idx(W, h, 0, side, k, lane_id() + 64 * i);
  }
}

template <class S, int kThreads, int P>
__device__ __forceinline__ void fetch_strips_pre(Fetch<S, kThreads, P>& f, const StripFetchPre<S, kThreads, P>& r,
                                                 const Geo& g, int l) {
  constexpr int NV = S::NV;
#pragma unroll
  for (int j = 0; j < Fetch<S, kThreads, P>::J; ++j) {
    // Loads issued on every path, as in fetch_ring_pre.
    const int len = r.has[j] ? g.n - 2 * l : 0;
    const typename S::V* src = r.base[j] + (l * r.d1[j] - 2 * NV * l * l);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      f.val[j][i] = src[t < len ? t : 0];
      f.dst[j][i] = t < len ? r.a0[j][i] + l * r.da[j] : -1;
    }
  }
}

// Strip prefetch from the staged LDS runs (as RingPre): unit u = (side,
// slot v, row k); the window index of element t is linear in the level
// (from strip_idx), its staged offset
// run0 + 2 NV up_levels_len(n, l) + rem (n - 2l) + t, with
// up_levels_len(n, l) = l (n + 1 - l), is a0s + l bs - 2 NV l^2, and it
// exists at level l when 2l < n - t.
template <class S, int kThreads, int P, int G>
struct StripPre {
  static constexpr int J = Fetch<S, kThreads, P, G>::J;
  int a0[J][P];
  int a0s[J][P];  // G > 1
  int lim[J][P];  // G > 1: n - t; negative for lanes without a unit
  int s0[J];      // G = 1 (one unit per wave slot): a0s - t
  int lz[J];      // G = 1: n; negative for waves without a unit
  int da[J];
  int bs[J];
};

template <class S, int kThreads, int P, int G>
__device__ __forceinline__ void strip_pre_init(StripPre<S, kThreads, P, G>& r, const Geo& g, int LH) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, LG = 64 / G;
  const int n = g.n, h = g.h, W = g.W, plane = W * W;
  const int sub = G > 1 ? lane_id() / LG : 0, t0 = lane_id() - sub * LG;
#pragma unroll
  for (int j = 0; j < StripPre<S, kThreads, P, G>::J; ++j) {
    const int u = (lwave<kThreads>() + j * kWaves) * G + sub;
    const bool has = sub < G && u < 4 * NV;
    const int uu = has ? u : 0;
    const int side = uu / (2 * NV), rem = uu - side * 2 * NV, v = rem >> 1, k = rem & 1;
    r.da[j] = side ? W + 1 : 1 - W;
    r.bs[j] = 2 * NV * (n + 1) - 2 * rem;
    r.s0[j] = side * LH + rem * n;
    r.lz[j] = has ? n : -(1 << 28);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = t0 + 64 * i;
      r.a0[j][i] = v * plane + strip_idx(W, h, 0, side, k, t);
      if constexpr (G > 1) {
        r.a0s[j][i] = r.s0[j] + t;
        r.lim[j][i] = has ? n - t : -1;
      }
    }
  }
}

template <class S, int kThreads, int P, int G>
__device__ __forceinline__ void fetch_strips_stg(Fetch<S, kThreads, P, G>& f, const StripPre<S, kThreads, P, G>& r,
                                                 const typename S::V* __restrict__ stg, int l) {
  constexpr int NV = S::NV;
  const int sq = 2 * NV * l * l;
#pragma unroll
  for (int j = 0; j < StripPre<S, kThreads, P, G>::J; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      const bool ok = G == 1 ? t < r.lz[j] - 2 * l : 2 * l < r.lim[j][i];
      const int off = G == 1 ? r.s0[j] + l * r.bs[j] - sq + t : r.a0s[j][i] + l * r.bs[j] - sq;
      f.val[j][i] = stg[ok ? off : 0];
      f.dst[j][i] = ok ? r.a0[j][i] + l * r.da[j] : -1;
    }
}

// Bridge panels of level l (Alg. 2-3), read from the buffer where level l's
// band survives (as up_strips_read). x-bridge: rows y = l+1+k (N end) and
// n-l-k (S end), x = h-l-1 .. h+l+2 (the band and the pyramid corners
// placed beside it), which in its transposed window are columns. y-bridge:
// columns x = l+1+k (W end) and n-l-k (E end), rows y = h+1-l .. h+l. Both
// are window columns read down the rows. Per wave unit, set up once: the
// panel offset 2 NV levels_len(l) + rem len(l) is d0 + l d1 + 2 NV l^2
// (levels_len = l^2 + 3l, len = 2l + 4 for the x-bridge; l^2 - l and 2l for
// the y-bridge) and the window start s0 + l ds.
template <class S, int kThreads>
struct BridgeEmitPre {
  static constexpr int J = EmitSlot<S, kThreads, 1, 4 * S::NV>::J;
  typename S::V* base[J];  // panel of the unit's end and slot row, null: no unit
  int d1[J], s0[J], ds[J];
};

template <class S, int kThreads>
__device__ __forceinline__ void bridge_emit_init(BridgeEmitPre<S, kThreads>& r, typename S::V* __restrict__ out,
                                                 bool isx, const Geo& g, int e) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, per = 4 * NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W;
  const int w = kWaves - 1 - lwave<kThreads>();
#pragma unroll
  for (int j = 0; j < BridgeEmitPre<S, kThreads>::J; ++j) {
    const int u = w + j * kWaves;
    const int uu = u < per ? u : 0;
    const int end = uu / (2 * NV), rem = uu - end * 2 * NV, v = rem >> 1, k = rem & 1;
    r.base[j] = u < per ? out + (isx ? xb_end(g, NV, e, end) + 4 * rem : yb_end(g, NV, e, end)) : nullptr;
    r.d1[j] = isx ? 6 * NV + 2 * rem : 2 * rem - 2 * NV;
    r.s0[j] = v * plane + (isx ? h - 1 : h + 1) * W + (end ? n - k : 1 + k);
    r.ds[j] = end ? -W - 1 : 1 - W;
  }
}

template <class S, int kThreads, int P>
__device__ __forceinline__ void bridge_ends_read(EmitSlot<S, kThreads, P, 4 * S::NV>& es,
                                                 const BridgeEmitPre<S, kThreads>& r,
                                                 const typename S::V* __restrict__ win, bool isx, const Geo& g,
                                                 int l) {
  constexpr int NV = S::NV;
  const int W = g.W, len = isx ? 2 * l + 4 : 2 * l;
#pragma unroll
  for (int j = 0; j < EmitSlot<S, kThreads, P, 4 * NV>::J; ++j) {
    es.len[j] = 0;
    if (r.base[j] == nullptr || len == 0) continue;
    es.len[j] = len;
    es.dst[j] = r.base[j] + (l * r.d1[j] + 2 * NV * l * l);
    const typename S::V* src = win + r.s0[j] + l * r.ds[j];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      es.val[j][i] = src[(t < len ? t : 0) * W];
    }
  }
}

// The same panels with every term worked out at each level (as
// up_strips_read_direct).
template <class S, int kThreads, int P>
__device__ __forceinline__ void bridge_ends_read_direct(EmitSlot<S, kThreads, P, 4 * S::NV>& es,
                                                 const typename S::V* __restrict__ win,
                                                 typename S::V* __restrict__ out, bool isx, const Geo& g, int e,
                                                 int l) {
  constexpr int kWaves = kThreads / 64, NV = S::NV, per = 4 * NV;
  const int n = g.n, h = g.h, W = g.W, plane = W * W;
  const int len = isx ? 2 * l + 4 : 2 * l;
  const int w = kWaves - 1 - lwave<kThreads>();
#pragma unroll
  for (int j = 0; j < EmitSlot<S, kThreads, P, per>::J; ++j) {
    const int u = w + j * kWaves;
    es.len[j] = 0;
    if (u >= per || len == 0) continue;
    const int end = u / (2 * NV), rem = u - end * 2 * NV, v = rem >> 1, k = rem & 1;
    es.len[j] = len;
    es.dst[j] = out +
                (isx ? xb_end(g, NV, e, end) + 2 * NV * xb_levels_len(l)
                     : yb_end(g, NV, e, end) + 2 * NV * yb_levels_len(l)) +
                (size_t)rem * len;
    const int across = end ? (n - l - k) : (l + 1 + k);
    const typename S::V* src = win + v * plane + (isx ? h - l - 1 : h + 1 - l) * W + across;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int t = lane_id() + 64 * i;
      es.val[j][i] = src[(t < len ? t : 0) * W];
    }
  }
}

// Window-only values (NW > NV) start at zero in both buffers: a point's
// value that arrives from the state or a panel comes without them, and a
// point computed in this window overwrites them level by level. (A value
// placed at level l never sits where this window computed an earlier level
// of the same parity.) The caller's first barrier orders this before any
// read.
template <class S, int NT>
__device__ __forceinline__ void clear_window_only(typename S::V* buf0, typename S::V* buf1, int W) {
  if constexpr (S::NW > S::NV) {
    const int cnt = (S::NW - S::NV) * W * W;
    typename S::V* a = buf0 + S::NV * W * W;
    typename S::V* b = buf1 + S::NV * W * W;
    for (int q = ltid<NT>(); q < cnt; q += NT) {
      a[q] = 0;
      b[q] = 0;
    }
  }
}

// ----------------------------------------------------------------- kernels

// Stage items. Each runs on one workgroup of NT threads with `smem` as its
// LDS; a stage kernel runs item blockIdx.x, the batched persistent kernel
// the items it takes from its queue.

// Upward pyramid of one tile, from the state (Alg. 1).
template <class S, int WC, int NT>
__device__ void up_item(const Geo& g, int H, typename S::V* __restrict__ state, const PanelPtrs& pp,
                        const SchemeParams& sp, int tile, double* smem) {
  using V = typename S::V;
  V* buf0 = reinterpret_cast<V*>(smem);
  V* buf1 = buf0 + S::NW * g.W * g.W;
  clear_window_only<S, NT>(buf0, buf1, g.W);  // ordered by the barrier after the gather
  const int a = tile % g.ntx, b = tile / g.ntx;
  const int x0 = g.off + a * g.n, y0 = g.off + b * g.n;
  const int n = g.n, W = g.W, plane = W * W;
  const size_t gplane = (size_t)g.nx * g.ny;
  const float invn = 1.0f / (float)n;
  gather<NT, V>(
      S::NV * n * n,
      [&](int q) -> V {
        int vr, c, v, r;
        fdivmod(q, n, invn, vr, c);
        fdivmod(vr, n, invn, v, r);
        return state[v * gplane + (size_t)wrap(y0 + r, g.ny) * g.nx + wrap(x0 + c, g.nx)];
      },
      [&](int q, V val) {
        int vr, c, v, r;
        fdivmod(q, n, invn, vr, c);
        fdivmod(vr, n, invn, v, r);
        buf0[v * plane + (r + 1) * W + (c + 1)] = val;
      });
  __syncthreads();
  up_levels<S, WC, NT>(buf0, buf1, 0, g, tile, x0, y0, level_base(g), H, state, static_cast<V*>(pp.up), sp);
}

// The bridge between tiles A = e and B = tB across A's east edge (isx, the
// x-bridge, Alg. 3) or south edge (the y-bridge, Alg. 2), both in the
// y-bridge's window layout (the x-bridge's window transposed): at level l the
// rectangle of window columns l+1 .. n-l and rows h+1-l .. h+l. Runs on a
// group of NT threads with `smem` as its LDS; the level loop (and its
// barriers) is the same for both directions, so two groups of one
// workgroup may run an x- and a y-bridge side by side.
template <class S, int WC, int NT, bool STAGED>
__device__ __forceinline__ void bridge_body(const Geo& g, int H, bool isx,
                                            typename S::V* __restrict__ state, const PanelPtrs& pp,
                                            const SchemeParams& sp, int e, int tB, int xw0, int yw0, double* smem) {
  using V = typename S::V;
  constexpr int NV = S::NV;
  V* buf0 = reinterpret_cast<V*>(smem);
  V* buf1 = buf0 + S::NW * g.W * g.W;
  V* stg = buf1 + S::NW * g.W * g.W;
  clear_window_only<S, NT>(buf0, buf1, g.W);  // ordered by the barrier after level 0 is placed
  const int n = g.n, h = g.h;
  const V* up = static_cast<const V*>(pp.up);
  V* out = static_cast<V*>(isx ? pp.xb : pp.yb);
  const long long T0 = level_base(g);
  const int LH = 2 * NV * up_levels_len(n, H);
  // One-wave groups always stage (their panels are a few KB), which keeps
  // the per-level fetch registers out of them. Staging is a compile-time
  // choice: with one fetch path per kernel the prefetched values are not
  // merged between paths, and their loads are waited for only where placed.
  static_assert(STAGED || NT != 64, "one-wave groups stage");
  constexpr bool staged = STAGED;
  // Strips are at most n long: one position per lane up to n = 64, and
  // when staged 64 / n runs side by side in one slot for n <= 32.
  constexpr int kP = (WC != 0 && WC <= 66) ? 1 : 2;
  constexpr int kG = (staged && WC != 0 && WC - 2 <= 32) ? 64 / (WC - 2) : 1;
  using F = Fetch<S, NT, kP, kG>;
  constexpr bool prefetch = F::J * kP <= 16;
  // Level l's pass also emits the panels of level l-1; they are at most
  // n + 2 long (the x-bridge's), one position per lane up to n = 62.
  constexpr int kPe = (WC != 0 && WC <= 64) ? 1 : 2;
  constexpr bool kPre = BridgeEmitPre<S, NT>::J <= 2;  // as in up_levels
  constexpr bool kPack = !kPre && WC != 0 && WC <= 32;   // 64 / (n + 2) runs per wave slot
  constexpr int kGb = kPack ? 64 / (WC ? WC : 1) : 1;
  using PK = PackPre<S, NT, kGb, 4 * NV>;
  using E = std::conditional_t<kPack, EmitLanes<S, PK::J>, EmitSlot<S, NT, kPe, 4 * NV>>;
  [[maybe_unused]] BridgeEmitPre<S, NT> ep;
  [[maybe_unused]] PK pk;
  if constexpr (kPre) bridge_emit_init<S, NT>(ep, out, isx, g, e);
  if constexpr (kPack) bridge_pack_init<S, NT, kGb>(pk, out, isx, g, e);
  auto ends_read = [&](E& es, const V* win, int l) {
    if constexpr (kPre)
      bridge_ends_read<S, NT, kPe>(es, ep, win, isx, g, l);
    else if constexpr (kPack)
      bridge_pack_read<S, NT, kGb>(es, pk, win, l);
    else
      bridge_ends_read_direct<S, NT, kPe>(es, win, out, isx, g, e, l);
  };
  if constexpr (staged) {
    const V* sA = up + up_end(g, NV, e, isx ? 3 : 1);
    const V* sB = up + up_end(g, NV, tB, isx ? 2 : 0);
    // Runs of at most 2 NV up_levels_len(n, h) values.
    constexpr int kH = (WC - 2) / 2;
    constexpr int kC = stage_fixed_count<V, NT>(WC ? 2 * NV * kH * (WC - 2 - kH + 1) : 0, 2);
    if constexpr (kC > 0)
      stage_runs_fixed<NT, kC, 2, V>(stg, sA, LH, sB, LH, sA, 0, sA, 0);
    else
      stage_runs<NT, V>(stg, sA, LH, sB, LH, sA, 0, sA, 0);
    __syncthreads();
  }
  StripPre<S, NT, kP, kG> pre;
  if constexpr (staged && prefetch) strip_pre_init<S, NT, kP, kG>(pre, g, LH);
  // Level l: place the strips of level l, after computing the band of level l
  // (1 <= l <= h-1) from level l-1. The first level only places, the last (H)
  // only computes (a full half cycle has no level h in a bridge); they are
  // peeled off so the loop body tests nothing per level. H >= 1.
  // The fetch path keeps each wave's run terms precomputed when a wave has
  // at most two units.
  constexpr bool kFetchPre = !staged && F::J <= 2;
  [[maybe_unused]] StripFetchPre<S, NT, kP> fpre;
  if constexpr (kFetchPre) strip_fetch_init<S, NT, kP>(fpre, isx, g, up, e, tB);
  auto strips_fetch = [&](F& f, int l) {
    if constexpr (staged) {
      if constexpr (prefetch) fetch_strips_stg<S, NT, kP, kG>(f, pre, stg, l);
    } else if constexpr (kFetchPre) {
      fetch_strips_pre<S, NT, kP>(f, fpre, g, l);
    } else {
      fetch_strips<S, NT, kP>(f, isx, g, l, up, e, tB);
    }
  };
  auto strips_place = [&](const F& f, V* cur, int l) {
    if constexpr (staged && !prefetch)
      place_strips_flat<S, NT>(stg, cur, g, l, LH);
    else
      place_fetched(f, cur);
  };
  // The x-bridge's window is transposed; a scheme whose step is symmetric in
  // x and y reads it with the plain accessor, so both directions share one
  // compute path.
  auto band = [&](const V* prv, V* cur, int l) {
    if (S::XY_SYM || !isx)
      compute_level<S, WC, NT, false>(prv, cur, g.W, l + 1, h + 1 - l, n - 2 * l, 2 * l, T0 + l - 1, sp);
    else
      compute_level<S, WC, NT, true>(prv, cur, g.W, l + 1, h + 1 - l, n - 2 * l, 2 * l, T0 + l - 1, sp);
  };
  if constexpr (staged) {
    {
      // Declared per level: the prefetched values are not carried round the
      // loop.
      F f;
      strips_fetch(f, 0);
      strips_place(f, buf0, 0);
      __syncthreads();
    }
    for (int l = 1; l < H; ++l) {
      F f;
      E es;
      V* cur = (l & 1) ? buf1 : buf0;
      const V* prv = (l & 1) ? buf0 : buf1;
      if constexpr (emit_early<S>()) ends_read(es, prv, l - 1);
      strips_fetch(f, l);
      band(prv, cur, l);
      strips_place(f, cur, l);
      if constexpr (!emit_early<S>()) ends_read(es, prv, l - 1);
      emit_write(es);
      __syncthreads();
    }
  } else {
    // From HBM, each level's strips are fetched kAhead levels before they
    // are placed, so their loads have kAhead band passes to arrive: slot
    // l mod kAhead holds level l, refilled with level l + kAhead once level
    // l is placed. The loop is unrolled by kAhead so that every slot is a
    // fixed set of registers. Lookahead is kept to a few registers per slot.
    constexpr int kAhead = F::J * kP * (int)sizeof(V) <= 32 ? 3 : 1;
    F f[kAhead];
#pragma unroll
    for (int i = 0; i < kAhead; ++i)
      strips_fetch(f[i], opaque_level(i < H ? i : H - 1));
    strips_place(f[0], buf0, 0);
    strips_fetch(f[0], opaque_level(kAhead < H ? kAhead : H - 1));
    __syncthreads();
    // Each level's band is planned before the barrier that precedes it.
    auto plan = [&](int l) { return level_plan<S, WC, NT>(l + 1, h + 1 - l, n - 2 * l, 2 * l); };
    auto pl = plan(1);
    auto level = [&](F& fl, int l, bool refill) {
      E es;
      V* cur = (l & 1) ? buf1 : buf0;
      const V* prv = (l & 1) ? buf0 : buf1;
      if constexpr (emit_early<S>()) ends_read(es, prv, l - 1);
      if (S::XY_SYM || !isx)
        level_run<S, WC, NT, false>(prv, cur, g.W, pl, T0 + l - 1, sp);
      else
        level_run<S, WC, NT, true>(prv, cur, g.W, pl, T0 + l - 1, sp);
      strips_place(fl, cur, l);
      if (refill) strips_fetch(fl, l + kAhead);
      if constexpr (!emit_early<S>()) ends_read(es, prv, l - 1);
      emit_write(es);
      pl = plan(l + 1);
      __syncthreads();
    };
    // Unconditional refills in whole blocks, then the last levels with tests
    // (as in the octahedron's fetch loop).
    int l0 = 1;  // level l0 + i is held in slot (1 + i) mod kAhead
    for (; l0 + 2 * kAhead - 1 < H; l0 += kAhead) {
#pragma unroll
      for (int i = 0; i < kAhead; ++i) level(f[(1 + i) % kAhead], l0 + i, true);
    }
    for (; l0 < H; l0 += kAhead) {
#pragma unroll
      for (int i = 0; i < kAhead; ++i)
        if (l0 + i < H) level(f[(1 + i) % kAhead], l0 + i, l0 + i + kAhead < H);
    }
  }
  {
    // The last emitted level, H - 1, beside the band of level H when H < h.
    E es;
    ends_read(es, (H & 1) ? buf0 : buf1, H - 1);
    if (H < h) band((H & 1) ? buf0 : buf1, (H & 1) ? buf1 : buf0, H);
    emit_write(es);
  }
  __syncthreads();
  if (H < h) {
    const V* fin = (H & 1) ? buf1 : buf0;
    if (isx)
      write_rect<S, NT, true>(fin, state, g, xw0, yw0, h + 1 - H, H + 1, 2 * H, n - 2 * H);
    else
      write_rect<S, NT>(fin, state, g, xw0, yw0, H + 1, h + 1 - H, n - 2 * H, 2 * H);
  }
}

// Window origin and the far tile of the bridge over the east (isx) or south
// edge of tile e.
__device__ __forceinline__ void bridge_frame(const Geo& g, bool isx, int e, int& tB, int& xw0, int& yw0) {
  const int a = e % g.ntx, b = e / g.ntx;
  const int n = g.n, h = g.h;
  if (isx) {
    xw0 = g.off + (a + 1) * n - h - 1;
    yw0 = g.off + b * n - 1;
    tB = b * g.ntx + (a + 1 == g.ntx ? 0 : a + 1);
  } else {
    xw0 = g.off + a * n - 1;
    yw0 = g.off + (b + 1) * n - h - 1;
    tB = (b + 1 == g.nty ? 0 : b + 1) * g.ntx + a;
  }
}

// Item i < ntiles: the x-bridge over the east edge of tile i; item
// ntiles + i: the y-bridge over the south edge of tile i (Alg. 2-3).
template <class S, int WC, int NT, bool STAGED>
__device__ void bridge_item(const Geo& g, int H, typename S::V* __restrict__ state, const PanelPtrs& pp,
                            const SchemeParams& sp, int item, double* smem) {
  const int ntiles = g.ntx * g.nty;
  const bool isx = item < ntiles;
  const int e = isx ? item : item - ntiles;
  int tB, xw0, yw0;
  bridge_frame(g, isx, e, tB, xw0, yw0);
  bridge_body<S, WC, NT, STAGED>(g, H, isx, state, pp, sp, e, tB, xw0, yw0, smem);
}

// LDS values (doubles) of one bridge group: two windows and, when staged,
// the two facing strips of all levels.
template <class S>
__host__ __device__ inline size_t bridge_group_doubles(int n, bool staged) {
  const size_t win = 2 * (size_t)(n + 2) * (size_t)(n + 2) * S::NW;
  const size_t stg = staged ? (size_t)2 * 2 * S::NV * (size_t)up_levels_len(n, n / 2) : 0;
  return ((win + stg) * sizeof(typename S::V) + 7) / 8;
}

// Both bridges of tile e in one workgroup of 2 NTI threads: threads
// 0 .. NTI-1 run the x-bridge, NTI .. 2 NTI-1 the y-bridge, each with its own
// LDS. The two run the same level loop under the workgroup's barriers, so the
// bridge stage takes one round of workgroups instead of two.
template <class S, int WC, int NTI, bool STAGED>
__device__ void bridge_pair_item(const Geo& g, int H, typename S::V* __restrict__ state, const PanelPtrs& pp,
                                 const SchemeParams& sp, int e, double* smem) {
  const bool isx = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / NTI)) == 0;
  int tB, xw0, yw0;
  bridge_frame(g, isx, e, tB, xw0, yw0);
  double* mine = smem + (isx ? 0 : bridge_group_doubles<S>(g.n, STAGED));
  bridge_body<S, WC, NTI, STAGED>(g, H, isx, state, pp, sp, e, tB, xw0, yw0, mine);
}

// Downward pyramid at the south-east corner of tile c (Alg. 4), fused with
// the next half cycle's upward pyramid of the tile centred on that corner
// (an octahedron): the level-h tile never leaves LDS.
template <class S, int WC, int NT, bool STAGED>
__device__ void oct_item(const Geo& g, int Hd, int Hu, typename S::V* __restrict__ state, const PanelPtrs& pp,
                         const SchemeParams& sp, int c, double* smem) {
  using V = typename S::V;
  constexpr int NV = S::NV;
  V* buf0 = reinterpret_cast<V*>(smem);
  V* buf1 = buf0 + S::NW * g.W * g.W;
  V* stg = buf1 + S::NW * g.W * g.W;
  clear_window_only<S, NT>(buf0, buf1, g.W);  // ordered by the barrier after level 0 is placed
  const int a = c % g.ntx, b = c / g.ntx;
  const int n = g.n, h = g.h;
  const int a1 = (a + 1 == g.ntx) ? 0 : a + 1, b1 = (b + 1 == g.nty) ? 0 : b + 1;
  const int eTop = c, eBot = b1 * g.ntx + a, eLeft = c, eRight = b * g.ntx + a1;
  const int xw0 = g.off + (a + 1) * n - h - 1, yw0 = g.off + (b + 1) * n - h - 1;
  const V* xb = static_cast<const V*>(pp.xb);
  const V* yb = static_cast<const V*>(pp.yb);
  V* up = static_cast<V*>(pp.up);
  const long long T0 = level_base(g);
  const int LxH = 2 * NV * xb_levels_len(Hd), LyH = 2 * NV * yb_levels_len(Hd);
  // The tile centred on this corner is tile (a, b) of the tiling shifted by h
  // (tile (a+1, b+1) of the unshifted one when the shift wraps to 0).
  Geo g2 = g;
  g2.off = g.off + h;
  int a2 = a, b2 = b;
  if (g2.off == n) {
    g2.off = 0;
    a2 = a1;
    b2 = b1;
  }
  const int tile2 = b2 * g.ntx + a2;
  static_assert(STAGED || NT != 64, "one-wave groups stage");  // as in the bridges
  constexpr bool staged = STAGED;
  // Ring runs are at most n + 2 long: at window pitches up to 64 they take
  // one position per lane, and up to 32, 64 / (n + 2) of them lie side by
  // side in one staged slot. The fetch path with per-wave terms (a wave
  // holds at most two of the 8 NV units) takes one position per lane at
  // pitch 66 as well and places the two elements past 64 of its last level's
  // runs across the tile from values loaded at its start (kPast).
  constexpr int kWavesO = NT / 64;
  constexpr bool kPast = !staged && WC == 66 && (8 * NV + kWavesO - 1) / kWavesO <= 2;
  constexpr int kP = (kPast || (WC != 0 && WC <= 64)) ? 1 : 2;
  constexpr int kG = (staged && WC != 0 && WC <= 32) ? 64 / (WC ? WC : 1) : 1;
  using F = Fetch<S, NT, kP, kG>;
  constexpr bool prefetch = F::J * kP <= 16;
  if constexpr (staged) {
    // Runs of at most 2 NV xb_levels_len(h) values (the x-bridges'; the
    // y-bridges' are shorter).
    constexpr int kH = (WC - 2) / 2;
    constexpr int kC = stage_fixed_count<V, NT>(WC ? 2 * NV * kH * (kH + 3) : 0, 4);
    if constexpr (kC > 0)
      stage_runs_fixed<NT, kC, 4, V>(stg, xb + xb_end(g, NV, eTop, 1), LxH, xb + xb_end(g, NV, eBot, 0), LxH,
                                     yb + yb_end(g, NV, eLeft, 1), LyH, yb + yb_end(g, NV, eRight, 0), LyH);
    else
      stage_runs<NT, V>(stg, xb + xb_end(g, NV, eTop, 1), LxH, xb + xb_end(g, NV, eBot, 0), LxH,
                        yb + yb_end(g, NV, eLeft, 1), LyH, yb + yb_end(g, NV, eRight, 0), LyH);
    __syncthreads();
  }
  RingPre<S, NT, kP, kG> pre;
  if constexpr (staged && prefetch) ring_pre_init<S, NT, kP, kG>(pre, g, LxH, LyH);
  // Level l: place the ring of level l, after computing the square of level l
  // (l >= 1) from level l-1. The first level only places, the last (Hd) only
  // computes; they are peeled off so the loop body tests nothing per level.
  auto ring_fetch = [&](F& f, int l) {
    if constexpr (staged) {
      if constexpr (prefetch) fetch_ring_stg<S, NT, kP, kG>(f, pre, stg, l);
    } else {
      fetch_ring<S, NT, kP>(f, g, l, xb, yb, eTop, eBot, eLeft, eRight);
    }
  };
  auto ring_place = [&](const F& f, V* cur, int l) {
    if constexpr (staged && !prefetch)
      place_ring_flat<S, NT>(stg, cur, g, l, LxH, LyH);
    else
      place_fetched(f, cur);
  };
  // From HBM with few units per wave, each level's ring is fetched kAhead
  // levels before it is placed (slots as in the bridges).
  constexpr bool kFetchPre = !staged && F::J <= 2;
  if constexpr (kFetchPre) {
    constexpr int kAhead = F::J * kP * (int)sizeof(V) <= 32 ? 3 : 1;
    RingFetchPre<S, NT, kP> fpre;
    ring_fetch_init<S, NT, kP>(fpre, g, xb, yb, eTop, eBot, eLeft, eRight);
    [[maybe_unused]] RingPast<S, NT, kP> past;
    if constexpr (kPast) fetch_ring_past<S, NT, kP>(past, fpre, h - 1);
    F f[kAhead];
    if (Hd > 0) {
#pragma unroll
      for (int i = 0; i < kAhead; ++i)
        fetch_ring_pre<S, NT, kP>(f[i], fpre, opaque_level(i < Hd ? i : Hd - 1));
      place_fetched(f[0], buf0);
      fetch_ring_pre<S, NT, kP>(f[0], fpre, opaque_level(kAhead < Hd ? kAhead : Hd - 1));
      __syncthreads();
    }
    // Each level's square is planned before the barrier that precedes it.
    auto plan = [&](int l) { return level_plan<S, WC, NT>(h + 1 - l, h + 1 - l, 2 * l, 2 * l); };
    auto pl = plan(1);
    auto level = [&](F& fl, int l, bool refill) {
      V* cur = (l & 1) ? buf1 : buf0;
      const V* prv = (l & 1) ? buf0 : buf1;
      level_run<S, WC, NT>(prv, cur, g.W, pl, T0 + l - 1, sp);
      place_fetched(fl, cur);
      if constexpr (kPast) {
        if (l == h - 1) {
#pragma unroll
          for (int j = 0; j < F::J; ++j)
            if (past.dst[j] >= 0) cur[past.dst[j]] = past.val[j];
        }
      }
      if (refill) fetch_ring_pre<S, NT, kP>(fl, fpre, l + kAhead);
      pl = plan(l + 1);
      __syncthreads();
    };
    // Blocks whose every level refills its slot issue their loads
    // unconditionally, so the wait before a slot's placement counts only the
    // loads of the later slots (a refill that might be skipped would make the
    // compiler wait for all of them); the last levels follow with tests.
    int l0 = 1;  // level l0 + i is held in slot (1 + i) mod kAhead
    for (; l0 + 2 * kAhead - 1 < Hd; l0 += kAhead) {
#pragma unroll
      for (int i = 0; i < kAhead; ++i) level(f[(1 + i) % kAhead], l0 + i, true);
    }
    for (; l0 < Hd; l0 += kAhead) {
#pragma unroll
      for (int i = 0; i < kAhead; ++i)
        if (l0 + i < Hd) level(f[(1 + i) % kAhead], l0 + i, l0 + i + kAhead < Hd);
    }
  } else {
    if (Hd > 0) {
      F f;
      ring_fetch(f, 0);
      ring_place(f, buf0, 0);
      __syncthreads();
    }
    for (int l = 1; l < Hd; ++l) {
      F f;  // per level, as in the bridges
      V* cur = (l & 1) ? buf1 : buf0;
      const V* prv = (l & 1) ? buf0 : buf1;
      ring_fetch(f, l);
      compute_level<S, WC, NT>(prv, cur, g.W, h + 1 - l, h + 1 - l, 2 * l, 2 * l, T0 + l - 1, sp);
      ring_place(f, cur, l);
      __syncthreads();
    }
  }
  if (Hd > 0) {
    V* cur = (Hd & 1) ? buf1 : buf0;
    const V* prv = (Hd & 1) ? buf0 : buf1;
    if (Hd < h)
      compute_level<S, WC, NT>(prv, cur, g.W, h + 1 - Hd, h + 1 - Hd, 2 * Hd, 2 * Hd, T0 + Hd - 1, sp);
    else
      compute_level<S, WC, NT, false, true>(prv, cur, g.W, 1, 1, n, n, T0 + Hd - 1, sp);
    __syncthreads();
  }
  const V* top = (Hd & 1) ? buf1 : buf0;
  if (Hd < h) {
    write_rect<S, NT>(top, state, g, xw0, yw0, h + 1 - Hd, h + 1 - Hd, 2 * Hd, 2 * Hd);
    return;
  }
  if (Hu == 0) {
    write_rect<S, NT>(top, state, g, xw0, yw0, 1, 1, n, n);
    return;
  }
  up_levels<S, WC, NT>(buf0, buf1, h & 1, g2, tile2, xw0 + 1, yw0 + 1, T0 + h, Hu, state, up, sp);
}

template <class S, int WC, int NT>
__global__ __launch_bounds__(NT) void k_up(Geo g, int H, typename S::V* __restrict__ state, PanelPtrs pp,
                                           SchemeParams sp) {
  extern __shared__ double smem_d[];
  up_item<S, WC, NT>(g, H, state, pp, sp, (int)blockIdx.x, smem_d);
}

template <class S, int WC, int NT, bool STAGED>
__global__ __launch_bounds__(NT) void k_bridge(Geo g, int H, typename S::V* __restrict__ state, PanelPtrs pp,
                                               SchemeParams sp) {
  extern __shared__ double smem_d[];
  bridge_item<S, WC, NT, STAGED>(g, H, state, pp, sp, (int)blockIdx.x, smem_d);
}

template <class S, int WC, int NTI, bool STAGED>
__global__ __launch_bounds__(2 * NTI) void k_bridge_pair(Geo g, int H, typename S::V* __restrict__ state, PanelPtrs pp,
                                                         SchemeParams sp) {
  extern __shared__ double smem_d[];
  bridge_pair_item<S, WC, NTI, STAGED>(g, H, state, pp, sp, (int)blockIdx.x, smem_d);
}

template <class S, int WC, int NT, bool STAGED>
__global__ __launch_bounds__(NT) void k_oct(Geo g, int Hd, int Hu, typename S::V* __restrict__ state, PanelPtrs pp,
                                            SchemeParams sp) {
  extern __shared__ double smem_d[];
  oct_item<S, WC, NT, STAGED>(g, Hd, Hu, state, pp, sp, (int)blockIdx.x, smem_d);
}

template <class S>
constexpr int plain_rows() {
  return S::NV >= 8 ? 2 : 8;
}

// Neighbour access for the per-step kernel below: rw[row][column][v] with
// CW register columns; the point sits at column c + 1 of row 1.
template <class V, int NWv, int CW>
struct ColsNb {
  const V (*rw)[CW][NWv];
  int c;
  __device__ __forceinline__ V operator()(int di, int dj, int v) const { return rw[dj + 1][c + di + 1][v]; }
};

// Per-step kernel of the light schemes (at most 16 bytes per point in the
// window). A thread computes C adjacent columns (C = 2 on grids of even
// width: one 2-value load and store per row and value) of PR rows, with all
// PR + 2 input rows loaded before the first update, so every load of a
// thread is in flight at once; 128 threads cover 128 C columns. Workgroups
// are dealt round robin to the 8 XCDs in workgroup order, so the blocks are
// renumbered to give each XCD a contiguous band of rows: the rows two
// vertically adjacent blocks both read then meet in one XCD's L2.
constexpr int kPlainRows = 4;
constexpr int kXcds = 8;
template <class S, int C>
__global__ __launch_bounds__(128) void k_plain_cols(const typename S::V* __restrict__ in,
                                                    typename S::V* __restrict__ out, int nx, int ny, long long Trel,
                                                    const long long* tbase, SchemeParams sp) {
  using V = typename S::V;
  constexpr int NV = S::NV, NW = S::NW, PR = kPlainRows, CW = C + 2;
  const long long T = Trel + (tbase ? *tbase : 0LL);
  const int nbx = (nx + 128 * C - 1) / (128 * C);
  const int nb = nbx * ((ny + PR - 1) / PR);
  const int per = (nb + kXcds - 1) / kXcds;
  const int L = (int)blockIdx.x;
  const int t = (L % kXcds) * per + L / kXcds;
  if (t >= nb) return;
  const int bx = t % nbx, by = t / nbx;
  const int x = (bx * 128 + (int)threadIdx.x) * C;
  if (x >= nx) return;
  const int ys = by * PR;
  const int xw = x == 0 ? nx - 1 : x - 1;
  const int xe = x + C == nx ? 0 : x + C;
  const size_t plane = (size_t)nx * ny;
  // window-only values of the scheme are zero: every sub-step is a launch of
  // its own, so none survives one
  V rw[PR + 2][CW][NW] = {};
#pragma unroll
  for (int k = 0; k < PR + 2; ++k) {
    const int y = ((ys + k - 1) % ny + ny) % ny;
    const V* row = in + (size_t)y * nx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (C == 2) {
        using V2 = HIP_vector_type<V, 2>;
        const V2 m = *reinterpret_cast<const V2*>(row + v * plane + x);
        rw[k][1][v] = m.x;
        rw[k][2][v] = m.y;
      } else {
        rw[k][1][v] = row[v * plane + x];
      }
      rw[k][0][v] = row[v * plane + xw];
      rw[k][CW - 1][v] = row[v * plane + xe];
    }
  }
#pragma unroll
  for (int k = 0; k < PR; ++k) {
    if (ys + k >= ny) break;
    V o[C][NW];
#pragma unroll
    for (int c = 0; c < C; ++c) S::step(T, ColsNb<V, NW, CW>{&rw[k], c}, o[c], sp);
    V* dst = out + (size_t)(ys + k) * nx + x;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (C == 2) {
        using V2 = HIP_vector_type<V, 2>;
        *reinterpret_cast<V2*>(dst + v * plane) = V2(o[0][v], o[1][v]);
      } else {
        dst[v * plane] = o[0][v];
      }
    }
  }
}

// One sub-step of every point (the classical per-step update). Block 64 x 4;
// each thread walks plain_rows rows of one column, keeping three rows of its
// 3-wide neighbourhood in registers.
template <class S>
__global__ __launch_bounds__(256) void k_plain(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                               int nx, int ny, long long Trel, const long long* tbase,
                                               SchemeParams sp) {
  using V = typename S::V;
  constexpr int NV = S::NV, NW = S::NW;
  constexpr int R = plain_rows<S>();
  const long long T = Trel + (tbase ? *tbase : 0LL);
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int ys = (blockIdx.y * 4 + threadIdx.y) * R;
  if (x >= nx || ys >= ny) return;
  const int xw = (x == 0) ? nx - 1 : x - 1;
  const int xe = (x == nx - 1) ? 0 : x + 1;
  const size_t plane = (size_t)nx * ny;
  // window-only values of the scheme are zero here: every sub-step is a
  // launch of its own, so none survives one
  V rw[3][3][NW] = {};
  auto load = [&](V(&row)[3][NW], int y) {
    if (y < 0) y += ny;
    if (y >= ny) y -= ny;
    const V* base = in + (size_t)y * nx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      row[0][v] = base[v * plane + xw];
      row[1][v] = base[v * plane + x];
      row[2][v] = base[v * plane + xe];
    }
  };
  load(rw[0], ys - 1);
  load(rw[1], ys);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = ys + r;
    if (y >= ny) break;
    load(rw[2], y + 1);
    const RegNb<V, NW> nb{rw};
    V o[NW];
    S::step(T, nb, o, sp);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * plane + (size_t)y * nx + x] = o[v];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        rw[0][i][v] = rw[1][i][v];
        rw[1][i][v] = rw[2][i][v];
      }
  }
}

// ------------------------------------------------------------ launchers

template <class S>
SchemeInfo info_of() {
  return SchemeInfo{S::NV, S::NW, S::NVAR, S::SUB, (int)sizeof(typename S::V)};
}

// Workgroup size of the generic stage code for tile sides up to 22: one wave
// for the light schemes.
template <class S>
constexpr int small_threads() {
  return Lay<S, 0>::light ? 64 : Lay<S, 0>::NT;
}

// Window pitch as a compile-time constant for tile sides 16, 32 and 64; the
// workgroup size follows the instantiation's layout, one wave for small
// tiles of the light schemes.
#define SWEPT_BY_PITCH(KERNEL, S, n, GRID, LDS, STREAM, ...)                                                   \
  do {                                                                                                         \
    if ((n) == 64)                                                                                             \
      hipLaunchKernelGGL((KERNEL<S, 66, Lay<S, 66>::NT>), GRID, dim3(Lay<S, 66>::NT), LDS, STREAM, __VA_ARGS__); \
    else if ((n) == 32)                                                                                        \
      hipLaunchKernelGGL((KERNEL<S, 34, Lay<S, 34>::NT>), GRID, dim3(Lay<S, 34>::NT), LDS, STREAM, __VA_ARGS__); \
    else if ((n) == 16)                                                                                        \
      hipLaunchKernelGGL((KERNEL<S, 18, Lay<S, 18>::NT>), GRID, dim3(Lay<S, 18>::NT), LDS, STREAM, __VA_ARGS__); \
    else if ((n) <= 22)                                                                                        \
      hipLaunchKernelGGL((KERNEL<S, 0, small_threads<S>()>), GRID, dim3(small_threads<S>()), LDS, STREAM,       \
                         __VA_ARGS__);                                                                         \
    else                                                                                                       \
      hipLaunchKernelGGL((KERNEL<S, 0, Lay<S, 0>::NT>), GRID, dim3(Lay<S, 0>::NT), LDS, STREAM, __VA_ARGS__);   \
  } while (0)

// The same with the staging choice ST (a compile-time kernel parameter; the
// one-wave instantiations exist staged only).
#define SWEPT_BY_PITCH_ST(KERNEL, S, n, ST, GRID, LDS, STREAM, ...)                                           \
  do {                                                                                                        \
    constexpr int nt66 = Lay<S, 66>::NT, nt34 = Lay<S, 34>::NT, nts = small_threads<S>(), nt0 = Lay<S, 0>::NT; \
    constexpr int nt18 = Lay<S, 18>::NT;                                                                      \
    if ((n) == 16) {                                                                                          \
      if constexpr (nt18 == 64) {                                                                             \
        hipLaunchKernelGGL((KERNEL<S, 18, nt18, true>), GRID, dim3(nt18), LDS, STREAM, __VA_ARGS__);          \
      } else {                                                                                                \
        if (ST)                                                                                               \
          hipLaunchKernelGGL((KERNEL<S, 18, nt18, true>), GRID, dim3(nt18), LDS, STREAM, __VA_ARGS__);        \
        else                                                                                                  \
          hipLaunchKernelGGL((KERNEL<S, 18, nt18, false>), GRID, dim3(nt18), LDS, STREAM, __VA_ARGS__);       \
      }                                                                                                       \
    } else if ((n) == 64) {                                                                                   \
      if (ST)                                                                                                 \
        hipLaunchKernelGGL((KERNEL<S, 66, nt66, true>), GRID, dim3(nt66), LDS, STREAM, __VA_ARGS__);          \
      else                                                                                                    \
        hipLaunchKernelGGL((KERNEL<S, 66, nt66, false>), GRID, dim3(nt66), LDS, STREAM, __VA_ARGS__);         \
    } else if ((n) == 32) {                                                                                   \
      if (ST)                                                                                                 \
        hipLaunchKernelGGL((KERNEL<S, 34, nt34, true>), GRID, dim3(nt34), LDS, STREAM, __VA_ARGS__);          \
      else                                                                                                    \
        hipLaunchKernelGGL((KERNEL<S, 34, nt34, false>), GRID, dim3(nt34), LDS, STREAM, __VA_ARGS__);         \
    } else if ((n) <= 22) {                                                                                   \
      if constexpr (nts == 64) {                                                                              \
        hipLaunchKernelGGL((KERNEL<S, 0, nts, true>), GRID, dim3(nts), LDS, STREAM, __VA_ARGS__);             \
      } else {                                                                                                \
        if (ST)                                                                                               \
          hipLaunchKernelGGL((KERNEL<S, 0, nts, true>), GRID, dim3(nts), LDS, STREAM, __VA_ARGS__);           \
        else                                                                                                  \
          hipLaunchKernelGGL((KERNEL<S, 0, nts, false>), GRID, dim3(nts), LDS, STREAM, __VA_ARGS__);          \
      }                                                                                                       \
    } else {                                                                                                  \
      if (ST)                                                                                                 \
        hipLaunchKernelGGL((KERNEL<S, 0, nt0, true>), GRID, dim3(nt0), LDS, STREAM, __VA_ARGS__);             \
      else                                                                                                    \
        hipLaunchKernelGGL((KERNEL<S, 0, nt0, false>), GRID, dim3(nt0), LDS, STREAM, __VA_ARGS__);            \
    }                                                                                                         \
  } while (0)

template <class S>
hipError_t up_t(const Geo& g, int H, void* state, PanelPtrs p, const SchemeParams& sp, hipStream_t s) {
  const size_t lds = window_lds_bytes(info_of<S>(), g.n);
  SWEPT_BY_PITCH(k_up, S, g.n, dim3(g.ntx * g.nty), lds, s, g, H, static_cast<typename S::V*>(state),
                 p, sp);
  return hipGetLastError();
}

// Workgroup size of the instantiation that runs tile side n.
template <class S>
constexpr int threads_for(int n) {
  return n == 64 ? Lay<S, 66>::NT
                 : (n == 32 ? Lay<S, 34>::NT : (n == 16 ? Lay<S, 18>::NT : (n <= 22 ? small_threads<S>() : Lay<S, 0>::NT)));
}

// One-wave instantiations always stage their panel inputs.
template <class S>
bool forced_staging(int n) {
  return threads_for<S>(n) == 64;
}

// Whether the octahedron of tile side n, fetching its ring runs from HBM,
// keeps each wave's run terms precomputed and fetches a few levels ahead
// (a wave holds at most two of the 8 NV ring units); it then has no need
// to stage the runs in LDS.
template <class S>
bool oct_fetch_ahead(int n) {
  const int waves = threads_for<S>(n) / 64;
  return (8 * S::NV + waves - 1) / waves <= 2;
}

// Threads of one group of a bridge pair: 8 waves at tile side 64, half the
// stage workgroup otherwise.
template <class S, int WC>
constexpr int pair_threads() {
  return WC == 66 ? 512 : Lay<S, WC>::NT / 2;
}

// Bridge pairs (both bridges of a tile in one workgroup) for the column
// layouts when two bridge groups fit the workgroup LDS, staged if that
// fits too.
template <class S, int WC>
bool bridge_pair_launch(const Geo& g, int H, bool staged, void* state, PanelPtrs p, const SchemeParams& sp,
                        hipStream_t s, hipError_t* err) {
  constexpr int NT = 2 * pair_threads<S, WC>();
  if constexpr (!Lay<S, WC>::cols || NT < 128) {
    return false;
  } else {
    const size_t lim = device_lds_limit();
    bool st = staged && 2 * 8 * bridge_group_doubles<S>(g.n, true) <= lim;
    const size_t lds = 2 * 8 * bridge_group_doubles<S>(g.n, st);
    if (lds > lim) return false;
    if (st)
      hipLaunchKernelGGL((k_bridge_pair<S, WC, NT / 2, true>), dim3(g.ntx * g.nty), dim3(NT), lds, s, g, H,
                         static_cast<typename S::V*>(state), p, sp);
    else
      hipLaunchKernelGGL((k_bridge_pair<S, WC, NT / 2, false>), dim3(g.ntx * g.nty), dim3(NT), lds, s, g, H,
                         static_cast<typename S::V*>(state), p, sp);
    *err = hipGetLastError();
    return true;
  }
}

template <class S>
hipError_t bridge_t(const Geo& g, int H, bool staged, bool pair_ok, void* state, PanelPtrs p, const SchemeParams& sp,
                    hipStream_t s) {
  hipError_t e = hipSuccess;
  if (pair_ok && g.n == 64 && bridge_pair_launch<S, 66>(g, H, staged, state, p, sp, s, &e)) return e;
  if (pair_ok && g.n == 32 && bridge_pair_launch<S, 34>(g, H, staged, state, p, sp, s, &e)) return e;
  staged = staged || forced_staging<S>(g.n);
  const size_t lds = window_lds_bytes(info_of<S>(), g.n) + (staged ? bridge_stage_bytes(info_of<S>(), g.n) : 0);
  SWEPT_BY_PITCH_ST(k_bridge, S, g.n, staged, dim3(2 * g.ntx * g.nty), lds, s, g, H,
                    static_cast<typename S::V*>(state), p, sp);
  return hipGetLastError();
}

template <class S>
hipError_t oct_t(const Geo& g, int Hd, int Hu, bool staged, void* state, PanelPtrs p, const SchemeParams& sp,
                 hipStream_t s) {
  staged = staged || forced_staging<S>(g.n);
  const size_t lds = window_lds_bytes(info_of<S>(), g.n) + (staged ? oct_stage_bytes(info_of<S>(), g.n) : 0);
  SWEPT_BY_PITCH_ST(k_oct, S, g.n, staged, dim3(g.ntx * g.nty), lds, s, g, Hd, Hu,
                    static_cast<typename S::V*>(state), p, sp);
  return hipGetLastError();
}

template <class S>
hipError_t plain_t(int nx, int ny, long long T, const long long* tbase, const void* in, void* out,
                   const SchemeParams& sp, hipStream_t s) {
  if constexpr (Lay<S, 0>::light) {
    // two columns per thread need an even width and buffers aligned to two values
    const uintptr_t al = 2 * sizeof(typename S::V);
    const bool two = nx % 2 == 0 && (reinterpret_cast<uintptr_t>(in) % al) == 0 &&
                     (reinterpret_cast<uintptr_t>(out) % al) == 0;
    const int C = two ? 2 : 1;
    const int nb = ((nx + 128 * C - 1) / (128 * C)) * ((ny + kPlainRows - 1) / kPlainRows);
    const dim3 grid(((nb + kXcds - 1) / kXcds) * kXcds);
    if (C == 2)
      hipLaunchKernelGGL((k_plain_cols<S, 2>), grid, dim3(128), 0, s, static_cast<const typename S::V*>(in),
                         static_cast<typename S::V*>(out), nx, ny, T, tbase, sp);
    else
      hipLaunchKernelGGL((k_plain_cols<S, 1>), grid, dim3(128), 0, s, static_cast<const typename S::V*>(in),
                         static_cast<typename S::V*>(out), nx, ny, T, tbase, sp);
    return hipGetLastError();
  }
  constexpr int R = plain_rows<S>();
  const dim3 grid((nx + 63) / 64, (ny + 4 * R - 1) / (4 * R));
  hipLaunchKernelGGL(k_plain<S>, grid, dim3(64, 4), 0, s, static_cast<const typename S::V*>(in),
                     static_cast<typename S::V*>(out), nx, ny, T, tbase, sp);
  return hipGetLastError();
}

template <class S, int WC, int NT, bool ST>
hipError_t lds_staged(int b) {
  if constexpr (WC != 0 && Lay<S, WC>::cols && NT == Lay<S, WC>::NT && 2 * pair_threads<S, WC>() >= 128) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bridge_pair<S, WC, pair_threads<S, WC>(), ST>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bridge<S, WC, NT, ST>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_oct<S, WC, NT, ST>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

#include "rect.hpp"

template <class S, int WC, int NT>
hipError_t lds_one(int b) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_up<S, WC, NT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e != hipSuccess) return e;
  e = lds_staged<S, WC, NT, true>(b);
  if (e != hipSuccess) return e;
  if constexpr (NT != 64) e = lds_staged<S, WC, NT, false>(b);
  return e;
}

template <class S>
hipError_t lds_t(size_t bytes) {
  const int b = (int)bytes;
  hipError_t e = lds_one<S, 0, Lay<S, 0>::NT>(b);
  if (e != hipSuccess) return e;
  e = lds_one<S, 0, small_threads<S>()>(b);
  if (e != hipSuccess) return e;
  e = lds_one<S, 34, Lay<S, 34>::NT>(b);
  if (e != hipSuccess) return e;
  e = lds_one<S, 18, Lay<S, 18>::NT>(b);
  if (e != hipSuccess) return e;
  e = rect_lds_t<S>(b);
  if (e != hipSuccess) return e;
  return lds_one<S, 66, Lay<S, 66>::NT>(b);
}

// ------------------------------------------------------------------ batch

// One sub-step of the 64 x 64 block `blk` of a grid (per-step grids of a
// batch); thread (x, y) walks 64 / (NT / 64) rows of one column.
template <class S, int NT>
__device__ void plain_item(const typename S::V* __restrict__ in, typename S::V* __restrict__ out, int nx, int ny,
                           long long T, const SchemeParams& sp, int blk) {
  using V = typename S::V;
  constexpr int NV = S::NV, NW = S::NW, TY = NT / 64, R = kBatchBlock / TY;
  static_assert(TY * R == kBatchBlock, "block geometry");
  const int bx = (nx + kBatchBlock - 1) / kBatchBlock;
  const int x = (blk % bx) * kBatchBlock + (int)(threadIdx.x & 63);
  const int ys = (blk / bx) * kBatchBlock + (int)(threadIdx.x >> 6) * R;
  if (x >= nx || ys >= ny) return;
  const int xw = (x == 0) ? nx - 1 : x - 1;
  const int xe = (x == nx - 1) ? 0 : x + 1;
  const size_t plane = (size_t)nx * ny;
  // window-only values of the scheme are zero here: every sub-step is a
  // launch of its own, so none survives one
  V rw[3][3][NW] = {};
  auto load = [&](V(&row)[3][NW], int y) {
    if (y < 0) y += ny;
    if (y >= ny) y -= ny;
    const V* base = in + (size_t)y * nx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      row[0][v] = base[v * plane + xw];
      row[1][v] = base[v * plane + x];
      row[2][v] = base[v * plane + xe];
    }
  };
  load(rw[0], ys - 1);
  load(rw[1], ys);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = ys + r;
    if (y >= ny) break;
    load(rw[2], y + 1);
    V o[NW];
    S::step(T, RegNb<V, NW>{rw}, o, sp);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * plane + (size_t)y * nx + x] = o[v];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        rw[0][i][v] = rw[1][i][v];
        rw[1][i][v] = rw[2][i][v];
      }
  }
}

template <class S, int NT>
__device__ void copy_item(const typename S::V* __restrict__ in, typename S::V* __restrict__ out, int nx, int ny,
                          int blk) {
  constexpr int TY = NT / 64, R = kBatchBlock / TY;
  const int bx = (nx + kBatchBlock - 1) / kBatchBlock;
  const int x = (blk % bx) * kBatchBlock + (int)(threadIdx.x & 63);
  const int ys = (blk / bx) * kBatchBlock + (int)(threadIdx.x >> 6) * R;
  if (x >= nx) return;
  const size_t plane = (size_t)nx * ny;
  for (int r = 0; r < R; ++r) {
    const int y = ys + r;
    if (y >= ny) break;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) out[v * plane + (size_t)y * nx + x] = in[v * plane + (size_t)y * nx + x];
  }
}

// Run item `item` of phase p of grid G with the stage code at pitch WC on NT
// threads. Phase 0: upward pyramid; odd phases: bridges of half cycle
// (p - 1) / 2; even phases: octahedra (the last one of the advance writes the
// state). A per-step grid: phase p < S is sub-step p, alternating between the
// state and the second buffer; after an odd count a copy back.
template <class S, int WC, int NT>
__device__ __forceinline__ void batch_stage(const BatchGrid& G, const BatchPlan& P, int p, int item, double* smem) {
  using V = typename S::V;
  V* state = static_cast<V*>(G.state);
  if constexpr (WC < 0) {
    // Rectangular tiles (WC = rect_marker(pitch)): phase 0 the first
    // frustums, odd phases the bridges of half cycle (p - 1) / 2 on tiling
    // ((p - 1) / 2) mod 2, even phases the stage that finishes its downward
    // pyramids and starts the next frustums (the last one of the advance
    // writes its squares).
    constexpr int RW = WC == -1 ? 0 : -WC;
    if constexpr (S::NW == S::NV && (RW == 0 || Lay<S, 66>::light)) {
      RGeo g = G.rg;
      g.tbase = nullptr;
      const int h = g.h;
      V* sm = reinterpret_cast<V*>(smem);
      if (p == 0) {
        g.T0 = G.g0.T0;
        rect_oct_item<S, RW, NT>(g, 0, 0, P.q > 0 ? h : P.r, state, G.pp, G.sp, item, sm);
        return;
      }
      const int hc = (p - 1) / 2;
      g.T0 = G.g0.T0 + (long long)hc * h;
      const int H = hc < P.q ? h : P.r;
      if (p & 1) {
        rect_bridge_item<S, RW, NT>(g, hc & 1, H, state, G.pp, G.sp, item, sm);
      } else {
        const int Hu = (hc + 1 < P.q) ? h : (hc + 1 == P.q ? P.r : 0);
        rect_oct_item<S, RW, NT>(g, 1 - (hc & 1), H, Hu, state, G.pp, G.sp, item, sm);
      }
    }
    return;
  } else {
  if constexpr (WC == 0 && NT == 256) {
    if (G.kind == kBatchPlain) {
      V* s2 = static_cast<V*>(G.state2);
      if (p < P.S) {
        const bool even = (p & 1) == 0;
        plain_item<S, NT>(even ? state : s2, even ? s2 : state, G.g0.nx, G.g0.ny, G.g0.T0 + p, G.sp, item);
      } else {
        copy_item<S, NT>(s2, state, G.g0.nx, G.g0.ny, item);
      }
      return;
    }
  }
  Geo g = G.g0;
  const int h = g.h;
  if (p == 0) {
    up_item<S, WC, NT>(g, P.q > 0 ? h : P.r, state, G.pp, G.sp, item, smem);
    return;
  }
  const int hc = (p - 1) / 2;
  g.off = (hc & 1) ? h : 0;
  g.T0 = G.g0.T0 + (long long)hc * h;
  const int H = hc < P.q ? h : P.r;
  // One-wave items (tile sides up to 22) always stage their panel inputs
  // (a few KB), which keeps the per-level fetch registers out of the kernel.
  constexpr bool always_staged = NT == 64;
  if (p & 1) {
    if (always_staged || G.staged_bridge) {
      bridge_item<S, WC, NT, true>(g, H, state, G.pp, G.sp, item, smem);
    } else if constexpr (!always_staged) {
      bridge_item<S, WC, NT, false>(g, H, state, G.pp, G.sp, item, smem);
    }
  } else {
    const int Hu = (hc + 1 < P.q) ? h : (hc + 1 == P.q ? P.r : 0);
    if (always_staged || G.staged_oct) {
      oct_item<S, WC, NT, true>(g, H, Hu, state, G.pp, G.sp, item, smem);
    } else if constexpr (!always_staged) {
      oct_item<S, WC, NT, false>(g, H, Hu, state, G.pp, G.sp, item, smem);
    }
  }
  }
}

// One launch of a slot of the phased batch: workgroup b finds its entry by
// binary search over the launch's item offsets (all reads are uniform) and
// runs one item. No workgroup waits for another: the slot's launches order
// the phases.
template <int WC, int NT>
__global__ __launch_bounds__(NT) void k_batch_phase(PhaseLaunch L) {
  extern __shared__ double smem_d[];
  const int b = (int)blockIdx.x;
  int lo = 0, hi = L.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (L.cum[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  const int g = L.grid[lo], p = L.phase[lo], item = b - L.cum[lo];
  const BatchGrid& G = L.grids[g];
  const BatchPlan& P = L.plans[g];
  switch (G.scheme) {
    case kHeat64: batch_stage<Heat64, WC, NT>(G, P, p, item, smem_d); break;
    case kWave64: batch_stage<Wave64, WC, NT>(G, P, p, item, smem_d); break;
    case kHash64: batch_stage<Hash64, WC, NT>(G, P, p, item, smem_d); break;
    case kHeat32C: batch_stage<Heat32C, WC, NT>(G, P, p, item, smem_d); break;
    case kWave32C: batch_stage<Wave32C, WC, NT>(G, P, p, item, smem_d); break;
    default: break;
  }
}

#ifdef SWEPT2D_BUILD_PERSISTENT_BATCH
// Items of grid `G` completed before its phase p.
__device__ __forceinline__ long long batch_need(const BatchGrid& G, int p) {
  if (G.kind == kBatchPlain) return (long long)G.units * p;
  if (p == 0) return 0;
  return (long long)G.units * (1 + 2 * (p / 2) + ((p + 1) / 2 - 1));
}

template <class S, int WC>
__device__ __noinline__ void batch_stage_persistent(const BatchGrid& G, const BatchPlan& P, int p, int item,
                                                    double* smem) {
  if (G.kind == kBatchPlain) {
    using V = typename S::V;
    V* state = static_cast<V*>(G.state);
    V* s2 = static_cast<V*>(G.state2);
    if (p < P.S) {
      const bool even = (p & 1) == 0;
      plain_item<S, kBatchThreads>(even ? state : s2, even ? s2 : state, G.g0.nx, G.g0.ny, G.g0.T0 + p, G.sp, item);
    } else {
      copy_item<S, kBatchThreads>(s2, state, G.g0.nx, G.g0.ny, item);
    }
    return;
  }
  batch_stage<S, WC, kBatchThreads>(G, P, p, item, smem);
}

template <class S>
__device__ void batch_scheme(const BatchGrid& G, const BatchPlan& P, int p, int item, double* smem) {
  if (G.wc == 66)
    batch_stage_persistent<S, 66>(G, P, p, item, smem);
  else if (G.wc == 34)
    batch_stage_persistent<S, 34>(G, P, p, item, smem);
  else
    batch_stage_persistent<S, 0>(G, P, p, item, smem);
}

// Largest i in [lo, hi) with a[i] <= key (a nondecreasing, a[lo] <= key).
__device__ __forceinline__ int last_le(const long long* a, int lo, int hi, long long key) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= key)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The persistent work loop. One thread takes the next ticket (first counting
// the workgroup's previous item as done), decodes it and waits for its
// dependency; the workgroup then runs the item. The loop's exit and every
// value the item depends on are read back as scalars (readfirstlane), so
// the whole workgroup goes round the loop together.
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchSched s) {
  extern __shared__ double smem_d[];
  __shared__ int sh_stop, sh_phase, sh_grid, sh_item;
  int prev = -1;  // grid of the previous item (uniform)
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev >= 0) __hip_atomic_fetch_add(&s.done[prev], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      int stop = __hip_atomic_load(s.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      int p = 0, g = 0, item = 0;
      if (!stop) {
        const long long k = (long long)atomicAdd(s.head, 1ull);
        if (k >= s.total) {
          stop = 1;
        } else {
          p = last_le(s.phase_base, 0, s.nphases, k);
          const long long local = k - s.phase_base[p];
          const long long* cum = (p & 1) ? s.cum2 : s.cum1;
          const int j = last_le(cum, 0, s.phase_active[p], local);
          g = s.order[j];
          item = (int)(local - cum[j]);
          const unsigned need = (unsigned)batch_need(s.grids[g], p);
          const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
          while (__hip_atomic_load(&s.done[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > (unsigned long long)s.wait_ticks ||
                __hip_atomic_load(s.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              __hip_atomic_store(s.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              stop = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(16);
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      sh_stop = stop;
      sh_phase = p;
      sh_grid = g;
      sh_item = item;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(sh_stop)) break;
    const int g = __builtin_amdgcn_readfirstlane(sh_grid);
    const int p = __builtin_amdgcn_readfirstlane(sh_phase);
    const int item = __builtin_amdgcn_readfirstlane(sh_item);
    const BatchGrid& G = s.grids[g];
    const BatchPlan& P = s.plans[g];
    switch (__builtin_amdgcn_readfirstlane(G.scheme)) {
      case kHeat64: batch_scheme<Heat64>(G, P, p, item, smem_d); break;
      case kWave64: batch_scheme<Wave64>(G, P, p, item, smem_d); break;
      case kHash64: batch_scheme<Hash64>(G, P, p, item, smem_d); break;
      case kHeat32C: batch_scheme<Heat32C>(G, P, p, item, smem_d); break;
      case kWave32C: batch_scheme<Wave32C>(G, P, p, item, smem_d); break;
      default: break;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    prev = g;
  }
}

__global__ void k_batch_reset(unsigned* done, int ngrids, unsigned long long* head) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ngrids) done[i] = 0u;
  if (i == 0) *head = 0ull;
}
#endif  // SWEPT2D_BUILD_PERSISTENT_BATCH

}  // namespace

// ------------------------------------------------- explicit instantiation

template <class S>
SchemeInfo Stages<S>::info() {
  return info_of<S>();
}
template <class S>
hipError_t Stages<S>::up(const Geo& g, int H, void* state, PanelPtrs p, const SchemeParams& sp, hipStream_t s) {
  return up_t<S>(g, H, state, p, sp, s);
}
template <class S>
hipError_t Stages<S>::bridge(const Geo& g, int H, bool staged, bool pair_ok, void* state, PanelPtrs p,
                             const SchemeParams& sp, hipStream_t s) {
  return bridge_t<S>(g, H, staged, pair_ok, state, p, sp, s);
}
template <class S>
hipError_t Stages<S>::oct(const Geo& g, int Hd, int Hu, bool staged, void* state, PanelPtrs p, const SchemeParams& sp,
                          hipStream_t s) {
  return oct_t<S>(g, Hd, Hu, staged, state, p, sp, s);
}
template <class S>
hipError_t Stages<S>::plain(int nx, int ny, long long T, const long long* tbase, const void* in, void* out,
                            const SchemeParams& sp, hipStream_t s) {
  return plain_t<S>(nx, ny, T, tbase, in, out, sp, s);
}
template <class S>
bool Stages<S>::fetch_ahead(int n) {
  return oct_fetch_ahead<S>(n);
}
template <class S>
hipError_t Stages<S>::lds(size_t bytes) {
  return lds_t<S>(bytes);
}
template <class S>
hipError_t Stages<S>::rect_oct(const RGeo& g, int upar, int Hd, int Hu, void* state, PanelPtrs p,
                               const SchemeParams& sp, hipStream_t s) {
  return rect_oct_t<S>(g, upar, Hd, Hu, state, p, sp, s);
}
template <class S>
hipError_t Stages<S>::rect_bridge(const RGeo& g, int par, int H, void* state, PanelPtrs p, const SchemeParams& sp,
                                  hipStream_t s) {
  return rect_bridge_t<S>(g, par, H, state, p, sp, s);
}

template <int WC, int NT>
hipError_t BatchPhase<WC, NT>::launch(const PhaseLaunch& L, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_batch_phase<WC, NT>), dim3(blocks), dim3(NT), lds, st, L);
  return hipGetLastError();
}
template <int WC, int NT>
hipError_t BatchPhase<WC, NT>::lds(int bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_phase<WC, NT>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
template <int WC, int NT>
hipError_t BatchPhase<WC, NT>::resident(size_t lds, int* out) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_batch_phase<WC, NT>, NT, lds);
}

}  // namespace swept
