// Swept stages on rectangular tiles of any side of at least 2h (the tiling
// is described with RGeo in engine.hpp). Included by stages.hpp inside its
// anonymous namespace; the launchers at the end of stages.hpp instantiate
// these kernels once per scheme.
//
// These stages serve grids that no even square tile side divides (an odd
// side, a prime) and tiles wider than the square ones. The tile sizes are
// run-time values; the window pitch WC is 66 when every tile is at most 64
// wide and the scheme is light (levels in the column layout with lane
// shifts of the square tiles' code, 16 waves), 34 when at most 32 wide
// (one point per thread at a fixed pitch, 4 waves), and otherwise the
// run-time widest tile + 2 (WC = 0: one rectangle point per thread with its
// 3x3 neighbourhood read from LDS, 4 waves). The component structure is the square tiles':
// a workgroup keeps its component's window in LDS, double buffered by level
// parity; panel levels are stored as soon as their level is complete (the
// band of level l stays untouched in buffer l mod 2 while later levels of
// that parity are computed strictly inside it).
//
// Panel conventions (per tile, end and level l = 0..H-1; row k = 0 nearer
// the edge the panel faces, value t along that edge; row stride R per value
// slot and row):
//  up   ends N, S, W, E (0..3): the two outermost rows or columns of the
//       frustum's level-l rectangle [l, w-1-l] in tile coordinates,
//       t = 0 at tile position l; R = urow.
//  xb   ends N, S (0, 1) of the x-bridge over the east edge E of tile
//       (a, b): rows l, l+1 (N) or w_y-1-l, w_y-2-l (S) of the tile, for
//       x in [E-l-2, E+l+2) (the band and the frustum corners); R = 2h + 4.
//  yb   ends W, E (0, 1) of the y-bridge over the south edge F of tile
//       (a, b): columns l, l+1 (W) or w_x-1-l, w_x-2-l (E) of the tile, for
//       y in [F-l, F+l); R = 2h.
// The downward pyramid at the south-east corner of tile (a, b) reads the S
// end of xb(a, b), the N end of xb(a, b+1), the E end of yb(a, b) and the W
// end of yb(a+1, b): the ring two wide around its level-l square, corners
// included.

// Cell x + c, with x + c in [-L, 2L), brought into [0, L).
__device__ __forceinline__ int rect_wrap(int x, int L) { return x < 0 ? x + L : (x >= L ? x - L : x); }

// One level: every point of the window rectangle [x0, x0+w) x [y0, y0+hg)
// gets sub-step T from `in` into `out`. At pitch 66 the column layout takes
// its side neighbours by lane shifts where the rectangle lies within window
// columns 2..63, and from LDS otherwise; at pitch 34 one point per thread;
// at a run-time pitch the flux schemes walk columns and the others take one
// point per thread.
template <class S, int WC, int NT>
__device__ __forceinline__ void rect_level(const typename S::V* __restrict__ in, typename S::V* __restrict__ out,
                                           int P, int x0, int y0, int w, int hg, long long T, const SchemeParams& sp) {
  using V = typename S::V;
  constexpr int NV = S::NV;
  if (w <= 0 || hg <= 0) return;
  if constexpr (WC == 66) {
    if (x0 >= 2 && x0 + w <= 64)
      compute_level<S, 66, NT, false, false>(in, out, 66, x0, y0, w, hg, T, sp);
    else
      compute_level<S, 66, NT, false, true>(in, out, 66, x0, y0, w, hg, T, sp);
    return;
  } else if constexpr (WC == 34) {
    compute_level<S, 34, NT, false>(in, out, 34, x0, y0, w, hg, T, sp);
    return;
  } else if constexpr (walks<S>::value) {
    // the flux schemes' column walk at the run-time pitch (their tiles are
    // at most 33 wide: the window of two buffers fills the LDS)
    compute_level<S, 0, NT, false>(in, out, P, x0, y0, w, hg, T, sp);
    return;
  }
  const int plane = P * P, npts = w * hg;
  const float inv = __builtin_amdgcn_rcpf((float)w);
  for (int k = (int)threadIdx.x; k < npts; k += NT) {
    int dy, dx;
    fdivmod(k, w, inv, dy, dx);
    const int o = (y0 + dy) * P + x0 + dx;
    V nb[3][3][NV];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) nb[r][c][v] = in[v * plane + o + (r - 1) * P + (c - 1)];
    V res[NV];
    S::step(T, RegNb<V, NV>{&nb[0]}, res, sp);
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * plane + o] = res[v];
  }
}

// A panel level <-> two window rows of `len` values per value slot: value t
// of row k of slot v sits at window column c0 + t dc + k kc, row
// r0 + t dr + k kr, and at pan[(2 v + k) R + t]. TO_PANEL: window -> panel.
struct RectRun {
  int c0, r0, dc, dr, kc, kr, len;
};

template <class S, int NT, bool TO_PANEL>
__device__ __forceinline__ void rect_copy(typename S::V* __restrict__ win, int P, const RectRun& q,
                                          typename S::V* __restrict__ pan, int R) {
  constexpr int NV = S::NV;
  if (q.len <= 0) return;
  const int plane = P * P, total = 2 * NV * q.len;
  const float inv = __builtin_amdgcn_rcpf((float)q.len);
  for (int e = (int)threadIdx.x; e < total; e += NT) {
    int vk, t;
    fdivmod(e, q.len, inv, vk, t);
    const int k = vk & 1, v = vk >> 1;
    const int wi = v * plane + (q.r0 + t * q.dr + k * q.kr) * P + q.c0 + t * q.dc + k * q.kc;
    if (TO_PANEL)
      pan[vk * R + t] = win[wi];
    else
      win[wi] = pan[vk * R + t];
  }
}

// Panel runs placed in the window, fetched into registers a level ahead
// (the fixed-pitch instantiations): up to four runs of one level, each
// thread holding elements threadIdx.x + j NT (j < KR) of every run with
// their window positions (-1: none). KR covers the longest run those
// instantiations meet (a ring run of 2h + 4 values, h <= 32 at pitch 66 and
// <= 16 at pitch 34).
template <class S, int WC, int NT>
constexpr int rect_kr() {
  return WC == 66 ? (136 * S::NV + NT - 1) / NT : (WC == 34 ? (72 * S::NV + NT - 1) / NT : 1);
}

template <class V, int KR>
struct RectFetch {
  V val[4][KR];
  int wi[4][KR];
};

// The fixed-pitch instantiations describe each kind of run once for all
// levels: level l of the run starts at window cell (c0 + l dc0, r0 + l dr0)
// with len0 + l dlen values per row, value t of row k of slot v lying at
// (+ t dc + k kc, + t dr + k kr) and at src[l sstride + (2 v + k) R + t].
// A thread keeps its elements of a run for every level (element
// threadIdx.x + j NT is row e / S, value e mod S, S the run's longest
// level), so a level costs it one test and two additions per element.
struct RunLin {
  int c0, r0, dc0, dr0, dc, dr, kc, kr, len0, dlen, R, sstride;
};

template <int KR>
struct RunLanes {
  int wi[KR];  // window index at level 0 (buffer-relative)
  int pi[KR];  // panel index at level 0
  int t[KR];   // value index along the run
  bool ok[KR];
};

template <class S, int NT, int KR>
__device__ __forceinline__ RunLanes<KR> run_lanes(const RunLin& q, int S_len, int P) {
  constexpr int NV = S::NV;
  RunLanes<KR> L;
  const float inv = __builtin_amdgcn_rcpf((float)(S_len > 0 ? S_len : 1));
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int e = (int)threadIdx.x + j * NT;
    int vk, t;
    fdivmod(e, S_len > 0 ? S_len : 1, inv, vk, t);
    const int k = vk & 1, v = vk >> 1;
    L.ok[j] = S_len > 0 && vk < 2 * NV;
    L.t[j] = t;
    L.wi[j] = v * P * P + (q.r0 + t * q.dr + k * q.kr) * P + q.c0 + t * q.dc + k * q.kc;
    L.pi[j] = vk * q.R + t;
  }
  return L;
}

// Level l of up to four runs into registers (window positions -1: none).
template <class S, int KR>
__device__ __forceinline__ void lin_fetch(RectFetch<typename S::V, KR>& f, const RunLanes<KR> (&L)[4],
                                          const RunLin (&q)[4], const typename S::V* const (&src)[4], int n, int l,
                                          int P) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int len = q[r].len0 + l * q[r].dlen, dw = l * (q[r].dr0 * P + q[r].dc0);
    const typename S::V* sp = src[r] + (long long)l * q[r].sstride;
#pragma unroll
    for (int j = 0; j < KR; ++j) {
      f.wi[r][j] = -1;
      if (r < n && L[r].ok[j] && L[r].t[j] < len) {
        f.wi[r][j] = L[r].wi[j] + dw;
        f.val[r][j] = sp[L[r].pi[j]];
      }
    }
  }
}

// Level l of one run, window -> panel.
template <class S, int KR>
__device__ __forceinline__ void lin_emit(const typename S::V* __restrict__ win, const RunLanes<KR>& L, const RunLin& q,
                                         typename S::V* __restrict__ dst, int l, int P) {
  const int len = q.len0 + l * q.dlen, dw = l * (q.dr0 * P + q.dc0);
  typename S::V* dp = dst + (long long)l * q.sstride;
#pragma unroll
  for (int j = 0; j < KR; ++j)
    if (L.ok[j] && L.t[j] < len) dp[L.pi[j]] = win[L.wi[j] + dw];
}

struct RectRuns {
  int n;
  RectRun q[4];
  const void* src[4];
  int R[4];
};

template <class S, int KR>
__device__ __forceinline__ void rect_place(const RectFetch<typename S::V, KR>& f, typename S::V* __restrict__ win) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int j = 0; j < KR; ++j)
      if (f.wi[r][j] >= 0) win[f.wi[r][j]] = f.val[r][j];
}

template <class S, int NT>
__device__ __forceinline__ void rect_copy_runs(typename S::V* __restrict__ win, int P, const RectRuns& rs) {
  for (int r = 0; r < rs.n; ++r)
    rect_copy<S, NT, false>(win, P, rs.q[r], const_cast<typename S::V*>(static_cast<const typename S::V*>(rs.src[r])),
                            rs.R[r]);
}

// Window cells [cx0, cx0+w) x [cy0, cy0+hg) <-> state cells
// (gx0 + cx, gy0 + cy) modulo the grid (gx0 + cx and gy0 + cy in
// [-L, 2L)), skipping the window square [qx0, qx0+qs) x [qy0, qy0+qs).
// LOAD: state -> window.
template <class S, int NT, bool LOAD>
__device__ __forceinline__ void rect_move(typename S::V* __restrict__ win, int P, typename S::V* __restrict__ state,
                                          int nx, int ny, int cx0, int cy0, int w, int hg, int gx0, int gy0, int qx0,
                                          int qy0, int qs) {
  constexpr int NV = S::NV;
  if (w <= 0 || hg <= 0) return;
  const int plane = P * P, npts = w * hg;
  const size_t splane = (size_t)nx * ny;
  const float inv = __builtin_amdgcn_rcpf((float)w);
  for (int k = (int)threadIdx.x; k < npts; k += NT) {
    int dy, dx;
    fdivmod(k, w, inv, dy, dx);
    const int cx = cx0 + dx, cy = cy0 + dy;
    if (cx >= qx0 && cx < qx0 + qs && cy >= qy0 && cy < qy0 + qs) continue;
    const size_t gi = (size_t)rect_wrap(gy0 + cy, ny) * nx + rect_wrap(gx0 + cx, nx);
    const int wi = cy * P + cx;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (LOAD)
        win[v * plane + wi] = state[v * splane + gi];
      else
        state[v * splane + gi] = win[v * plane + wi];
    }
  }
}

__device__ __forceinline__ size_t rect_up_at(const RGeo& g, int nv, int tile, int end, int l) {
  return ((size_t)(tile * 4 + end) * g.h + l) * (size_t)(2 * nv * g.urow);
}
__device__ __forceinline__ size_t rect_xb_at(const RGeo& g, int nv, int tile, int end, int l) {
  return ((size_t)(tile * 2 + end) * g.h + l) * (size_t)(2 * nv * (2 * g.h + 4));
}
__device__ __forceinline__ size_t rect_yb_at(const RGeo& g, int nv, int tile, int end, int l) {
  return ((size_t)(tile * 2 + end) * g.h + l) * (size_t)(2 * nv * (2 * g.h));
}

// Tile `item` of tiling upar: the downward pyramid (height Hd) at the corner
// of tiling 1 - upar inside it, the rest of the tile from the state, then
// the upward frustum of the tile (height Hu). Window cell (cx, cy) is tile
// cell (cx - 1, cy - 1).
template <class S, int WC, int NT>
__device__ __forceinline__ void rect_oct_item(const RGeo& g, int upar, int Hd, int Hu, typename S::V* __restrict__ state,
                              const PanelPtrs& pp, const SchemeParams& sp, int item, typename S::V* smem) {
  using V = typename S::V;
  constexpr int NV = S::NV;
  const int tx = g.ax.t, ty = g.ay.t, P = g.P;
  const int j = item / tx, i = item - j * tx;
  int sx, wx, sy, wy;
  rect_span(g.ax, upar, i, sx, wx);
  rect_span(g.ay, upar, j, sy, wy);
  // The two level buffers, chosen by parity with a select (an array of
  // pointers would hide from the compiler that they point into LDS).
  V* const buf0 = smem;
  V* const buf1 = smem + NV * P * P;
  auto buf = [&](int k) { return (k & 1) ? buf1 : buf0; };
  const long long base = g.T0 + (g.tbase ? *g.tbase : 0LL);
  const int nx = g.ax.L, ny = g.ay.L;
  // The corner of the other tiling inside this tile, and the downward
  // pyramid (tile (di, dj) of that tiling) it belongs to.
  int ox, oy, di, dj;
  if (upar == 1) {  // corners of tiling 0: the south-east corner of tile (i, j)
    ox = rect_width0(g.ax, i) - rect_width0(g.ax, i) / 2;
    oy = rect_width0(g.ay, j) - rect_width0(g.ay, j) / 2;
    di = i;
    dj = j;
  } else {  // corners of tiling 1: the south-east corner of tile (i-1, j-1)
    ox = rect_width0(g.ax, i) / 2;
    oy = rect_width0(g.ay, j) / 2;
    di = i == 0 ? tx - 1 : i - 1;
    dj = j == 0 ? ty - 1 : j - 1;
  }
  const int cE = 1 + ox, cF = 1 + oy;
  const V* xb = static_cast<const V*>(pp.xb);
  const V* yb = static_cast<const V*>(pp.yb);
  const int tN = di + dj * tx, tS = di + (dj + 1 == ty ? 0 : dj + 1) * tx;
  const int tE = (di + 1 == tx ? 0 : di + 1) + dj * tx;
  const int Rx = 2 * g.h + 4, Ry = 2 * g.h;
  // Ring of the downward pyramid's level l (for its level l + 1).
  auto ring = [&](int l) {
    return RectRuns{4,
                    {RectRun{cE - l - 2, cF - 1 - l, 1, 0, 0, -1, 2 * l + 4},
                     RectRun{cE - l - 2, cF + l, 1, 0, 0, 1, 2 * l + 4}, RectRun{cE - 1 - l, cF - l, 0, 1, -1, 0, 2 * l},
                     RectRun{cE + l, cF - l, 0, 1, 1, 0, 2 * l}},
                    {xb + rect_xb_at(g, NV, tN, 1, l), xb + rect_xb_at(g, NV, tS, 0, l),
                     yb + rect_yb_at(g, NV, tN, 1, l), yb + rect_yb_at(g, NV, tE, 0, l)},
                    {Rx, Rx, Ry, Ry}};
  };
  // The tile's cells outside the level-Hd square (all of them if Hd == 0),
  // at level Hd, from the state; they go to the buffer level Hd ends in,
  // where no ring or square of an earlier level reaches.
  if (Hu > 0)
    rect_move<S, NT, true>(buf(Hd), P, state, nx, ny, 1, 1, wx, wy, sx - 1, sy - 1, cE - Hd, cF - Hd, 2 * Hd);
  if (Hd > 0) rect_copy_runs<S, NT>(buf(0), P, ring(0));
  if constexpr (WC != 0) {
    // Each level's ring is fetched during the level before and placed at
    // the start of its own (beside the square it surrounds).
    constexpr int KR = rect_kr<S, WC, NT>();
    const RunLin rq[4] = {{cE - 2, cF - 1, -1, -1, 1, 0, 0, -1, 4, 2, Rx, 2 * NV * Rx},
                          {cE - 2, cF, -1, 1, 1, 0, 0, 1, 4, 2, Rx, 2 * NV * Rx},
                          {cE - 1, cF, -1, -1, 0, 1, -1, 0, 0, 2, Ry, 2 * NV * Ry},
                          {cE, cF, 1, -1, 0, 1, 1, 0, 0, 2, Ry, 2 * NV * Ry}};
    const V* const rsrc[4] = {xb + rect_xb_at(g, NV, tN, 1, 0), xb + rect_xb_at(g, NV, tS, 0, 0),
                              yb + rect_yb_at(g, NV, tN, 1, 0), yb + rect_yb_at(g, NV, tE, 0, 0)};
    const int Smax = 2 * Hd + 2;
    const RunLanes<KR> rl[4] = {run_lanes<S, NT, KR>(rq[0], Smax, P), run_lanes<S, NT, KR>(rq[1], Smax, P),
                                run_lanes<S, NT, KR>(rq[2], Smax, P), run_lanes<S, NT, KR>(rq[3], Smax, P)};
    RectFetch<V, KR> f;
    if (Hd > 1) lin_fetch<S, KR>(f, rl, rq, rsrc, 4, 1, P);
    __syncthreads();
    for (int l = 1; l <= Hd; ++l) {
      if (l < Hd) {
        rect_place<S, KR>(f, buf(l));
        if (l + 1 < Hd) lin_fetch<S, KR>(f, rl, rq, rsrc, 4, l + 1, P);
      }
      rect_level<S, WC, NT>(buf(l - 1), buf(l), P, cE - l, cF - l, 2 * l, 2 * l, base + l - 1, sp);
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int l = 1; l <= Hd; ++l) {
      rect_level<S, WC, NT>(buf(l - 1), buf(l), P, cE - l, cF - l, 2 * l, 2 * l, base + l - 1, sp);
      if (l < Hd) rect_copy_runs<S, NT>(buf(l), P, ring(l));
      __syncthreads();
    }
  }
  if (Hu == 0) {
    rect_move<S, NT, false>(buf(Hd), P, state, nx, ny, cE - Hd, cF - Hd, 2 * Hd, 2 * Hd, sx - 1, sy - 1, 0, 0, 0);
    return;
  }
  V* up = static_cast<V*>(pp.up);
  const int tile = item, R = g.urow;
  if constexpr (WC != 0) {
    // the frustum's strips of level l (rectangle [l, w-1-l] in tile cells)
    constexpr int KR = rect_kr<S, WC, NT>();
    const int us = 2 * NV * R;
    const RunLin uq[4] = {{1, 1, 1, 1, 1, 0, 0, 1, wx, -2, R, us}, {1, wy, 1, -1, 1, 0, 0, -1, wx, -2, R, us},
                          {1, 1, 1, 1, 0, 1, 1, 0, wy, -2, R, us}, {wx, 1, -1, 1, 0, 1, -1, 0, wy, -2, R, us}};
    const int Smax = wx > wy ? wx : wy;
    const RunLanes<KR> ul[4] = {run_lanes<S, NT, KR>(uq[0], Smax, P), run_lanes<S, NT, KR>(uq[1], Smax, P),
                                run_lanes<S, NT, KR>(uq[2], Smax, P), run_lanes<S, NT, KR>(uq[3], Smax, P)};
    V* const ub[4] = {up + rect_up_at(g, NV, tile, 0, 0), up + rect_up_at(g, NV, tile, 1, 0),
                      up + rect_up_at(g, NV, tile, 2, 0), up + rect_up_at(g, NV, tile, 3, 0)};
    for (int m = 1; m <= Hu; ++m) {
      V* in = buf(Hd + m - 1);
      rect_level<S, WC, NT>(in, buf(Hd + m), P, 1 + m, 1 + m, wx - 2 * m, wy - 2 * m, base + Hd + m - 1, sp);
#pragma unroll
      for (int r = 0; r < 4; ++r) lin_emit<S, KR>(in, ul[r], uq[r], ub[r], m - 1, P);
      __syncthreads();
    }
  } else {
    for (int m = 1; m <= Hu; ++m) {
      V* in = buf(Hd + m - 1);
      rect_level<S, WC, NT>(in, buf(Hd + m), P, 1 + m, 1 + m, wx - 2 * m, wy - 2 * m, base + Hd + m - 1, sp);
      // panels of level m - 1: rectangle [m-1, w-m] in tile cells
      const int l = m - 1, lx = wx - 2 * l, ly = wy - 2 * l;
      rect_copy<S, NT, true>(in, P, RectRun{m, m, 1, 0, 0, 1, lx}, up + rect_up_at(g, NV, tile, 0, l), R);
      rect_copy<S, NT, true>(in, P, RectRun{m, wy - l, 1, 0, 0, -1, lx}, up + rect_up_at(g, NV, tile, 1, l), R);
      rect_copy<S, NT, true>(in, P, RectRun{m, m, 0, 1, 1, 0, ly}, up + rect_up_at(g, NV, tile, 2, l), R);
      rect_copy<S, NT, true>(in, P, RectRun{wx - l, m, 0, 1, -1, 0, ly}, up + rect_up_at(g, NV, tile, 3, l), R);
      __syncthreads();
    }
  }
  rect_move<S, NT, false>(buf(Hd + Hu), P, state, nx, ny, 1 + Hu, 1 + Hu, wx - 2 * Hu, wy - 2 * Hu, sx - 1, sy - 1,
                      0, 0, 0);
}

// Bridge `item` of tiling par: items 0 .. t_x t_y - 1 are the x-bridges over
// the east edge of tile (a, b), the rest the y-bridges over the south edge.
// The window's columns run across the edge, 2H + 2 of them (cell
// E - H - 1 + c), its rows along it over the tile's extent; the y-bridge's
// window is the transpose (row c across the edge).
template <class S, int WC, int NT>
__device__ __forceinline__ void rect_bridge_item(const RGeo& g, int par, int H, typename S::V* __restrict__ state,
                                 const PanelPtrs& pp, const SchemeParams& sp, int item, typename S::V* smem) {
  using V = typename S::V;
  constexpr int NV = S::NV;
  const int tx = g.ax.t, ty = g.ay.t, P = g.P;
  const bool isx = item < tx * ty;
  const int e = isx ? item : item - tx * ty;
  const int b = e / tx, a = e - b * tx;
  int sx, wx, sy, wy;
  rect_span(g.ax, par, a, sx, wx);
  rect_span(g.ay, par, b, sy, wy);
  // The two level buffers, chosen by parity with a select (an array of
  // pointers would hide from the compiler that they point into LDS).
  V* const buf0 = smem;
  V* const buf1 = smem + NV * P * P;
  auto buf = [&](int k) { return (k & 1) ? buf1 : buf0; };
  const long long base = g.T0 + (g.tbase ? *g.tbase : 0LL);
  const int nx = g.ax.L, ny = g.ay.L;
  const int wal = isx ? wy : wx;  // extent along the edge
  // Window position of (across, along) as (column, row).
  auto run = [&](int ac, int al, int dac, int dal, int kac, int kal, int len) {
    return isx ? RectRun{ac, al, dac, dal, kac, kal, len} : RectRun{al, ac, dal, dac, kal, kac, len};
  };
  const V* up = static_cast<const V*>(pp.up);
  const int tnear = e;
  const int tfar = isx ? (a + 1 == tx ? 0 : a + 1) + b * tx : a + (b + 1 == ty ? 0 : b + 1) * tx;
  const int enear = isx ? 3 : 1, efar = isx ? 2 : 0;  // E / S end of the near tile, W / N of the far
  const int R = g.urow;
  // Frustum strips of level m: the near tile's at across H - m (k = 0) and
  // H - m - 1, the far tile's at H + 1 + m and H + 2 + m; along m + t.
  auto strips = [&](int m) {
    return RectRuns{2,
                    {run(H - m, m, 0, 1, -1, 0, wal - 2 * m), run(H + 1 + m, m, 0, 1, 1, 0, wal - 2 * m), RectRun{},
                     RectRun{}},
                    {up + rect_up_at(g, NV, tnear, enear, m), up + rect_up_at(g, NV, tfar, efar, m), nullptr, nullptr},
                    {R, R, 0, 0}};
  };
  V* out = static_cast<V*>(isx ? pp.xb : pp.yb);
  const int Ro = isx ? 2 * g.h + 4 : 2 * g.h;
  auto at = [&](int end, int l) {
    return isx ? rect_xb_at(g, NV, e, end, l) : rect_yb_at(g, NV, e, end, l);
  };
  rect_copy_runs<S, NT>(buf(0), P, strips(0));
  if constexpr (WC != 0) {
    // Each level's strips are fetched during the level before and placed at
    // the start of their own; the runs are described once for all levels.
    constexpr int KR = rect_kr<S, WC, NT>();
    const int ss = 2 * NV * R;
    const RunLin sq[4] = {isx ? RunLin{H, 0, -1, 1, 0, 1, -1, 0, wal, -2, R, ss} : RunLin{0, H, 1, -1, 1, 0, 0, -1, wal, -2, R, ss},
                          isx ? RunLin{H + 1, 0, 1, 1, 0, 1, 1, 0, wal, -2, R, ss}
                              : RunLin{0, H + 1, 1, 1, 1, 0, 0, 1, wal, -2, R, ss},
                          RunLin{}, RunLin{}};
    const V* const ssrc[4] = {up + rect_up_at(g, NV, tnear, enear, 0), up + rect_up_at(g, NV, tfar, efar, 0), nullptr,
                              nullptr};
    const RunLanes<KR> sl[4] = {run_lanes<S, NT, KR>(sq[0], wal, P), run_lanes<S, NT, KR>(sq[1], wal, P),
                                RunLanes<KR>{}, RunLanes<KR>{}};
    RectFetch<V, KR> f;
    if (H > 1) lin_fetch<S, KR>(f, sl, sq, ssrc, 2, 1, P);
    __syncthreads();
    for (int l = 1; l <= H; ++l) {
      const V* in = buf(l - 1);
      if (l < H) {
        rect_place<S, KR>(f, buf(l));
        if (l + 1 < H) lin_fetch<S, KR>(f, sl, sq, ssrc, 2, l + 1, P);
      }
      if (isx)
        rect_level<S, WC, NT>(in, buf(l), P, H + 1 - l, l, 2 * l, wal - 2 * l, base + l - 1, sp);
      else
        rect_level<S, WC, NT>(in, buf(l), P, l, H + 1 - l, wal - 2 * l, 2 * l, base + l - 1, sp);
      __syncthreads();
    }
    // The ends of every level m, stored once all levels are done (their
    // cells stay untouched in buffer m mod 2: later levels of that parity
    // write only inside them), so that no level waits for panel stores
    // before it places its prefetched strips: rows (x-bridge) or columns
    // (y-bridge) m, m+1 and wal-1-m, wal-2-m of the tile; across, the
    // x-bridge's run covers its band and the frustum corners, the y-bridge's
    // its band only.
    const int os = 2 * NV * Ro;
    const RunLin eq[2] = {isx ? RunLin{H - 1, 0, -1, 1, 1, 0, 0, 1, 4, 2, Ro, os}
                              : RunLin{0, H + 1, 1, -1, 0, 1, 1, 0, 0, 2, Ro, os},
                          isx ? RunLin{H - 1, wal - 1, -1, -1, 1, 0, 0, -1, 4, 2, Ro, os}
                              : RunLin{wal - 1, H + 1, -1, -1, 0, 1, -1, 0, 0, 2, Ro, os}};
    const RunLanes<KR> el[2] = {run_lanes<S, NT, KR>(eq[0], 2 * H + 2, P), run_lanes<S, NT, KR>(eq[1], 2 * H + 2, P)};
    V* const eb[2] = {out + at(0, 0), out + at(1, 0)};
    for (int m = 0; m < H; ++m) {
      lin_emit<S, KR>(buf(m), el[0], eq[0], eb[0], m, P);
      lin_emit<S, KR>(buf(m), el[1], eq[1], eb[1], m, P);
    }
  } else {
    __syncthreads();
    for (int l = 1; l <= H; ++l) {
      const V* in = buf(l - 1);
      if (l < H) rect_copy_runs<S, NT>(buf(l), P, strips(l));
      if (isx)
        rect_level<S, WC, NT>(in, buf(l), P, H + 1 - l, l, 2 * l, wal - 2 * l, base + l - 1, sp);
      else
        rect_level<S, WC, NT>(in, buf(l), P, l, H + 1 - l, wal - 2 * l, 2 * l, base + l - 1, sp);
      __syncthreads();
    }
    // The ends of every level m, stored once all levels are done (as above).
    for (int m = 0; m < H; ++m) {
      V* in = buf(m);
      const int ac0 = isx ? H - m - 1 : H + 1 - m, len = isx ? 2 * m + 4 : 2 * m;
      rect_copy<S, NT, true>(in, P, run(ac0, m, 1, 0, 0, 1, len), out + at(0, m), Ro);
      rect_copy<S, NT, true>(in, P, run(ac0, wal - 1 - m, 1, 0, 0, -1, len), out + at(1, m), Ro);
    }
  }
  // the band at level H: across [1, 2H + 1), along [H, wal - H)
  if (isx) {
    const int E = sx + wx >= nx ? sx + wx - nx : sx + wx;
    rect_move<S, NT, false>(buf(H), P, state, nx, ny, 1, H, 2 * H, wal - 2 * H, E - H - 1, sy, 0, 0, 0);
  } else {
    const int F = sy + wy >= ny ? sy + wy - ny : sy + wy;
    rect_move<S, NT, false>(buf(H), P, state, nx, ny, H, 1, wal - 2 * H, 2 * H, sx, F - H - 1, 0, 0, 0);
  }
}

template <class S, int WC, int NT>
__global__ __launch_bounds__(NT) void k_rect_oct(RGeo g, int upar, int Hd, int Hu, typename S::V* __restrict__ state,
                                                 PanelPtrs pp, SchemeParams sp) {
  extern __shared__ double smem_d[];
  rect_oct_item<S, WC, NT>(g, upar, Hd, Hu, state, pp, sp, (int)blockIdx.x, reinterpret_cast<typename S::V*>(smem_d));
}

template <class S, int WC, int NT>
__global__ __launch_bounds__(NT) void k_rect_bridge(RGeo g, int par, int H, typename S::V* __restrict__ state,
                                                    PanelPtrs pp, SchemeParams sp) {
  extern __shared__ double smem_d[];
  rect_bridge_item<S, WC, NT>(g, par, H, state, pp, sp, (int)blockIdx.x, reinterpret_cast<typename S::V*>(smem_d));
}

// The instantiation that runs window pitch P: 66 and 34 for light schemes
// (rect_geo picks those pitches only for them), the run-time pitch otherwise,
// on 4 waves, or on 8 for the flux schemes' column walk from pitch 22 (tiles
// of 20 and more: Rusanov Euler on 511 x 509, full RK2 steps/s, height 12
// 5.6e9 on 4 waves, 6.4e9 on 8; height 6 6.3e9 and 3.7e9).
constexpr int kRectWalkWidePitch = 22;
template <class S, class F>
hipError_t rect_by_pitch(int P, F&& f) {
  if constexpr (Lay<S, 66>::light) {
    if (P == 66) return f(std::integral_constant<int, 66>{}, std::integral_constant<int, 1024>{});
    if (P == 34) return f(std::integral_constant<int, 34>{}, std::integral_constant<int, 256>{});
  }
  if constexpr (walks<S>::value) {
    if (P >= kRectWalkWidePitch) return f(std::integral_constant<int, 0>{}, std::integral_constant<int, 512>{});
  }
  return f(std::integral_constant<int, 0>{}, std::integral_constant<int, kRectThreads>{});
}

template <class S>
hipError_t rect_oct_t(const RGeo& g, int upar, int Hd, int Hu, void* state, PanelPtrs p, const SchemeParams& sp,
                      hipStream_t s) {
  if constexpr (S::NW != S::NV) {
    return hipErrorNotSupported;
  } else {
    const size_t lds = rect_lds_bytes(info_of<S>(), g);
    return rect_by_pitch<S>(g.P, [&](auto wc, auto nt) {
      hipLaunchKernelGGL((k_rect_oct<S, decltype(wc)::value, decltype(nt)::value>), dim3(rect_tiles(g)),
                         dim3(decltype(nt)::value), lds, s, g, upar, Hd, Hu, static_cast<typename S::V*>(state), p, sp);
      return hipGetLastError();
    });
  }
}

template <class S>
hipError_t rect_bridge_t(const RGeo& g, int par, int H, void* state, PanelPtrs p, const SchemeParams& sp,
                         hipStream_t s) {
  if constexpr (S::NW != S::NV) {
    return hipErrorNotSupported;
  } else {
    const size_t lds = rect_lds_bytes(info_of<S>(), g);
    return rect_by_pitch<S>(g.P, [&](auto wc, auto nt) {
      hipLaunchKernelGGL((k_rect_bridge<S, decltype(wc)::value, decltype(nt)::value>), dim3(2 * rect_tiles(g)),
                         dim3(decltype(nt)::value), lds, s, g, par, H, static_cast<typename S::V*>(state), p, sp);
      return hipGetLastError();
    });
  }
}

template <class S, int WC, int NT>
hipError_t rect_lds_one(int bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_rect_oct<S, WC, NT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_rect_bridge<S, WC, NT>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <class S>
hipError_t rect_lds_t(int bytes) {
  if constexpr (S::NW != S::NV) {
    return hipSuccess;
  } else {
    hipError_t e = rect_lds_one<S, 0, kRectThreads>(bytes);
    if constexpr (walks<S>::value) {
      if (e == hipSuccess) e = rect_lds_one<S, 0, 512>(bytes);
    }
    if constexpr (Lay<S, 66>::light) {
      if (e == hipSuccess) e = rect_lds_one<S, 66, 1024>(bytes);
      if (e == hipSuccess) e = rect_lds_one<S, 34, 256>(bytes);
    }
    return e;
  }
}
