#pragma once
// 2D matrix-free C0IP operator and fused smoother step for gfx950 (shared by
// op2d.hip and op2d_avs64.hip / op2d_avs32.hip, which instantiate them)
//
// Operator (Sec. 4, eq. c0iptensorvp used
// on the whole Cartesian mesh):
//   A x = (B (x) M + 2 L (x) L + M (x) B) x,  first factor along x,
// i.e. with X[j][i] (i = x index, fastest)
//   Y = M_y (X B_x) + 2 L_y (X L_x) + B_y (X M_x).
//
// One workgroup owns a tile of TY x TX output nodes (whole cells, so a
// node's position in its cell is its tile-local index mod k).  X is staged
// once, with a 2k-node halo, in LDS.  The three Kronecker terms are then
// applied one after the other through a single LDS buffer T:
//   T = X B_x  (rows the M_y band reaches),  acc  = M_y T,
//   T = X L_x,                              acc += 2 L_y T,
//   T = X M_x  (all staged rows),           acc += B_y T,
// with acc in registers.  Each pass needs the band coefficients of one 1D
// factor only, which keeps them in scalar registers on interior tiles (all
// rows of a tile in the periodic row classes); a factor whose bands exceed
// the scalar budget is applied in groups of cell positions.  Boundary tiles
// read per-lane row classes from the global table.
#include <algorithm>

#include "fdm.h"
#include "kernels.h"
#include "tiles.h"

namespace c0ip {
namespace {

using tile::Band;
using tile::band_row;
using tile::clampi;
using tile::stage_eig;

// Cell positions [p0, end) whose bands of factor OP fit the scalar budget
// (80 SGPRs of coefficients).
template <typename T, int OP, int K>
constexpr int group_end(int p0) {
  constexpr int budget = sizeof(T) == 8 ? 40 : 80;
  int s = 0, p = p0;
  while (p < K && s + Band<OP, K>::width(p) <= budget) s += Band<OP, K>::width(p++);
  return p == p0 ? p0 + 1 : p;
}


// Tile geometry: TXC x TYC cells, NTH threads, x items of CW cells, y items
// of RW cell rows.
template <int K_, int TXC_, int TYC_, int NTH_, int CW_, int RW_>
struct Geo {
  static constexpr int K = K_, TXC = TXC_, TYC = TYC_, NTH = NTH_, CW = CW_, RW = RW_;
  static constexpr int H = 2 * K, TX = TXC * K, TY = TYC * K, RX = TX + 2 * H, RY = TY + 2 * H, W = 4 * K + 1;
  static constexpr int NIT_Y = TX * (TYC / RW), NI = (NIT_Y + NTH - 1) / NTH;
  static constexpr int TABMAX = 3 * (5 * K + 2) * W;  // row classes: at most 5k+2
  static_assert(TXC % CW == 0 && TYC % RW == 0, "item sizes must divide the tile");
};

// T[r][.] = X[r][.] op_x for rows [r0, r1) and cell positions [P0, P1).
template <typename T, class G, int OP, int P0, int P1, bool XIN>
__device__ __forceinline__ void xpass(const T* __restrict__ sX, T* __restrict__ sT, int r0, int r1,
                                      const T* __restrict__ tab, const T* __restrict__ sTab, int nclass, int left,
                                      int right0, int periodic, int x0, int n1) {
  constexpr int K = G::K, CW = G::CW, H = G::H;
  constexpr int NG = G::TXC / CW;
  constexpr int LO = Band<OP, K>::win_lo(P0), HI = Band<OP, K>::win_hi() + (CW - 1) * K;
  const int nit = (r1 - r0) * NG;
  for (int it = threadIdx.x; it < nit; it += G::NTH) {
    const int rr = it / NG, g = it - rr * NG, r = r0 + rr;
    T in[HI - LO + 1];
#pragma unroll
    for (int j = LO; j <= HI; ++j) in[j - LO] = sX[r * G::RX + g * CW * K + j];
#pragma unroll
    for (int p = P0; p < P1; ++p) {
#pragma unroll
      for (int w = 0; w < CW; ++w) {
        const int cl = XIN ? 2 * left + p
                           : tile::row_class(clampi(x0 + (g * CW + w) * K + p, 0, n1 - 1), n1, K, left, right0,
                                             periodic);
        sT[r * G::TX + (g * CW + w) * K + p] = band_row<T, OP, K, XIN>(tab, sTab, nclass, left, periodic, cl, in + (w * K + p + H - LO), p);
      }
    }
  }
}

template <typename T, class G, int OP, int P0, bool XIN>
__device__ __forceinline__ void xpass_all(const T* __restrict__ sX, T* __restrict__ sT, int r0, int r1,
                                          const T* __restrict__ tab, const T* __restrict__ sTab, int nclass,
                                          int left, int right0, int periodic, int x0, int n1) {
  constexpr int P1 = group_end<T, OP, G::K>(P0);
  xpass<T, G, OP, P0, P1, XIN>(sX, sT, r0, r1, tab, sTab, nclass, left, right0, periodic, x0, n1);
  if constexpr (P1 < G::K)
    xpass_all<T, G, OP, P1, XIN>(sX, sT, r0, r1, tab, sTab, nclass, left, right0, periodic, x0, n1);
}

// acc (+)= scale * op_y T for cell positions [P0, P1) of every y item.
template <typename T, class G, int OP, int P0, int P1, bool YIN, bool SET>
__device__ __forceinline__ void ypass(const T* __restrict__ sT, T (&acc)[G::NI][G::RW * G::K], T scale,
                                      const T* __restrict__ tab, const T* __restrict__ sTab, int nclass, int left,
                                      int right0, int periodic, int y0, int n1) {
  constexpr int K = G::K, RW = G::RW, H = G::H, TX = G::TX;
  constexpr int LO = Band<OP, K>::win_lo(P0), HI = Band<OP, K>::win_hi() + (RW - 1) * K;
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * G::NTH;
    if (G::NIT_Y % G::NTH != 0 && it >= G::NIT_Y) break;
    const int cg = it / TX, l = it - cg * TX;
    T t[HI - LO + 1];
#pragma unroll
    for (int j = LO; j <= HI; ++j) t[j - LO] = sT[(cg * RW * K + j) * TX + l];
#pragma unroll
    for (int p = P0; p < P1; ++p) {
#pragma unroll
      for (int w = 0; w < RW; ++w) {
        const int cl = YIN ? 2 * left + p
                           : tile::row_class(clampi(y0 + (cg * RW + w) * K + p, 0, n1 - 1), n1, K, left, right0,
                                             periodic);
        const T a = band_row<T, OP, K, YIN>(tab, sTab, nclass, left, periodic, cl, t + (w * K + p + H - LO), p);
        acc[q][w * K + p] = SET ? scale * a : acc[q][w * K + p] + scale * a;
      }
    }
  }
}

template <typename T, class G, int OP, int P0, bool YIN, bool SET>
__device__ __forceinline__ void ypass_all(const T* __restrict__ sT, T (&acc)[G::NI][G::RW * G::K], T scale,
                                          const T* __restrict__ tab, const T* __restrict__ sTab, int nclass,
                                          int left, int right0, int periodic, int y0, int n1) {
  constexpr int P1 = group_end<T, OP, G::K>(P0);
  ypass<T, G, OP, P0, P1, YIN, SET>(sT, acc, scale, tab, sTab, nclass, left, right0, periodic, y0, n1);
  if constexpr (P1 < G::K)
    ypass_all<T, G, OP, P1, YIN, SET>(sT, acc, scale, tab, sTab, nclass, left, right0, periodic, y0, n1);
}

// acc = (A X) on the tile's output nodes, X staged in sX and, on tiles
// that are not interior in both directions, the coefficient table in sTab
// (a barrier after the staging is the caller's); sT is overwritten.  Ends
// after the last y pass (no barrier).
template <typename T, class G, bool XIN, bool YIN>
__device__ __forceinline__ void op_tile(const T* __restrict__ sX, T* __restrict__ sT, T (&acc)[G::NI][G::RW * G::K],
                                        const T* __restrict__ tab, const T* __restrict__ sTab, int nclass, int left,
                                        int right0, int periodic, int x0, int y0, int n1) {
  constexpr int K = G::K, RY = G::RY;
  xpass_all<T, G, 2, 0, XIN>(sX, sT, K, RY - K, tab, sTab, nclass, left, right0, periodic, x0, n1);
  __syncthreads();
  ypass_all<T, G, 0, 0, YIN, true>(sT, acc, T(1), tab, sTab, nclass, left, right0, periodic, y0, n1);
  __syncthreads();
  xpass_all<T, G, 1, 0, XIN>(sX, sT, K, RY - K, tab, sTab, nclass, left, right0, periodic, x0, n1);
  __syncthreads();
  ypass_all<T, G, 1, 0, YIN, false>(sT, acc, T(2), tab, sTab, nclass, left, right0, periodic, y0, n1);
  __syncthreads();
  xpass_all<T, G, 0, 0, XIN>(sX, sT, 0, RY, tab, sTab, nclass, left, right0, periodic, x0, n1);
  __syncthreads();
  ypass_all<T, G, 2, 0, YIN, false>(sT, acc, T(1), tab, sTab, nclass, left, right0, periodic, y0, n1);
}

template <class G>
__device__ __forceinline__ bool tile_xin(int periodic, int left, int right0, int x0) {
  return periodic && x0 >= left && x0 + G::TX <= right0;
}
template <class G>
__device__ __forceinline__ bool tile_yin(int periodic, int left, int right0, int y0) {
  return periodic && y0 >= left && y0 + G::TY <= right0;
}

// Copy the coefficient table to LDS on tiles that need per-lane classes.
// Here and in the other staging helpers every global load of a thread is
// issued before its first LDS store, so that the loads' latencies overlap.
template <typename T, class G>
__device__ __forceinline__ void stage_tab(const T* __restrict__ tab, T* __restrict__ sTab, int nclass, bool need) {
  if (!need) return;
  constexpr int NL = (G::TABMAX + G::NTH - 1) / G::NTH;
  const int cnt = 3 * nclass * G::W;
  T v[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = threadIdx.x + q * G::NTH;
    v[q] = e < cnt ? tab[e] : T(0);
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = threadIdx.x + q * G::NTH;
    if (e < cnt) sTab[e] = v[q];
  }
}


template <typename T, class G>
__device__ __forceinline__ void op_tile_any(const T* __restrict__ sX, T* __restrict__ sT,
                                            T (&acc)[G::NI][G::RW * G::K], const T* __restrict__ tab,
                                            const T* __restrict__ sTab, int nclass, int left, int right0,
                                            int periodic, int x0, int y0, int n1) {
  const bool xin = tile_xin<G>(periodic, left, right0, x0), yin = tile_yin<G>(periodic, left, right0, y0);
  if (xin && yin)
    op_tile<T, G, true, true>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
  else if (xin)
    op_tile<T, G, true, false>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
  else if (yin)
    op_tile<T, G, false, true>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
  else
    op_tile<T, G, false, false>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
}

// Stage X on [x0 - 2k, x0 + TX + 2k) x [y0 - 2k, y0 + TY + 2k) (zero outside the mesh).
template <typename Tin, typename T, class G>
__device__ __forceinline__ void stage_x(const Tin* __restrict__ x, T* __restrict__ sX, int x0, int y0, int n1) {
  constexpr int NL = (G::RY * G::RX + G::NTH - 1) / G::NTH;
  T v[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = threadIdx.x + q * G::NTH;
    const int r = e / G::RX, c = e - r * G::RX;
    const int gy = y0 - G::H + r, gx = x0 - G::H + c;
    v[q] = (e < G::RY * G::RX && gy >= 0 && gy < n1 && gx >= 0 && gx < n1) ? (T)x[(size_t)gy * n1 + gx] : T(0);
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = threadIdx.x + q * G::NTH;
    if (e < G::RY * G::RX) sX[e] = v[q];
  }
}

template <typename Tin, typename T, class G, bool RES>
__global__ __launch_bounds__(G::NTH) void apply2d_kernel(const Tin* __restrict__ x, const T* __restrict__ b,
                                                         T* __restrict__ y, int n1, const T* __restrict__ tab,
                                                         int nclass, int left, int right0, int periodic, int64_t zs,
                                                         const int* __restrict__ active, tile::TileOrder ord,
                                                         Tin* __restrict__ xc) {
  if (active && !active[blockIdx.z]) return;
  int bx, by;
  if (!tile::tile_of_block(ord, blockIdx.x, bx, by)) return;
  x += blockIdx.z * zs;
  y += blockIdx.z * zs;
  if (RES) b += blockIdx.z * zs;
  __shared__ T sX[G::RY * G::RX];
  __shared__ T sT[G::RY * G::TX];
  __shared__ T sTab[G::TABMAX];
  const int x0 = bx * G::TX, y0 = by * G::TY;
  stage_x<Tin, T, G>(x, sX, x0, y0, n1);
  stage_tab<T, G>(tab, sTab, nclass,
                  !(tile_xin<G>(periodic, left, right0, x0) && tile_yin<G>(periodic, left, right0, y0)));
  // b of the outputs (residual form), loaded now to overlap the passes
  T bv[RES ? G::NI : 1][G::RW * G::K];
  if constexpr (RES) {
#pragma unroll
    for (int q = 0; q < G::NI; ++q) {
      const int it = threadIdx.x + q * G::NTH;
      const int cg = it / G::TX, l = it - cg * G::TX;
      const int gx = x0 + l;
#pragma unroll
      for (int w = 0; w < G::RW * G::K; ++w) {
        const int gy = y0 + cg * G::RW * G::K + w;
        const bool inner = it < G::NIT_Y && gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2;
        bv[q][w] = inner ? b[(size_t)gy * n1 + gx] : T(0);
      }
    }
  }
  T acc[G::NI][G::RW * G::K];
  __syncthreads();
  op_tile_any<T, G>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * G::NTH;
    if (G::NIT_Y % G::NTH != 0 && it >= G::NIT_Y) break;
    const int cg = it / G::TX, l = it - cg * G::TX;
    const int gx = x0 + l;
#pragma unroll
    for (int w = 0; w < G::RW * G::K; ++w) {
      const int gy = y0 + cg * G::RW * G::K + w;
      if (gx < n1 && gy < n1) {
        const size_t idx = (size_t)gy * n1 + gx;
        if (xc) xc[idx] = (Tin)sX[(cg * G::RW * G::K + w + G::H) * G::RX + l + G::H];  // exact: T holds every Tin
        if constexpr (RES) {
          const bool bnd = gx == 0 || gy == 0 || gx == n1 - 1 || gy == n1 - 1;
          y[idx] = bnd ? T(0) : bv[q][w] - acc[q][w];
        } else {
          y[idx] = acc[q][w];
        }
      }
    }
  }
}

// Tile configuration of the operator per degree: TXC x TYC cells, threads,
// x items of CW cells, y items of RW cell rows.
template <int K> struct ApplyCfg;
template <> struct ApplyCfg<2> { using G = Geo<2, 24, 12, 256, 2, 2>; };
template <> struct ApplyCfg<3> { using G = Geo<3, 16, 8, 256, 2, 2>; };
template <> struct ApplyCfg<4> { using G = Geo<4, 12, 6, 256, 2, 2>; };
template <> struct ApplyCfg<5> { using G = Geo<5, 8, 4, 256, 2, 2>; };
template <> struct ApplyCfg<6> { using G = Geo<6, 8, 4, 256, 2, 2>; };
template <> struct ApplyCfg<7> { using G = Geo<7, 6, 4, 256, 2, 2>; };

// Small meshes (fewer big tiles than compute units) are latency bound: a
// one-wave workgroup per small tile shortens each block's chain of passes
// and spreads the mesh over more compute units.
template <int K> struct ApplyCfgSmall;
template <> struct ApplyCfgSmall<2> { using G = Geo<2, 6, 6, 64, 2, 2>; };
template <> struct ApplyCfgSmall<3> { using G = Geo<3, 4, 4, 64, 2, 2>; };
template <> struct ApplyCfgSmall<4> { using G = Geo<4, 4, 4, 64, 2, 2>; };
template <> struct ApplyCfgSmall<5> { using G = Geo<5, 2, 2, 64, 2, 2>; };
template <> struct ApplyCfgSmall<6> { using G = Geo<6, 2, 2, 64, 2, 2>; };
template <> struct ApplyCfgSmall<7> { using G = Geo<7, 2, 2, 64, 2, 2>; };

template <typename Tin, typename T, class G>
hipError_t apply2d_g(int n1, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s, int nsys,
                     int64_t zs, const int* active, Tin* xc) {
  if (xc && nsys != 1) return hipErrorInvalidValue;
  const int tx = (n1 + G::TX - 1) / G::TX, ty = (n1 + G::TY - 1) / G::TY;
  const tile::TileOrder ord = tile::make_order(
      tx, ty, [&](int bx) { return c.periodic && bx * G::TX >= c.left && bx * G::TX + G::TX <= c.right0; },
      [&](int by) { return c.periodic && by * G::TY >= c.left && by * G::TY + G::TY <= c.right0; });
  const dim3 grid(tile::order_blocks(ord), 1, nsys);
  if (b)
    apply2d_kernel<Tin, T, G, true><<<grid, G::NTH, 0, s>>>(x, b, y, n1, c.tab, c.nclass, c.left, c.right0,
                                                            c.periodic, zs, active, ord, xc);
  else
    apply2d_kernel<Tin, T, G, false><<<grid, G::NTH, 0, s>>>(x, b, y, n1, c.tab, c.nclass, c.left, c.right0,
                                                             c.periodic, zs, active, ord, xc);
  return hipGetLastError();
}

template <typename Tin, typename T, int K>
hipError_t apply2d_k(int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s, int nsys,
                     int64_t zs, const int* active, Tin* xc) {
  using G = typename ApplyCfg<K>::G;
  const int n1 = K * N + 1;
  const int64_t big = (int64_t)((n1 + G::TX - 1) / G::TX) * ((n1 + G::TY - 1) / G::TY) * nsys;
  if (big < 256) return apply2d_g<Tin, T, typename ApplyCfgSmall<K>::G>(n1, c, x, b, y, s, nsys, zs, active, xc);
  return apply2d_g<Tin, T, G>(n1, c, x, b, y, s, nsys, zs, active, xc);
}

// ------------------------------------------------------------------ smoother
// One step of the additive vertex-patch smoother (Sec. 3; local solver of
// eq. localsolverbila inverted by eq. inverse):
//   x_out = x + omega * sum_v R_v^T (Q_y (x) Q_x) D_v^{-1} (Q_y (x) Q_x)^T R_v (b - A x),
// fused in one launch.  A workgroup owns TC x TC cells; the residual on the
// owned tile extended by one cell (the support of every patch touching the
// tile) is computed with the operator's passes above and kept in LDS; the
// (TC+1)^2 patches touching the tile are solved there (neighbouring tiles
// solve shared patches twice instead of racing on writes) and each owned
// DoF is written once, summing its covering patches (owner computes; no
// atomics, deterministic).  The patch solves run in place in one LDS buffer
// (forward along x, then along y with the division by lambda_x + lambda_y
// and back, then back along x).  On interior tiles every patch has the
// interior eigenbasis: its reciprocal eigenvalue sums are tabulated once per
// workgroup and the basis is read with wave-uniform addresses.
template <typename T, int K_, int TC_, int NTH_>
struct SmGeo {
  static constexpr int K = K_, TC = TC_, NTH = NTH_;
  using G = Geo<K, TC + 2, TC + 2, NTH, 2, 2>;
  static constexpr int n = 2 * K - 1, NN = n * n, NP = TC + 1;
  static constexpr int SZA = G::RY * G::RX + G::RY * G::TX, SZB = NP * NP * NN;
  // coarse nodes per side of the staged region, and the prolongation scratch
  // (coarse values and their x-pass) placed after the staged x
  static constexpr int CX = ((G::RX - 1) / (2 * K) + 2) * K + 1;
  static constexpr int SZP = G::RY * G::RX + CX * CX + CX * G::RX;
  static constexpr int POOL = SZA > SZB ? SZA : SZB;
  static constexpr int POOLP = POOL > SZP ? POOL : SZP;
  // eigenbasis through scalar registers when it fits 64 of them
  static constexpr bool QS = NN * (int)sizeof(T) / 4 <= 64;
};

template <typename T, class S, bool INTERIOR>
__device__ __forceinline__ void patch_solves(const T* __restrict__ sRr, T* __restrict__ sA, const T* __restrict__ Qg,
                                             const T* __restrict__ sQ, const T* __restrict__ sLam,
                                             const T* __restrict__ sD, int N, int cx0, int cy0) {
  constexpr int K = S::K, n = S::n, NN = S::NN, NP = S::NP, TX = S::G::TX, NTH = S::NTH;
  const T* Q0 = (INTERIOR && S::QS) ? Qg : sQ;
  // forward along x: A[a][c] = sum_c' Qx[c'][c] r[a][c']
  for (int it = threadIdx.x; it < NP * NP * n; it += NTH) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const T* q = INTERIOR ? Q0 : sQ + tile::variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sRr[(pyl * K + 1 + a) * TX + pxl * K + 1 + c];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int cp = 0; cp < n; ++cp) s += q[cp * n + c] * in[cp];
      sA[p * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  // along y, in place per column: forward with Qy^T, scale, back with Qy
  for (int it = threadIdx.x; it < NP * NP * n; it += NTH) {
    const int p = it / n, c = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const int ty = INTERIOR ? 0 : tile::variant(vy, N), tx = INTERIOR ? 0 : tile::variant(vx, N);
    const T* q = INTERIOR ? Q0 : sQ + ty * NN;
    T col[n], t[n];
#pragma unroll
    for (int a = 0; a < n; ++a) col[a] = sA[p * NN + a * n + c];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += q[a * n + ap] * col[a];
      // the same rounding on every path: s times the rounded reciprocal
      t[ap] = s * (INTERIOR ? sD[ap * n + c] : T(1) / (sLam[tx * n + c] + sLam[ty * n + ap]));
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += q[a * n + ap] * t[ap];
      sA[p * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  // back along x, in place per row: A[a][c'] = sum_c Qx[c'][c] A[a][c]
  for (int it = threadIdx.x; it < NP * NP * n; it += NTH) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const T* q = INTERIOR ? Q0 : sQ + tile::variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sA[p * NN + a * n + c];
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += q[cp * n + c] * in[c];
      sA[p * NN + a * n + cp] = s;
    }
  }
  __syncthreads();
}

// sX += (P ec) on the staged region (fine nodes [x0 - 2k, ..) x [y0 - 2k, ..)):
// the coarse values covering it are staged in sC, interpolated along x into
// sP, then along y (the 1D embedding table T[s][p][a]: coarse-cell basis a
// at position p of fine cell 2 cc + s).  P ec is 0 on the mesh boundary.
// Ends with a barrier.
template <typename T, class S>
__device__ __forceinline__ void prolong_into(T* __restrict__ sX, T* __restrict__ sC, T* __restrict__ sP,
                                             T* __restrict__ sPT, const T* __restrict__ ec,
                                             const T* __restrict__ ptab, int nf, int x0, int y0) {
  using G = typename S::G;
  constexpr int K = S::K, CX = S::CX, RX = G::RX, RY = G::RY, NTH = S::NTH, NT = 2 * K * (K + 1);
  const int nc = (nf - 1) / 2 + 1;
  const int f0x = x0 - G::H, f0y = y0 - G::H;
  const int cxl = ((f0x > 0 ? f0x : 0) / K >> 1) * K, cyl = ((f0y > 0 ? f0y : 0) / K >> 1) * K;
  {
    constexpr int NLC = (CX * CX + NTH - 1) / NTH, NLT = (NT + NTH - 1) / NTH;
    T v[NLC], t[NLT];
#pragma unroll
    for (int q = 0; q < NLC; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int r = e / CX, c = e - r * CX;
      const int gy = cyl + r, gx = cxl + c;
      v[q] = (e < CX * CX && gy < nc && gx < nc) ? ec[(size_t)gy * nc + gx] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NLT; ++q) {
      const int e = threadIdx.x + q * NTH;
      t[q] = e < NT ? ptab[e] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NLC; ++q) {
      const int e = threadIdx.x + q * NTH;
      if (e < CX * CX) sC[e] = v[q];
    }
#pragma unroll
    for (int q = 0; q < NLT; ++q) {
      const int e = threadIdx.x + q * NTH;
      if (e < NT) sPT[e] = t[q];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < CX * RX; e += NTH) {
    const int r = e / RX, c = e - r * RX;
    const int f = f0x + c;
    T v = 0;
    if (f >= 1 && f <= nf - 2) {
      const int cf = f / K, p = f - cf * K, cc = cf >> 1, sh = cf & 1;
      const T* tb = sPT + (sh * K + p) * (K + 1);
      const T* src = sC + r * CX + cc * K - cxl;
#pragma unroll
      for (int a = 0; a <= K; ++a) v += tb[a] * src[a];
    }
    sP[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RY * RX; e += NTH) {
    const int r = e / RX, c = e - r * RX;
    const int f = f0y + r;
    if (f >= 1 && f <= nf - 2) {
      const int cf = f / K, p = f - cf * K, cc = cf >> 1, sh = cf & 1;
      const T* tb = sPT + (sh * K + p) * (K + 1);
      const T* src = sP + (cc * K - cyl) * RX + c;
      T v = 0;
#pragma unroll
      for (int a = 0; a <= K; ++a) v += tb[a] * src[a * RX];
      sX[e] += v;
    }
  }
  __syncthreads();
}

template <typename T, class S, bool PRO>
__global__ __launch_bounds__(S::NTH) void avs2d_kernel(const T* __restrict__ x, const T* __restrict__ b,
                                                       T* __restrict__ xout, int N, int n1, const T* __restrict__ tab,
                                                       int nclass, int left, int right0, int periodic,
                                                       const T* __restrict__ Qg, const T* __restrict__ lamg, T omega,
                                                       int64_t zs, const int* __restrict__ active,
                                                       tile::TileOrder ord, const T* __restrict__ ec,
                                                       const T* __restrict__ ptab, int64_t zc) {
  using G = typename S::G;
  constexpr int K = S::K, TC = S::TC, n = S::n, NN = S::NN, NP = S::NP, NTH = S::NTH;
  __shared__ T pool[PRO ? S::POOLP : S::POOL];
  __shared__ T sRr[G::TY * G::TX];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  __shared__ T sD[NN];
  __shared__ T sTab[G::TABMAX];
  __shared__ T sPT[PRO ? 2 * K * (K + 1) : 1];
  if (active && !active[blockIdx.z]) return;
  int tbx, tby;
  if (!tile::tile_of_block(ord, blockIdx.x, tbx, tby)) return;
  x += blockIdx.z * zs;
  b += blockIdx.z * zs;
  xout += blockIdx.z * zs;
  if (PRO) ec += blockIdx.z * zc;
  const int cx0 = tbx * TC, cy0 = tby * TC;
  const int x0 = (cx0 - 1) * K, y0 = (cy0 - 1) * K;  // residual tile origin (a vertex node)
  T* sX = pool;
  T* sT = pool + G::RY * G::RX;
  stage_x<T, T, G>(x, sX, x0, y0, n1);
  stage_tab<T, G>(tab, sTab, nclass,
                  !(tile_xin<G>(periodic, left, right0, x0) && tile_yin<G>(periodic, left, right0, y0)));
  stage_eig<T, n, NTH>(Qg, lamg, sQ, sLam, sD);
  // b on the residual tile, loaded now so that its latency overlaps the passes
  T bv[G::NI][G::RW * K];
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * NTH;
    const int cg = it / G::TX, l = it - cg * G::TX;
    const int gx = x0 + l;
#pragma unroll
    for (int w = 0; w < G::RW * K; ++w) {
      const int gy = y0 + cg * G::RW * K + w;
      const bool inner = it < G::NIT_Y && gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2;
      bv[q][w] = inner ? b[(size_t)gy * n1 + gx] : T(0);
    }
  }
  T acc[G::NI][G::RW * K];
  // x_in = x + P ec (the first post-smoothing step of a V-cycle level)
  if (PRO)
    prolong_into<T, S>(sX, pool + G::RY * G::RX, pool + G::RY * G::RX + S::CX * S::CX, sPT, ec, ptab, n1, x0, y0);
  __syncthreads();
  op_tile_any<T, G>(sX, sT, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
  // residual r = b - A x on the tile (0 on and outside the boundary)
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * NTH;
    if (G::NIT_Y % NTH != 0 && it >= G::NIT_Y) break;
    const int cg = it / G::TX, l = it - cg * G::TX;
    const int gx = x0 + l;
#pragma unroll
    for (int w = 0; w < G::RW * K; ++w) {
      const int rt = cg * G::RW * K + w, gy = y0 + rt;
      const bool inner = gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2;
      sRr[rt * G::TX + l] = inner ? bv[q][w] - acc[q][w] : T(0);
    }
  }
  // x at the owned nodes, from the staged tile before the patch solves reuse it
  constexpr int OW = TC * K + 1, NG = (OW * OW + NTH - 1) / NTH;
  T xv[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int e = threadIdx.x + q * NTH;
    const int jj = e / OW, ii = e - jj * OW;
    xv[q] = e < OW * OW ? sX[(jj + K + G::H) * G::RX + ii + K + G::H] : T(0);
  }
  __syncthreads();
  const bool interior = cx0 >= 2 && cx0 + TC <= N - 2 && cy0 >= 2 && cy0 + TC <= N - 2;
  T* sA = pool;
  if (interior)
    patch_solves<T, S, true>(sRr, sA, Qg, sQ, sLam, sD, N, cx0, cy0);
  else
    patch_solves<T, S, false>(sRr, sA, Qg, sQ, sLam, sD, N, cx0, cy0);
  // owned DoFs: x + omega * (sum of the covering patches' corrections)
  const int gx0 = cx0 * K, gy0 = cy0 * K;
  const int gx1 = (cx0 + TC >= N) ? n1 : (cx0 + TC) * K;
  const int gy1 = (cy0 + TC >= N) ? n1 : (cy0 + TC) * K;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int e = threadIdx.x + q * NTH;
    if (e >= OW * OW) break;
    const int jj = e / OW, ii = e - jj * OW;
    const int gx = gx0 + ii, gy = gy0 + jj;
    if (gx >= gx1 || gy >= gy1) continue;
    const size_t idx = (size_t)gy * n1 + gx;
    if (gx == 0 || gx == n1 - 1 || gy == 0 || gy == n1 - 1) {
      xout[idx] = T(0);
      continue;
    }
    const int vxa = gx / K, vxb = (gx % K == 0) ? vxa : vxa + 1;
    const int vya = gy / K, vyb = (gy % K == 0) ? vya : vya + 1;
    T a = 0;
    for (int vy = vya; vy <= vyb; ++vy) {
      if (vy < 1 || vy > N - 1) continue;
      for (int vx = vxa; vx <= vxb; ++vx) {
        if (vx < 1 || vx > N - 1) continue;
        const int p = (vy - cy0) * NP + (vx - cx0);
        const int c = gx - ((vx - 1) * K + 1), r = gy - ((vy - 1) * K + 1);
        a += sA[p * NN + r * n + c];
      }
    }
    xout[idx] = xv[q] + omega * a;
  }
}

// Tile sizes (owned cells per side) the fused smoother is compiled for;
// variant 0 is the default, the autotuner may pick any of them per level.
// ------------------------------------------------------------- pre-smoothing
// The first pre-smoothing step of a V-cycle level and the residual after it,
// in one launch:  x1 = S(0, b) = omega sum_v R_v^T A~_v^{-1} R_v b  and
// r = b - A x1.  A workgroup owns TC x TC cells.  The residual on its nodes
// needs x1 on the tile extended by 2k nodes (two cells), so the workgroup
// solves every patch covering that region ((TC + 5)^2 patches, from b
// staged on the tile extended by three cells), sums their corrections into
// the operator's staged input, and applies the operator's passes.  x1 and r
// are written on the owned nodes only (owner computes, deterministic).
// The patches of neighbouring tiles are solved redundantly instead of
// passing x1 through HBM and a second launch.
template <typename T, int K_, int TC_, int NTH_>
struct PreGeo {
  static constexpr int K = K_, TC = TC_, NTH = NTH_;
  using G = Geo<K, TC, TC, NTH, 2, 2>;
  static constexpr int n = 2 * K - 1, NN = n * n;
  static constexpr int NV = TC + 5;               // patches per direction (vertices cx0-2 .. cx0+TC+2)
  static constexpr int SB = (TC + 6) * K - 1;     // staged b per direction: nodes (cx0-3)K+1 ..
  static constexpr int REG_A = SB * SB > G::RY * G::RX ? SB * SB : G::RY * G::RX;   // b, then x1 (operator input)
  static constexpr int REG_B = NV * NV * NN > G::RY * G::TX ? NV * NV * NN : G::RY * G::TX;  // corrections, then T
  static constexpr bool OK = NN <= 25;  // register patch solves (k <= 3; measured slower above)
};

template <typename T, class S>
__global__ __launch_bounds__(S::NTH) void pre2d_kernel(const T* __restrict__ b, T* __restrict__ x1out,
                                                       T* __restrict__ rout, int N, int n1, const T* __restrict__ tab,
                                                       int nclass, int left, int right0, int periodic,
                                                       const T* __restrict__ Qg, const T* __restrict__ lamg, T omega,
                                                       tile::TileOrder ord) {
  using G = typename S::G;
  constexpr int K = S::K, TC = S::TC, n = S::n, NN = S::NN, NV = S::NV, SB = S::SB, NTH = S::NTH;
  __shared__ T regA[S::REG_A];
  __shared__ T regB[S::REG_B];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  __shared__ T sD[NN];
  __shared__ T sTab[G::TABMAX];
  int tbx, tby;
  if (!tile::tile_of_block(ord, blockIdx.x, tbx, tby)) return;
  const int cx0 = tbx * TC, cy0 = tby * TC;
  const int x0 = cx0 * K, y0 = cy0 * K;  // operator tile origin (owned nodes)
  const int bx0 = (cx0 - 3) * K + 1, by0 = (cy0 - 3) * K + 1;  // staged b origin
  // b on the staged region (0 outside the interior nodes)
  {
    constexpr int NLB = (SB * SB + NTH - 1) / NTH;
    T v[NLB];
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      const int e = threadIdx.x + q * NTH;
      const int rr = e / SB, cc = e - rr * SB;
      const int gy = by0 + rr, gx = bx0 + cc;
      v[q] = (e < SB * SB && gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2) ? b[(size_t)gy * n1 + gx] : T(0);
    }
    stage_eig<T, n, NTH>(Qg, lamg, sQ, sLam, sD);
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      const int e = threadIdx.x + q * NTH;
      if (e < SB * SB) regA[e] = v[q];
    }
  }
  stage_tab<T, G>(tab, sTab, nclass,
                  !(tile_xin<G>(periodic, left, right0, x0) && tile_yin<G>(periodic, left, right0, y0)));
  __syncthreads();
  // patch solves for the vertices cx0-2+i, cy0-2+j (i, j < NV) inside the mesh
  const bool interior = cx0 >= 4 && cx0 + TC <= N - 4 && cy0 >= 4 && cy0 + TC <= N - 4;
  for (int p = threadIdx.x; p < NV * NV; p += NTH) {
    const int pyl = p / NV, pxl = p - pyl * NV;
    const int vx = cx0 - 2 + pxl, vy = cy0 - 2 + pyl;
    if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
    // patch nodes start at (v-1)K+1 = staged origin + (pxl) K
    const T* src = regA + (pyl * K) * SB + pxl * K;
    if (interior) {
      fdm::patch_reg<T, n>(src, SB, regB + p * NN, [&](int i) { return Qg[i]; }, [&](int i) { return Qg[i]; },
                           [&](int ap, int c) { return sD[ap * n + c]; });
    } else {
      const int tx = tile::variant(vx, N), ty = tile::variant(vy, N);
      const T* qx = sQ + tx * NN;
      const T* qy = sQ + ty * NN;
      const T* lx = sLam + tx * n;
      const T* ly = sLam + ty * n;
      fdm::patch_reg<T, n>(src, SB, regB + p * NN, [&](int i) { return qx[i]; }, [&](int i) { return qy[i]; },
                           [&](int ap, int c) { return T(1) / (lx[c] + ly[ap]); });
    }
  }
  // b on the owned nodes, kept in registers for the residual (regA is overwritten next)
  T bv[G::NI][G::RW * K];
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * NTH;
    const int cg = it / G::TX, l = it - cg * G::TX;
#pragma unroll
    for (int w = 0; w < G::RW * K; ++w) {
      const int rt = cg * G::RW * K + w;
      // owned node (x0 + l, y0 + rt) = staged b index (3K - 1 + rt, 3K - 1 + l)
      bv[q][w] = it < G::NIT_Y ? regA[(3 * K - 1 + rt) * SB + 3 * K - 1 + l] : T(0);
    }
  }
  __syncthreads();
  // x1 = omega * sum of covering corrections on the operator's staged region
  // (nodes x0 - 2K .. x0 + TC K + 2K), 0 outside the interior nodes
  T* sX = regA;
  for (int e = threadIdx.x; e < G::RY * G::RX; e += NTH) {
    const int rr = e / G::RX, cc = e - rr * G::RX;
    const int gx = x0 - G::H + cc, gy = y0 - G::H + rr;
    T a = 0;
    if (gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2) {
      const int vxa = gx / K, vxb = (gx % K == 0) ? vxa : vxa + 1;
      const int vya = gy / K, vyb = (gy % K == 0) ? vya : vya + 1;
      for (int vy = vya; vy <= vyb; ++vy) {
        if (vy < 1 || vy > N - 1) continue;
        for (int vx = vxa; vx <= vxb; ++vx) {
          if (vx < 1 || vx > N - 1) continue;
          const int p = (vy - cy0 + 2) * NV + (vx - cx0 + 2);
          const int c = gx - ((vx - 1) * K + 1), r = gy - ((vy - 1) * K + 1);
          a += regB[p * NN + r * n + c];
        }
      }
      a *= omega;
    }
    sX[e] = a;
  }
  __syncthreads();
  T acc[G::NI][G::RW * K];
  op_tile_any<T, G>(sX, regB, acc, tab, sTab, nclass, left, right0, periodic, x0, y0, n1);
#pragma unroll
  for (int q = 0; q < G::NI; ++q) {
    const int it = threadIdx.x + q * NTH;
    if (G::NIT_Y % NTH != 0 && it >= G::NIT_Y) break;
    const int cg = it / G::TX, l = it - cg * G::TX;
    const int gx = x0 + l;
#pragma unroll
    for (int w = 0; w < G::RW * K; ++w) {
      const int rt = cg * G::RW * K + w, gy = y0 + rt;
      if (gx < n1 && gy < n1) {
        const size_t idx = (size_t)gy * n1 + gx;
        const bool bnd = gx == 0 || gy == 0 || gx == n1 - 1 || gy == n1 - 1;
        rout[idx] = bnd ? T(0) : bv[q][w] - acc[q][w];
        x1out[idx] = bnd ? T(0) : sX[(rt + G::H) * G::RX + l + G::H];
      }
    }
  }
}

template <int K> struct PreTile { static constexpr int TC = K <= 2 ? 8 : 4; };

template <typename T, int K>
hipError_t pre2d_k(int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* b, T* x1, T* r, T omega,
                   hipStream_t s) {
  if constexpr (!PreGeo<T, K, PreTile<K>::TC, 256>::OK) {
    return hipErrorNotSupported;
  } else {
    constexpr int TC = PreTile<K>::TC;
    using S = PreGeo<T, K, TC, 256>;
    using G = typename S::G;
    const int n1 = K * N + 1;
    // tiles over the nodes (the last one holds the boundary node k N), as for the operator
    const int nt = (n1 + G::TX - 1) / G::TX;
    auto in = [&](int bt) { return c.periodic && bt * G::TX >= c.left && bt * G::TX + G::TX <= c.right0; };
    const tile::TileOrder ord = tile::make_order(nt, nt, in, in);
    pre2d_kernel<T, S><<<tile::order_blocks(ord), S::NTH, 0, s>>>(b, x1, r, N, n1, c.tab, c.nclass, c.left, c.right0,
                                                                   c.periodic, e.Q, e.lam, omega, ord);
    return hipGetLastError();
  }
}

template <int K> struct FusedTiles;
template <> struct FusedTiles<2> { static constexpr int n = 3, tc[3] = {16, 8, 24}; };
template <> struct FusedTiles<3> { static constexpr int n = 3, tc[3] = {8, 4, 12}; };
template <> struct FusedTiles<4> { static constexpr int n = 2, tc[3] = {8, 4, 8}; };
template <> struct FusedTiles<5> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };
template <> struct FusedTiles<6> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };
template <> struct FusedTiles<7> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };

template <typename T, int K, int TC>
hipError_t avs2d_tc(int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout, T omega,
                    hipStream_t s, int nsys, int64_t zs, const int* active, const T* ec, const T* ptab,
                    int64_t zc) {
  using S = SmGeo<T, K, TC, 256>;
  const int n1 = K * N + 1;
  const int nt = (N + TC - 1) / TC;
  // interior: residual tile in the periodic row classes and every patch of the interior type
  auto in = [&](int bt) {
    const int c0 = bt * TC, o = (c0 - 1) * K;
    return c.periodic && o >= c.left && o + (TC + 2) * K <= c.right0 && c0 >= 2 && c0 + TC <= N - 2;
  };
  const tile::TileOrder ord = tile::make_order(nt, nt, in, in);
  const dim3 grid(tile::order_blocks(ord), 1, nsys);
  if (ec)
    avs2d_kernel<T, S, true><<<grid, S::NTH, 0, s>>>(x, b, xout, N, n1, c.tab, c.nclass, c.left, c.right0,
                                                     c.periodic, e.Q, e.lam, omega, zs, active, ord, ec, ptab, zc);
  else
    avs2d_kernel<T, S, false><<<grid, S::NTH, 0, s>>>(x, b, xout, N, n1, c.tab, c.nclass, c.left, c.right0,
                                                      c.periodic, e.Q, e.lam, omega, zs, active, ord, ec, ptab, zc);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t avs2d_k(int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout, T omega,
                   hipStream_t s, int nsys, int64_t zs, const int* active, int variant, const T* ec, const T* ptab,
                   int64_t zc) {
  using F = FusedTiles<K>;
  switch (variant < F::n ? variant : 0) {
    case 1: return avs2d_tc<T, K, F::tc[1]>(N, c, e, x, b, xout, omega, s, nsys, zs, active, ec, ptab, zc);
    case 2: return avs2d_tc<T, K, F::tc[2]>(N, c, e, x, b, xout, omega, s, nsys, zs, active, ec, ptab, zc);
    default: return avs2d_tc<T, K, F::tc[0]>(N, c, e, x, b, xout, omega, s, nsys, zs, active, ec, ptab, zc);
  }
}

}  // namespace

template <typename Tin, typename T>
hipError_t launch_apply2d(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s,
                          int nsys, int64_t zs, const int* active, Tin* xc) {
#define CALL(K) apply2d_k<Tin, T, K>(N, c, x, b, y, s, nsys, zs, active, xc)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_pre2d(int k, int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* b, T* x1, T* r, T omega,
                        hipStream_t s) {
#define CALL(K) pre2d_k<T, K>(N, c, e, b, x1, r, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_avs2d(int k, int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout,
                        T omega, hipStream_t s, int nsys, int64_t zs, const int* active, int variant, const T* ec,
                        const T* ptab, int64_t zc) {
#define CALL(K) avs2d_k<T, K>(N, c, e, x, b, xout, omega, s, nsys, zs, active, variant, ec, ptab, zc)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}
}  // namespace c0ip
