// Device helpers shared by the tile kernels (row classes of the 1D
// factors, structural bands and band products, XCD-aware tile order).
#pragma once

#include <hip/hip_runtime.h>

namespace c0ip {
namespace tile {

constexpr int kThreads = 256;

// Row class of global 1D row g: rows within 2k of either end are their own
// class; the others repeat with the node's position in its cell.
__device__ __forceinline__ int row_class(int g, int n1, int k, int left, int right0, int periodic) {
  if (!periodic) return g;
  if (g < left) return g;
  if (g >= right0) return left + (n1 - 1 - g);
  return 2 * left + g % k;
}

// Boundary type of the vertex patch at vertex v in [1, N-1] along one axis.
__device__ __forceinline__ int variant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap the (x, y) tile index so that XCD c walks one contiguous band
// of tiles (row-major): neighbouring tiles, whose halos overlap, then share
// that XCD's L2.  A bijection for any grid size.
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int gx = gridDim.x, T = gx * gridDim.y;
  const int L = blockIdx.x + blockIdx.y * gx;
  const int c = L & 7, q = L >> 3;
  const int logical = c * (T >> 3) + min(c, T & 7) + q;
  bx = logical % gx;
  by = logical / gx;
}

// Block-to-tile order of a launch.  Tiles outside the rectangle
// [bx_lo, bx_hi] x [by_lo, by_hi] (those that need per-lane row classes or
// boundary patches, and run slower) take the first block indices so that
// they start first and do not trail the launch.  The interior rectangle
// follows, each XCD walking one contiguous band of it (row-major), which
// keeps the halos that neighbouring tiles share in one L2.  Blocks
// [nb, nbp) pad the ring to a multiple of 8 and do nothing.
struct TileOrder {
  int tx = 0, ty = 0, bx_lo = 0, bx_hi = -1, by_lo = 0, by_hi = -1, nb = 0, nbp = 0;
};

// in[b] for b = 0..n-1 must be true exactly on one range; returns it (lo > hi if empty)
template <class F>
inline void interior_range(int n, F in, int& lo, int& hi) {
  lo = 0;
  hi = -1;
  int b = 0;
  while (b < n && !in(b)) ++b;
  lo = b;
  while (b < n && in(b)) ++b;
  hi = b - 1;
  if (lo > hi) {
    lo = 0;
    hi = -1;
  }
}

template <class FX, class FY>
inline TileOrder make_order(int tx, int ty, FX xin, FY yin) {
  TileOrder o;
  o.tx = tx;
  o.ty = ty;
  interior_range(tx, xin, o.bx_lo, o.bx_hi);
  interior_range(ty, yin, o.by_lo, o.by_hi);
  if (o.bx_lo > o.bx_hi || o.by_lo > o.by_hi) {
    o.bx_lo = o.by_lo = 0;
    o.bx_hi = o.by_hi = -1;
  }
  const int ni = (o.bx_hi - o.bx_lo + 1) * (o.by_hi - o.by_lo + 1);
  o.nb = tx * ty - ni;
  o.nbp = (o.nb + 7) & ~7;
  return o;
}
__host__ __device__ inline int order_blocks(const TileOrder& o) {
  return o.nbp + (o.bx_hi - o.bx_lo + 1) * (o.by_hi - o.by_lo + 1);
}

__host__ __device__ inline bool tile_of_block(const TileOrder& o, int L, int& bx, int& by) {
  const int iw = o.bx_hi - o.bx_lo + 1, ih = o.by_hi - o.by_lo + 1;
  if (L < o.nb) {
    if (iw <= 0) {
      bx = L % o.tx;
      by = L / o.tx;
      return true;
    }
    const int ntop = o.by_lo * o.tx;
    if (L < ntop) {
      by = L / o.tx;
      bx = L - by * o.tx;
      return true;
    }
    L -= ntop;
    const int side = o.tx - iw, nmid = ih * side;
    if (L < nmid) {
      const int r = L / side, c = L - r * side;
      by = o.by_lo + r;
      bx = c < o.bx_lo ? c : c + iw;
      return true;
    }
    L -= nmid;
    by = o.by_hi + 1 + L / o.tx;
    bx = L % o.tx;
    return true;
  }
  if (L < o.nbp) return false;
  const int Li = L - o.nbp, T = iw * ih;
  if (Li >= T) return false;
  const int c = Li & 7, q = Li >> 3;
  const int logical = c * (T >> 3) + (c < (T & 7) ? c : (T & 7)) + q;
  bx = o.bx_lo + logical % iw;
  by = o.by_lo + logical / iw;
  return true;
}

// Structural band of a row at position p in its cell (p = 0: vertex node)
// for the three 1D factors, OP = 0 (M), 1 (L), 2 (B): M and L couple the
// nodes of the one (p > 0) or two (p = 0) cells containing the row; B
// reaches one cell further on each side through the point terms.
template <int OP, int K>
struct Band {
  static constexpr int lo(int p) { return OP == 2 ? (p == 0 ? -2 * K : -K - p) : (p == 0 ? -K : -p); }
  static constexpr int hi(int p) { return OP == 2 ? (p == 0 ? 2 * K : 2 * K - p) : (p == 0 ? K : K - p); }
  static constexpr int width(int p) { return hi(p) - lo(p) + 1; }
  // input window (relative to the cell's first node minus 2K) of rows p0..K-1
  static constexpr int win_lo(int p0) { return 2 * K + (p0 == 0 ? lo(0) : lo(1) + 1); }
  static constexpr int win_hi() { return 2 * K + (OP == 2 ? 2 * K : K); }
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Band product of factor OP for the row at cell position p with
// coefficients c (centred) and inputs v (v[0] = the band's first tap).
template <typename T, int OP, int K>
__device__ __forceinline__ T band_dot(const T* __restrict__ c, const T* v, int p) {
  T a = 0;
#pragma unroll
  for (int o = Band<OP, K>::lo(p); o <= Band<OP, K>::hi(p); ++o) a += c[o] * v[o];
  return a;
}

// Rows of the periodic classes share one coefficient row per cell
// position, read with wave-uniform addresses from the global table.  On
// interior tiles (UNIFORM) every row is periodic.  Elsewhere the few lanes
// whose row is in a boundary class (or every lane on meshes too small to
// have periodic rows) redo the product with their own row from the
// workgroup's LDS copy of the table.
template <typename T, int OP, int K, bool UNIFORM>
__device__ __forceinline__ T band_row(const T* __restrict__ tab, const T* __restrict__ sTab, int nclass, int left,
                                      int periodic, int cl, const T* v, int p) {
  constexpr int W = 4 * K + 1, H = 2 * K;
  if constexpr (UNIFORM) {
    return band_dot<T, OP, K>(tab + (size_t)(OP * nclass + 2 * left + p) * W + H, v, p);
  } else {
    T a = 0;
    if (periodic) a = band_dot<T, OP, K>(tab + (size_t)(OP * nclass + 2 * left + p) * W + H, v, p);
    if (!periodic || cl != 2 * left + p) a = band_dot<T, OP, K>(sTab + (OP * nclass + cl) * W + H, v, p);
    return a;
  }
}

// LDS copies of a level's fast-diagonalisation data, every global load of
// a thread issued before its first LDS store: sQ = the four
// eigenbases (4 n^2), sLam = their eigenvalues (4 n), and the interior
// patch's inverse eigenvalue sums sD[ap][c] = 1 / (lambda_c + lambda_ap).
template <typename T, int n, int NTH>
__device__ __forceinline__ void stage_eig(const T* __restrict__ Qg, const T* __restrict__ lamg, T* __restrict__ sQ,
                                          T* __restrict__ sLam, T* __restrict__ sD) {
  constexpr int NN = n * n, LQ = (4 * NN + NTH - 1) / NTH, LL = (4 * n + NTH - 1) / NTH, LD = (NN + NTH - 1) / NTH;
  T q[LQ], l[LL], da[LD], db[LD];
#pragma unroll
  for (int u = 0; u < LQ; ++u) {
    const int e = threadIdx.x + u * NTH;
    q[u] = e < 4 * NN ? Qg[e] : T(0);
  }
#pragma unroll
  for (int u = 0; u < LL; ++u) {
    const int e = threadIdx.x + u * NTH;
    l[u] = e < 4 * n ? lamg[e] : T(0);
  }
#pragma unroll
  for (int u = 0; u < LD; ++u) {
    const int e = threadIdx.x + u * NTH;
    da[u] = e < NN ? lamg[e % n] : T(1);
    db[u] = e < NN ? lamg[e / n] : T(1);
  }
#pragma unroll
  for (int u = 0; u < LQ; ++u) {
    const int e = threadIdx.x + u * NTH;
    if (e < 4 * NN) sQ[e] = q[u];
  }
#pragma unroll
  for (int u = 0; u < LL; ++u) {
    const int e = threadIdx.x + u * NTH;
    if (e < 4 * n) sLam[e] = l[u];
  }
#pragma unroll
  for (int u = 0; u < LD; ++u) {
    const int e = threadIdx.x + u * NTH;
    if (e < NN) sD[e] = T(1) / (da[u] + db[u]);  // [ap][c]
  }
}

}  // namespace tile
}  // namespace c0ip
