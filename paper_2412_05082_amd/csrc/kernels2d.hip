// 2D kernels: matrix-free C0IP operator and the additive vertex-patch
// smoother with fast-diagonalisation local solves, for gfx950.
//
// Operator (Sec. 4, eq. c0iptensorvp, used globally on the Cartesian mesh):
//   A x = (B (x) M + 2 L (x) L + M (x) B) x,  first factor along x.
// In matrix form with X[j][i] (i = x index, fastest):
//   Y = M_y (X B_x) + 2 L_y (X L_x) + B_y (X M_x).
// One workgroup owns a tile of TY x TX output nodes (whole cells, so a
// node's position in its cell is its tile-local index mod k).  It stages
// X on the tile plus a 2k-node halo in LDS, runs the three x-sweeps into
// LDS (X M_x on the 2k halo rows, X L_x and X B_x on the k halo rows), then
// the three y-sweeps straight to HBM.  Band coefficients depend only on the
// node's position in its cell away from the boundary; interior tiles read
// them with wave-uniform addresses (scalar loads).
//
// Smoother (Sec. 3 additive vertex-patch Schwarz; local solver of eq.
// localsolverbila inverted by eq. inverse):
//   x_out = x_in + omega * sum_v R_v^T (Q_y (x) Q_x) D_v^{-1} (Q_y (x) Q_x)^T R_v r.
// Owner-computes: a workgroup owns a tile of TC x TC cells, solves the
// (TC+1)^2 patches that touch it (neighbouring tiles solve shared patches
// twice instead of racing on writes), and writes each owned DoF once.
#include <algorithm>

#include "kernels.h"

namespace c0ip {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int row_class(int g, int n1, int k, int left, int right0, int periodic) {
  if (!periodic) return g;
  if (g < left) return g;
  if (g >= right0) return left + (n1 - 1 - g);
  return 2 * left + g % k;
}

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

// Structural band of a row at position p in its cell (p = 0: vertex node).
// M and L: support of one (p > 0) or two (p = 0) cells; B: one more cell
// on each side through the point terms.
template <int K> __host__ __device__ constexpr int m_lo(int p) { return p == 0 ? -K : -p; }
template <int K> __host__ __device__ constexpr int m_hi(int p) { return p == 0 ? K : K - p; }
template <int K> __host__ __device__ constexpr int b_lo(int p) { return p == 0 ? -2 * K : -K - p; }
template <int K> __host__ __device__ constexpr int b_hi(int p) { return p == 0 ? 2 * K : 2 * K - p; }

// ------------------------------------------------------------------ operator

template <typename T, int K, int TXC, int TYC, bool INTERIOR>
__device__ __forceinline__ void x_sweeps(const T* __restrict__ sX, T* __restrict__ sU, T* __restrict__ sV,
                                         T* __restrict__ sW, int x0, int n1, const T* __restrict__ tab,
                                         int nclass, int left, int right0, int periodic) {
  constexpr int H = 2 * K, TX = TXC * K, TY = TYC * K, RX = TX + 2 * H, RY = TY + 2 * H, W = 4 * K + 1;
  for (int it = threadIdx.x; it < RY * TXC; it += kThreads) {
    const int r = it / TXC, cc = it - r * TXC;
    T in[4 * K + 1];
#pragma unroll
    for (int j = 0; j <= 4 * K; ++j) in[j] = sX[r * RX + cc * K + j];
    const bool vw = (r >= K) && (r < RY - K);
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const int g = max(0, min(x0 + cc * K + p, n1 - 1));
      const int cls = INTERIOR ? (2 * left + p) : row_class(g, n1, K, left, right0, periodic);
      const T* cM = tab + (size_t)cls * W + H;
      const T* cL = tab + (size_t)(nclass + cls) * W + H;
      const T* cB = tab + (size_t)(2 * nclass + cls) * W + H;
      T u = 0;
#pragma unroll
      for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) u += cM[o] * in[p + o + H];
      sU[r * TX + cc * K + p] = u;
      if (vw) {
        T v = 0, w = 0;
#pragma unroll
        for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) v += cL[o] * in[p + o + H];
#pragma unroll
        for (int o = b_lo<K>(p); o <= b_hi<K>(p); ++o) w += cB[o] * in[p + o + H];
        sV[(r - K) * TX + cc * K + p] = v;
        sW[(r - K) * TX + cc * K + p] = w;
      }
    }
  }
}

template <typename T, int K, int TXC, int TYC, bool INTERIOR, bool RES>
__device__ __forceinline__ void y_sweeps(const T* __restrict__ sU, const T* __restrict__ sV,
                                         const T* __restrict__ sW, int x0, int y0, int n1,
                                         const T* __restrict__ tab, int nclass, int left, int right0,
                                         int periodic, const T* __restrict__ b, T* __restrict__ y) {
  constexpr int H = 2 * K, TX = TXC * K, W = 4 * K + 1;
  for (int it = threadIdx.x; it < TX * TYC; it += kThreads) {
    const int cr = it / TX, l = it - cr * TX;
    const int gx = x0 + l;
    if (gx >= n1) continue;
    T u[4 * K + 1], v[2 * K + 1], w[2 * K + 1];
#pragma unroll
    for (int j = 0; j <= 4 * K; ++j) u[j] = sU[(cr * K + j) * TX + l];
#pragma unroll
    for (int j = 0; j <= 2 * K; ++j) {
      v[j] = sV[(cr * K + j) * TX + l];
      w[j] = sW[(cr * K + j) * TX + l];
    }
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const int gy = y0 + cr * K + p;
      if (gy >= n1) break;
      const int cls = INTERIOR ? (2 * left + p) : row_class(gy, n1, K, left, right0, periodic);
      const T* cM = tab + (size_t)cls * W + H;
      const T* cL = tab + (size_t)(nclass + cls) * W + H;
      const T* cB = tab + (size_t)(2 * nclass + cls) * W + H;
      T am = 0, al = 0, ab = 0;
#pragma unroll
      for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) {
        am += cM[o] * w[p + o + K];
        al += cL[o] * v[p + o + K];
      }
#pragma unroll
      for (int o = b_lo<K>(p); o <= b_hi<K>(p); ++o) ab += cB[o] * u[p + o + H];
      const T acc = am + 2 * al + ab;
      const size_t idx = (size_t)gy * n1 + gx;
      if (RES) {
        const bool bnd = (gx == 0) | (gx == n1 - 1) | (gy == 0) | (gy == n1 - 1);
        y[idx] = bnd ? T(0) : (b[idx] - acc);
      } else {
        y[idx] = acc;
      }
    }
  }
}

// Row-class tables have at most 5k+2 classes (2k+1 per boundary end plus k
// periodic ones, or one per row on levels with kN+1 <= 5k+2 nodes).
template <int K> __host__ __device__ constexpr int tab_max() { return 3 * (5 * K + 2) * (4 * K + 1); }

// Persistent form: a workgroup walks several tiles of its XCD's band (see
// xcd_tile); the global loads of the next tile are issued into registers
// before the current tile's sweeps, so their latency overlaps compute.
// XCD c owns tiles [start_c, start_c + len_c) (row-major over the tile grid);
// its g_c workgroups take every g_c-th tile of that band.
__device__ __forceinline__ void band_of_block(int ntiles, int& t0, int& tend, int& stride) {
  const int G = gridDim.x, bi = blockIdx.x, c = bi & 7, i = bi >> 3;
  const int g = (G - c + 7) >> 3;
  const int len = (ntiles >> 3) + (c < (ntiles & 7) ? 1 : 0);
  const int start = c * (ntiles >> 3) + min(c, ntiles & 7);
  t0 = start + i;
  tend = start + len;
  stride = g;
}

template <typename Tin, typename T, int K, int TXC, int TYC, bool RES>
__global__ __launch_bounds__(kThreads) void apply2d_kernel(const Tin* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ y, int n1, int tiles_x, int ntiles,
                                                           const T* __restrict__ tab, int nclass, int left,
                                                           int right0, int periodic, int64_t zs,
                                                           const int* __restrict__ active) {
  constexpr int H = 2 * K, TX = TXC * K, TY = TYC * K, RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int NL = (RY * RX + kThreads - 1) / kThreads;
  if (active && !active[blockIdx.z]) return;
  // system blockIdx.z of a batch of equally sized vectors zs apart
  x += blockIdx.z * zs;
  y += blockIdx.z * zs;
  if (RES) b += blockIdx.z * zs;
  __shared__ T sX[RY * RX];
  __shared__ T sU[RY * TX];
  __shared__ T sV[(TY + 2 * K) * TX];
  __shared__ T sW[(TY + 2 * K) * TX];
  __shared__ T sTab[tab_max<K>()];
  {
    const int ntab = 3 * nclass * (4 * K + 1);
    for (int e = threadIdx.x; e < ntab; e += kThreads) sTab[e] = tab[e];
  }
  int t, tend, stride;
  band_of_block(ntiles, t, tend, stride);
  T v[NL];
#define C0IP_LOAD_TILE(tt)                                                                              \
  {                                                                                                     \
    const int lx0 = ((tt) % tiles_x) * TX, ly0 = ((tt) / tiles_x) * TY;                                 \
    _Pragma("unroll") for (int q = 0; q < NL; ++q) {                                                    \
      const int e = threadIdx.x + q * kThreads;                                                         \
      const int r = e / RX, c = e - r * RX;                                                             \
      const int gy = ly0 - H + r, gx = lx0 - H + c;                                                     \
      v[q] = (e < RY * RX && gy >= 0 && gy < n1 && gx >= 0 && gx < n1) ? (T)x[(size_t)gy * n1 + gx]     \
                                                                        : T(0);                         \
    }                                                                                                   \
  }
  if (t < tend) C0IP_LOAD_TILE(t)
  for (; t < tend; t += stride) {
    const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
    __syncthreads();  // the previous tile is done with sX, sU, sV, sW
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < RY * RX) sX[e] = v[q];
    }
    __syncthreads();
    if (t + stride < tend) C0IP_LOAD_TILE(t + stride)  // in flight during the sweeps below
    const bool xin = periodic && x0 >= left && x0 + TX <= right0;
    const bool yin = periodic && y0 >= left && y0 + TY <= right0;
    // interior tiles: wave-uniform coefficient addresses in the global table
    // (scalar loads); boundary tiles: per-lane class rows from the LDS copy
    if (xin)
      x_sweeps<T, K, TXC, TYC, true>(sX, sU, sV, sW, x0, n1, tab, nclass, left, right0, periodic);
    else
      x_sweeps<T, K, TXC, TYC, false>(sX, sU, sV, sW, x0, n1, sTab, nclass, left, right0, periodic);
    __syncthreads();
    if (yin)
      y_sweeps<T, K, TXC, TYC, true, RES>(sU, sV, sW, x0, y0, n1, tab, nclass, left, right0, periodic, b, y);
    else
      y_sweeps<T, K, TXC, TYC, false, RES>(sU, sV, sW, x0, y0, n1, sTab, nclass, left, right0, periodic, b, y);
  }
#undef C0IP_LOAD_TILE
}

// Resident workgroups of a kernel on the whole device (cached per kernel).
template <typename KernelT>
int device_slots(KernelT kernel) {
  static int slots = 0;
  if (slots == 0) {
    int dev = 0, ncu = 0, occ = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kThreads, 0);
    slots = std::max(8, ncu * std::max(occ, 1));
  }
  return slots;
}

inline int persistent_grid(int ntiles, int slots) {
  if (ntiles <= 8) return ntiles;
  int g = std::min(ntiles, slots);
  return g >= 8 ? (g & ~7) : g;
}

template <int K> struct ApplyTile2D;
template <> struct ApplyTile2D<2> { static constexpr int TXC = 16, TYC = 16; };
template <> struct ApplyTile2D<3> { static constexpr int TXC = 16, TYC = 8; };
template <> struct ApplyTile2D<4> { static constexpr int TXC = 8, TYC = 8; };
template <> struct ApplyTile2D<5> { static constexpr int TXC = 8, TYC = 4; };
template <> struct ApplyTile2D<6> { static constexpr int TXC = 4, TYC = 4; };
template <> struct ApplyTile2D<7> { static constexpr int TXC = 4, TYC = 4; };

template <typename Tin, typename T, int K>
hipError_t apply2d_k(int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s, int nsys,
                     int64_t zs, const int* active) {
  constexpr int TXC = ApplyTile2D<K>::TXC, TYC = ApplyTile2D<K>::TYC;
  const int n1 = K * N + 1;
  const int tx = (n1 + TXC * K - 1) / (TXC * K), ty = (n1 + TYC * K - 1) / (TYC * K);
  const int nt = tx * ty;
  if (b) {
    auto kern = apply2d_kernel<Tin, T, K, TXC, TYC, true>;
    const int G = persistent_grid(nt, device_slots(kern));
    kern<<<dim3(G, 1, nsys), kThreads, 0, s>>>(x, b, y, n1, tx, nt, c.tab, c.nclass, c.left, c.right0, c.periodic,
                                               zs, active);
  } else {
    auto kern = apply2d_kernel<Tin, T, K, TXC, TYC, false>;
    const int G = persistent_grid(nt, device_slots(kern));
    kern<<<dim3(G, 1, nsys), kThreads, 0, s>>>(x, b, y, n1, tx, nt, c.tab, c.nclass, c.left, c.right0, c.periodic,
                                               zs, active);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ smoother

__device__ __forceinline__ int variant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void patch2d_kernel(const T* __restrict__ r, const T* __restrict__ xin,
                                                           T* __restrict__ xout, int N, int n1,
                                                           const T* __restrict__ Qg, const T* __restrict__ lamg,
                                                           T omega, int64_t zs, const int* __restrict__ active) {
  constexpr int n = 2 * K - 1, NN = n * n, NP = TC + 1, S = (TC + 2) * K - 1;
  if (active && !active[blockIdx.z]) return;
  r += blockIdx.z * zs;
  xout += blockIdx.z * zs;
  if (xin) xin += blockIdx.z * zs;
  constexpr int NL = (S * S + kThreads - 1) / kThreads;
  __shared__ T sR[S * S];
  __shared__ T sA[NP * NP * NN];
  __shared__ T sB[NP * NP * NN];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int cx0 = tbx * TC, cy0 = tby * TC;
  const int ox = (cx0 - 1) * K + 1, oy = (cy0 - 1) * K + 1;  // global node of region (0,0)
  {
    T v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int rr = e / S, cc = e - rr * S;
      const int gy = oy + rr, gx = ox + cc;
      v[q] = (e < S * S && gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2) ? r[(size_t)gy * n1 + gx] : T(0);
    }
    for (int e = threadIdx.x; e < 4 * NN; e += kThreads) sQ[e] = Qg[e];
    for (int e = threadIdx.x; e < 4 * n; e += kThreads) sLam[e] = lamg[e];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < S * S) sR[e] = v[q];
    }
  }
  __syncthreads();
  const T* Q = sQ;
  const T* lam = sLam;
  // forward along x: t[a][c] = sum_c' Qx[c'][c] r[a][c']
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
    const T* q = Q + variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sR[(pyl * K + a) * S + pxl * K + c];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int cp = 0; cp < n; ++cp) s += q[cp * n + c] * in[cp];
      sA[p * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  // along y: forward with Qy^T, divide by lambda_x + lambda_y, back with Qy
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, c = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
    const int ty = variant(vy, N), tx = variant(vx, N);
    const T* q = Q + ty * NN;
    const T lx = lam[tx * n + c];
    T col[n], t[n];
#pragma unroll
    for (int a = 0; a < n; ++a) col[a] = sA[p * NN + a * n + c];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += q[a * n + ap] * col[a];
      t[ap] = s / (lx + lam[ty * n + ap]);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += q[a * n + ap] * t[ap];
      sB[p * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  // back along x: u[a][c'] = sum_c Qx[c'][c] t[a][c]
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
    const T* q = Q + variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sB[p * NN + a * n + c];
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += q[cp * n + c] * in[c];
      sA[p * NN + a * n + cp] = s;
    }
  }
  __syncthreads();
  // owned DoFs: sum the covering patches' corrections
  constexpr int OW = TC * K + 1;
  const int gx0 = cx0 * K, gy0 = cy0 * K;
  const int gx1 = (cx0 + TC >= N) ? n1 : (cx0 + TC) * K;
  const int gy1 = (cy0 + TC >= N) ? n1 : (cy0 + TC) * K;
  for (int e = threadIdx.x; e < OW * OW; e += kThreads) {
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
    T acc = 0;
    for (int vy = vya; vy <= vyb; ++vy) {
      if (vy < 1 || vy > N - 1) continue;
      for (int vx = vxa; vx <= vxb; ++vx) {
        if (vx < 1 || vx > N - 1) continue;
        const int p = (vy - cy0) * NP + (vx - cx0);
        const int c = gx - ((vx - 1) * K + 1), a = gy - ((vy - 1) * K + 1);
        acc += sA[p * NN + a * n + c];
      }
    }
    xout[idx] = (xin ? xin[idx] : T(0)) + omega * acc;
  }
}

// ------------------------------------------------------------------ fused smoother
// One step S(x, b) = x + omega sum_v R_v^T A~_v^{-1} R_v (b - A x) in one
// launch: the residual is computed on the owned tile extended by one cell
// (the support of every patch touching the tile) with the operator's
// sweeps, kept in LDS, and consumed by the patch solves; r never goes to
// HBM.  Tile TC x TC owned cells; the residual tile is (TC+2) x (TC+2)
// cells starting one cell before the owned one.

template <typename T, int K, int TXC, int TYC, bool INTERIOR>
__device__ __forceinline__ void y_sweeps_residual_lds(const T* __restrict__ sU, const T* __restrict__ sV,
                                                      const T* __restrict__ sW, int x0, int y0, int n1,
                                                      const T* __restrict__ tab, int nclass, int left, int right0,
                                                      int periodic, const T* __restrict__ b, T* __restrict__ sRr) {
  constexpr int H = 2 * K, TX = TXC * K, W = 4 * K + 1;
  for (int it = threadIdx.x; it < TX * TYC; it += kThreads) {
    const int cr = it / TX, l = it - cr * TX;
    const int gx = x0 + l;
    T u[4 * K + 1], v[2 * K + 1], w[2 * K + 1];
#pragma unroll
    for (int j = 0; j <= 4 * K; ++j) u[j] = sU[(cr * K + j) * TX + l];
#pragma unroll
    for (int j = 0; j <= 2 * K; ++j) {
      v[j] = sV[(cr * K + j) * TX + l];
      w[j] = sW[(cr * K + j) * TX + l];
    }
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const int gy = y0 + cr * K + p;
      const int cls = INTERIOR ? (2 * left + p) : row_class(max(0, min(gy, n1 - 1)), n1, K, left, right0, periodic);
      const T* cM = tab + (size_t)cls * W + H;
      const T* cL = tab + (size_t)(nclass + cls) * W + H;
      const T* cB = tab + (size_t)(2 * nclass + cls) * W + H;
      T am = 0, al = 0, ab = 0;
#pragma unroll
      for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) {
        am += cM[o] * w[p + o + K];
        al += cL[o] * v[p + o + K];
      }
#pragma unroll
      for (int o = b_lo<K>(p); o <= b_hi<K>(p); ++o) ab += cB[o] * u[p + o + H];
      const bool inner = gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2;
      sRr[(cr * K + p) * TX + l] = inner ? b[(size_t)gy * n1 + gx] - (am + 2 * al + ab) : T(0);
    }
  }
}

// Patch solves of the fused smoother.  Interior tiles (every patch of
// variant 0) index Q and lambda with loop-invariant addresses, so the
// eigenbasis stays in registers across the items of a thread.
template <typename T, int K, int TC, bool INTERIOR>
__device__ __forceinline__ void fused_patches(const T* __restrict__ sRr, T* __restrict__ pool,
                                              const T* __restrict__ Q, const T* __restrict__ lam, int N, int cx0,
                                              int cy0) {
  constexpr int TX = (TC + 2) * K, n = 2 * K - 1, NN = n * n, NP = TC + 1;
  T* sA = pool;
  T* sB = pool + NP * NP * NN;
  // patch solves, as in patch2d_kernel; the residual tile node of patch (vx,vy),
  // entry (a, c), is ((vy - cy0) K + 1 + a, (vx - cx0) K + 1 + c)
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const T* q = INTERIOR ? Q : Q + variant(vx, N) * NN;
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
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, c = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const int ty = INTERIOR ? 0 : variant(vy, N), tx = INTERIOR ? 0 : variant(vx, N);
    const T* q = Q + ty * NN;
    const T lx = lam[tx * n + c];
    T col[n], t[n];
#pragma unroll
    for (int a = 0; a < n; ++a) col[a] = sA[p * NN + a * n + c];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += q[a * n + ap] * col[a];
      t[ap] = s / (lx + lam[ty * n + ap]);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += q[a * n + ap] * t[ap];
      sB[p * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (!INTERIOR && (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1)) continue;
    const T* q = INTERIOR ? Q : Q + variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sB[p * NN + a * n + c];
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

template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void avs2d_kernel(const T* __restrict__ x, const T* __restrict__ b,
                                                         T* __restrict__ xout, int N, int n1,
                                                         const T* __restrict__ tab, int nclass, int left,
                                                         int right0, int periodic, const T* __restrict__ Qg,
                                                         const T* __restrict__ lamg, T omega, int64_t zs,
                                                         const int* __restrict__ active) {
  constexpr int TXC = TC + 2, TYC = TC + 2, H = 2 * K, TX = TXC * K, TY = TYC * K, RX = TX + 2 * H,
                RY = TY + 2 * H;
  constexpr int n = 2 * K - 1, NN = n * n, NP = TC + 1;
  constexpr int SZA = RY * RX + RY * TX + 2 * (TY + 2 * K) * TX, SZB = 2 * NP * NP * NN;
  constexpr int NL = (RY * RX + kThreads - 1) / kThreads;
  __shared__ T pool[SZA > SZB ? SZA : SZB];
  __shared__ T sRr[TY * TX];
  __shared__ T sTab[tab_max<K>()];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  if (active && !active[blockIdx.z]) return;
  x += blockIdx.z * zs;
  b += blockIdx.z * zs;
  xout += blockIdx.z * zs;
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int cx0 = tbx * TC, cy0 = tby * TC;
  const int x0 = (cx0 - 1) * K, y0 = (cy0 - 1) * K;  // residual tile origin (a vertex node)
  T* sX = pool;
  T* sU = sX + RY * RX;
  T* sV = sU + RY * TX;
  T* sW = sV + (TY + 2 * K) * TX;
  {
    T v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int r = e / RX, c = e - r * RX;
      const int gy = y0 - H + r, gx = x0 - H + c;
      v[q] = (e < RY * RX && gy >= 0 && gy < n1 && gx >= 0 && gx < n1) ? x[(size_t)gy * n1 + gx] : T(0);
    }
    const int ntab = 3 * nclass * (4 * K + 1);
    for (int e = threadIdx.x; e < ntab; e += kThreads) sTab[e] = tab[e];
    for (int e = threadIdx.x; e < 4 * NN; e += kThreads) sQ[e] = Qg[e];
    for (int e = threadIdx.x; e < 4 * n; e += kThreads) sLam[e] = lamg[e];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < RY * RX) sX[e] = v[q];
    }
  }
  __syncthreads();
  const bool xin = periodic && x0 >= left && x0 + TX <= right0;
  const bool yin = periodic && y0 >= left && y0 + TY <= right0;
  if (xin)
    x_sweeps<T, K, TXC, TYC, true>(sX, sU, sV, sW, x0, n1, tab, nclass, left, right0, periodic);
  else
    x_sweeps<T, K, TXC, TYC, false>(sX, sU, sV, sW, x0, n1, sTab, nclass, left, right0, periodic);
  __syncthreads();
  if (yin)
    y_sweeps_residual_lds<T, K, TXC, TYC, true>(sU, sV, sW, x0, y0, n1, tab, nclass, left, right0, periodic, b,
                                                sRr);
  else
    y_sweeps_residual_lds<T, K, TXC, TYC, false>(sU, sV, sW, x0, y0, n1, sTab, nclass, left, right0, periodic, b,
                                                 sRr);
  __syncthreads();
  // all patches of the tile interior (vertices in [2, N-2]): one eigenbasis
  const bool interior = cx0 >= 2 && cx0 + TC <= N - 2 && cy0 >= 2 && cy0 + TC <= N - 2;
  T* sA = pool;
  if (interior)
    fused_patches<T, K, TC, true>(sRr, pool, sQ, sLam, N, cx0, cy0);
  else
    fused_patches<T, K, TC, false>(sRr, pool, sQ, sLam, N, cx0, cy0);
  constexpr int OW = TC * K + 1;
  const int gx0 = cx0 * K, gy0 = cy0 * K;
  const int gx1 = (cx0 + TC >= N) ? n1 : (cx0 + TC) * K;
  const int gy1 = (cy0 + TC >= N) ? n1 : (cy0 + TC) * K;
  for (int e = threadIdx.x; e < OW * OW; e += kThreads) {
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
    T acc = 0;
    for (int vy = vya; vy <= vyb; ++vy) {
      if (vy < 1 || vy > N - 1) continue;
      for (int vx = vxa; vx <= vxb; ++vx) {
        if (vx < 1 || vx > N - 1) continue;
        const int p = (vy - cy0) * NP + (vx - cx0);
        const int c = gx - ((vx - 1) * K + 1), a = gy - ((vy - 1) * K + 1);
        acc += sA[p * NN + a * n + c];
      }
    }
    xout[idx] = x[idx] + omega * acc;
  }
}

// Tile sizes (owned cells per side) the fused smoother is compiled for;
// variant 0 is the default, the autotuner may pick any of them per level.
template <int K> struct FusedTiles;
template <> struct FusedTiles<2> { static constexpr int n = 3, tc[3] = {16, 8, 24}; };
template <> struct FusedTiles<3> { static constexpr int n = 3, tc[3] = {8, 4, 12}; };
template <> struct FusedTiles<4> { static constexpr int n = 2, tc[3] = {8, 4, 8}; };
template <> struct FusedTiles<5> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };
template <> struct FusedTiles<6> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };
template <> struct FusedTiles<7> { static constexpr int n = 2, tc[3] = {4, 2, 4}; };

template <typename T, int K, int TC>
hipError_t avs2d_tc(int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout, T omega,
                    hipStream_t s, int nsys, int64_t zs, const int* active) {
  const int n1 = K * N + 1;
  const int nt = (N + TC - 1) / TC;
  avs2d_kernel<T, K, TC><<<dim3(nt, nt, nsys), kThreads, 0, s>>>(x, b, xout, N, n1, c.tab, c.nclass, c.left,
                                                                 c.right0, c.periodic, e.Q, e.lam, omega, zs,
                                                                 active);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t avs2d_k(int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout, T omega,
                   hipStream_t s, int nsys, int64_t zs, const int* active, int variant) {
  using F = FusedTiles<K>;
  switch (variant < F::n ? variant : 0) {
    case 1: return avs2d_tc<T, K, F::tc[1]>(N, c, e, x, b, xout, omega, s, nsys, zs, active);
    case 2: return avs2d_tc<T, K, F::tc[2]>(N, c, e, x, b, xout, omega, s, nsys, zs, active);
    default: return avs2d_tc<T, K, F::tc[0]>(N, c, e, x, b, xout, omega, s, nsys, zs, active);
  }
}

template <int K> struct PatchTile2D;
template <> struct PatchTile2D<2> { static constexpr int TC = 16; };
template <> struct PatchTile2D<3> { static constexpr int TC = 8; };
template <> struct PatchTile2D<4> { static constexpr int TC = 8; };
template <> struct PatchTile2D<5> { static constexpr int TC = 4; };
template <> struct PatchTile2D<6> { static constexpr int TC = 4; };
template <> struct PatchTile2D<7> { static constexpr int TC = 4; };

template <typename T, int K>
hipError_t patch2d_k(int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega, hipStream_t s,
                     int nsys, int64_t zs, const int* active) {
  constexpr int TC = PatchTile2D<K>::TC;
  const int n1 = K * N + 1;
  const int nt = (N + TC - 1) / TC;
  dim3 grid(nt, nt, nsys);
  patch2d_kernel<T, K, TC><<<grid, kThreads, 0, s>>>(r, xin, xout, N, n1, e.Q, e.lam, omega, zs, active);
  return hipGetLastError();
}

// ------------------------------------------------------------------ transfers
// Restriction b_c = P^T r_f and prolongation x_f += P e_c in one launch each:
// a workgroup owns TCC x TCC coarse cells, stages its fine (or coarse)
// window in LDS and applies the 1D embedding table along x, then along y.
// Table T[s][p][a]: value of coarse-cell basis a at the fine node of
// position p in fine cell 2cc+s.

template <int K> struct TransferTile2D { static constexpr int TCC = K <= 4 ? 8 : 4; };

template <typename T, int K, int TCC>
__global__ __launch_bounds__(kThreads) void restrict2d_kernel(const T* __restrict__ rf, T* __restrict__ bc, int Nc,
                                                              const T* __restrict__ tab, int64_t zf, int64_t zc,
                                                              const int* __restrict__ active) {
  constexpr int CT = TCC * K, F = 2 * K * (TCC + 1), NT = 2 * K * (K + 1);
  if (active && !active[blockIdx.z]) return;
  rf += blockIdx.z * zf;
  bc += blockIdx.z * zc;
  constexpr int NL = (F * F + kThreads - 1) / kThreads;
  __shared__ T sF[F * F];
  __shared__ T sT[F * CT];
  __shared__ T sTb[NT];
  const int nf = 2 * K * Nc + 1, nc = K * Nc + 1;
  const int c0x = blockIdx.x * TCC, c0y = blockIdx.y * TCC;
  const int fx0 = 2 * K * (c0x - 1), fy0 = 2 * K * (c0y - 1);
  {
    T v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int rr = e / F, cc = e - rr * F;
      const int gy = fy0 + rr, gx = fx0 + cc;
      v[q] = (e < F * F && gy >= 0 && gy < nf && gx >= 0 && gx < nf) ? rf[(size_t)gy * nf + gx] : T(0);
    }
    for (int e = threadIdx.x; e < NT; e += kThreads) sTb[e] = tab[e];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < F * F) sF[e] = v[q];
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < F * CT; it += kThreads) {
    const int rr = it / CT, l = it - rr * CT;
    const int I = c0x * K + l, cl = l / K, a = l - cl * K;  // coarse cell c0x+cl, position a
    const T* row = sF + rr * F + 2 * K * (cl + 1);
    T v = 0;
#pragma unroll
    for (int q = 0; q < 2 * K; ++q) v += sTb[q * (K + 1) + a] * row[q];
    if (a == 0) {
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) v += sTb[q * (K + 1) + K] * row[q - 2 * K];
    }
    sT[it] = (I > 0 && I < nc - 1) ? v : T(0);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < CT * CT; it += kThreads) {
    const int m = it / CT, l = it - m * CT;
    const int I = c0x * K + l, J = c0y * K + m;
    if (I >= nc || J >= nc) continue;
    const int cm = m / K, a = m - cm * K;
    const T* col = sT + (2 * K * (cm + 1)) * CT + l;
    T v = 0;
#pragma unroll
    for (int q = 0; q < 2 * K; ++q) v += sTb[q * (K + 1) + a] * col[q * CT];
    if (a == 0) {
#pragma unroll
      for (int q = 0; q < 2 * K; ++q) v += sTb[q * (K + 1) + K] * col[(q - 2 * K) * CT];
    }
    bc[(size_t)J * nc + I] = (J > 0 && J < nc - 1) ? v : T(0);
  }
}

template <typename T, int K, int TCC>
__global__ __launch_bounds__(kThreads) void prolong2d_kernel(const T* __restrict__ ec, const T* xin, T* xf, int Nc,
                                                             const T* __restrict__ tab, int64_t zc, int64_t zf,
                                                             const int* __restrict__ active) {
  constexpr int CW = TCC * K + 1, FT = 2 * K * TCC, NT = 2 * K * (K + 1);
  if (active && !active[blockIdx.z]) return;
  ec += blockIdx.z * zc;
  xf += blockIdx.z * zf;
  xin += blockIdx.z * zf;
  constexpr int NL = (CW * CW + kThreads - 1) / kThreads;
  __shared__ T sC[CW * CW];
  __shared__ T sT[CW * FT];
  __shared__ T sTb[NT];
  const int nf = 2 * K * Nc + 1, nc = K * Nc + 1;
  const int c0x = blockIdx.x * TCC, c0y = blockIdx.y * TCC;
  {
    T v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      const int rr = e / CW, cc = e - rr * CW;
      const int gy = c0y * K + rr, gx = c0x * K + cc;
      v[q] = (e < CW * CW && gy < nc && gx < nc) ? ec[(size_t)gy * nc + gx] : T(0);
    }
    for (int e = threadIdx.x; e < NT; e += kThreads) sTb[e] = tab[e];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < CW * CW) sC[e] = v[q];
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < CW * FT; it += kThreads) {
    const int rr = it / FT, l = it - rr * FT;
    const int cf = l / K, p = l - cf * K, cl = cf >> 1, s2 = cf & 1;  // local coarse cell cl
    const T* tb = sTb + (s2 * K + p) * (K + 1);
    const T* src = sC + rr * CW + cl * K;
    T v = 0;
#pragma unroll
    for (int a = 0; a <= K; ++a) v += tb[a] * src[a];
    sT[it] = v;
  }
  __syncthreads();
  // fine nodes [2k c0, 2k (c0 + TCC)) of this tile, plus the last (boundary)
  // node of the mesh for the last tile, so that every output is written
  constexpr int FO = FT + 1;
  for (int it = threadIdx.x; it < FO * FO; it += kThreads) {
    const int m = it / FO, l = it - m * FO;
    const int fx = 2 * K * c0x + l, fy = 2 * K * c0y + m;
    if (fx >= nf || fy >= nf) continue;
    if ((l == FT && fx != nf - 1) || (m == FT && fy != nf - 1)) continue;
    const size_t idx = (size_t)fy * nf + fx;
    if (fx == 0 || fy == 0 || fx == nf - 1 || fy == nf - 1) {
      xf[idx] = T(0);
      continue;
    }
    const int cf = m / K, p = m - cf * K, cl = cf >> 1, s2 = cf & 1;
    const T* tb = sTb + (s2 * K + p) * (K + 1);
    const T* src = sT + (cl * K) * FT + l;
    T v = 0;
#pragma unroll
    for (int a = 0; a <= K; ++a) v += tb[a] * src[a * FT];
    xf[idx] = xin[idx] + v;
  }
}

template <typename T, int K>
hipError_t restrict2d_k(int Nc, const T* tab, const T* rf, T* bc, hipStream_t s, int nsys, int64_t zf,
                        int64_t zc, const int* active) {
  constexpr int TCC = TransferTile2D<K>::TCC;
  const int nt = (Nc + TCC - 1) / TCC;
  restrict2d_kernel<T, K, TCC><<<dim3(nt, nt, nsys), kThreads, 0, s>>>(rf, bc, Nc, tab, zf, zc, active);
  return hipGetLastError();
}

template <typename T, int K>
hipError_t prolong2d_k(int Nc, const T* tab, const T* ec, const T* xin, T* xf, hipStream_t s, int nsys,
                       int64_t zc, int64_t zf, const int* active) {
  constexpr int TCC = TransferTile2D<K>::TCC;
  const int nt = (Nc + TCC - 1) / TCC;
  prolong2d_kernel<T, K, TCC><<<dim3(nt, nt, nsys), kThreads, 0, s>>>(ec, xin, xf, Nc, tab, zc, zf, active);
  return hipGetLastError();
}

}  // namespace

template <typename Tin, typename T>
hipError_t launch_apply2d(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s,
                          int nsys, int64_t zs, const int* active) {
#define CALL(K) apply2d_k<Tin, T, K>(N, c, x, b, y, s, nsys, zs, active)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_patch2d(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s, int nsys, int64_t zs, const int* active) {
#define CALL(K) patch2d_k<T, K>(N, e, r, xin, xout, omega, s, nsys, zs, active)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_restrict2d(int k, int Nc, const T* table, const T* rf, T* bc, hipStream_t s, int nsys,
                             int64_t zf, int64_t zc, const int* active) {
#define CALL(K) restrict2d_k<T, K>(Nc, table, rf, bc, s, nsys, zf, zc, active)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_prolong2d(int k, int Nc, const T* table, const T* ec, const T* xin, T* xf, hipStream_t s,
                            int nsys, int64_t zc, int64_t zf, const int* active) {
#define CALL(K) prolong2d_k<T, K>(Nc, table, ec, xin, xf, s, nsys, zc, zf, active)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template hipError_t launch_restrict2d<double>(int, int, const double*, const double*, double*, hipStream_t, int,
                                              int64_t, int64_t, const int*);
template hipError_t launch_restrict2d<float>(int, int, const float*, const float*, float*, hipStream_t, int, int64_t,
                                             int64_t, const int*);
template hipError_t launch_prolong2d<double>(int, int, const double*, const double*, const double*, double*,
                                             hipStream_t, int, int64_t, int64_t, const int*);
template hipError_t launch_prolong2d<float>(int, int, const float*, const float*, const float*, float*, hipStream_t,
                                            int, int64_t, int64_t, const int*);
template <typename T>
hipError_t launch_avs2d(int k, int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout,
                        T omega, hipStream_t s, int nsys, int64_t zs, const int* active, int variant) {
#define CALL(K) avs2d_k<T, K>(N, c, e, x, b, xout, omega, s, nsys, zs, active, variant)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}
int avs2d_variants(int k) {
  switch (k) {
    case 2: return FusedTiles<2>::n;
    case 3: return FusedTiles<3>::n;
    case 4: return FusedTiles<4>::n;
    case 5: return FusedTiles<5>::n;
    case 6: return FusedTiles<6>::n;
    case 7: return FusedTiles<7>::n;
    default: return 1;
  }
}
template hipError_t launch_avs2d<double>(int, int, const LevelCoef<double>&, const LevelEig<double>&, const double*,
                                         const double*, double*, double, hipStream_t, int, int64_t, const int*, int);
template hipError_t launch_avs2d<float>(int, int, const LevelCoef<float>&, const LevelEig<float>&, const float*,
                                        const float*, float*, float, hipStream_t, int, int64_t, const int*, int);
template hipError_t launch_apply2d<double, double>(int, int, const LevelCoef<double>&, const double*,
                                                   const double*, double*, hipStream_t, int, int64_t, const int*);
template hipError_t launch_apply2d<float, double>(int, int, const LevelCoef<double>&, const float*,
                                                  const double*, double*, hipStream_t, int, int64_t, const int*);
template hipError_t launch_apply2d<float, float>(int, int, const LevelCoef<float>&, const float*, const float*,
                                                 float*, hipStream_t, int, int64_t, const int*);
template hipError_t launch_patch2d<double>(int, int, const LevelEig<double>&, const double*, const double*,
                                           double*, double, hipStream_t, int, int64_t, const int*);
template hipError_t launch_patch2d<float>(int, int, const LevelEig<float>&, const float*, const float*, float*,
                                          float, hipStream_t, int, int64_t, const int*);

}  // namespace c0ip
