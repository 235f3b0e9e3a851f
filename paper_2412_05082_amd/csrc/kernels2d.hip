// 2D kernels for gfx950: the unfused vertex-patch smoother step and the
// grid transfers (the operator and the fused smoother are in op2d.hip).
//
// Smoother (Sec. 3 additive vertex-patch Schwarz; local solver of eq.
// localsolverbila inverted by eq. inverse):
//   x_out = x_in + omega * sum_v R_v^T (Q_y (x) Q_x) D_v^{-1} (Q_y (x) Q_x)^T R_v r.
// Owner-computes: a workgroup owns a tile of TC x TC cells, solves the
// (TC+1)^2 patches that touch it (neighbouring tiles solve shared patches
// twice instead of racing on writes), and writes each owned DoF once.
#include <algorithm>

#include "exact.h"
#include "fdm.h"
#include "kernels.h"
#include "tiles.h"

namespace c0ip {
namespace {

constexpr int kThreads = tile::kThreads;
using tile::variant;
using tile::xcd_tile;

// ------------------------------------------------------------------ smoother

template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void patch2d_kernel(const T* __restrict__ r, const T* __restrict__ xin,
                                                           T* __restrict__ xout, int N, int n1,
                                                           const T* __restrict__ Qg, const T* __restrict__ lamg,
                                                           T omega, int64_t zs, const int* __restrict__ active) {
  constexpr int n = 2 * K - 1, NN = n * n, NP = TC + 1, S = (TC + 2) * K - 1;
  // small patches (k <= 3): one thread per patch, transforms in registers (for k = 4 this was measured
  // several times slower than the passes below)
  constexpr bool REG = NN <= 25;
  if (active && !active[blockIdx.z]) return;
  r += blockIdx.z * zs;
  xout += blockIdx.z * zs;
  if (xin) xin += blockIdx.z * zs;
  constexpr int NL = (S * S + kThreads - 1) / kThreads;
  __shared__ T sR[S * S];
  __shared__ T sA[NP * NP * NN];
  __shared__ T sB[REG ? 1 : NP * NP * NN];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  __shared__ T sD[NN];
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
    tile::stage_eig<T, n, kThreads>(Qg, lamg, sQ, sLam, sD);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * kThreads;
      if (e < S * S) sR[e] = v[q];
    }
  }
  __syncthreads();
  if constexpr (REG) {
    // every patch of an interior tile has the interior basis (wave-uniform reads)
    const bool interior = cx0 >= 2 && cx0 + TC <= N - 2 && cy0 >= 2 && cy0 + TC <= N - 2;
    for (int p = threadIdx.x; p < NP * NP; p += kThreads) {
      const int pyl = p / NP, pxl = p - pyl * NP;
      const int vx = cx0 + pxl, vy = cy0 + pyl;
      if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
      const T* src = sR + (pyl * K) * S + pxl * K;
      if (interior) {
        fdm::patch_reg<T, n>(src, S, sA + p * NN, [&](int i) { return Qg[i]; }, [&](int i) { return Qg[i]; },
                             [&](int ap, int c) { return sD[ap * n + c]; });
      } else {
        const int tx = variant(vx, N), ty = variant(vy, N);
        const T* qx = sQ + tx * NN;
        const T* qy = sQ + ty * NN;
        const T* lx = sLam + tx * n;
        const T* ly = sLam + ty * n;
        fdm::patch_reg<T, n>(src, S, sA + p * NN, [&](int i) { return qx[i]; }, [&](int i) { return qy[i]; },
                             [&](int ap, int c) { return T(1) / (lx[c] + ly[ap]); });
      }
    }
    __syncthreads();
  } else {
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
  }
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

template <int K> struct PatchTile2D;
template <> struct PatchTile2D<2> { static constexpr int TC = 15; };  // 256 patches: one per thread
template <> struct PatchTile2D<3> { static constexpr int TC = 15; };
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

// Owner-computes smoother step with exact local solves: as patch2d_kernel,
// but each patch correction is the dense product A_v^{-1} r_v (one inverse
// per patch type, read through the cache; on interior tiles every patch has
// the interior type, so the reads are wave-uniform across patches).
template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void patch2d_exact_kernel(const T* __restrict__ r, const T* __restrict__ xin,
                                                                 T* __restrict__ xout, int N, int n1,
                                                                 const T* __restrict__ Aex, T omega) {
  constexpr int n = 2 * K - 1, NN = n * n, NP = TC + 1, S = (TC + 2) * K - 1;
  __shared__ T sR[S * S];
  __shared__ T sA[NP * NP * NN];
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int cx0 = tbx * TC, cy0 = tby * TC;
  const int ox = (cx0 - 1) * K + 1, oy = (cy0 - 1) * K + 1;  // global node of region (0,0)
  for (int e = threadIdx.x; e < S * S; e += kThreads) {
    const int rr = e / S, cc = e - rr * S;
    const int gy = oy + rr, gx = ox + cc;
    sR[e] = (gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2) ? r[(size_t)gy * n1 + gx] : T(0);
  }
  __syncthreads();
  // u[i] = sum_j A_v^{-1}[i][j] r_v[j] for every patch touching the tile
  for (int it = threadIdx.x; it < NP * NP * NN; it += kThreads) {
    const int p = it / NN, i = it - p * NN;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = cx0 + pxl, vy = cy0 + pyl;
    if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1) continue;
    const T* row = Aex + (size_t)(variant(vy, N) * 4 + variant(vx, N)) * NN * NN + (size_t)i * NN;
    T s = 0;
    for (int a = 0; a < n; ++a) {
      const T* rr = sR + (pyl * K + a) * S + pxl * K;
#pragma unroll
      for (int c = 0; c < n; ++c) s += row[a * n + c] * rr[c];
    }
    sA[it] = s;
  }
  __syncthreads();
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

template <int K> struct ExactTile2D { static constexpr int TC = K <= 3 ? 8 : 4; };

template <typename T, int K>
hipError_t patch2d_exact_k(int N, const T* Aex, const T* r, const T* xin, T* xout, T omega, hipStream_t s) {
  constexpr int TC = ExactTile2D<K>::TC;
  const int nt = (N + TC - 1) / TC;
  patch2d_exact_kernel<T, K, TC><<<dim3(nt, nt), kThreads, 0, s>>>(r, xin, xout, N, K * N + 1, Aex, omega);
  return hipGetLastError();
}

// Atomic-scatter form of the smoother step (the comparison variant): a
// workgroup solves TC x TC patches, each exactly once (no redundant border
// patches), and adds omega times every patch correction into x_out with
// hardware floating-point atomics.  The caller initialises x_out (x_in or
// 0); the summation order of overlapping patches is not fixed, so results
// agree with the owner-computes kernels to rounding, not bit for bit.
template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void patch2d_atomic_kernel(const T* __restrict__ r, T* __restrict__ xout,
                                                                  int N, int n1, const T* __restrict__ Qg,
                                                                  const T* __restrict__ lamg, T omega) {
  constexpr int n = 2 * K - 1, NN = n * n, NP = TC, S = (TC + 1) * K - 1;
  __shared__ T sR[S * S];
  __shared__ T sA[NP * NP * NN];
  __shared__ T sB[NP * NP * NN];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int vx0 = tbx * TC + 1, vy0 = tby * TC + 1;  // first vertex of the block
  const int ox = (vx0 - 1) * K + 1, oy = (vy0 - 1) * K + 1;
  for (int e = threadIdx.x; e < S * S; e += kThreads) {
    const int rr = e / S, cc = e - rr * S;
    const int gy = oy + rr, gx = ox + cc;
    sR[e] = (gx >= 1 && gx <= n1 - 2 && gy >= 1 && gy <= n1 - 2) ? r[(size_t)gy * n1 + gx] : T(0);
  }
  for (int e = threadIdx.x; e < 4 * NN; e += kThreads) sQ[e] = Qg[e];
  for (int e = threadIdx.x; e < 4 * n; e += kThreads) sLam[e] = lamg[e];
  __syncthreads();
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, a = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = vx0 + pxl, vy = vy0 + pyl;
    if (vx > N - 1 || vy > N - 1) continue;
    const T* q = sQ + variant(vx, N) * NN;
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
  for (int it = threadIdx.x; it < NP * NP * n; it += kThreads) {
    const int p = it / n, c = it - p * n;
    const int pyl = p / NP, pxl = p - pyl * NP;
    const int vx = vx0 + pxl, vy = vy0 + pyl;
    if (vx > N - 1 || vy > N - 1) continue;
    const int ty = variant(vy, N), tx = variant(vx, N);
    const T* q = sQ + ty * NN;
    T col[n], t[n];
#pragma unroll
    for (int a = 0; a < n; ++a) col[a] = sA[p * NN + a * n + c];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += q[a * n + ap] * col[a];
      t[ap] = s / (sLam[tx * n + c] + sLam[ty * n + ap]);
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
    const int vx = vx0 + pxl, vy = vy0 + pyl;
    if (vx > N - 1 || vy > N - 1) continue;
    const T* q = sQ + variant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = sB[p * NN + a * n + c];
    const int gy = (vy - 1) * K + 1 + a, gx0 = (vx - 1) * K + 1;
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += q[cp * n + c] * in[c];
      unsafeAtomicAdd(xout + (size_t)gy * n1 + gx0 + cp, omega * s);
    }
  }
}

template <typename T, int K>
hipError_t patch2d_atomic_k(int N, const LevelEig<T>& e, const T* r, T* xout, T omega, hipStream_t s) {
  constexpr int TC = PatchTile2D<K>::TC;
  const int n1 = K * N + 1;
  const int nt = (N - 1 + TC - 1) / TC;
  patch2d_atomic_kernel<T, K, TC><<<dim3(nt, nt), kThreads, 0, s>>>(r, xout, N, n1, e.Q, e.lam, omega);
  return hipGetLastError();
}

// ------------------------------------------------------ coloured multiplicative
// One colour of the coloured multiplicative smoother (Sec. 3, Fig. 2):
//   x <- x + omega * sum_{v of colour c} R_v^T A~_v^{-1} R_v r,   r = b - A x
// taken after the previous colour.  Colour c = px + 2 py + 4 rb holds the
// vertices v = (2a + px, 2b + py) in [1, N-1]^2 with (a + b) mod 2 = rb;
// their patches share no node and no entry of A couples two of them, so
// each patch is solved once and its correction is added in place with a
// plain store (no other patch of the colour touches its nodes).  The
// vertices of a colour are numbered row by row of b; rows alternate
// between two lengths.

struct ColourRows {
  int a_lo, a_hi, b_lo, nb;  // lattice ranges of a and b
  int rb;
  int cnt0, cnt1;            // patches in rows b_lo + 2i and b_lo + 2i + 1
  int total;
};

__host__ __device__ inline int colour_row_count(int a_lo, int a_hi, int b, int rb) {
  const int af = a_lo + (((rb - a_lo - b) % 2) + 2) % 2;
  return af <= a_hi ? (a_hi - af) / 2 + 1 : 0;
}

inline ColourRows colour_rows(int N, int c) {
  const int px = c & 1, py = (c >> 1) & 1;
  ColourRows cr;
  cr.rb = (c >> 2) & 1;
  cr.a_lo = px == 0 ? 1 : 0;
  cr.a_hi = (N - 1 - px) / 2;
  cr.b_lo = py == 0 ? 1 : 0;
  const int b_hi = (N - 1 - py) / 2;
  cr.nb = b_hi >= cr.b_lo ? b_hi - cr.b_lo + 1 : 0;
  cr.cnt0 = colour_row_count(cr.a_lo, cr.a_hi, cr.b_lo, cr.rb);
  cr.cnt1 = colour_row_count(cr.a_lo, cr.a_hi, cr.b_lo + 1, cr.rb);
  cr.total = (cr.nb / 2) * (cr.cnt0 + cr.cnt1) + (cr.nb % 2) * cr.cnt0;
  return cr;
}

// vertex (vx, vy) of the patch with number q of the colour
__device__ __forceinline__ void colour_vertex(const ColourRows& cr, int px, int py, int q, int& vx, int& vy) {
  const int pair = cr.cnt0 + cr.cnt1;
  const int i = q / pair, rem = q - i * pair;
  const int b = cr.b_lo + 2 * i + (rem >= cr.cnt0 ? 1 : 0);
  const int t = rem >= cr.cnt0 ? rem - cr.cnt0 : rem;
  const int af = cr.a_lo + (((cr.rb - cr.a_lo - b) % 2) + 2) % 2;
  vx = 2 * (af + 2 * t) + px;
  vy = 2 * b + py;
}

// Patches per workgroup of the colour kernel and its LDS strips.  A patch's
// residual rows (its (2k-1)^2 interior nodes) reach, through the bands of
// the 1D factors, the nodes of the patch's cells (M, L: 2k+1 per axis) and
// of the cells next to them (B: 4k+1 per axis).  The operator is
// M_y (X B_x) + 2 L_y (X L_x) + B_y (X M_x), so two strips of x suffice:
// the patch rows over 4k+1 columns (for X B_x and X L_x) and 4k+1 rows over
// the patch columns (for X M_x).  Neither strip holds a node interior to
// another patch of the colour: patches of one colour are 4 cells apart
// along an axis or 2 cells apart along both, so their interiors never fall
// inside the closed patch rows or columns.  NP patches fill a workgroup
// with one local-solve output per thread; the coefficient table (at most
// 5k+2 row classes) is staged in LDS.
template <int K>
struct ColourFused {
  static constexpr int n = 2 * K - 1, NN = n * n, C = 2 * K + 1, W = 4 * K + 1, R = C * W;
  static constexpr int NP = kThreads / NN > 0 ? kThreads / NN : 1;
  static constexpr int MAXCLASS = 5 * K + 2, TAB = 3 * MAXCLASS * W;
  static_assert(NP * NN <= kThreads, "one node per thread in the y passes and the update");
};

// Band products for a row at cell position P (compile time), taps `stride`
// apart from the row's own tap v[0]; c: the row's coefficients, centred.
// Each accumulates its taps from the band's low end up, as the tiled
// operator does.
template <typename T, int OP, int K, int P>
__device__ __forceinline__ T band_fixed(const T* c, const T* v, int stride) {
  T a = 0;
#pragma unroll
  for (int o = tile::Band<OP, K>::lo(P); o <= tile::Band<OP, K>::hi(P); ++o) a += c[o] * v[o * stride];
  return a;
}

// OP at the row's cell position p (a runtime value, nearly uniform over a wave).
template <typename T, int OP, int K, int P = 0>
__device__ __forceinline__ T band_at(const T* c, int p, const T* v, int stride) {
  if constexpr (P + 1 < K) {
    if (p != P) return band_at<T, OP, K, P + 1>(c, p, v, stride);
  }
  return band_fixed<T, OP, K, P>(c, v, stride);
}

// B and L of one row over the same taps (B's band contains L's), sharing the loads.
template <typename T, int K, int P>
__device__ __forceinline__ void band_bl_fixed(const T* cB, const T* cL, const T* v, T& aB, T& aL) {
  using BB = tile::Band<2, K>;
  using BL = tile::Band<1, K>;
  aB = 0;
  aL = 0;
#pragma unroll
  for (int o = BB::lo(P); o <= BB::hi(P); ++o) {
    const T w = v[o];
    aB += cB[o] * w;
    if (o >= BL::lo(P) && o <= BL::hi(P)) aL += cL[o] * w;
  }
}

template <typename T, int K, int P = 0>
__device__ __forceinline__ void band_bl_at(const T* cB, const T* cL, int p, const T* v, T& aB, T& aL) {
  if constexpr (P + 1 < K) {
    if (p != P) {
      band_bl_at<T, K, P + 1>(cB, cL, p, v, aB, aL);
      return;
    }
  }
  band_bl_fixed<T, K, P>(cB, cL, v, aB, aL);
}

// Row cl of factor OP in the LDS table, centred on its own tap.
template <typename T, int OP, int K>
__device__ __forceinline__ const T* table_row(const T* sTab, int nclass, int cl) {
  return sTab + (OP * nclass + cl) * (4 * K + 1) + 2 * K;
}

// x <- x + omega * sum over the colour's patches of R_v^T A~_v^{-1} R_v r
// (or of R_v^T A_v^{-1} R_v r with the exact local matrices), r = b - A x
// formed on the patch rows in LDS, or read from rsrc when that is given (a
// residual computed beforehand, or b when x is 0).
template <typename T, int K, bool EXACT>
__global__ __launch_bounds__(kThreads) void mvs2d_colour_kernel(const T* __restrict__ b, T* __restrict__ x, int N,
                                                                int n1, ColourRows cr, int px, int py,
                                                                const T* __restrict__ tab, int nclass, int left,
                                                                int right0, int periodic, const T* __restrict__ rsrc,
                                                                const T* __restrict__ Qg, const T* __restrict__ lamg,
                                                                const T* __restrict__ Aex, T omega) {
  using F = ColourFused<K>;
  constexpr int n = F::n, NN = F::NN, C = F::C, W = F::W, R = F::R, NP = F::NP;
  __shared__ T sRow[NP * R];   // rows (vy-1)K .. (vy+1)K, columns (vx-2)K .. (vx+2)K
  __shared__ T sCol[NP * R];   // rows (vy-2)K .. (vy+2)K, columns (vx-1)K .. (vx+1)K
  __shared__ T sTB[NP * C * n];
  __shared__ T sTL[NP * C * n];
  __shared__ T sTM[NP * W * n];
  __shared__ T sA[NP * NN];
  __shared__ T sB[NP * NN];
  __shared__ T sTab[F::TAB];
  __shared__ T sQ[EXACT ? 1 : 4 * NN];
  __shared__ T sLam[EXACT ? 1 : 4 * n];
  const int q0 = blockIdx.x * NP;
  const int np = min(NP, cr.total - q0);
  if (np <= 0) return;
  // This thread's node of the y passes and the update (at most one: NP (2K-1)^2 <= kThreads; rows
  // slowest).  Its b (or r) and x are loaded first, so that their latency overlaps the staging.
  const bool mine = threadIdx.x < np * NN;
  int ya = 0, yp = 0, yc = 0, vxm = 1, vym = 1;
  if (mine) {
    ya = threadIdx.x / (np * n);
    const int rem = threadIdx.x - ya * (np * n);
    yp = rem / n;
    yc = rem - yp * n;
    colour_vertex(cr, px, py, q0 + yp, vxm, vym);
  }
  const size_t gm = (size_t)((vym - 1) * K + 1 + ya) * n1 + (vxm - 1) * K + 1 + yc;
  const T bm = mine ? (rsrc ? rsrc[gm] : b[gm]) : T(0);
  const T xm = mine ? x[gm] : T(0);
  if (rsrc) {
    if (mine) sB[yp * NN + ya * n + yc] = bm;
  } else {
    // stage the two strips of x (zero outside the mesh) and the table, every load issued before the stores
    constexpr int NS = (NP * R + kThreads - 1) / kThreads, NT = (F::TAB + kThreads - 1) / kThreads;
    T vr[NS], vc[NS], vt[NT];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = threadIdx.x + u * kThreads;
      vr[u] = vc[u] = T(0);
      if (e < np * R) {
        const int p = e / R, loc = e - p * R;
        int vx, vy;
        colour_vertex(cr, px, py, q0 + p, vx, vy);
        const int i = loc / W, j = loc - i * W;
        const int gy = (vy - 1) * K + i, gx = (vx - 2) * K + j;
        if (gx >= 0 && gx < n1) vr[u] = x[(size_t)gy * n1 + gx];
        const int i2 = loc / C, j2 = loc - i2 * C;
        const int gy2 = (vy - 2) * K + i2, gx2 = (vx - 1) * K + j2;
        if (gy2 >= 0 && gy2 < n1) vc[u] = x[(size_t)gy2 * n1 + gx2];
      }
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int e = threadIdx.x + u * kThreads;
      vt[u] = e < 3 * nclass * W ? tab[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = threadIdx.x + u * kThreads;
      if (e < np * R) {
        sRow[e] = vr[u];
        sCol[e] = vc[u];
      }
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int e = threadIdx.x + u * kThreads;
      if (e < 3 * nclass * W) sTab[e] = vt[u];
    }
    __syncthreads();
    // x passes at the patch's interior columns: X B_x and X L_x on the patch
    // rows, X M_x on 4K+1 rows (items ordered column-major, so that the
    // lanes of a wave mostly share a column and its band extent)
    for (int e = threadIdx.x; e < np * (C + W) * n; e += kThreads) {
      const int c = e / (np * (C + W)), rem = e - c * (np * (C + W)), p = rem / (C + W), i = rem - p * (C + W);
      int vx, vy;
      colour_vertex(cr, px, py, q0 + p, vx, vy);
      const int gx = (vx - 1) * K + 1 + c, pc = (1 + c) % K;
      const int cl = tile::row_class(gx, n1, K, left, right0, periodic);
      if (i < C) {
        T aB, aL;
        band_bl_at<T, K>(table_row<T, 2, K>(sTab, nclass, cl), table_row<T, 1, K>(sTab, nclass, cl), pc,
                         sRow + p * R + i * W + K + 1 + c, aB, aL);
        sTB[(p * C + i) * n + c] = aB;
        sTL[(p * C + i) * n + c] = aL;
      } else {
        const int iw = i - C;
        sTM[(p * W + iw) * n + c] =
            band_at<T, 0, K>(table_row<T, 0, K>(sTab, nclass, cl), pc, sCol + p * R + iw * C + 1 + c, 1);
      }
    }
    __syncthreads();
    // y passes: r = b - (M_y TB + 2 L_y TL + B_y TM) at this thread's node
    if (mine) {
      const int gy = (vym - 1) * K + 1 + ya, pa = (1 + ya) % K;
      const int cl = tile::row_class(gy, n1, K, left, right0, periodic);
      const T ax = band_at<T, 0, K>(table_row<T, 0, K>(sTab, nclass, cl), pa, sTB + (yp * C + 1 + ya) * n + yc, n) +
                   T(2) * band_at<T, 1, K>(table_row<T, 1, K>(sTab, nclass, cl), pa,
                                           sTL + (yp * C + 1 + ya) * n + yc, n) +
                   band_at<T, 2, K>(table_row<T, 2, K>(sTab, nclass, cl), pa, sTM + (yp * W + K + 1 + ya) * n + yc,
                                    n);
      sB[yp * NN + ya * n + yc] = bm - ax;
    }
  }
  if constexpr (EXACT) {
    // exact local solves: u = A_v^{-1} r_v, one dense row per thread and patch
    __syncthreads();
    for (int it = threadIdx.x; it < np * NN; it += kThreads) {
      const int p = it / NN, i = it - p * NN;
      int vx, vy;
      colour_vertex(cr, px, py, q0 + p, vx, vy);
      const T* row = Aex + (size_t)(variant(vy, N) * 4 + variant(vx, N)) * NN * NN + (size_t)i * NN;
      const T* rv = sB + p * NN;
      T s = 0;
      for (int j = 0; j < NN; ++j) s += row[j] * rv[j];
      sA[it] = s;
    }
  } else {
    // fast diagonalisation, one output per thread and stage:
    // r (sB) -> Q_x^T along x (sA) -> Q_y^T along y, / (lambda_x + lambda_y) (sB)
    //        -> Q_y along y (sA) -> Q_x along x (sB)
    for (int e = threadIdx.x; e < 4 * NN; e += kThreads) sQ[e] = Qg[e];
    for (int e = threadIdx.x; e < 4 * n; e += kThreads) sLam[e] = lamg[e];
    __syncthreads();
    const int e = threadIdx.x;
    const bool on = e < np * NN;
    const int p = on ? e / NN : 0, loc = e - p * NN, a = loc / n, c = loc - a * n;
    int vx = 1, vy = 1;
    if (on) colour_vertex(cr, px, py, q0 + p, vx, vy);
    const int tx = variant(vx, N), ty = variant(vy, N);
    const T* qx = sQ + tx * NN;
    const T* qy = sQ + ty * NN;
    T* pA = sA + p * NN;
    T* pB = sB + p * NN;
    if (on) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) s += qx[j * n + c] * pB[a * n + j];
      pA[a * n + c] = s;
    }
    __syncthreads();
    if (on) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) s += qy[j * n + a] * pA[j * n + c];
      pB[a * n + c] = s / (sLam[tx * n + c] + sLam[ty * n + a]);
    }
    __syncthreads();
    if (on) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) s += qy[a * n + j] * pB[j * n + c];
      pA[a * n + c] = s;
    }
    __syncthreads();
    if (on) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < n; ++j) s += qx[c * n + j] * pA[a * n + j];
      pB[a * n + c] = s;
    }
  }
  __syncthreads();
  // x += omega u at this thread's node (no other workgroup of the launch reads or writes it)
  const T* u = EXACT ? sA : sB;
  if (mine) x[gm] = xm + omega * u[yp * NN + ya * n + yc];
}

template <typename T, int K, bool EXACT>
hipError_t mvs2d_colour_k(int N, int colour, const LevelCoef<T>& cf, const T* Q, const T* lam, const T* Aex,
                          const T* b, const T* r, T* x, T omega, hipStream_t s) {
  constexpr int NP = ColourFused<K>::NP;
  const ColourRows cr = colour_rows(N, colour);
  if (cr.total <= 0) return hipSuccess;
  if (cf.nclass > ColourFused<K>::MAXCLASS) return hipErrorInvalidValue;
  const int nblk = (cr.total + NP - 1) / NP;
  mvs2d_colour_kernel<T, K, EXACT><<<nblk, kThreads, 0, s>>>(b, x, N, K * N + 1, cr, colour & 1, (colour >> 1) & 1,
                                                            cf.tab, cf.nclass, cf.left, cf.right0, cf.periodic,
                                                            r, Q, lam, Aex, omega);
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

template <typename T>
hipError_t launch_patch2d(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s, int nsys, int64_t zs, const int* active) {
#define CALL(K) patch2d_k<T, K>(N, e, r, xin, xout, omega, s, nsys, zs, active)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_patch2d_atomic(int k, int N, const LevelEig<T>& e, const T* r, T* xout, T omega, hipStream_t s) {
#define CALL(K) patch2d_atomic_k<T, K>(N, e, r, xout, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_mvs2d_colour(int k, int N, int colour, const LevelCoef<T>& c, const LevelEig<T>& e, const T* b,
                               const T* r, T* x, T omega, hipStream_t s) {
#define CALL(K) mvs2d_colour_k<T, K, false>(N, colour, c, e.Q, e.lam, nullptr, b, r, x, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_patch2d_exact(int k, int N, const T* Aex, const T* r, const T* xin, T* xout, T omega,
                                hipStream_t s) {
#define CALL(K) patch2d_exact_k<T, K>(N, Aex, r, xin, xout, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_mvs2d_colour_exact(int k, int N, int colour, const LevelCoef<T>& c, const T* Aex, const T* b,
                                     const T* r, T* x, T omega, hipStream_t s) {
#define CALL(K) mvs2d_colour_k<T, K, true>(N, colour, c, nullptr, nullptr, Aex, b, r, x, omega, s)
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
template hipError_t launch_patch2d_atomic<double>(int, int, const LevelEig<double>&, const double*, double*,
                                                  double, hipStream_t);
template hipError_t launch_patch2d_atomic<float>(int, int, const LevelEig<float>&, const float*, float*, float,
                                                 hipStream_t);
template hipError_t launch_mvs2d_colour<double>(int, int, int, const LevelCoef<double>&, const LevelEig<double>&,
                                                const double*, const double*, double*, double, hipStream_t);
template hipError_t launch_mvs2d_colour<float>(int, int, int, const LevelCoef<float>&, const LevelEig<float>&,
                                                const float*, const float*, float*, float, hipStream_t);
template hipError_t launch_patch2d_exact<double>(int, int, const double*, const double*, const double*, double*,
                                                 double, hipStream_t);
template hipError_t launch_patch2d_exact<float>(int, int, const float*, const float*, const float*, float*, float,
                                                hipStream_t);
template hipError_t launch_mvs2d_colour_exact<double>(int, int, int, const LevelCoef<double>&, const double*,
                                                      const double*, const double*, double*, double, hipStream_t);
template hipError_t launch_mvs2d_colour_exact<float>(int, int, int, const LevelCoef<float>&, const float*,
                                                      const float*, const float*, float*, float, hipStream_t);
template hipError_t launch_patch2d<double>(int, int, const LevelEig<double>&, const double*, const double*,
                                           double*, double, hipStream_t, int, int64_t, const int*);
template hipError_t launch_patch2d<float>(int, int, const LevelEig<float>&, const float*, const float*, float*,
                                          float, hipStream_t, int, int64_t, const int*);

}  // namespace c0ip
