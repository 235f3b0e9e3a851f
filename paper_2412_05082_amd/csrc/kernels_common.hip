// Dimension-independent kernels: grid transfers, the level-0 solve and the
// Krylov vector kernels.
//
// Transfers (Sec. 3): prolongation = embedding of Q_k on the coarse mesh
// into Q_k on the refined mesh, restriction = its transpose.  Both are
// tensor products of one 1D matrix and are applied one axis at a time;
// along an axis a vector is viewed as [outer][n_axis][inner].
#include "kernels.h"

namespace c0ip {
namespace {

constexpr int kThreads = 256;

// Division by a divisor fixed for a launch (Granlund-Montgomery): q = n / d
// for 0 <= n < 2^31 and 1 <= d < 2^31 with one high multiply, an add and a
// shift instead of a 64-bit division per element.
struct FastDiv {
  uint32_t d = 1, m = 0, l = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t dv) : d(dv) {
    while ((1ull << l) < d) ++l;
    m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)__umulhi(n, m) + n) >> l);
  }
};

inline int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > (1 << 20)) b = 1 << 20;
  if (b < 1) b = 1;
  return (int)b;
}

// out[i_f] (+)= sum_a T[s][p][a] in[cc k + a],  fine node i_f = (2cc+s) k + p.
// One item per (inner index, coarse cell, outer index), item indices below
// 2^31 (checked by the launcher): ii = idx mod inner, cc = (idx / inner) mod
// ncell, io = idx / (inner ncell), by fixed divisors.  The item's positions
// in the cell are compile-time, so the table entries are wave-uniform.

// Prolongation along one axis: coarse cell cc (coarse nodes cc k .. cc k + k)
// gives the 2k fine nodes of fine cells 2cc, 2cc+1:
//   out[(2cc+s) k + p] (+)= sum_a T[s][p][a] in[cc k + a];
// the cell cc = Nc - 1 also writes the last fine node, and the first and
// last fine nodes (boundary) get 0.
template <typename T, int K, bool ACC>
__global__ __launch_bounds__(kThreads) void prolong1d_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                             int64_t inner, int nin, int nout, int64_t outer,
                                                             const T* __restrict__ tab, FastDiv dinner,
                                                             FastDiv dcell) {
  const int ncell = nin / K;  // Nc
  const uint32_t total = (uint32_t)(inner * ncell * outer);
  for (uint32_t idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
    const uint32_t rest = dinner.div(idx), iq = dcell.div(rest);
    const int64_t ii = idx - rest * (uint32_t)inner;
    const int cc = (int)(rest - iq * (uint32_t)ncell);
    const int64_t io = iq;
    const T* base = in + ii + inner * ((int64_t)cc * K + (int64_t)nin * io);
    T c[K + 1];
#pragma unroll
    for (int a = 0; a <= K; ++a) c[a] = base[a * inner];
    T* o = out + ii + inner * ((int64_t)nout * io);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int p = 0; p < K; ++p) {
        const int f = (2 * cc + s) * K + p;
        T v = 0;
#pragma unroll
        for (int a = 0; a <= K; ++a) v += tab[(s * K + p) * (K + 1) + a] * c[a];
        if (f == 0) v = T(0);
        if (ACC)
          o[inner * f] += v;
        else
          o[inner * f] = v;
      }
    if (cc == ncell - 1 && !ACC) o[inner * (nout - 1)] = T(0);
  }
}

// Restriction along one axis (the transpose): coarse cell cc gives the
// coarse nodes cc k + a, a < k, from the fine nodes of fine cells 2cc-2 ..
// 2cc+1 (the vertex a = 0 also collects the coarse basis of cell cc-1):
//   out[cc k + a] = sum_{s,p} T[s][p][a] in[(2cc+s) k + p]
//                 + [a = 0] sum_{s,p} T[s][p][k] in[(2cc-2+s) k + p];
// cc = Nc writes the last coarse node; boundary nodes get 0.
template <typename T, int K>
__global__ __launch_bounds__(kThreads) void restrict1d_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                              int64_t inner, int nin, int nout, int64_t outer,
                                                              const T* __restrict__ tab, FastDiv dinner,
                                                              FastDiv dcell) {
  const int ncell = nout / K + 1;  // Nc + 1
  const uint32_t total = (uint32_t)(inner * ncell * outer);
  for (uint32_t idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += gridDim.x * kThreads) {
    const uint32_t rest = dinner.div(idx), iq = dcell.div(rest);
    const int64_t ii = idx - rest * (uint32_t)inner;
    const int cc = (int)(rest - iq * (uint32_t)ncell);
    const int64_t io = iq;
    T* o = out + ii + inner * ((int64_t)nout * io);
    if (cc == ncell - 1) {  // the last coarse node (boundary)
      o[inner * (int64_t)(nout - 1)] = T(0);
      continue;
    }
    const T* base = in + ii + inner * ((int64_t)nin * io);
    // fine nodes (2cc-2) k .. (2cc+2) k - 1 (the lower half only for cc >= 1)
    T w[4 * K];
#pragma unroll
    for (int j = 0; j < 4 * K; ++j) {
      const int f = (2 * cc - 2) * K + j;
      w[j] = (f >= 0 && f < nin) ? base[inner * (int64_t)f] : T(0);
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
      T v = 0;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int p = 0; p < K; ++p) v += tab[(s * K + p) * (K + 1) + a] * w[2 * K + s * K + p];
      if (a == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int p = 0; p < K; ++p) v += tab[(s * K + p) * (K + 1) + K] * w[s * K + p];
      }
      const int I = cc * K + a;
      o[inner * (int64_t)I] = (I == 0) ? T(0) : v;
    }
  }
}

template <typename T, int K>
hipError_t restrict_k(int dim, int Nc, const T* tab, const T* rf, T* bc, T* scratch, hipStream_t s) {
  const int64_t nf = (int64_t)K * 2 * Nc + 1, nc = (int64_t)K * Nc + 1;
  // sizes along axes after each pass, x fastest
  int64_t sz[3] = {nf, nf, dim == 3 ? nf : 1};
  const T* src = rf;
  T* bufs[2] = {scratch, scratch + (dim == 3 ? nf * nf * nc : 0)};
  for (int ax = 0; ax < dim; ++ax) {
    int64_t inner = 1, outer = 1;
    for (int m = 0; m < ax; ++m) inner *= sz[m];
    for (int m = ax + 1; m < dim; ++m) outer *= sz[m];
    T* dst = (ax == dim - 1) ? bc : bufs[ax & 1];
    const int64_t total = inner * (Nc + 1) * outer;  // items: coarse cells 0..Nc
    if (inner * nf * outer >= (1ll << 31)) return hipErrorInvalidValue;
    restrict1d_kernel<T, K><<<grid_for(total), kThreads, 0, s>>>(src, dst, inner, (int)nf, (int)nc, outer, tab,
                                                                 FastDiv((uint32_t)inner),
                                                                 FastDiv((uint32_t)(Nc + 1)));
    sz[ax] = nc;
    src = dst;
  }
  return hipGetLastError();
}

template <typename T, int K>
hipError_t prolong_k(int dim, int Nc, const T* tab, const T* ec, T* xf, T* scratch, hipStream_t s) {
  const int64_t nf = (int64_t)K * 2 * Nc + 1, nc = (int64_t)K * Nc + 1;
  int64_t sz[3] = {nc, nc, dim == 3 ? nc : 1};
  const T* src = ec;
  T* bufs[2] = {scratch, scratch + (dim == 3 ? nf * nf * nc : 0)};
  for (int ax = 0; ax < dim; ++ax) {
    int64_t inner = 1, outer = 1;
    for (int m = 0; m < ax; ++m) inner *= sz[m];
    for (int m = ax + 1; m < dim; ++m) outer *= sz[m];
    const int64_t total = inner * Nc * outer;  // items: coarse cells 0..Nc-1
    if (inner * nf * outer >= (1ll << 31)) return hipErrorInvalidValue;
    const FastDiv di((uint32_t)inner), dn((uint32_t)Nc);
    if (ax == dim - 1) {
      prolong1d_kernel<T, K, true><<<grid_for(total), kThreads, 0, s>>>(src, xf, inner, (int)nc, (int)nf, outer,
                                                                         tab, di, dn);
    } else {
      T* dst = bufs[ax & 1];
      prolong1d_kernel<T, K, false><<<grid_for(total), kThreads, 0, s>>>(src, dst, inner, (int)nc, (int)nf,
                                                                          outer, tab, di, dn);
      src = dst;
    }
    sz[ax] = nf;
  }
  return hipGetLastError();
}

// Level 0: n1 = 2k+1 nodes per axis, interior nodes 1..2k-1; x = A0^{-1} b
// on the interior, 0 on the boundary.
template <typename T>
__global__ __launch_bounds__(kThreads) void coarse_kernel(int dim, int k, const double* __restrict__ Ainv,
                                                          const T* __restrict__ b, T* __restrict__ x, int64_t zs,
                                                          const int* __restrict__ active) {
  if (active && !active[blockIdx.y]) return;
  b += blockIdx.y * zs;
  x += blockIdx.y * zs;
  const int n1 = 2 * k + 1, n = 2 * k - 1;
  const int ntot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
  const int n0 = dim == 2 ? n * n : n * n * n;
  for (int g = blockIdx.x * kThreads + threadIdx.x; g < ntot; g += gridDim.x * kThreads) {
    const int i0 = g % n1, i1 = (g / n1) % n1, i2 = dim == 3 ? g / (n1 * n1) : 1;
    const bool interior = i0 >= 1 && i0 <= n && i1 >= 1 && i1 <= n && i2 >= 1 && i2 <= n;
    double s = 0;
    if (interior) {
      const int row = (i0 - 1) + n * (i1 - 1) + (dim == 3 ? n * n * (i2 - 1) : 0);
      for (int c = 0; c < n0; ++c) {
        const int c0 = c % n + 1, c1 = (c / n) % n + 1, c2 = c / (n * n) + 1;
        const int gc = c0 + n1 * c1 + (dim == 3 ? n1 * n1 * c2 : 0);
        s += Ainv[(size_t)row * n0 + c] * (double)b[gc];
      }
    }
    x[g] = (T)s;
  }
}

template <typename Ta, typename Tb>
__global__ __launch_bounds__(kThreads) void cast_kernel(int64_t n, const Ta* __restrict__ a, Tb* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    b[i] = (Tb)a[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_kernel(int64_t n, T v, T* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    a[i] = v;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Each block reduces a contiguous chunk against the m vectors, eight at a
// time: every w element loaded feeds eight products.
constexpr int kDotPerThread = 8;
constexpr int kMaxDot = 64;
constexpr int kDotGroup = 8;

__global__ __launch_bounds__(kThreads) void multidot_kernel(int64_t n, int m, const double* __restrict__ V,
                                                            int64_t ldv, const double* __restrict__ w,
                                                            double* __restrict__ partial, int nblk) {
  __shared__ double red[kThreads / 64][kDotGroup];
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int j0 = 0; j0 < m; j0 += kDotGroup) {
    double acc[kDotGroup];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) acc[q] = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q)
        if (j0 + q < m) acc[q] += V[(int64_t)(j0 + q) * ldv + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0) red[wid][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDotGroup && j0 + threadIdx.x < m) {
      double s = 0;
      for (int q = 0; q < kThreads / 64; ++q) s += red[q][threadIdx.x];
      partial[(int64_t)(j0 + threadIdx.x) * nblk + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void reduce_partials_kernel(int nblk, const double* __restrict__ partial,
                                                                   double* __restrict__ out, int accumulate) {
  __shared__ double red[kThreads / 64];
  const int j = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += partial[(int64_t)j * nblk + b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < kThreads / 64; ++q) t += red[q];
    out[j] = accumulate ? out[j] + t : t;
  }
}


__global__ __launch_bounds__(kThreads) void normalize_kernel(int64_t n, const double* __restrict__ w,
                                                             const double* __restrict__ nrm2,
                                                             double* __restrict__ v) {
  const double inv = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    v[i] = w[i] * inv;
}

template <typename Tz>
__global__ __launch_bounds__(kThreads) void update_solution_kernel(int64_t n, int m, const Tz* __restrict__ Z,
                                                                   int64_t ldz, const double* __restrict__ y,
                                                                   double* __restrict__ x) {
  __shared__ double sy[kMaxDot];
  for (int j0 = 0; j0 < m; j0 += kMaxDot) {
    const int mj = min(kMaxDot, m - j0);
    __syncthreads();
    if (threadIdx.x < mj) sy[threadIdx.x] = y[j0 + threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
      double s = x[i];
      for (int j = 0; j < mj; ++j) s += sy[j] * (double)Z[(int64_t)(j0 + j) * ldz + i];
      x[i] = s;
    }
  }
}


// ---- Arnoldi step with delayed re-orthogonalisation (classical Gram-Schmidt
// applied twice, the second pass of vector j fused into step j+1).
//
// State at step j: final orthonormal V_0..V_{j-1}; lagged vector u (the
// new direction after one projection, not yet re-orthogonalised); w = A z_j.
// One reduction gives a = V^T u, c = V^T w, u.u, u.w, w.w; then
//   s = a, alpha = sqrt(u.u - |s|^2), V_j = (u - V s) / alpha,
//   h_v = (u.w - s.c) / alpha  (= V_j . w),
//   u_new = w - V c - V_j h_v = w - V (c - s h_v/alpha) - u h_v/alpha.
constexpr int kArnGroup = 8;

// Each block owns kArnChunk consecutive entries: u and w stay in registers
// (kArnPer per lane) while the basis vectors stream past, four at a time.
constexpr int kArnPer = 8;
constexpr int kArnChunk = kThreads * kArnPer;
constexpr int kArnVec = 4;

// NT: the basis is read with non-temporal loads (taken when it is larger
// than the last-level cache, which it would only flush).
template <bool NT>
__global__ __launch_bounds__(kThreads) void arnoldi_dots_kernel(int64_t n, int j, const double* __restrict__ V,
                                                                int64_t ldv, const double* __restrict__ u,
                                                                const double* __restrict__ w,
                                                                double* __restrict__ partial, int nblk) {
  // partial rows: [0, j): V_i.u ; [j, 2j): V_i.w ; 2j: u.u ; 2j+1: u.w ; 2j+2: w.w
  __shared__ double red[kThreads / 64][2 * kArnVec];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kArnChunk + threadIdx.x;
  double ur[kArnPer], wr[kArnPer];
  double e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int e = 0; e < kArnPer; ++e) {
    const int64_t i = base + (int64_t)e * kThreads;
    ur[e] = i < n ? u[i] : 0.0;
    wr[e] = i < n ? w[i] : 0.0;
    e0 += ur[e] * ur[e];
    e1 += ur[e] * wr[e];
    e2 += wr[e] * wr[e];
  }
  {
    const double x0 = wave_sum(e0), x1 = wave_sum(e1), x2 = wave_sum(e2);
    if (lane == 0) {
      red[wid][0] = x0;
      red[wid][1] = x1;
      red[wid][2] = x2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double sum = 0;
      for (int q = 0; q < kThreads / 64; ++q) sum += red[q][threadIdx.x];
      partial[(int64_t)(2 * j + threadIdx.x) * nblk + blockIdx.x] = sum;
    }
    __syncthreads();
  }
  for (int i0 = 0; i0 < j; i0 += kArnVec) {
    double au[kArnVec], aw[kArnVec];
#pragma unroll
    for (int q = 0; q < kArnVec; ++q) {
      au[q] = aw[q] = 0;
      if (i0 + q < j) {
        const double* vq = V + (int64_t)(i0 + q) * ldv;
#pragma unroll
        for (int e = 0; e < kArnPer; ++e) {
          const int64_t i = base + (int64_t)e * kThreads;
          double v = 0.0;
          if (i < n) v = NT ? __builtin_nontemporal_load(vq + i) : vq[i];
          au[q] += v * ur[e];
          aw[q] += v * wr[e];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kArnVec; ++q) {
      const double x = wave_sum(au[q]), y = wave_sum(aw[q]);
      if (lane == 0) {
        red[wid][q] = x;
        red[wid][kArnVec + q] = y;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kArnVec) {
      const int t = threadIdx.x, q = t % kArnVec;
      if (i0 + q < j) {
        double sum = 0;
        for (int r = 0; r < kThreads / 64; ++r) sum += red[r][t];
        const int row = t < kArnVec ? i0 + q : j + i0 + q;
        partial[(int64_t)row * nblk + blockIdx.x] = sum;
      }
    }
    __syncthreads();
  }
}

// One thread: coefficients of the update from the reduced dots d[0..2j+2].
// coef layout: [0, j): e_i = s_i / alpha ; [j, 2j): f_i = c_i - s_i h_v / alpha ;
// 2j: 1/alpha ; 2j+1: h_v/alpha ; 2j+2: alpha ; 2j+3: h_v ; 2j+4: |s|^2/u.u
__device__ void arnoldi_coef(int j, const double* __restrict__ d, double* __restrict__ coef) {
  double ss = 0, sc = 0;
  for (int i = 0; i < j; ++i) {
    ss += d[i] * d[i];
    sc += d[i] * d[j + i];
  }
  const double uu = d[2 * j], uw = d[2 * j + 1];
  const double a2 = uu - ss;
  const double alpha = a2 > 0 ? sqrt(a2) : 0.0;
  const double inv = alpha > 0 ? 1.0 / alpha : 0.0;
  const double hv = (uw - sc) * inv;
  for (int i = 0; i < j; ++i) {
    coef[i] = d[i] * inv;
    coef[j + i] = d[j + i] - d[i] * hv * inv;
  }
  coef[2 * j] = inv;
  coef[2 * j + 1] = hv * inv;
  coef[2 * j + 2] = alpha;
  coef[2 * j + 3] = hv;
  coef[2 * j + 4] = uu > 0 ? ss / uu : 0.0;
}

// One block: the update coefficients from the reduced sums d (written by the
// previous launch) into coef and, when host is not NULL, the sums and the
// coefficients into host memory (host[0, 2j+3) and host[hoff, hoff+2j+5)),
// so that no copy follows; the host reads them once the launch has
// completed (an event).
__global__ __launch_bounds__(kThreads) void arnoldi_coef_kernel(int j, const double* __restrict__ d,
                                                                double* __restrict__ coef,
                                                                double* __restrict__ host, int hoff) {
  __shared__ double sd[2 * kMaxDot + 3], sc[2 * kMaxDot + 5];
  const int nd = 2 * j + 3, nc = 2 * j + 5;
  for (int i = threadIdx.x; i < nd; i += kThreads) sd[i] = d[i];
  __syncthreads();
  if (threadIdx.x == 0) arnoldi_coef(j, sd, sc);
  __syncthreads();
  for (int i = threadIdx.x; i < nc; i += kThreads) coef[i] = sc[i];
  if (host) {
    for (int i = threadIdx.x; i < nd; i += kThreads) host[i] = sd[i];
    for (int i = threadIdx.x; i < nc; i += kThreads) host[hoff + i] = sc[i];
  }
}

__global__ __launch_bounds__(kThreads) void arnoldi_update_kernel(int64_t n, int j, const double* __restrict__ V,
                                                                  int64_t ldv, double* __restrict__ u,
                                                                  const double* __restrict__ w,
                                                                  const double* __restrict__ coef,
                                                                  double* __restrict__ vout,
                                                                  float* __restrict__ u32) {
  __shared__ double se[kMaxDot], sf[kMaxDot];
  for (int t = threadIdx.x; t < kMaxDot; t += kThreads) {
    se[t] = t < j ? coef[t] : 0.0;
    sf[t] = t < j ? coef[j + t] : 0.0;
  }
  __syncthreads();
  const double inv = coef[2 * j], d = coef[2 * j + 1];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double ui = u[i], wi = w[i];
    double sv = 0, sw = 0;
    int q = 0;
    for (; q + 4 <= j; q += 4) {
      double v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = V[(int64_t)(q + t) * ldv + i];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        sv += se[q + t] * v[t];
        sw += sf[q + t] * v[t];
      }
    }
    for (; q < j; ++q) {
      const double v = V[(int64_t)q * ldv + i];
      sv += se[q] * v;
      sw += sf[q] * v;
    }
    vout[i] = ui * inv - sv;
    const double un = wi - sw - d * ui;
    u[i] = un;
    if (u32) u32[i] = (float)un;
  }
}

}  // namespace

int multidot_blocks(int64_t n) {
  int64_t b = (n + kThreads * kDotPerThread - 1) / (kThreads * kDotPerThread);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename Tin, typename T>
hipError_t launch_apply(int dim, int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y,
                        hipStream_t s) {
  return dim == 2 ? launch_apply2d<Tin, T>(k, N, c, x, b, y, s) : launch_apply3d<Tin, T>(k, N, c, x, b, y, s);
}

template <typename T>
hipError_t launch_patch_smooth(int dim, int k, int N, const LevelEig<T>& e, const T* r, const T* x_in, T* x_out,
                               T omega, hipStream_t s) {
  return dim == 2 ? launch_patch2d<T>(k, N, e, r, x_in, x_out, omega, s)
                  : launch_patch3d<T>(k, N, e, r, x_in, x_out, omega, s);
}

template <typename T>
hipError_t launch_restrict(int dim, int k, int Nc, const T* table, const T* rf, T* bc, T* scratch, hipStream_t s) {
  if (dim == 2) return launch_restrict2d<T>(k, Nc, table, rf, bc, s);
#define CALL(K) restrict_k<T, K>(dim, Nc, table, rf, bc, scratch, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_prolong_add(int dim, int k, int Nc, const T* table, const T* ec, T* xf, T* scratch,
                              hipStream_t s) {
  if (dim == 2) return launch_prolong2d<T>(k, Nc, table, ec, xf, xf, s);
#define CALL(K) prolong_k<T, K>(dim, Nc, table, ec, xf, scratch, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_coarse(int dim, int k, const double* Ainv, const T* b, T* x, hipStream_t s, int nsys, int64_t zs,
                         const int* active) {
  const int n1 = 2 * k + 1, ntot = dim == 2 ? n1 * n1 : n1 * n1 * n1;
  coarse_kernel<T><<<dim3((ntot + kThreads - 1) / kThreads, nsys), kThreads, 0, s>>>(dim, k, Ainv, b, x, zs, active);
  return hipGetLastError();
}

template <typename Ta, typename Tb>
hipError_t launch_cast(int64_t n, const Ta* a, Tb* b, hipStream_t s) {
  cast_kernel<Ta, Tb><<<grid_for(n), kThreads, 0, s>>>(n, a, b);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double* a, hipStream_t s) {
  fill_kernel<double><<<grid_for(n), kThreads, 0, s>>>(n, v, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_t(int64_t n, T v, T* a, hipStream_t s) {
  fill_kernel<T><<<grid_for(n), kThreads, 0, s>>>(n, v, a);
  return hipGetLastError();
}

hipError_t launch_multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* partial,
                           int nblk, hipStream_t s) {
  multidot_kernel<<<nblk, kThreads, 0, s>>>(n, m, V, ldv, w, partial, nblk);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(int m, int nblk, const double* partial, double* out, int accumulate,
                                  hipStream_t s) {
  reduce_partials_kernel<<<m, kThreads, 0, s>>>(nblk, partial, out, accumulate);
  return hipGetLastError();
}


hipError_t launch_normalize(int64_t n, const double* w, const double* nrm2, double* v, hipStream_t s) {
  normalize_kernel<<<grid_for(n), kThreads, 0, s>>>(n, w, nrm2, v);
  return hipGetLastError();
}

template <typename Tz>
hipError_t launch_update_solution(int64_t n, int m, const Tz* Z, int64_t ldz, const double* y, double* x,
                                  hipStream_t s) {
  update_solution_kernel<Tz><<<grid_for(n), kThreads, 0, s>>>(n, m, Z, ldz, y, x);
  return hipGetLastError();
}

int arnoldi_blocks(int64_t n) { return (int)((n + kArnChunk - 1) / kArnChunk); }

hipError_t launch_arnoldi_dots(int64_t n, int j, const double* V, int64_t ldv, const double* u, const double* w,
                               double* partial, int nblk, hipStream_t s) {
  if ((int64_t)nblk * kArnChunk < n) return hipErrorInvalidValue;
  // measured on a 2.36 M-entry basis: non-temporal loads are 10 % faster
  // once the basis exceeds the 256 MiB last-level cache, slower below
  if ((double)j * (double)n * sizeof(double) > 256.0 * (1 << 20))
    arnoldi_dots_kernel<true><<<nblk, kThreads, 0, s>>>(n, j, V, ldv, u, w, partial, nblk);
  else
    arnoldi_dots_kernel<false><<<nblk, kThreads, 0, s>>>(n, j, V, ldv, u, w, partial, nblk);
  return hipGetLastError();
}

hipError_t launch_arnoldi_reduce_coef(int j, int nblk, const double* partial, double* d, double* coef,
                                      double* host, int hoff, hipStream_t s) {
  if (j < 0 || j > kMaxDot) return hipErrorInvalidValue;
  reduce_partials_kernel<<<2 * j + 3, kThreads, 0, s>>>(nblk, partial, d, 0);
  arnoldi_coef_kernel<<<1, kThreads, 0, s>>>(j, d, coef, host, hoff);
  return hipGetLastError();
}

hipError_t launch_arnoldi_update(int64_t n, int j, const double* V, int64_t ldv, double* u, const double* w,
                                 const double* coef, double* vout, hipStream_t s, float* u32) {
  arnoldi_update_kernel<<<grid_for(n), kThreads, 0, s>>>(n, j, V, ldv, u, w, coef, vout, u32);
  return hipGetLastError();
}


template hipError_t launch_apply<double, double>(int, int, int, const LevelCoef<double>&, const double*,
                                                 const double*, double*, hipStream_t);
template hipError_t launch_apply<float, double>(int, int, int, const LevelCoef<double>&, const float*,
                                                const double*, double*, hipStream_t);
template hipError_t launch_apply<float, float>(int, int, int, const LevelCoef<float>&, const float*, const float*,
                                               float*, hipStream_t);
template hipError_t launch_patch_smooth<double>(int, int, int, const LevelEig<double>&, const double*,
                                                const double*, double*, double, hipStream_t);
template hipError_t launch_patch_smooth<float>(int, int, int, const LevelEig<float>&, const float*, const float*,
                                               float*, float, hipStream_t);
template hipError_t launch_restrict<double>(int, int, int, const double*, const double*, double*, double*,
                                            hipStream_t);
template hipError_t launch_restrict<float>(int, int, int, const float*, const float*, float*, float*, hipStream_t);
template hipError_t launch_prolong_add<double>(int, int, int, const double*, const double*, double*, double*,
                                               hipStream_t);
template hipError_t launch_prolong_add<float>(int, int, int, const float*, const float*, float*, float*,
                                              hipStream_t);
template hipError_t launch_coarse<double>(int, int, const double*, const double*, double*, hipStream_t, int, int64_t,
                                          const int*);
template hipError_t launch_coarse<float>(int, int, const double*, const float*, float*, hipStream_t, int, int64_t,
                                         const int*);
template hipError_t launch_cast<double, float>(int64_t, const double*, float*, hipStream_t);
template hipError_t launch_cast<float, double>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_fill_t<float>(int64_t, float, float*, hipStream_t);
template hipError_t launch_fill_t<double>(int64_t, double, double*, hipStream_t);
template hipError_t launch_update_solution<double>(int64_t, int, const double*, int64_t, const double*, double*,
                                                   hipStream_t);
template hipError_t launch_update_solution<float>(int64_t, int, const float*, int64_t, const double*, double*,
                                                  hipStream_t);

}  // namespace c0ip
