// Vector kernels of the flexible conjugate-gradient solve (Sec. 5.1: the
// paper's Krylov method for the symmetric additive smoother).  One
// iteration with preconditioned residual z = MG(r):
//   beta = (z . q_old) / (p_old . q_old),  p = z - beta p_old,  q = A p,
//   alpha = (r . p) / (p . q),  x += alpha p,  r -= alpha q.
// Every scalar is formed on the device (reductions write sc[]), so an
// iteration needs one host read only, of r . r for the stopping test.
#include "krylov_cg.h"

namespace c0ip {
namespace cg {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 8;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block sum of v (every thread passes its value; thread 0 gets the sum)
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kThreads / 64; ++q) t += red[q];
  __syncthreads();
  return t;
}

template <typename Tz>
__global__ __launch_bounds__(kThreads) void dot_kernel(int64_t n, const Tz* __restrict__ z,
                                                       const double* __restrict__ q, double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  double a = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) a += (double)z[i] * q[i];
  const double t = block_sum(a, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void dot2_kernel(int64_t n, const double* __restrict__ p,
                                                        const double* __restrict__ q, const double* __restrict__ r,
                                                        double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  double a = 0, c = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double pi = p[i];
    a += pi * q[i];
    c += pi * r[i];
  }
  const double ta = block_sum(a, red);
  const double tc = block_sum(c, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = ta;
    partial[gridDim.x + blockIdx.x] = tc;
  }
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(int m, int nblk, const double* __restrict__ partial,
                                                          double* __restrict__ sc, int slot, int stage) {
  __shared__ double red[kThreads / 64];
  __shared__ double tot[4];
  for (int j = 0; j < m; ++j) {
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) s += partial[(int64_t)j * nblk + b];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) tot[j] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < m; ++j) sc[slot + j] = tot[j];
    if (stage == 1) sc[kBETA] = sc[kZQ] / sc[kPQOLD];
    if (stage == 2) {
      sc[kALPHA] = sc[kRP] / sc[kPQ];
      sc[kPQOLD] = sc[kPQ];
    }
  }
}

template <typename Tz>
__global__ __launch_bounds__(kThreads) void update_p_kernel(int64_t n, const Tz* __restrict__ z,
                                                            const double* __restrict__ sc, double* __restrict__ p,
                                                            int first) {
  const double beta = first ? 0.0 : sc[kBETA];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = first ? (double)z[i] : (double)z[i] - beta * p[i];
}

__global__ __launch_bounds__(kThreads) void update_xr_kernel(int64_t n, const double* __restrict__ sc,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ q, double* __restrict__ x,
                                                             double* __restrict__ r, double* __restrict__ partial,
                                                             float* __restrict__ r32) {
  __shared__ double red[kThreads / 64];
  const double alpha = sc[kALPHA];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  double a = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    a += ri * ri;
  }
  const double t = block_sum(a, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int blocks(int64_t n) {
  int64_t b = (n + kThreads * kPerThread - 1) / (kThreads * kPerThread);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename Tz>
hipError_t launch_dot(int64_t n, const Tz* z, const double* q, double* partial, int nblk, hipStream_t s) {
  dot_kernel<Tz><<<nblk, kThreads, 0, s>>>(n, z, q, partial);
  return hipGetLastError();
}

hipError_t launch_dot2(int64_t n, const double* p, const double* q, const double* r, double* partial, int nblk,
                       hipStream_t s) {
  dot2_kernel<<<nblk, kThreads, 0, s>>>(n, p, q, r, partial);
  return hipGetLastError();
}

hipError_t launch_reduce(int m, int nblk, const double* partial, double* sc, int slot, int stage, hipStream_t s) {
  if (m < 1 || m > 4) return hipErrorInvalidValue;
  reduce_kernel<<<1, kThreads, 0, s>>>(m, nblk, partial, sc, slot, stage);
  return hipGetLastError();
}

template <typename Tz>
hipError_t launch_update_p(int64_t n, const Tz* z, const double* sc, double* p, int first, hipStream_t s) {
  update_p_kernel<Tz><<<grid_for(n), kThreads, 0, s>>>(n, z, sc, p, first);
  return hipGetLastError();
}

hipError_t launch_update_xr(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                            double* partial, int nblk, hipStream_t s, float* r32) {
  update_xr_kernel<<<nblk, kThreads, 0, s>>>(n, sc, p, q, x, r, partial, r32);
  return hipGetLastError();
}

template hipError_t launch_dot<float>(int64_t, const float*, const double*, double*, int, hipStream_t);
template hipError_t launch_dot<double>(int64_t, const double*, const double*, double*, int, hipStream_t);
template hipError_t launch_update_p<float>(int64_t, const float*, const double*, double*, int, hipStream_t);
template hipError_t launch_update_p<double>(int64_t, const double*, const double*, double*, int, hipStream_t);

}  // namespace cg
}  // namespace c0ip
