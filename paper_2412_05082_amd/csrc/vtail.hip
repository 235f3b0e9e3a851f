// The lowest levels of the V-cycle (Algorithm 1) in one workgroup per
// system, with every vector of those levels in LDS.
//
// Below a few thousand DoFs per level each kernel of the V-cycle is bound
// by its own launch and memory latency (about 5 us each, six of them per
// level).  Here levels 0..LT run in a single launch: the right-hand side
// of level LT is read once, pre-smoothing, residual, restriction, the
// coarse solve, prolongation and post-smoothing of every level below run
// from LDS with workgroup barriers between steps, and x of level LT is
// written once.  The operations are the same as the tiled kernels':
// sum-factorised operator with the row-class band tables, fast-
// diagonalisation patch solves gathered per node, the 1D embedding table.
#include <algorithm>

#include "kernels.h"

namespace c0ip {
namespace {

constexpr int kTailThreads = 1024;

// dst[0..n) = src[0..n), four loads in flight per thread
template <typename Td, typename Ts>
__device__ __forceinline__ void t_copy(Td* __restrict__ dst, const Ts* __restrict__ src, int n) {
  for (int e0 = threadIdx.x; e0 < n; e0 += 4 * kTailThreads) {
    Ts v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kTailThreads;
      v[u] = e < n ? src[e] : Ts(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kTailThreads;
      if (e < n) dst[e] = (Td)v[u];
    }
  }
}

__device__ __forceinline__ int clampn(int v, int n1) { return v < 0 ? 0 : (v > n1 - 1 ? n1 - 1 : v); }

__device__ __forceinline__ int rclass(int g, int n1, int k, int left, int right0, int periodic) {
  if (!periodic) return g;
  if (g < left) return g;
  if (g >= right0) return left + (n1 - 1 - g);
  return 2 * left + g % k;
}
__device__ __forceinline__ int pvariant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

// LDS layout (element offsets; the same function sizes the launch).  x and
// b live on every level; r and the sweep/patch scratch only on the level
// being worked on, so they are allocated once at the top level's size.  The
// patch corrections PR share memory with the sweep buffers U, V, W (each
// phase's scratch is dead by the time the other is written); the transfer
// scratch is U.
struct TailLayout {
  int x[kTailMaxLevels], b[kTailMaxLevels], tab[kTailMaxLevels], q[kTailMaxLevels], lam[kTailMaxLevels];
  int r, u, v, w, pr, pt, total;  // in T elements
  int a0;                         // offset of the float64 level-0 inverse, in doubles
  int bytes;
};

__host__ __device__ inline TailLayout tail_layout(int k, int LT, const int* nclass, int tsize) {
  TailLayout L{};
  int off = 0;
  for (int l = 0; l <= LT; ++l) {
    const int n1 = k * (2 << l) + 1;
    L.x[l] = off;
    off += n1 * n1;
    L.b[l] = off;
    off += n1 * n1;
  }
  const int n1max = k * (2 << LT) + 1, nnmax = n1max * n1max;
  const int n = 2 * k - 1, NP = (2 << LT) - 1;
  L.r = off;
  off += nnmax;
  L.u = off;
  L.v = off + nnmax;
  L.w = off + 2 * nnmax;
  L.pr = off;
  off += 3 * nnmax > NP * NP * n * n ? 3 * nnmax : NP * NP * n * n;
  for (int l = 0; l <= LT; ++l) {
    L.tab[l] = off;
    off += 3 * nclass[l] * (4 * k + 1);
    L.q[l] = off;
    off += 4 * n * n;
    L.lam[l] = off;
    off += 4 * n;
  }
  L.pt = off;
  off += 2 * k * (k + 1);
  L.total = off;
  const int tbytes = ((off * tsize + 15) / 16) * 16;
  L.a0 = tbytes / 8;
  L.bytes = tbytes + n * n * n * n * 8;
  return L;
}

// y = A x (b == nullptr) or y = b - A x (0 on the boundary).  Every tap
// runs over the widest band with the table's zero entries outside a row's
// structural band (and outside the mesh), so the loops have fixed trip
// counts; indices past the mesh edge are clamped (their coefficient is 0).
template <typename T, int K>
__device__ void t_apply(int N, const T* x, const T* b, T* y, T* U, T* V, T* W, const T* tab, int nclass, int left,
                        int right0, int periodic) {
  const int n1 = K * N + 1, nn = n1 * n1;
  constexpr int Wd = 4 * K + 1, H = 2 * K;
  for (int e = threadIdx.x; e < nn; e += kTailThreads) {
    const int j = e / n1, i = e - j * n1;
    const int cls = rclass(i, n1, K, left, right0, periodic);
    const T* cM = tab + cls * Wd + H;
    const T* cL = tab + (nclass + cls) * Wd + H;
    const T* cB = tab + (2 * nclass + cls) * Wd + H;
    const T* row = x + j * n1;
    T u = 0, v = 0, w = 0;
#pragma unroll
    for (int o = -2 * K; o <= 2 * K; ++o) {
      const T xv = row[clampn(i + o, n1)];
      if (o >= -K && o <= K) {
        u += cM[o] * xv;
        v += cL[o] * xv;
      }
      w += cB[o] * xv;
    }
    U[e] = u;
    V[e] = v;
    W[e] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nn; e += kTailThreads) {
    const int j = e / n1, i = e - j * n1;
    const int cls = rclass(j, n1, K, left, right0, periodic);
    const T* cM = tab + cls * Wd + H;
    const T* cL = tab + (nclass + cls) * Wd + H;
    const T* cB = tab + (2 * nclass + cls) * Wd + H;
    T acc = 0;
#pragma unroll
    for (int o = -2 * K; o <= 2 * K; ++o) {
      const int q = clampn(j + o, n1) * n1 + i;
      if (o >= -K && o <= K) acc += cM[o] * W[q] + 2 * cL[o] * V[q];
      acc += cB[o] * U[q];
    }
    if (b) {
      const bool bnd = i == 0 || j == 0 || i == n1 - 1 || j == n1 - 1;
      y[e] = bnd ? T(0) : b[e] - acc;
    } else {
      y[e] = acc;
    }
  }
  __syncthreads();
}

// Patch solves of all (N-1)^2 patches of the level from r, into PR
// (patch-major, n x n each): forward along x, along y (with the division
// by lambda_x + lambda_y) and back, back along x; one patch row or column
// per thread, in place.
template <typename T, int K>
__device__ void t_patches(int N, const T* r, T* PR, const T* Q, const T* lam) {
  constexpr int n = 2 * K - 1, NN = n * n;
  const int n1 = K * N + 1, NP = N - 1, items = NP * NP * n;
  for (int it = threadIdx.x; it < items; it += kTailThreads) {
    const int pi = it / n, a = it - pi * n;
    const int vy = pi / NP + 1, vx = pi - (vy - 1) * NP + 1;
    const T* qx = Q + pvariant(vx, N) * NN;
    const T* src = r + ((vy - 1) * K + 1 + a) * n1 + (vx - 1) * K + 1;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = src[c];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int cp = 0; cp < n; ++cp) s += qx[cp * n + c] * in[cp];
      PR[pi * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < items; it += kTailThreads) {
    const int pi = it / n, c = it - pi * n;
    const int vy = pi / NP + 1, vx = pi - (vy - 1) * NP + 1;
    const int tx = pvariant(vx, N), ty = pvariant(vy, N);
    const T* qy = Q + ty * NN;
    T col[n], t[n];
#pragma unroll
    for (int a = 0; a < n; ++a) col[a] = PR[pi * NN + a * n + c];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += qy[a * n + ap] * col[a];
      t[ap] = s / (lam[tx * n + c] + lam[ty * n + ap]);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += qy[a * n + ap] * t[ap];
      PR[pi * NN + a * n + c] = s;
    }
  }
  __syncthreads();
  for (int it = threadIdx.x; it < items; it += kTailThreads) {
    const int pi = it / n, a = it - pi * n;
    const int vy = pi / NP + 1, vx = pi - (vy - 1) * NP + 1;
    const T* qx = Q + pvariant(vx, N) * NN;
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = PR[pi * NN + a * n + c];
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += qx[cp * n + c] * in[c];
      PR[pi * NN + a * n + cp] = s;
    }
  }
  __syncthreads();
}

// x = (x_is_zero ? 0 : x) + omega * sum of the covering patches' corrections
template <typename T, int K>
__device__ void t_gather(int N, T* x, const T* PR, T omega, bool x_is_zero) {
  constexpr int n = 2 * K - 1, NN = n * n;
  const int n1 = K * N + 1, NP = N - 1;
  for (int e = threadIdx.x; e < n1 * n1; e += kTailThreads) {
    const int i = e % n1, j = e / n1;
    if (i == 0 || j == 0 || i == n1 - 1 || j == n1 - 1) {
      x[e] = T(0);
      continue;
    }
    const int vxa = i / K, vxb = (i % K == 0) ? vxa : vxa + 1;
    const int vya = j / K, vyb = (j % K == 0) ? vya : vya + 1;
    T acc = 0;
    for (int vy = vya; vy <= vyb; ++vy) {
      if (vy < 1 || vy > N - 1) continue;
      for (int vx = vxa; vx <= vxb; ++vx) {
        if (vx < 1 || vx > N - 1) continue;
        acc += PR[((vy - 1) * NP + (vx - 1)) * NN + (j - ((vy - 1) * K + 1)) * n + (i - ((vx - 1) * K + 1))];
      }
    }
    x[e] = (x_is_zero ? T(0) : x[e]) + omega * acc;
  }
  __syncthreads();
}

// bc = P^T rf (Nc coarse cells); S: scratch of n1f * n1c
template <typename T, int K>
__device__ void t_restrict(int Nc, const T* rf, T* bc, T* S, const T* pt) {
  const int nf = 2 * K * Nc + 1, nc = K * Nc + 1;
  for (int e = threadIdx.x; e < nf * nc; e += kTailThreads) {
    const int I = e % nc, jf = e / nc;
    T v = 0;
    if (I > 0 && I < nc - 1) {
      const int cc = I / K, a = I - cc * K;
      const T* row = rf + jf * nf;
      for (int q = 0; q < 2 * K; ++q) v += pt[q * (K + 1) + a] * row[2 * cc * K + q];
      if (a == 0)
        for (int q = 0; q < 2 * K; ++q) v += pt[q * (K + 1) + K] * row[(2 * cc - 2) * K + q];
    }
    S[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nc * nc; e += kTailThreads) {
    const int I = e % nc, J = e / nc;
    T v = 0;
    if (J > 0 && J < nc - 1) {
      const int cc = J / K, a = J - cc * K;
      for (int q = 0; q < 2 * K; ++q) v += pt[q * (K + 1) + a] * S[(2 * cc * K + q) * nc + I];
      if (a == 0)
        for (int q = 0; q < 2 * K; ++q) v += pt[q * (K + 1) + K] * S[((2 * cc - 2) * K + q) * nc + I];
    }
    bc[e] = v;
  }
  __syncthreads();
}

// xf += P ec
template <typename T, int K>
__device__ void t_prolong_add(int Nc, const T* ec, T* xf, T* S, const T* pt) {
  const int nf = 2 * K * Nc + 1, nc = K * Nc + 1;
  for (int e = threadIdx.x; e < nc * nf; e += kTailThreads) {
    const int f = e % nf, J = e / nf;
    T v = 0;
    if (f > 0 && f < nf - 1) {
      const int cf = f / K, p = f - cf * K, cc = cf >> 1, s = cf & 1;
      for (int a = 0; a <= K; ++a) v += pt[(s * K + p) * (K + 1) + a] * ec[J * nc + cc * K + a];
    }
    S[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nf * nf; e += kTailThreads) {
    const int fx = e % nf, fy = e / nf;
    if (fx == 0 || fy == 0 || fx == nf - 1 || fy == nf - 1) continue;
    const int cf = fy / K, p = fy - cf * K, cc = cf >> 1, s = cf & 1;
    T v = 0;
    for (int a = 0; a <= K; ++a) v += pt[(s * K + p) * (K + 1) + a] * S[(cc * K + a) * nf + fx];
    xf[e] += v;
  }
  __syncthreads();
}

template <typename T, int K>
__global__ __launch_bounds__(kTailThreads) void vtail_kernel(TailParams<T> P, TailIO<T> io) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int sys = blockIdx.x;
  if (io.active && !io.active[sys]) return;
  int top = 0;
  for (int l = 1; l <= P.LT; ++l)
    if (sys < io.nA[l]) top = l;
  const TailLayout L = tail_layout(K, P.LT, P.nclass, sizeof(T));
  T* S = reinterpret_cast<T*>(smem);
  double* A0 = reinterpret_cast<double*>(smem) + L.a0;
  constexpr int n = 2 * K - 1, n0 = n * n;
  {
    const int n1 = K * (2 << top) + 1;
    t_copy(S + L.b[top], io.b[top] + (int64_t)sys * io.stride[top], n1 * n1);
  }
  for (int l = 0; l <= top; ++l) {
    t_copy(S + L.tab[l], P.tab[l], 3 * P.nclass[l] * (4 * K + 1));
    t_copy(S + L.q[l], P.Q[l], 4 * n * n);
    t_copy(S + L.lam[l], P.lam[l], 4 * n);
  }
  t_copy(S + L.pt, P.ptab, 2 * K * (K + 1));
  if (P.coarse_mode == 0) t_copy(A0, P.Ainv, n0 * n0);
  __syncthreads();
  const T om = P.omega;
  T* r = S + L.r;
  T* U = S + L.u;
  T* V = S + L.v;
  T* W = S + L.w;
  T* PR = S + L.pr;
  const T* pt = S + L.pt;
  for (int l = top; l >= 1; --l) {
    const int N = 2 << l, nn = (K * N + 1) * (K * N + 1);
    T *x = S + L.x[l], *b = S + L.b[l];
    const T* tab = S + L.tab[l];
    const int nc = P.nclass[l], le = P.left[l], r0 = P.right0[l], per = P.periodic[l];
    if (P.pre == 0) {
      for (int e = threadIdx.x; e < nn; e += kTailThreads) x[e] = T(0);
      __syncthreads();
    }
    for (int st = 0; st < P.pre; ++st) {
      if (st == 0) {
        t_patches<T, K>(N, b, PR, S + L.q[l], S + L.lam[l]);
        t_gather<T, K>(N, x, PR, om, true);
      } else {
        t_apply<T, K>(N, x, b, r, U, V, W, tab, nc, le, r0, per);
        t_patches<T, K>(N, r, PR, S + L.q[l], S + L.lam[l]);
        t_gather<T, K>(N, x, PR, om, false);
      }
    }
    t_apply<T, K>(N, x, b, r, U, V, W, tab, nc, le, r0, per);
    t_restrict<T, K>(N / 2, r, S + L.b[l - 1], U, pt);
  }
  {  // level 0
    T* b0 = S + L.b[0];
    T* x0 = S + L.x[0];
    constexpr int n1 = 2 * K + 1;
    if (P.coarse_mode == 0) {
      for (int g = threadIdx.x; g < n1 * n1; g += kTailThreads) {
        const int i0 = g % n1, i1 = g / n1;
        double s = 0;
        if (i0 >= 1 && i0 <= n && i1 >= 1 && i1 <= n) {
          const int row = (i0 - 1) + n * (i1 - 1);
          for (int c = 0; c < n0; ++c) s += A0[row * n0 + c] * (double)b0[(c % n + 1) + n1 * (c / n + 1)];
        }
        x0[g] = (T)s;
      }
      __syncthreads();
    } else {
      t_patches<T, K>(2, b0, PR, S + L.q[0], S + L.lam[0]);
      t_gather<T, K>(2, x0, PR, T(1), true);
    }
  }
  for (int l = 1; l <= top; ++l) {
    const int N = 2 << l;
    T *x = S + L.x[l], *b = S + L.b[l];
    const T* tab = S + L.tab[l];
    const int nc = P.nclass[l], le = P.left[l], r0 = P.right0[l], per = P.periodic[l];
    t_prolong_add<T, K>(N / 2, S + L.x[l - 1], x, U, pt);
    for (int st = 0; st < P.post; ++st) {
      t_apply<T, K>(N, x, b, r, U, V, W, tab, nc, le, r0, per);
      t_patches<T, K>(N, r, PR, S + L.q[l], S + L.lam[l]);
      t_gather<T, K>(N, x, PR, om, false);
    }
  }
  {
    const int n1 = K * (2 << top) + 1;
    t_copy(io.x[top] + (int64_t)sys * io.stride[top], S + L.x[top], n1 * n1);
  }
}

template <typename T, int K>
hipError_t vtail_configure_k(int bytes) {
  return hipFuncSetAttribute((const void*)vtail_kernel<T, K>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename T, int K>
hipError_t vtail_k(const TailParams<T>& P, const TailIO<T>& io, int nsys, hipStream_t s) {
  const TailLayout L = tail_layout(K, P.LT, P.nclass, sizeof(T));
  vtail_kernel<T, K><<<nsys, kTailThreads, L.bytes, s>>>(P, io);
  return hipGetLastError();
}

}  // namespace

int tail_bytes(int k, int LT, const int* nclass, int elem_size) {
  return tail_layout(k, LT, nclass, elem_size).bytes;
}

int tail_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return v;
}

template <typename T>
hipError_t configure_vtail(int k, int bytes) {
  switch (k) {
    case 2: return vtail_configure_k<T, 2>(bytes);
    case 3: return vtail_configure_k<T, 3>(bytes);
    case 4: return vtail_configure_k<T, 4>(bytes);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_vtail(int k, const TailParams<T>& P, const TailIO<T>& io, int nsys, hipStream_t s) {
  switch (k) {
    case 2: return vtail_k<T, 2>(P, io, nsys, s);
    case 3: return vtail_k<T, 3>(P, io, nsys, s);
    case 4: return vtail_k<T, 4>(P, io, nsys, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t configure_vtail<double>(int, int);
template hipError_t configure_vtail<float>(int, int);
template hipError_t launch_vtail<double>(int, const TailParams<double>&, const TailIO<double>&, int, hipStream_t);
template hipError_t launch_vtail<float>(int, const TailParams<float>&, const TailIO<float>&, int, hipStream_t);

}  // namespace c0ip
