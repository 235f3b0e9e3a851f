// One colour of the coloured multiplicative vertex-patch smoother on a 3D
// mesh (Sec. 3, Fig. 2 extended to three dimensions: 16 colours).
//   x <- x + omega * sum_{v of colour c} R_v^T A~_v^{-1} R_v r,   r = b - A x.
// Colour c = px + 2 py + 4 pz + 8 rb holds the vertices
// v = (2a + px, 2b + py, 2cc + pz) in [1, N-1]^3 with (a + b + cc) mod 2 = rb;
// their patches share no node and no entry of A couples two of them, so
// every patch is solved once and added in place.  Numbering: plane by plane
// of cc; within a plane the vertices with (a + b) mod 2 = (rb - cc) mod 2,
// row by row of b (rows alternate between two lengths, and so do planes).
// Local solve: fast diagonalisation (eq. inverse) as three passes of 1D
// transforms along x, y and z.
#include "mvs3d.h"
#include "tiles.h"

namespace c0ip {
namespace {

constexpr int kThreads = tile::kThreads;
using tile::variant;

struct Lat {
  int lo, hi;  // lattice index range along one axis
};

__host__ __device__ inline Lat lat(int N, int par) { return {par == 0 ? 1 : 0, (N - 1 - par) / 2}; }

__host__ __device__ inline int row_count(Lat a, int b, int par) {
  const int af = a.lo + (((par - a.lo - b) % 2) + 2) % 2;
  return af <= a.hi ? (a.hi - af) / 2 + 1 : 0;
}

// vertices of one plane whose (a + b) has parity par
__host__ __device__ inline int plane_count(Lat a, Lat b, int par) {
  const int nb = b.hi >= b.lo ? b.hi - b.lo + 1 : 0;
  const int c0 = row_count(a, b.lo, par), c1 = row_count(a, b.lo + 1, par);
  return (nb / 2) * (c0 + c1) + (nb % 2) * c0;
}

struct Colour3 {
  Lat a, b, c;
  int px, py, pz, rb;
  int t0, t1;  // vertices in planes c.lo + 2i and c.lo + 2i + 1
  int total;
};

Colour3 colour3(int N, int col) {
  Colour3 k;
  k.px = col & 1;
  k.py = (col >> 1) & 1;
  k.pz = (col >> 2) & 1;
  k.rb = (col >> 3) & 1;
  k.a = lat(N, k.px);
  k.b = lat(N, k.py);
  k.c = lat(N, k.pz);
  const int nc = k.c.hi >= k.c.lo ? k.c.hi - k.c.lo + 1 : 0;
  k.t0 = plane_count(k.a, k.b, (((k.rb - k.c.lo) % 2) + 2) % 2);
  k.t1 = plane_count(k.a, k.b, (((k.rb - k.c.lo - 1) % 2) + 2) % 2);
  k.total = (nc / 2) * (k.t0 + k.t1) + (nc % 2) * k.t0;
  return k;
}

__device__ __forceinline__ void vertex3(const Colour3& k, int q, int& vx, int& vy, int& vz) {
  const int pp = k.t0 + k.t1;
  const int i = q / pp, rem = q - i * pp;
  const int cc = k.c.lo + 2 * i + (rem >= k.t0 ? 1 : 0);
  int q2 = rem >= k.t0 ? rem - k.t0 : rem;
  const int par = (((k.rb - cc) % 2) + 2) % 2;
  const int c0 = row_count(k.a, k.b.lo, par), c1 = row_count(k.a, k.b.lo + 1, par);
  const int rp = c0 + c1;
  const int j = q2 / rp, rem2 = q2 - j * rp;
  const int b = k.b.lo + 2 * j + (rem2 >= c0 ? 1 : 0);
  const int t = rem2 >= c0 ? rem2 - c0 : rem2;
  const int af = k.a.lo + (((par - k.a.lo - b) % 2) + 2) % 2;
  vx = 2 * (af + 2 * t) + k.px;
  vy = 2 * b + k.py;
  vz = 2 * cc + k.pz;
}

template <int K> struct ColourPatches3 {
  static constexpr int n = 2 * K - 1;
  static constexpr int NPW = kThreads / (n * n) > 0 ? kThreads / (n * n) : 1;
  static_assert(4 * n <= kThreads, "one eigenvalue per thread");
};

template <typename T, int K>
__global__ __launch_bounds__(kThreads) void mvs3d_colour_kernel(const T* __restrict__ r, T* __restrict__ x, int N,
                                                                int n1, Colour3 col, const T* __restrict__ Qg,
                                                                const T* __restrict__ lamg, T omega) {
  constexpr int n = 2 * K - 1, NN = n * n, N3 = NN * n, NPW = ColourPatches3<K>::NPW;
  __shared__ T sA[NPW * N3];
  __shared__ T sB[NPW * N3];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  const int q0 = blockIdx.x * NPW;
  const int np = min(NPW, col.total - q0);
  if (np <= 0) return;
  const size_t s1 = n1, s2 = (size_t)n1 * n1;
  // gather r on the patches' nodes (x fastest), and x there for the final
  // update (no other workgroup of the colour reads or writes those nodes):
  // every global load is issued before the first LDS store
  constexpr int NL = (NPW * N3 + kThreads - 1) / kThreads, LQ = (4 * NN + kThreads - 1) / kThreads;
  T rv[NL], xv[NL], qv[LQ];
  size_t gi[NL];
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * kThreads;
    rv[u] = xv[u] = T(0);
    gi[u] = 0;
    if (e < np * N3) {
      const int p = e / N3, loc = e - p * N3;
      const int zz = loc / NN, yy = (loc / n) % n, xx = loc % n;
      int vx, vy, vz;
      vertex3(col, q0 + p, vx, vy, vz);
      gi[u] = (size_t)((vz - 1) * K + 1 + zz) * s2 + (size_t)((vy - 1) * K + 1 + yy) * s1 + (vx - 1) * K + 1 + xx;
      rv[u] = r[gi[u]];
      xv[u] = x[gi[u]];
    }
  }
#pragma unroll
  for (int u = 0; u < LQ; ++u) {
    const int e = threadIdx.x + u * kThreads;
    qv[u] = e < 4 * NN ? Qg[e] : T(0);
  }
  const T lv = threadIdx.x < 4 * n ? lamg[threadIdx.x] : T(0);
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * kThreads;
    if (e < np * N3) sB[e] = rv[u];
  }
#pragma unroll
  for (int u = 0; u < LQ; ++u) {
    const int e = threadIdx.x + u * kThreads;
    if (e < 4 * NN) sQ[e] = qv[u];
  }
  if (threadIdx.x < 4 * n) sLam[threadIdx.x] = lv;
  __syncthreads();
  // forward along x: sA[z][y][c] = sum_c' Qx[c'][c] sB[z][y][c']
  for (int it = threadIdx.x; it < np * NN; it += kThreads) {
    const int p = it / NN, line = it - p * NN;
    int vx, vy, vz;
    vertex3(col, q0 + p, vx, vy, vz);
    const T* q = sQ + variant(vx, N) * NN;
    const T* in = sB + p * N3 + line * n;
    T v[n];
#pragma unroll
    for (int c = 0; c < n; ++c) v[c] = in[c];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int cp = 0; cp < n; ++cp) s += q[cp * n + c] * v[cp];
      sA[p * N3 + line * n + c] = s;
    }
  }
  __syncthreads();
  // forward along y: sB[z][a][x] = sum_a' Qy[a'][a] sA[z][a'][x]
  for (int it = threadIdx.x; it < np * NN; it += kThreads) {
    const int p = it / NN, line = it - p * NN, zz = line / n, xx = line - zz * n;
    int vx, vy, vz;
    vertex3(col, q0 + p, vx, vy, vz);
    const T* q = sQ + variant(vy, N) * NN;
    const T* in = sA + p * N3 + zz * NN + xx;
    T v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) v[a] = in[a * n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += q[ap * n + a] * v[ap];
      sB[p * N3 + zz * NN + a * n + xx] = s;
    }
  }
  __syncthreads();
  // along z: forward with Qz^T, divide by lambda_x + lambda_y + lambda_z, back with Qz
  for (int it = threadIdx.x; it < np * NN; it += kThreads) {
    const int p = it / NN, line = it - p * NN, yy = line / n, xx = line - yy * n;
    int vx, vy, vz;
    vertex3(col, q0 + p, vx, vy, vz);
    const int tz = variant(vz, N);
    const T* q = sQ + tz * NN;
    const T lxy = sLam[variant(vx, N) * n + xx] + sLam[variant(vy, N) * n + yy];
    const T* in = sB + p * N3 + line;
    T v[n], t[n];
#pragma unroll
    for (int z = 0; z < n; ++z) v[z] = in[z * NN];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int z = 0; z < n; ++z) s += q[z * n + c] * v[z];
      t[c] = s / (lxy + sLam[tz * n + c]);
    }
#pragma unroll
    for (int z = 0; z < n; ++z) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += q[z * n + c] * t[c];
      sA[p * N3 + z * NN + line] = s;
    }
  }
  __syncthreads();
  // back along y: sB[z][a][x] = sum_a' Qy[a][a'] sA[z][a'][x]
  for (int it = threadIdx.x; it < np * NN; it += kThreads) {
    const int p = it / NN, line = it - p * NN, zz = line / n, xx = line - zz * n;
    int vx, vy, vz;
    vertex3(col, q0 + p, vx, vy, vz);
    const T* q = sQ + variant(vy, N) * NN;
    const T* in = sA + p * N3 + zz * NN + xx;
    T v[n];
#pragma unroll
    for (int a = 0; a < n; ++a) v[a] = in[a * n];
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += q[a * n + ap] * v[ap];
      sB[p * N3 + zz * NN + a * n + xx] = s;
    }
  }
  __syncthreads();
  // back along x into sA
  for (int it = threadIdx.x; it < np * NN; it += kThreads) {
    const int p = it / NN, line = it - p * NN;
    int vx, vy, vz;
    vertex3(col, q0 + p, vx, vy, vz);
    const T* q = sQ + variant(vx, N) * NN;
    const T* in = sB + p * N3 + line * n;
    T v[n];
#pragma unroll
    for (int c = 0; c < n; ++c) v[c] = in[c];
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += q[cp * n + c] * v[c];
      sA[p * N3 + line * n + cp] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int e = threadIdx.x + u * kThreads;
    if (e < np * N3) x[gi[u]] = xv[u] + omega * sA[e];
  }
}

template <typename T, int K>
hipError_t mvs3d_colour_k(int N, int colour, const LevelEig<T>& e, const T* r, T* x, T omega, hipStream_t s) {
  constexpr int NPW = ColourPatches3<K>::NPW;
  const Colour3 col = colour3(N, colour);
  if (col.total <= 0) return hipSuccess;
  const int nblk = (col.total + NPW - 1) / NPW;
  mvs3d_colour_kernel<T, K><<<nblk, kThreads, 0, s>>>(r, x, N, K * N + 1, col, e.Q, e.lam, omega);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_mvs3d_colour(int k, int N, int colour, const LevelEig<T>& e, const T* r, T* x, T omega,
                               hipStream_t s) {
#define CALL(K) mvs3d_colour_k<T, K>(N, colour, e, r, x, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template hipError_t launch_mvs3d_colour<double>(int, int, int, const LevelEig<double>&, const double*, double*,
                                                double, hipStream_t);
template hipError_t launch_mvs3d_colour<float>(int, int, int, const LevelEig<float>&, const float*, float*, float,
                                               hipStream_t);

}  // namespace c0ip
