// 3D additive vertex-patch smoother for gfx950, streaming along z (Sec. 3,
// the AVS definition with eq. localsolverbila in 3D, inverted by fast
// diagonalisation, eq. inverse):
//   x_out = x_in + omega sum_v R_v^T (Q (x) Q (x) Q) (L_x + L_y + L_z)^-1
//                                    (Q (x) Q (x) Q)^T R_v r.
// A workgroup owns a TC x TC tile of cells in x, y (owner computes) over a
// chunk of z cells, and walks the vertex layers vz of the chunk.  The
// patches of a layer are the (TC+1)^2 patches around the tile's vertices;
// each covers 2k-1 residual planes, of which k-1 are shared with the next
// layer.  Per residual plane, once: the forward x and y transforms of every
// patch's n x n block (n = 2k-1), kept in an LDS ring of 2k-1 planes.  Per
// layer: the z transform, the division by the eigenvalue sums and the
// inverse z transform along the n planes of each patch (the result of the
// lower k planes overwrites their ring slots, the upper k-1 go to k-1
// extra slots), then per plane the inverse y and x transforms in place,
// and a gather: each owned node sums the (at most 2 x 2) patches of the
// layer that contain it into a register accumulator of the layer's 2k-1
// planes.  The k lowest planes are then complete and are written out.
// All sums run in a fixed order (deterministic).
#include <algorithm>

#include "kernels.h"

namespace c0ip {
namespace {

// variant of the patch at vertex v in [1, N-1] along one axis (0 interior,
// 1 touching the lower boundary, 2 the upper one, 3 both)
__device__ __forceinline__ int pvariant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

constexpr unsigned kOff = 0x80000000u;  // an offset outside every buffer
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, T v) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}

template <int K_, int TC_>
struct SGeo {
  static constexpr int K = K_, TC = TC_, NTH = 256;
  static constexpr int n = 2 * K - 1, NN = n * n, P = TC + 1, PP = P * P;
  static constexpr int RS = (TC + 2) * K - 1;    // staged residual plane: RS x RS nodes
  static constexpr int SLOT = PP * NN;           // one plane of every patch's block
  static constexpr int NSLOT = 2 * K - 1 + K - 1;  // ring of 2k-1 planes + k-1 extra
  static constexpr int OWN = TC * K;             // owned nodes per direction
  static constexpr int NO = (OWN * OWN + NTH - 1) / NTH;  // owned nodes per thread
};

// One 1D transform of n values: out[c] = sum_a Q[a][c] in[a] (FWD, Q^T) or
// out[a] = sum_c Q[a][c] in[c] (inverse).  Q is either wave-uniform (held in
// registers) or a per-lane row in LDS.
template <typename T, int n, bool FWD>
__device__ __forceinline__ void tr1(const T* q, const T (&in)[n], T (&out)[n]) {
#pragma unroll
  for (int i = 0; i < n; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) s += (FWD ? q[j * n + i] : q[i * n + j]) * in[j];
    out[i] = s;
  }
}

// x (AX = 0) or y (AX = 1) transform of every patch block of one slot, in
// place, or from the staged residual plane into the slot (FROMR).  Items:
// (patch, line).
template <typename T, class G, int AX, bool FWD, bool FROMR, bool UNI>
__device__ __forceinline__ void pass_xy(T* __restrict__ slot, const T* __restrict__ sR, const T (&q0)[G::NN],
                                        const T* __restrict__ sQ, int cx0, int cy0, int N) {
  constexpr int n = G::n, K = G::K, P = G::P;
  for (int it = threadIdx.x; it < G::PP * n; it += G::NTH) {
    const int qd = it / n, ln = it - qd * n;
    const int px = qd % P, py = qd / P;
    const int vx = cx0 + px, vy = cy0 + py;
    const bool valid = vx >= 1 && vx <= N - 1 && vy >= 1 && vy <= N - 1;
    T* blk = slot + qd * G::NN;
    T in[n], out[n];
    if (FROMR) {
      // x transform of row ln (local y) of the patch's residual block
#pragma unroll
      for (int a = 0; a < n; ++a) in[a] = valid ? sR[(py * K + ln) * G::RS + px * K + a] : T(0);
    } else {
#pragma unroll
      for (int a = 0; a < n; ++a) in[a] = AX == 0 ? blk[ln * n + a] : blk[a * n + ln];
    }
    const int var = pvariant(AX == 0 ? vx : vy, N);
    if (UNI)
      tr1<T, n, FWD>(q0, in, out);
    else
      tr1<T, n, FWD>(sQ + var * G::NN, in, out);
#pragma unroll
    for (int a = 0; a < n; ++a) {
      if (AX == 0)
        blk[ln * n + a] = out[a];
      else
        blk[a * n + ln] = out[a];
    }
  }
}

template <typename T, class G, bool UNI>
__device__ __forceinline__ void smooth3d_tile(const T* __restrict__ r, const T* __restrict__ xin, T* __restrict__ xout,
                                              int N, const T* __restrict__ Qg, T omega, int cx0, int cy0, int c0,
                                              int c1, T* __restrict__ sF,
                                              T* __restrict__ sR, const T* __restrict__ sQ,
                                              const T* __restrict__ sLam) {
  constexpr int K = G::K, n = G::n, NN = G::NN, NTH = G::NTH, NO = G::NO, RING = 2 * K - 1;
  const int n1 = K * N + 1, NK = n1 - 1;
  const size_t plane = (size_t)n1 * n1;
  const unsigned pbytes = (unsigned)(plane * sizeof(T));
  // interior-variant eigenbasis in registers (wave-uniform)
  T q0[NN];
#pragma unroll
  for (int i = 0; i < NN; ++i) q0[i] = Qg[i];
  // owned nodes of this thread: in-plane offsets (kOff: none or boundary)
  unsigned ooff[NO];
  int ox[NO], oy[NO];
#pragma unroll
  for (int t = 0; t < NO; ++t) {
    const int e = threadIdx.x + t * NTH;
    ox[t] = e % G::OWN;
    oy[t] = e / G::OWN;
    const int gx = cx0 * K + ox[t], gy = cy0 * K + oy[t];
    const bool own = e < G::OWN * G::OWN && gx < NK && gy < NK;
    ooff[t] = own ? (unsigned)(gy * n1 + gx) * sizeof(T) : kOff;
    if (!own) oy[t] = -1;
  }
  // staged residual plane: node offsets (kOff outside [1, NK-1]^2)
  constexpr int NR = (G::RS * G::RS + NTH - 1) / NTH;
  unsigned roff[NR];
#pragma unroll
  for (int t = 0; t < NR; ++t) {
    const int e = threadIdx.x + t * NTH;
    const int i = e % G::RS, j = e / G::RS;
    const int gx = (cx0 - 1) * K + 1 + i, gy = (cy0 - 1) * K + 1 + j;
    roff[t] = (e < G::RS * G::RS && gx >= 1 && gx <= NK - 1 && gy >= 1 && gy <= NK - 1)
                  ? (unsigned)(gy * n1 + gx) * sizeof(T)
                  : kOff;
  }
  T acc[2 * K - 1][NO];
#pragma unroll
  for (int j = 0; j < 2 * K - 1; ++j)
#pragma unroll
    for (int t = 0; t < NO; ++t) acc[j][t] = T(0);
  auto emit = [&](int zp, const T (&a)[NO]) {  // plane zp complete: write the owned nodes
    if (zp < c0 * K || zp >= c1 * K || zp >= NK) return;
    const __amdgpu_buffer_rsrc_t ri = buf(xin + (size_t)zp * plane, xin ? pbytes : 0u);
    const __amdgpu_buffer_rsrc_t ro = buf(xout + (size_t)zp * plane, pbytes);
#pragma unroll
    for (int t = 0; t < NO; ++t) {
      const int gx = cx0 * K + ox[t], gy = cy0 * K + oy[t];
      const bool bnd = zp == 0 || gx == 0 || gy == 0;
      const T v = buf_load<T>(ri, ooff[t]) + omega * a[t];
      buf_store<T>(ro, ooff[t], bnd ? T(0) : v);
    }
  };
  const int v0 = max(c0, 1), v1 = min(c1, N - 1);
  if (c0 == 0) {  // plane 0 is boundary
    T z[NO];
#pragma unroll
    for (int t = 0; t < NO; ++t) z[t] = T(0);
    emit(0, z);
  }
  int zdone = (v0 - 1) * K;  // residual planes transformed so far: up to zdone
  for (int vz = v0; vz <= v1; ++vz) {
    const int zlo = (vz - 1) * K + 1;  // planes zlo .. zlo + n - 1
    // forward x, y transforms of the new planes
    for (int zp = max(zdone + 1, zlo); zp <= zlo + n - 1; ++zp) {
      const __amdgpu_buffer_rsrc_t rr = buf(r + (size_t)zp * plane, pbytes);
      T v[NR];
#pragma unroll
      for (int t = 0; t < NR; ++t) v[t] = buf_load<T>(rr, roff[t]);
#pragma unroll
      for (int t = 0; t < NR; ++t) {
        const int e = threadIdx.x + t * NTH;
        if (NR * NTH == G::RS * G::RS || e < G::RS * G::RS) sR[e] = v[t];
      }
      __syncthreads();
      T* slot = sF + (zp % RING) * G::SLOT;
      pass_xy<T, G, 0, true, true, UNI>(slot, sR, q0, sQ, cx0, cy0, N);
      __syncthreads();
      pass_xy<T, G, 1, true, false, UNI>(slot, sR, q0, sQ, cx0, cy0, N);
    }
    zdone = zlo + n - 1;
    __syncthreads();
    // z transform, division, inverse z transform: item (patch, y, x)
    {
      const int zv = pvariant(vz, N);
      const T* qz = Qg + zv * NN;
      const T* lz = sLam + zv * n;
      for (int it = threadIdx.x; it < G::PP * NN; it += NTH) {
        const int qd = it / NN, e = it - qd * NN, m = e / n, c = e - m * n;
        const int px = qd % G::P, py = qd / G::P;
        const T lxy = sLam[pvariant(cx0 + px, N) * n + c] + sLam[pvariant(cy0 + py, N) * n + m];
        T in[n], w[n];
#pragma unroll
        for (int j = 0; j < n; ++j) in[j] = sF[((zlo + j) % RING) * G::SLOT + it];
        tr1<T, n, true>(qz, in, w);
#pragma unroll
        for (int kz = 0; kz < n; ++kz) w[kz] = w[kz] / (lxy + lz[kz]);
        tr1<T, n, false>(qz, w, in);
#pragma unroll
        for (int j = 0; j < n; ++j) {
          const int s = j < K ? (zlo + j) % RING : RING + j - K;
          sF[s * G::SLOT + it] = in[j];
        }
      }
    }
    __syncthreads();
    // inverse y then x transforms of every plane of the layer
    for (int j = 0; j < n; ++j) {
      T* slot = sF + (j < K ? (zlo + j) % RING : RING + j - K) * G::SLOT;
      pass_xy<T, G, 1, false, false, UNI>(slot, sR, q0, sQ, cx0, cy0, N);
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
      T* slot = sF + (j < K ? (zlo + j) % RING : RING + j - K) * G::SLOT;
      pass_xy<T, G, 0, false, false, UNI>(slot, sR, q0, sQ, cx0, cy0, N);
    }
    __syncthreads();
    // gather: each owned node sums the patches of the layer containing it
#pragma unroll
    for (int t = 0; t < NO; ++t) {
      if (oy[t] < 0) continue;
      const int gx = cx0 * K + ox[t], gy = cy0 * K + oy[t];
      const int mx = gx / K, rx = gx - mx * K, my = gy / K, ry = gy - my * K;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const T* slot = sF + (j < K ? (zlo + j) % RING : RING + j - K) * G::SLOT;
        T s = 0;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          if (dy == 1 && ry == 0) continue;
          const int vy = my + dy, ay = gy - (vy - 1) * K - 1;
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            if (dx == 1 && rx == 0) continue;
            const int vx = mx + dx, ax = gx - (vx - 1) * K - 1;
            s += slot[((vy - cy0) * G::P + (vx - cx0)) * NN + ay * n + ax];
          }
        }
        acc[j][t] += s;
      }
    }
    // planes zlo .. zlo + k - 1 are complete
#pragma unroll
    for (int j = 0; j < K; ++j) emit(zlo + j, acc[j]);
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
#pragma unroll
      for (int t = 0; t < NO; ++t) acc[j][t] = acc[j + K][t];
#pragma unroll
    for (int j = K - 1; j < 2 * K - 1; ++j)
#pragma unroll
      for (int t = 0; t < NO; ++t) acc[j][t] = T(0);
    __syncthreads();  // the next layer overwrites the slots
  }
  // planes above the last layer's vertex plane that no later layer reaches
  if (v1 == N - 1 && v1 >= v0) {
#pragma unroll
    for (int j = 0; j < K - 1; ++j) emit(v1 * K + 1 + j, acc[j]);
  }
}

// Zeros on the faces x, y, z = kN (boundary nodes no tile owns).
template <typename T, int NTH>
__device__ __forceinline__ void zero_faces3(T* __restrict__ y, int n1, int fb) {
  const int NK = n1 - 1;
  const int64_t nf = (int64_t)n1 * n1;
  for (int q = 0; q < 16; ++q) {
    const int64_t f = ((int64_t)fb * 16 + q) * NTH + threadIdx.x;
    if (f >= 3 * nf) return;
    const int face = (int)(f / nf);
    const int64_t rem = f - face * nf;
    const int u = (int)(rem % n1), w = (int)(rem / n1);
    const int gx = face == 0 ? NK : u, gy = face == 0 ? u : (face == 1 ? NK : w), gz = face == 2 ? NK : w;
    y[((size_t)gz * n1 + gy) * n1 + gx] = T(0);
  }
}

template <typename T, class G>
__global__ __launch_bounds__(G::NTH) void smooth3d_kernel(const T* __restrict__ r, const T* __restrict__ xin,
                                                          T* __restrict__ xout, int N, const T* __restrict__ Qg,
                                                          const T* __restrict__ lamg, T omega, int tx, int zcc) {
  const int n1 = G::K * N + 1;
  const int nt = tx * tx;
  if ((int)blockIdx.x >= nt) {
    if (blockIdx.y == 0) zero_faces3<T, G::NTH>(xout, n1, blockIdx.x - nt);
    return;
  }
  __shared__ T sF[G::NSLOT * G::SLOT];
  __shared__ T sR[G::RS * G::RS];
  __shared__ T sQ[4 * G::NN];
  __shared__ T sLam[4 * G::n];
  for (int e = threadIdx.x; e < 4 * G::NN; e += G::NTH) sQ[e] = Qg[e];
  for (int e = threadIdx.x; e < 4 * G::n; e += G::NTH) sLam[e] = lamg[e];
  __syncthreads();
  const int bx = blockIdx.x % tx, by = blockIdx.x / tx;
  const int cx0 = bx * G::TC, cy0 = by * G::TC;
  const int c0 = blockIdx.y * zcc, c1 = min(c0 + zcc, N);
  // tiles whose patches are all interior in x and y take the basis in
  // scalar registers (when it fits them)
  constexpr bool kUniFits = G::NN * (int)sizeof(T) / 4 <= 50;
  const bool uni = kUniFits && cx0 >= 2 && cx0 + G::TC <= N - 2 && cy0 >= 2 && cy0 + G::TC <= N - 2;
  if constexpr (kUniFits) {
    if (uni) {
      smooth3d_tile<T, G, true>(r, xin, xout, N, Qg, omega, cx0, cy0, c0, c1, sF, sR, sQ, sLam);
      return;
    }
  }
  smooth3d_tile<T, G, false>(r, xin, xout, N, Qg, omega, cx0, cy0, c0, c1, sF, sR, sQ, sLam);
}

template <typename T, int K> struct SmoothCfg;
template <typename T> struct SmoothCfg<T, 2> { using G = SGeo<2, 8>; };
template <typename T> struct SmoothCfg<T, 3> { using G = SGeo<3, 6>; };
template <typename T> struct SmoothCfg<T, 4> { using G = SGeo<4, sizeof(T) == 4 ? 4 : 2>; };

template <typename T, class G>
hipError_t smooth3d_g(int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega, hipStream_t s) {
  const int n1 = G::K * N + 1;
  const int tx = (N + G::TC - 1) / G::TC;
  int zcc = N;
  while (zcc > 4 && (int64_t)tx * tx * ((N + zcc - 1) / zcc) < 2048) zcc = (zcc + 1) / 2;
  const int nface = (int)((3 * (int64_t)n1 * n1 + 16 * G::NTH - 1) / (16 * G::NTH));
  const dim3 grid(tx * tx + nface, (N + zcc - 1) / zcc);
  smooth3d_kernel<T, G><<<grid, G::NTH, 0, s>>>(r, xin, xout, N, e.Q, e.lam, omega, tx, zcc);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_patch3d(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s) {
  // raw buffer offsets of a plane must stay below 2^31 bytes
  if ((double)(k * N + 1) * (k * N + 1) * sizeof(T) >= 2147483648.0) return hipErrorInvalidValue;
  switch (k) {
    case 2: return smooth3d_g<T, typename SmoothCfg<T, 2>::G>(N, e, r, xin, xout, omega, s);
    case 3: return smooth3d_g<T, typename SmoothCfg<T, 3>::G>(N, e, r, xin, xout, omega, s);
    case 4: return smooth3d_g<T, typename SmoothCfg<T, 4>::G>(N, e, r, xin, xout, omega, s);
    default: return launch_patch3d_wide<T>(k, N, e, r, xin, xout, omega, s);
  }
}

template hipError_t launch_patch3d<double>(int, int, const LevelEig<double>&, const double*, const double*,
                                           double*, double, hipStream_t);
template hipError_t launch_patch3d<float>(int, int, const LevelEig<float>&, const float*, const float*, float*,
                                          float, hipStream_t);

}  // namespace c0ip
