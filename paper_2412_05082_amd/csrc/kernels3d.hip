// 3D kernels: matrix-free C0IP operator and the additive vertex-patch
// smoother with fast-diagonalisation local solves, for gfx950.
//
// Operator (Sec. 4, eq. c0iptensorvp3D, used globally on the Cartesian
// mesh), first factor along x:
//   A = B M M + M B M + M M B + 2 (L L M + M L L + L M L).
// Sum factorisation: x-sweeps X M_x, X L_x, X B_x; y-sweeps give
//   S1 = (B_x M_y + M_x B_y + 2 L_x L_y) X,  S2 = M_x M_y X,
//   S3 = 2 (M_x L_y + L_x M_y) X;
// and Y = M_z S1 + B_z S2 + L_z S3.
// A workgroup owns a 16 x 16 column of (x, y) nodes and streams along z:
// per plane it stages X on the tile plus a 2k halo in LDS, runs the x- and
// y-sweeps, and pushes S1, S2, S3 of its own column into register windows
// of 4k+1 planes, from which the z-sweep emits one output plane.
//
// Smoother (Sec. 3, eq. localsolverbila in 3D, eq. inverse):
// owner-computes over tiles of TC^3 cells.  The (TC+1)^3 patches touching
// a tile are solved in the 8 classes of vertex parity; patches of one
// class are disjoint, so their damped corrections are added to an LDS
// accumulator of the owned nodes without conflicts.  Each contraction
// is applied in place along lines of the patch.
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

template <int K> __host__ __device__ constexpr int m_lo(int p) { return p == 0 ? -K : -p; }
template <int K> __host__ __device__ constexpr int m_hi(int p) { return p == 0 ? K : K - p; }
template <int K> __host__ __device__ constexpr int b_lo(int p) { return p == 0 ? -2 * K : -K - p; }
template <int K> __host__ __device__ constexpr int b_hi(int p) { return p == 0 ? 2 * K : 2 * K - p; }
template <int K> __host__ __device__ constexpr int tab_max() { return 3 * (5 * K + 2) * (4 * K + 1); }

// ------------------------------------------------------------------ operator

constexpr int kT3 = 16;  // tile width in x and y (nodes)

template <typename Tin, typename T, int K, bool RES>
__global__ __launch_bounds__(kThreads) void apply3d_kernel(const Tin* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ y, int n1, int zc,
                                                           const T* __restrict__ tab, int nclass, int left,
                                                           int right0, int periodic) {
  constexpr int H = 2 * K, W = 4 * K + 1, R = kT3 + 2 * H;  // staged plane is R x R
  constexpr int NL = (R * R + kThreads - 1) / kThreads;
  __shared__ T sX[R * R];
  __shared__ T sM[R * kT3];              // X M_x on rows [-2k, T+2k)
  __shared__ T sL[(kT3 + 2 * K) * kT3];  // X L_x on rows [-k, T+k)
  __shared__ T sB[(kT3 + 2 * K) * kT3];  // X B_x on rows [-k, T+k)
  __shared__ T sTab[tab_max<K>()];
  const int x0 = blockIdx.x * kT3, y0 = blockIdx.y * kT3, z0 = blockIdx.z * zc;
  const int ntab = 3 * nclass * W;
  for (int e = threadIdx.x; e < ntab; e += kThreads) sTab[e] = tab[e];
  const int lx = threadIdx.x % kT3, ly = threadIdx.x / kT3;
  const int gx = x0 + lx, gy = y0 + ly;
  const int cy = row_class(min(gy, n1 - 1), n1, K, left, right0, periodic), py = min(gy, n1 - 1) % K;
  T w1[W], w2[W], w3[W];  // S1, S2, S3 at planes zp-4k .. zp
#pragma unroll
  for (int q = 0; q < W; ++q) w1[q] = w2[q] = w3[q] = T(0);
  const size_t plane = (size_t)n1 * n1;
  const int zend = min(z0 + zc, n1);
  for (int zp = z0 - H; zp < zend + H; ++zp) {
    // stage X on the plane (0 outside the mesh)
    {
      T v[NL];
      const bool zin = zp >= 0 && zp < n1;
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * kThreads;
        const int r = e / R, c = e - r * R;
        const int yy = y0 - H + r, xx = x0 - H + c;
        v[q] = (e < R * R && zin && yy >= 0 && yy < n1 && xx >= 0 && xx < n1)
                   ? (T)x[(size_t)zp * plane + (size_t)yy * n1 + xx]
                   : T(0);
      }
      __syncthreads();  // previous plane's sweeps are done with sX, sM, sL, sB
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int e = threadIdx.x + q * kThreads;
        if (e < R * R) sX[e] = v[q];
      }
    }
    __syncthreads();
    // x-sweeps: item (row r in [0, R), column l in [0, T))
    for (int it = threadIdx.x; it < R * kT3; it += kThreads) {
      const int r = it / kT3, l = it - r * kT3;
      const int g = min(x0 + l, n1 - 1);
      const int cls = row_class(g, n1, K, left, right0, periodic), p = g % K;
      const T* cM = sTab + cls * W + H;
      const T* cL = sTab + (nclass + cls) * W + H;
      const T* cB = sTab + (2 * nclass + cls) * W + H;
      const T* row = sX + r * R + l + H;  // row[o] = X at column x0 + l + o
      T m = 0;
      for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) m += cM[o] * row[o];
      sM[it] = m;
      if (r >= K && r < R - K) {
        T lv = 0, bv = 0;
        for (int o = m_lo<K>(p); o <= m_hi<K>(p); ++o) lv += cL[o] * row[o];
        for (int o = b_lo<K>(p); o <= b_hi<K>(p); ++o) bv += cB[o] * row[o];
        sL[(r - K) * kT3 + l] = lv;
        sB[(r - K) * kT3 + l] = bv;
      }
    }
    __syncthreads();
    // y-sweeps for this thread's column
    T s1, s2, s3;
    {
      const T* cM = sTab + cy * W + H;
      const T* cL = sTab + (nclass + cy) * W + H;
      const T* cB = sTab + (2 * nclass + cy) * W + H;
      T bm = 0, mb = 0, mm = 0, ml = 0, ll = 0, lm = 0;
      for (int o = m_lo<K>(py); o <= m_hi<K>(py); ++o) {
        const T xm = sM[(ly + H + o) * kT3 + lx], xl = sL[(ly + K + o) * kT3 + lx],
                xb = sB[(ly + K + o) * kT3 + lx];
        bm += cM[o] * xb;
        mm += cM[o] * xm;
        ml += cL[o] * xm;
        ll += cL[o] * xl;
        lm += cM[o] * xl;
      }
      for (int o = b_lo<K>(py); o <= b_hi<K>(py); ++o) mb += cB[o] * sM[(ly + H + o) * kT3 + lx];
      s1 = bm + mb + 2 * ll;
      s2 = mm;
      s3 = 2 * (ml + lm);
    }
#pragma unroll
    for (int q = 0; q < W - 1; ++q) {
      w1[q] = w1[q + 1];
      w2[q] = w2[q + 1];
      w3[q] = w3[q + 1];
    }
    w1[W - 1] = s1;
    w2[W - 1] = s2;
    w3[W - 1] = s3;
    // z-sweep for plane z = zp - 2k: window index 2k + o holds plane z + o
    const int z = zp - H;
    if (z >= z0 && z < zend && gx < n1 && gy < n1) {
      const int cz = row_class(z, n1, K, left, right0, periodic), pz = z % K;
      const T* cM = sTab + cz * W + H;
      const T* cL = sTab + (nclass + cz) * W + H;
      const T* cB = sTab + (2 * nclass + cz) * W + H;
      T acc = 0;
      for (int o = m_lo<K>(pz); o <= m_hi<K>(pz); ++o) acc += cM[o] * w1[H + o] + cL[o] * w3[H + o];
      for (int o = b_lo<K>(pz); o <= b_hi<K>(pz); ++o) acc += cB[o] * w2[H + o];
      const size_t idx = (size_t)z * plane + (size_t)gy * n1 + gx;
      if (RES) {
        const bool bnd = gx == 0 || gx == n1 - 1 || gy == 0 || gy == n1 - 1 || z == 0 || z == n1 - 1;
        y[idx] = bnd ? T(0) : b[idx] - acc;
      } else {
        y[idx] = acc;
      }
    }
  }
}

template <typename Tin, typename T, int K>
hipError_t apply3d_k(int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s) {
  const int n1 = K * N + 1;
  const int nt = (n1 + kT3 - 1) / kT3;
  // split z so that the grid has a few thousand workgroups; halo planes are recomputed
  int zc = n1;
  while (zc > 8 * K && (int64_t)nt * nt * ((n1 + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
  dim3 grid(nt, nt, (n1 + zc - 1) / zc);
  if (b)
    apply3d_kernel<Tin, T, K, true><<<grid, kThreads, 0, s>>>(x, b, y, n1, zc, c.tab, c.nclass, c.left, c.right0,
                                                               c.periodic);
  else
    apply3d_kernel<Tin, T, K, false><<<grid, kThreads, 0, s>>>(x, b, y, n1, zc, c.tab, c.nclass, c.left,
                                                                c.right0, c.periodic);
  return hipGetLastError();
}

// ------------------------------------------------------------------ smoother

__device__ __forceinline__ int variant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

template <int K> struct PatchTile3D;
template <> struct PatchTile3D<2> { static constexpr int TC = 4; };
template <> struct PatchTile3D<3> { static constexpr int TC = 3; };
template <> struct PatchTile3D<4> { static constexpr int TC = 2; };
template <> struct PatchTile3D<5> { static constexpr int TC = 1; };
template <> struct PatchTile3D<6> { static constexpr int TC = 1; };
template <> struct PatchTile3D<7> { static constexpr int TC = 1; };

template <typename T, int K, int TC>
__global__ __launch_bounds__(kThreads) void patch3d_kernel(const T* __restrict__ r, const T* __restrict__ xin,
                                                           T* __restrict__ xout, int N, int n1,
                                                           const T* __restrict__ Qg, const T* __restrict__ lamg,
                                                           T omega) {
  constexpr int n = 2 * K - 1, NN = n * n, N3 = NN * n, NP = TC + 1, S = (TC + 2) * K - 1;
  constexpr int PB = ((NP + 1) / 2) * ((NP + 1) / 2) * ((NP + 1) / 2);  // largest parity class
  constexpr int OW = TC * K + 1;
  __shared__ T sR[S * S * S];
  __shared__ T sP[PB * N3];
  __shared__ T sAcc[OW * OW * OW];
  __shared__ T sQ[4 * NN];
  __shared__ T sLam[4 * n];
  const int c0[3] = {(int)blockIdx.x * TC, (int)blockIdx.y * TC, (int)blockIdx.z * TC};
  const int o0 = (c0[0] - 1) * K + 1, o1 = (c0[1] - 1) * K + 1, o2 = (c0[2] - 1) * K + 1;
  const size_t plane = (size_t)n1 * n1;
  for (int e = threadIdx.x; e < S * S * S; e += kThreads) {
    const int i = e % S, j = (e / S) % S, l = e / (S * S);
    const int g0 = o0 + i, g1 = o1 + j, g2 = o2 + l;
    const bool in = g0 >= 1 && g0 <= n1 - 2 && g1 >= 1 && g1 <= n1 - 2 && g2 >= 1 && g2 <= n1 - 2;
    sR[e] = in ? r[(size_t)g2 * plane + (size_t)g1 * n1 + g0] : T(0);
  }
  for (int e = threadIdx.x; e < OW * OW * OW; e += kThreads) sAcc[e] = T(0);
  for (int e = threadIdx.x; e < 4 * NN; e += kThreads) sQ[e] = Qg[e];
  for (int e = threadIdx.x; e < 4 * n; e += kThreads) sLam[e] = lamg[e];
  __syncthreads();
  for (int par = 0; par < 8; ++par) {
    // patches of this tile whose vertex parity is par, numbered 0..np-1
    const int px = par & 1, py = (par >> 1) & 1, pz = par >> 2;
    const int vx0 = c0[0] + ((px - c0[0]) % 2 + 2) % 2, vy0 = c0[1] + ((py - c0[1]) % 2 + 2) % 2,
              vz0 = c0[2] + ((pz - c0[2]) % 2 + 2) % 2;
    const int cx = vx0 <= c0[0] + TC ? (c0[0] + TC - vx0) / 2 + 1 : 0;
    const int cyn = vy0 <= c0[1] + TC ? (c0[1] + TC - vy0) / 2 + 1 : 0;
    const int czn = vz0 <= c0[2] + TC ? (c0[2] + TC - vz0) / 2 + 1 : 0;
    const int np = cx * cyn * czn;
    // gather R_v r for each patch into sP
    for (int e = threadIdx.x; e < np * N3; e += kThreads) {
      const int pi = e / N3, t = e - pi * N3;
      const int a0 = t % n, a1 = (t / n) % n, a2 = t / NN;
      const int vx = vx0 + 2 * (pi % cx), vy = vy0 + 2 * ((pi / cx) % cyn), vz = vz0 + 2 * (pi / (cx * cyn));
      // region index of node (vx-1)k+1+a0 etc.
      const int i = (vx - c0[0]) * K + a0, j = (vy - c0[1]) * K + a1, l = (vz - c0[2]) * K + a2;
      sP[e] = sR[(l * S + j) * S + i];
    }
    __syncthreads();
    // six in-place line passes; pass d (0,1,2 forward along x,y,z; 3,4,5 back along z,y,x)
    for (int pass = 0; pass < 6; ++pass) {
      const int ax = pass < 3 ? pass : 5 - pass;
      const bool fwd = pass < 3;
      for (int e = threadIdx.x; e < np * NN; e += kThreads) {
        const int pi = e / NN, t = e - pi * NN;
        const int u0 = t % n, u1 = t / n;  // the two other coordinates
        const int vx = vx0 + 2 * (pi % cx), vy = vy0 + 2 * ((pi / cx) % cyn), vz = vz0 + 2 * (pi / (cx * cyn));
        const int vv = ax == 0 ? vx : (ax == 1 ? vy : vz);
        const T* q = sQ + variant(vv, N) * NN;
        int base, stride;
        if (ax == 0) { base = u0 * n + u1 * NN; stride = 1; }
        else if (ax == 1) { base = u0 + u1 * NN; stride = n; }
        else { base = u0 + u1 * n; stride = NN; }
        T* line = sP + pi * N3 + base;
        T in[n], out[n];
#pragma unroll
        for (int a = 0; a < n; ++a) in[a] = line[a * stride];
        if (fwd) {
#pragma unroll
          for (int c = 0; c < n; ++c) {
            T sacc = 0;
#pragma unroll
            for (int a = 0; a < n; ++a) sacc += q[a * n + c] * in[a];
            out[c] = sacc;
          }
          if (ax == 2) {  // divide by lambda_x + lambda_y + lambda_z, then back along z
            const T lxy = sLam[variant(vx, N) * n + u0] + sLam[variant(vy, N) * n + u1];
            const T* lz = sLam + variant(vz, N) * n;
#pragma unroll
            for (int c = 0; c < n; ++c) in[c] = out[c] / (lxy + lz[c]);
#pragma unroll
            for (int a = 0; a < n; ++a) {
              T sacc = 0;
#pragma unroll
              for (int c = 0; c < n; ++c) sacc += q[a * n + c] * in[c];
              out[a] = sacc;
            }
          }
        } else {
#pragma unroll
          for (int a = 0; a < n; ++a) {
            T sacc = 0;
#pragma unroll
            for (int c = 0; c < n; ++c) sacc += q[a * n + c] * in[c];
            out[a] = sacc;
          }
        }
#pragma unroll
        for (int a = 0; a < n; ++a) line[a * stride] = out[a];
      }
      if (pass == 2) ++pass;  // z forward and back were fused
      __syncthreads();
    }
    // add the corrections on owned nodes (patches of one class are disjoint)
    for (int e = threadIdx.x; e < np * N3; e += kThreads) {
      const int pi = e / N3, t = e - pi * N3;
      const int a0 = t % n, a1 = (t / n) % n, a2 = t / NN;
      const int vx = vx0 + 2 * (pi % cx), vy = vy0 + 2 * ((pi / cx) % cyn), vz = vz0 + 2 * (pi / (cx * cyn));
      if (vx < 1 || vx > N - 1 || vy < 1 || vy > N - 1 || vz < 1 || vz > N - 1) continue;
      const int g0 = (vx - 1) * K + 1 + a0 - c0[0] * K, g1 = (vy - 1) * K + 1 + a1 - c0[1] * K,
                g2 = (vz - 1) * K + 1 + a2 - c0[2] * K;  // owned-local
      if (g0 < 0 || g0 >= TC * K || g1 < 0 || g1 >= TC * K || g2 < 0 || g2 >= TC * K) continue;
      sAcc[(g2 * OW + g1) * OW + g0] += sP[e];
    }
    __syncthreads();
  }
  const int gx1 = (c0[0] + TC >= N) ? n1 : (c0[0] + TC) * K;
  const int gy1 = (c0[1] + TC >= N) ? n1 : (c0[1] + TC) * K;
  const int gz1 = (c0[2] + TC >= N) ? n1 : (c0[2] + TC) * K;
  for (int e = threadIdx.x; e < OW * OW * OW; e += kThreads) {
    const int i = e % OW, j = (e / OW) % OW, l = e / (OW * OW);
    const int g0 = c0[0] * K + i, g1 = c0[1] * K + j, g2 = c0[2] * K + l;
    if (g0 >= gx1 || g1 >= gy1 || g2 >= gz1) continue;
    const size_t idx = (size_t)g2 * plane + (size_t)g1 * n1 + g0;
    const bool bnd = g0 == 0 || g0 == n1 - 1 || g1 == 0 || g1 == n1 - 1 || g2 == 0 || g2 == n1 - 1;
    xout[idx] = bnd ? T(0) : (xin ? xin[idx] : T(0)) + omega * sAcc[e];
  }
}

template <typename T, int K>
hipError_t patch3d_k(int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega, hipStream_t s) {
  constexpr int TC = PatchTile3D<K>::TC;
  const int n1 = K * N + 1;
  const int nt = (N + TC - 1) / TC;
  patch3d_kernel<T, K, TC><<<dim3(nt, nt, nt), kThreads, 0, s>>>(r, xin, xout, N, n1, e.Q, e.lam, omega);
  return hipGetLastError();
}

}  // namespace

template <typename Tin, typename T>
hipError_t launch_apply3d_wide(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s) {
#define CALL(K) apply3d_k<Tin, T, K>(N, c, x, b, y, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template <typename T>
hipError_t launch_patch3d_wide(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s) {
#define CALL(K) patch3d_k<T, K>(N, e, r, xin, xout, omega, s)
  C0IP_DISPATCH_K(k, CALL)
#undef CALL
}

template hipError_t launch_apply3d_wide<double, double>(int, int, const LevelCoef<double>&, const double*,
                                                   const double*, double*, hipStream_t);
template hipError_t launch_apply3d_wide<float, double>(int, int, const LevelCoef<double>&, const float*,
                                                  const double*, double*, hipStream_t);
template hipError_t launch_apply3d_wide<float, float>(int, int, const LevelCoef<float>&, const float*, const float*,
                                                 float*, hipStream_t);
template hipError_t launch_patch3d_wide<double>(int, int, const LevelEig<double>&, const double*, const double*,
                                           double*, double, hipStream_t);
template hipError_t launch_patch3d_wide<float>(int, int, const LevelEig<float>&, const float*, const float*, float*,
                                          float, hipStream_t);

}  // namespace c0ip
