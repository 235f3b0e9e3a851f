// Fast-diagonalisation solve of one 2D vertex patch in registers (eq.
// inverse): u = (Q_y (x) Q_x) D^{-1} (Q_y (x) Q_x)^T r for the n x n patch
// block r (row a = y index, column c = x index), with the generalised
// eigenbases Q (Q[c' * n + c] = component c' of eigenvector c) and the
// reciprocal eigenvalue sums D[ap * n + c] = 1 / (lambda_x[c] + lambda_y[ap]).
// One thread solves one patch: four 1D transforms of n^3 products each, no
// intermediate trip through LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace c0ip {
namespace fdm {

// Dinv(ap, c): the reciprocal eigenvalue sum for (y mode ap, x mode c).
template <typename T, int n, class QX, class QY, class DINV>
__device__ __forceinline__ void patch_reg(const T* __restrict__ src, int stride, T* __restrict__ dst, QX qx, QY qy,
                                          DINV dinv) {
  T t[n][n];
  // forward along x: t[a][c] = sum_c' Qx[c'][c] r[a][c']
#pragma unroll
  for (int a = 0; a < n; ++a) {
    T in[n];
#pragma unroll
    for (int c = 0; c < n; ++c) in[c] = src[a * stride + c];
#pragma unroll
    for (int c = 0; c < n; ++c) {
      T s = 0;
#pragma unroll
      for (int cp = 0; cp < n; ++cp) s += qx(cp * n + c) * in[cp];
      t[a][c] = s;
    }
  }
  // along y per column: forward with Qy^T, scale, back with Qy
#pragma unroll
  for (int c = 0; c < n; ++c) {
    T f[n];
#pragma unroll
    for (int ap = 0; ap < n; ++ap) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < n; ++a) s += qy(a * n + ap) * t[a][c];
      f[ap] = s * dinv(ap, c);
    }
#pragma unroll
    for (int a = 0; a < n; ++a) {
      T s = 0;
#pragma unroll
      for (int ap = 0; ap < n; ++ap) s += qy(a * n + ap) * f[ap];
      t[a][c] = s;
    }
  }
  // back along x: u[a][c'] = sum_c Qx[c'][c] t[a][c]
#pragma unroll
  for (int a = 0; a < n; ++a)
#pragma unroll
    for (int cp = 0; cp < n; ++cp) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) s += qx(cp * n + c) * t[a][c];
      dst[a * n + cp] = s;
    }
}

}  // namespace fdm
}  // namespace c0ip

