// Launchers of the gfx950 kernels (internal to libc0ip; plain pointers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace c0ip {

// Coefficient tables of one level's 1D M, L, B (row classes, see setup.h).
template <typename T>
struct LevelCoef {
  const T* tab = nullptr;  // [3][nclass][4k+1]
  int nclass = 0, left = 0, right0 = 0, periodic = 0;
  // With the default penalty: the same table scaled to h = 1 (M / h, L h,
  // B h^3), whose periodic rows are the compile-time reference rows, and
  // 1/h; ref == nullptr otherwise.
  const T* ref = nullptr;
  T hinv = 0;
};

// Fast-diagonalisation data of one level: Q[4][n*n], lam[4][n].
template <typename T>
struct LevelEig {
  const T* Q = nullptr;
  const T* lam = nullptr;
};

// y = A x, or y = b - A x when b != nullptr (boundary entries of y are 0).
// Tin = type of x, T = compute/output type.
template <typename Tin, typename T>
hipError_t launch_apply(int dim, int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y,
                        hipStream_t s);

// x_out = x_in + omega * sum_v R_v^T A~_v^{-1} R_v r  (x_in == nullptr: 0).
template <typename T>
hipError_t launch_patch_smooth(int dim, int k, int N, const LevelEig<T>& e, const T* r, const T* x_in,
                               T* x_out, T omega, hipStream_t s);

// Grid transfers (tensor-product 1D embedding, table [2][k][k+1]).
// restrict: bc = P^T rf;  prolong: xf (+)= P ec.  scratch >= n1f^(dim-1) * n1c elements.
template <typename T>
hipError_t launch_restrict(int dim, int k, int Nc, const T* table, const T* rf, T* bc, T* scratch,
                           hipStream_t s);
template <typename T>
hipError_t launch_prolong_add(int dim, int k, int Nc, const T* table, const T* ec, T* xf, T* scratch,
                              hipStream_t s);

// Level-0 solve: x = A0^{-1} b on the (2k-1)^dim interior nodes (float64);
// batched over nsys systems zs apart, skipping those with active[z] == 0.
template <typename T>
hipError_t launch_coarse(int dim, int k, const double* Ainv, const T* b, T* x, hipStream_t s, int nsys = 1,
                         int64_t zs = 0, const int* active = nullptr);

// Vector kernels (n = length).
template <typename Ta, typename Tb>
hipError_t launch_cast(int64_t n, const Ta* a, Tb* b, hipStream_t s);
hipError_t launch_fill(int64_t n, double v, double* a, hipStream_t s);
template <typename T>
hipError_t launch_fill_t(int64_t n, T v, T* a, hipStream_t s);
// partial[j * nblk + blk] = partial sum of V_j . w (j < m), nblk blocks.
hipError_t launch_multidot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* partial,
                           int nblk, hipStream_t s);
// out[j] = sum_b partial[j * nblk + b] (+ out_add[j] if accumulate)
hipError_t launch_reduce_partials(int m, int nblk, const double* partial, double* out, int accumulate,
                                  hipStream_t s);
// v = w / *nrm (nrm = device pointer to a squared norm: v = w / sqrt(*nrm))
hipError_t launch_normalize(int64_t n, const double* w, const double* nrm2, double* v, hipStream_t s);
// x += sum_j y[j] Z_j  (Z of type Tz)
template <typename Tz>
hipError_t launch_update_solution(int64_t n, int m, const Tz* Z, int64_t ldz, const double* y, double* x,
                                  hipStream_t s);

int multidot_blocks(int64_t n);

// Arnoldi step with delayed re-orthogonalisation (see kernels_common.hip).
// dots: partial[(2j+3) * nblk]; reduce_coef: d[2j+3] and coef[2j+5];
// update: V_j = (u - V s)/alpha into vout, u <- w - V f - (h_v/alpha) u.
int arnoldi_blocks(int64_t n);
hipError_t launch_arnoldi_dots(int64_t n, int j, const double* V, int64_t ldv, const double* u, const double* w,
                               double* partial, int nblk, hipStream_t s);
// d[row] = sum of partial row (2j+3 rows), then coef from d (2j+5 values);
// host: NULL or device-visible pinned memory that receives d at [0, 2j+3)
// and coef at [hoff, hoff + 2j+5), readable once the launches have completed.
hipError_t launch_arnoldi_reduce_coef(int j, int nblk, const double* partial, double* d, double* coef,
                                      double* host, int hoff, hipStream_t s);
// u32: NULL, or receives (float) of the new u (the next float32 V-cycle's input).
hipError_t launch_arnoldi_update(int64_t n, int j, const double* V, int64_t ldv, double* u, const double* w,
                                 const double* coef, double* vout, hipStream_t s, float* u32 = nullptr);

// Per-dimension operator and smoother launchers (k dispatched at run time).
// Batched forms (2D): nsys systems whose vectors are zs elements apart
// (fine / coarse strides zf / zc for the transfers); nsys = 1 for one.
// xc: NULL, or (one system) receives a copy of x, written from the staged
// tiles (saves a separate copy where x is needed again).
template <typename Tin, typename T>
hipError_t launch_apply2d(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s,
                          int nsys = 1, int64_t zs = 0, const int* active = nullptr, Tin* xc = nullptr);
template <typename T>
hipError_t launch_patch2d(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s, int nsys = 1, int64_t zs = 0, const int* active = nullptr);
// xout += omega * sum_v R_v^T A~_v^{-1} R_v r with floating-point atomics
// (xout initialised by the caller; each patch solved once).
template <typename T>
hipError_t launch_patch2d_atomic(int k, int N, const LevelEig<T>& e, const T* r, T* xout, T omega, hipStream_t s);
// One colour of the coloured multiplicative smoother (2D, 8 colours):
// One colour of the 2D multiplicative smoother, in place on x:
// x += omega * sum over the colour's patches of R_v^T A~_v^{-1} R_v r.  With
// r == nullptr the launch forms r = b - A x on each patch's rows in LDS,
// from x as it is before the launch (the colour's patches are disjoint and
// A-orthogonal, and none reads the nodes another one writes); else r is
// read (a residual computed beforehand, or b when x is 0).
template <typename T>
hipError_t launch_mvs2d_colour(int k, int N, int colour, const LevelCoef<T>& c, const LevelEig<T>& e, const T* b,
                               const T* r, T* x, T omega, hipStream_t s);
// The same with exact local solves (dense inverses Aex, layout as in exact.h).
template <typename T>
hipError_t launch_mvs2d_colour_exact(int k, int N, int colour, const LevelCoef<T>& c, const T* Aex, const T* b,
                                     const T* r, T* x, T omega, hipStream_t s);
// One fused smoothing step S(x, b) (residual in LDS; x_out must not alias x).
// variant: tile-size variant (0 = default; see avs2d_variants).  With ec:
// the step starts from x + P ec instead (ec: coarse vector of the level
// below, zc apart between systems; ptab: the embedding table).
template <typename T>
hipError_t launch_avs2d(int k, int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* x, const T* b, T* xout,
                        T omega, hipStream_t s, int nsys = 1, int64_t zs = 0, const int* active = nullptr,
                        int variant = 0, const T* ec = nullptr, const T* ptab = nullptr, int64_t zc = 0);
int avs2d_variants(int k);
template <typename T>
hipError_t launch_restrict2d(int k, int Nc, const T* table, const T* rf, T* bc, hipStream_t s, int nsys = 1,
                             int64_t zf = 0, int64_t zc = 0, const int* active = nullptr);
// xf = xin + P ec (xin may equal xf)
template <typename T>
hipError_t launch_prolong2d(int k, int Nc, const T* table, const T* ec, const T* xin, T* xf, hipStream_t s,
                            int nsys = 1, int64_t zc = 0, int64_t zf = 0, const int* active = nullptr);
template <typename Tin, typename T>
hipError_t launch_apply3d(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s);
// z-streaming operator with per-lane band loops (any k; used for k >= 5).
template <typename Tin, typename T>
hipError_t launch_apply3d_wide(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s);
template <typename T>
hipError_t launch_patch3d(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                          hipStream_t s);
// owner-computes patch smoother over cubic tiles with per-lane bases (any k; used for k >= 5)
template <typename T>
hipError_t launch_patch3d_wide(int k, int N, const LevelEig<T>& e, const T* r, const T* xin, T* xout, T omega,
                               hipStream_t s);

// Lowest levels 0..LT of the 2D V-cycle in one launch, one workgroup per
// system, every vector in LDS (vtail.hip).  Tables as on the tiled path.
constexpr int kTailMaxLevels = 5;
template <typename T>
struct TailParams {
  int LT = 0;  // top level of the tail
  int nclass[kTailMaxLevels] = {}, left[kTailMaxLevels] = {}, right0[kTailMaxLevels] = {},
      periodic[kTailMaxLevels] = {};
  const T* tab[kTailMaxLevels] = {};
  const T* Q[kTailMaxLevels] = {};
  const T* lam[kTailMaxLevels] = {};
  const T* ptab = nullptr;       // embedding table [2][k][k+1]
  const double* Ainv = nullptr;  // level-0 inverse (coarse_mode 0)
  T omega = 0;
  int pre = 1, post = 1, coarse_mode = 0;
};
// Per-level slot buffers: system s exists on level l iff s < nA[l]; its
// vectors start at b[l] + s * stride[l] (x likewise).  A system's tail
// starts at its highest level <= LT: b there is read, x there is written.
template <typename T>
struct TailIO {
  const T* b[kTailMaxLevels] = {};
  T* x[kTailMaxLevels] = {};
  int64_t stride[kTailMaxLevels] = {};
  int nA[kTailMaxLevels] = {};
  const int* active = nullptr;
};
// LDS bytes of the tail kernel for degree k up to level LT (nclass per level).
int tail_bytes(int k, int LT, const int* nclass, int elem_size);
// Largest LDS a workgroup may use on the current device.
int tail_lds_limit();
// Allow the tail kernel of degree k `bytes` of dynamic LDS (before launch or capture).
template <typename T>
hipError_t configure_vtail(int k, int bytes);
template <typename T>
hipError_t launch_vtail(int k, const TailParams<T>& P, const TailIO<T>& io, int nsys, hipStream_t s);

#define C0IP_DISPATCH_K(k, CALL)          \
  switch (k) {                            \
    case 2: return CALL(2);               \
    case 3: return CALL(3);               \
    case 4: return CALL(4);               \
    case 5: return CALL(5);               \
    case 6: return CALL(6);               \
    case 7: return CALL(7);               \
    default: return hipErrorInvalidValue; \
  }

}  // namespace c0ip
