// 3D matrix-free C0IP operator for gfx950 (Sec. 4, eq. c0iptensorvp3D
// used on the whole Cartesian mesh).  With the factors listed (z, y, x),
//   A = B M M + M B M + M M B + 2 (L L M + M L L + L M L).
// Grouped by the z factor, with per-plane sums over x and y
//   S1 = M_y (X B_x) + B_y (X M_x) + 2 L_y (X L_x),
//   S2 = M_y (X M_x),
//   S3 = 2 (L_y (X M_x) + M_y (X L_x)),
// the output is Y = M_z S1 + B_z S2 + L_z S3.
//
// A workgroup owns a TY x TX column of output nodes (whole cells) over a
// chunk of z cells and streams through the planes of the chunk plus a
// 2k-plane halo on each side:
//   * the plane is staged once in LDS with a 2k-node halo in x and y (the
//     next plane is already on its way from HBM in registers);
//   * one x pass per window of input row computes X M_x, X L_x and X B_x
//     into three LDS buffers;
//   * each thread owns one x column and one cell of y rows, so the y
//     positions in the cell, and with them the band shapes, are known at
//     compile time; the y passes give S1, S2, S3 of its k nodes;
//   * the z factor is applied in scatter form: 1D matrices are symmetric,
//     so plane zs adds row zs of M_z, B_z, L_z times its S values into a
//     register window of the 4k+1 output planes it reaches; the oldest
//     cell of the window is complete after the first plane of each cell
//     and is written out.
// Coefficients: with the default penalty the rows of the periodic classes
// are h-scaled copies of reference rows (h = 1) that are compile-time
// constants (generated at build time by gen_refcoef.cpp); every term of the
// 3D operator then carries the same factor 1/h, applied to the output.  On
// tiles whose x (y) rows are all periodic the x (y) coefficients are these
// constants; elsewhere the lanes in boundary classes redo their product with
// their own row from an LDS copy of the reference-scaled table.  The row
// class of a plane is the same for the whole workgroup: the z rows are read
// with wave-uniform addresses.  Output nodes on the faces x, y or z = 1 (the last node) are
// boundary nodes (zero rows of every 1D factor): tiles cover nodes
// [0, kN), and extra workgroups write those faces as zeros.
#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "refcoef.h"
#include "tiles.h"

namespace c0ip {
namespace {

using tile::Band;
using tile::clampi;

// The coefficient loads of a boundary plane are loop invariant; hoisted
// out of the plane loop they would not fit the scalar registers.  Passing
// the row offset through an empty asm statement on a scalar register keeps
// them inside.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Reference row of factor OP (0 = M, 1 = L, 2 = B) at cell position p.
template <int K, int OP>
__device__ __forceinline__ constexpr double ref_coef(int p, int j) {
  if constexpr (OP == 0)
    return RefCoef<K>::m[p][j];
  else if constexpr (OP == 1)
    return RefCoef<K>::l[p][j];
  else
    return RefCoef<K>::b[p][j];
}

// Band product with the reference row (constants) of the periodic class at
// cell position p; v centred on the row.
template <typename T, int OP, int K>
__device__ __forceinline__ T band_ref(const T* v, int p) {
  T a = 0;
#pragma unroll
  for (int o = Band<OP, K>::lo(p); o <= Band<OP, K>::hi(p); ++o) a += (T)ref_coef<K, OP>(p, 2 * K + o) * v[o];
  return a;
}

// Band product of factor OP for the row at cell position p of class cl:
// the reference row on tiles whose rows are all periodic (UNIFORM);
// elsewhere the lanes in boundary classes (every lane on meshes without
// periodic rows) redo it with their own row of the reference-scaled table
// in LDS.
template <typename T, int OP, int K, bool UNIFORM>
__device__ __forceinline__ T band3(const T* __restrict__ sTab, int nclass, int left, int periodic, int cl,
                                   const T* v, int p) {
  constexpr int W = 4 * K + 1, H = 2 * K;
  if constexpr (UNIFORM) {
    return band_ref<T, OP, K>(v, p);
  } else {
    T a = 0;
    if (periodic) a = band_ref<T, OP, K>(v, p);
    if (!periodic || cl != 2 * left + p) a = tile::band_dot<T, OP, K>(sTab + (OP * nclass + cl) * W + H, v, p);
    return a;
  }
}

// Tile geometry: TXC x TYC cells, x items of CW cells.  One thread per
// (x column, y cell).
template <int K_, int TXC_, int TYC_, int CW_>
struct Geo3 {
  static constexpr int K = K_, TXC = TXC_, TYC = TYC_, CW = CW_;
  static constexpr int H = 2 * K, W = 4 * K + 1, TX = TXC * K, TY = TYC * K, RX = TX + 4 * K, RY = TY + 4 * K;
  // LDS row strides: odd, so that lanes walking down a column hit distinct banks
  static constexpr int RXP = RX | 1, TXP = TX | 1;
  static constexpr int NTH = TX * TYC;
  static constexpr int NXG = TXC / CW, NXI = RY * NXG;
  static constexpr int NST = RX * RY, NL = (NST + NTH - 1) / NTH;
  static constexpr int TABMAX = 3 * (5 * K + 2) * W;  // row classes: at most 5k+2
  static_assert(TXC % CW == 0, "x items must divide the tile");
  static_assert(NTH % 64 == 0 && NTH <= 1024, "whole waves");
};

// X M_x on all staged rows, X L_x and X B_x on rows [k, RY - k).  Item
// (row r, group g of CW cells), rows fastest across lanes.
template <typename T, class G, bool XIN>
__device__ __forceinline__ void xpass3(const T* __restrict__ sX, T* __restrict__ sTM, T* __restrict__ sTL,
                                       T* __restrict__ sTB, const T* __restrict__ sTab, int nclass, int left,
                                       int right0, int periodic, int x0, int n1) {
  constexpr int K = G::K, CW = G::CW, H = G::H;
  constexpr int LO = Band<2, K>::win_lo(0), HI = Band<2, K>::win_hi() + (CW - 1) * K;
  for (int it = threadIdx.x; it < G::NXI; it += G::NTH) {
    const int g = it / G::RY, r = it - g * G::RY;
    T in[HI - LO + 1];
#pragma unroll
    for (int j = LO; j <= HI; ++j) in[j - LO] = sX[r * G::RXP + g * CW * K + j];
    auto cls = [&](int col, int p) {
      return XIN ? 2 * left + p : tile::row_class(clampi(x0 + col, 0, n1 - 1), n1, K, left, right0, periodic);
    };
    auto pass = [&](auto opc, T* __restrict__ out) {
      constexpr int OP = decltype(opc)::value;
#pragma unroll
      for (int p = 0; p < K; ++p)
#pragma unroll
        for (int w = 0; w < CW; ++w) {
          const int col = (g * CW + w) * K + p;
          out[col] = band3<T, OP, K, XIN>(sTab, nclass, left, periodic, cls(col, p), in + (w * K + p + H - LO), p);
        }
    };
    pass(std::integral_constant<int, 0>{}, sTM + r * G::TXP);
    if (r >= K && r < G::RY - K) {
      pass(std::integral_constant<int, 1>{}, sTL + (r - K) * G::TXP);
      pass(std::integral_constant<int, 2>{}, sTB + (r - K) * G::TXP);
    }
  }
}

// S1, S2, S3 of this thread's k nodes (x column l, y cell cy).  T_B and
// T_L hold staged rows [k, RY - k) (node y0 + cy k + p + o is their row
// cy k + p + k + o), T_M all staged rows (row cy k + p + 2k + o).
template <typename T, class G, bool YIN>
__device__ __forceinline__ void ypass3(const T* __restrict__ sTM, const T* __restrict__ sTL,
                                       const T* __restrict__ sTB, T (&S1)[G::K], T (&S2)[G::K], T (&S3)[G::K],
                                       const T* __restrict__ sTab, int nclass, int left, int right0, int periodic,
                                       int y0, int n1) {
  constexpr int K = G::K, TX = G::TX;
  const int l = threadIdx.x % TX, cy = threadIdx.x / TX;
  int cls[K];
#pragma unroll
  for (int p = 0; p < K; ++p)
    cls[p] = YIN ? 2 * left + p
                 : tile::row_class(clampi(y0 + cy * K + p, 0, n1 - 1), n1, K, left, right0, periodic);
  constexpr int TXP = G::TXP;
  // one window at a time (the scheduling barriers keep the next window's
  // loads from being hoisted over the current one's products)
  {
    T t[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) t[j] = sTB[(cy * K + j) * TXP + l];
#pragma unroll
    for (int p = 0; p < K; ++p) S1[p] = band3<T, 0, K, YIN>(sTab, nclass, left, periodic, cls[p], t + p + K, p);
  }
  __builtin_amdgcn_sched_barrier(0);
  {
    T t[3 * K];
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) t[j] = sTL[(cy * K + j) * TXP + l];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      S1[p] += T(2) * band3<T, 1, K, YIN>(sTab, nclass, left, periodic, cls[p], t + p + K, p);
      S3[p] = band3<T, 0, K, YIN>(sTab, nclass, left, periodic, cls[p], t + p + K, p);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  {
    T t[5 * K];
#pragma unroll
    for (int j = 0; j < 5 * K; ++j) t[j] = sTM[(cy * K + j) * TXP + l];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const T* v = t + p + 2 * K;
      S2[p] = band3<T, 0, K, YIN>(sTab, nclass, left, periodic, cls[p], v, p);
      S3[p] = T(2) * (S3[p] + band3<T, 1, K, YIN>(sTab, nclass, left, periodic, cls[p], v, p));
      S1[p] += band3<T, 2, K, YIN>(sTab, nclass, left, periodic, cls[p], v, p);
    }
  }
}

// Plane zs at cell position PS adds row zs of M_z, L_z, B_z (reference
// scaled, read with wave-uniform addresses) times S1, S3, S2 into the
// window: slot j is output plane (c - 2) k + j when zs = c k + PS.
template <typename T, int K, int PS, int OP>
__device__ __forceinline__ void zterm(T (&acc)[4 * K + 1][K], const T (&S)[K], const T* __restrict__ c) {
  constexpr int J = 2 * K + PS;
#pragma unroll
  for (int o = Band<OP, K>::lo(PS); o <= Band<OP, K>::hi(PS); ++o) {
    const T cv = c[o];
#pragma unroll
    for (int p = 0; p < K; ++p) acc[J + o][p] += cv * S[p];
  }
}
template <typename T, int K, int PS>
__device__ __forceinline__ void zscatter(T (&acc)[4 * K + 1][K], const T (&S1)[K], const T (&S2)[K],
                                         const T (&S3)[K], const T* __restrict__ ref, int row, int nclass) {
  constexpr int W = 4 * K + 1, H = 2 * K;
  zterm<T, K, PS, 0>(acc, S1, ref + opaque(row * W + H));
  zterm<T, K, PS, 1>(acc, S3, ref + opaque((nclass + row) * W + H));
  zterm<T, K, PS, 2>(acc, S2, ref + opaque((2 * nclass + row) * W + H));
}

// Raw buffer access: an offset at or beyond the buffer's size reads 0 and
// drops a store, which replaces the per-lane bounds tests of the staging
// loads, the residual's right-hand side and the output stores.
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

template <typename Tin, typename T, class G, bool RES, bool XIN, bool YIN>
__device__ __forceinline__ void apply3d_tile(const Tin* __restrict__ x, const T* __restrict__ b, T* __restrict__ y,
                                             int n1, const T* __restrict__ ref, T hinv, int nclass, int left,
                                             int right0, int periodic, int x0, int y0, int c0, int c1, T* __restrict__ sX,
                                             T* __restrict__ sTM, T* __restrict__ sTL, T* __restrict__ sTB,
                                             const T* __restrict__ sTab) {
  constexpr int K = G::K, H = G::H, NL = G::NL, NTH = G::NTH;
  const int NK = n1 - 1;
  const size_t plane = (size_t)n1 * n1;
  const unsigned pin = (unsigned)(plane * sizeof(Tin)), pout = (unsigned)(plane * sizeof(T));
  const int l = threadIdx.x % G::TX, cy = threadIdx.x / G::TX;
  const int gx = x0 + l;
  // in-plane byte offsets of this thread's staged elements (kOff: outside the mesh)
  unsigned soff[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = threadIdx.x + q * NTH;
    const int r = e / G::RX, c = e - r * G::RX;
    const int sy = y0 - H + r, sx = x0 - H + c;
    soff[q] = (e < G::NST && sy >= 0 && sy < n1 && sx >= 0 && sx < n1) ? (unsigned)(sy * n1 + sx) * sizeof(Tin)
                                                                       : kOff;
  }
  // output offsets (nodes of the tile below kN) and right-hand side offsets
  // (interior nodes only: the residual is 0 on the boundary)
  unsigned yoff[K], boff[K];
#pragma unroll
  for (int p = 0; p < K; ++p) {
    const int gy = y0 + cy * K + p;
    const unsigned o = (unsigned)(gy * n1 + gx) * sizeof(T);
    yoff[p] = gx < NK && gy < NK ? o : kOff;
    boff[p] = gx >= 1 && gx < NK && gy >= 1 && gy < NK ? o : kOff;
  }
  T v[NL];
  // planes that contribute to outputs [c0 k, c1 k), without the boundary planes
  const int zA = max((c0 - 2) * K, 1), zB = min((c1 + 1) * K, NK - 1);
  auto load_plane = [&](int z) {  // zeros beyond plane zB
    const __amdgpu_buffer_rsrc_t r = buf(x + (size_t)z * plane, z <= zB ? pin : 0u);
#pragma unroll
    for (int q = 0; q < NL; ++q) v[q] = (T)buf_load<Tin>(r, soff[q]);
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = threadIdx.x + q * NTH, r = e / G::RX;
      sX[e + r * (G::RXP - G::RX)] = v[q];  // rows padded to RXP; sX also holds the tail of the last q
    }
  };
  T acc[4 * K + 1][K];
#pragma unroll
  for (int j = 0; j <= 4 * K; ++j)
#pragma unroll
    for (int p = 0; p < K; ++p) acc[j][p] = T(0);
  load_plane(zA);
  store_plane();
  load_plane(zA + 1);
  T bq[RES ? K : 1][K];
  for (int c = c0 - 2; c <= c1 + 1; ++c) {
    const int ce = c - 2;  // the cell written after this cell's first plane
    const bool emit_c = ce >= c0 && ce < c1;
    if constexpr (RES) {
      if (emit_c) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int gz = ce * K + j;  // plane 0 is boundary: an empty buffer reads 0
          const __amdgpu_buffer_rsrc_t r = buf(b + (size_t)gz * plane, gz >= 1 ? pout : 0u);
#pragma unroll
          for (int p = 0; p < K; ++p) bq[j][p] = buf_load<T>(r, boff[p]);
        }
      }
    }
    static_for<0, K>([&](auto psc) {
      constexpr int ps = decltype(psc)::value;
      if (ps > 0 && c == c1 + 1) return;
      const int zs = c * K + ps;
      if (zs >= zA && zs <= zB) {
        __syncthreads();  // sX holds plane zs; the previous y passes are done
        xpass3<T, G, XIN>(sX, sTM, sTL, sTB, sTab, nclass, left, right0, periodic, x0, n1);
        __syncthreads();
        store_plane();  // plane zs + 1 (unused after zB)
        load_plane(zs + 2);
        T S1[K], S2[K], S3[K];
        ypass3<T, G, YIN>(sTM, sTL, sTB, S1, S2, S3, sTab, nclass, left, right0, periodic, y0, n1);
        const int clz = tile::row_class(zs, n1, K, left, right0, periodic);
        zscatter<T, K, ps>(acc, S1, S2, S3, ref, clz, nclass);
      }
      if (ps == 0 && emit_c) {
        // boundary outputs: zero rows give acc = 0, and b reads 0 there
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const __amdgpu_buffer_rsrc_t r = buf(y + (size_t)(ce * K + j) * plane, pout);
#pragma unroll
          for (int p = 0; p < K; ++p) {
            const T a = hinv * acc[j][p];
            buf_store<T>(r, yoff[p], RES ? bq[j][p] - a : a);
          }
        }
      }
    });
#pragma unroll
    for (int j = 0; j <= 3 * K; ++j)
#pragma unroll
      for (int p = 0; p < K; ++p) acc[j][p] = acc[j + K][p];
#pragma unroll
    for (int j = 3 * K + 1; j <= 4 * K; ++j)
#pragma unroll
      for (int p = 0; p < K; ++p) acc[j][p] = T(0);
  }
}

template <class G>
__host__ __device__ inline bool tile3_xin(int periodic, int left, int right0, int x0) {
  return periodic && x0 >= left && x0 + G::TX <= right0;
}
template <class G>
__host__ __device__ inline bool tile3_yin(int periodic, int left, int right0, int y0) {
  return periodic && y0 >= left && y0 + G::TY <= right0;
}

// Zeros on the faces x = kN, y = kN, z = kN (boundary nodes that no tile
// owns): face element f of 3 n1^2, 16 per thread.
template <typename T, int NTH>
__device__ __forceinline__ void zero_faces(T* __restrict__ y, int n1, int fb) {
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
template <int NTH>
inline int face_blocks(int n1) {
  return (int)((3 * (int64_t)n1 * n1 + 16 * NTH - 1) / (16 * NTH));
}

// RING = false: one workgroup per (interior tile, z chunk), every x and y
// row periodic, so all band shapes and coefficients are compile-time.
// RING = true: the tiles of the boundary ring (per-lane row classes), then
// the workgroups that zero the faces.  Two launches keep the interior
// kernel's register budget, and so its occupancy, free of the boundary
// code.
template <typename Tin, typename T, class G, bool RES, bool RING>
__global__ __launch_bounds__(G::NTH) void apply3d_kernel(const Tin* __restrict__ x, const T* __restrict__ b,
                                                         T* __restrict__ y, int N, int n1, const T* __restrict__ ref,
                                                         T hinv, int nclass, int left, int right0, int periodic,
                                                         int zcc, tile::TileOrder ord) {
  int bx, by;
  if constexpr (RING) {
    if ((int)blockIdx.x >= ord.nb) {
      if (blockIdx.y == 0) zero_faces<T, G::NTH>(y, n1, blockIdx.x - ord.nb);
      return;
    }
    tile::tile_of_block(ord, blockIdx.x, bx, by);
  } else {
    if (!tile::tile_of_block(ord, ord.nbp + blockIdx.x, bx, by)) return;
  }
  __shared__ T sX[G::NL * G::NTH + (G::NL * G::NTH / G::RX + 1) * (G::RXP - G::RX)];
  __shared__ T sTM[G::RY * G::TXP];
  __shared__ T sTL[(G::RY - 2 * G::K) * G::TXP];
  __shared__ T sTB[(G::RY - 2 * G::K) * G::TXP];
  __shared__ T sTab[RING ? G::TABMAX : 1];
  const int x0 = bx * G::TX, y0 = by * G::TY;
  const int c0 = blockIdx.y * zcc, c1 = min(c0 + zcc, N);
#define C0IP_TILE(XI, YI)                                                                                        \
  apply3d_tile<Tin, T, G, RES, XI, YI>(x, b, y, n1, ref, hinv, nclass, left, right0, periodic, x0, y0, c0, c1, sX, \
                                       sTM, sTL, sTB, sTab)
  if constexpr (RING) {
    for (int e = threadIdx.x; e < 3 * nclass * G::W; e += G::NTH) sTab[e] = ref[e];
    // (the first barrier of the plane loop orders the table copy)
    const bool xin = tile3_xin<G>(periodic, left, right0, x0), yin = tile3_yin<G>(periodic, left, right0, y0);
    if (xin)
      C0IP_TILE(true, false);
    else if (yin)
      C0IP_TILE(false, true);
    else
      C0IP_TILE(false, false);
  } else {
    C0IP_TILE(true, true);
  }
#undef C0IP_TILE
}

// Tile configuration per degree (k <= 4; the register window of the z
// factor holds (4k+1) k values per thread).
template <int K> struct Apply3Cfg;
template <> struct Apply3Cfg<2> { using G = Geo3<2, 16, 8, 2>; };
template <> struct Apply3Cfg<3> { using G = Geo3<3, 16, 4, 2>; };
template <> struct Apply3Cfg<4> { using G = Geo3<4, 8, 4, 2>; };

template <typename Tin, typename T, class G>
hipError_t apply3d_g(int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s) {
  const int n1 = G::K * N + 1;
  const int tx = (N + G::TXC - 1) / G::TXC, ty = (N + G::TYC - 1) / G::TYC;
  const tile::TileOrder ord =
      tile::make_order(tx, ty, [&](int bx) { return tile3_xin<G>(c.periodic, c.left, c.right0, bx * G::TX); },
                       [&](int by) { return tile3_yin<G>(c.periodic, c.left, c.right0, by * G::TY); });
  // z chunks: enough workgroups for the whole chip, at most 3k + 1 halo
  // planes recomputed per chunk
  int zcc = N;
  while (zcc > 8 && (int64_t)tx * ty * ((N + zcc - 1) / zcc) < 1024) zcc = (zcc + 1) / 2;
  // the ring's slower workgroups take shorter z chunks: 16 per column
  // (measured best for k = 3 at 32^3, 64^3 and 128^3 cells)
  const int zcr = std::max(2, N / 16);
  const int nin = tile::order_blocks(ord) - ord.nbp;
  const dim3 gring(ord.nb + face_blocks<G::NTH>(n1), (N + zcr - 1) / zcr), gin(nin, (N + zcc - 1) / zcc);
#define C0IP_LAUNCH(RES, RING, GRID, ZC)                                                                         \
  apply3d_kernel<Tin, T, G, RES, RING><<<GRID, G::NTH, 0, s>>>(x, b, y, N, n1, c.ref, c.hinv, c.nclass, c.left, \
                                                               c.right0, c.periodic, ZC, ord)
  if (b) {
    C0IP_LAUNCH(true, true, gring, zcr);
    if (nin > 0) C0IP_LAUNCH(true, false, gin, zcc);
  } else {
    C0IP_LAUNCH(false, true, gring, zcr);
    if (nin > 0) C0IP_LAUNCH(false, false, gin, zcc);
  }
#undef C0IP_LAUNCH
  return hipGetLastError();
}

}  // namespace

template <typename Tin, typename T>
hipError_t launch_apply3d(int k, int N, const LevelCoef<T>& c, const Tin* x, const T* b, T* y, hipStream_t s) {
  if (!c.ref) return launch_apply3d_wide<Tin, T>(k, N, c, x, b, y, s);  // not the default penalty
  // raw buffer offsets of a plane must stay below 2^31 bytes
  if ((double)(k * N + 1) * (k * N + 1) * sizeof(T) >= 2147483648.0) return hipErrorInvalidValue;
  switch (k) {
    case 2: return apply3d_g<Tin, T, Apply3Cfg<2>::G>(N, c, x, b, y, s);
    case 3: return apply3d_g<Tin, T, Apply3Cfg<3>::G>(N, c, x, b, y, s);
    case 4: return apply3d_g<Tin, T, Apply3Cfg<4>::G>(N, c, x, b, y, s);
    default: return launch_apply3d_wide<Tin, T>(k, N, c, x, b, y, s);
  }
}

template hipError_t launch_apply3d<double, double>(int, int, const LevelCoef<double>&, const double*,
                                                   const double*, double*, hipStream_t);
template hipError_t launch_apply3d<float, double>(int, int, const LevelCoef<double>&, const float*,
                                                  const double*, double*, hipStream_t);
template hipError_t launch_apply3d<float, float>(int, int, const LevelCoef<float>&, const float*, const float*,
                                                 float*, hipStream_t);

}  // namespace c0ip
