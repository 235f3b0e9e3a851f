// Device helpers shared by the 2D tile kernels (row classes of the 1D
// factors, structural bands, XCD-aware tile order).
#pragma once

#include <hip/hip_runtime.h>

namespace c0ip {
namespace tile {

constexpr int kThreads = 256;

// Row class of global 1D row g: rows within 2k of either end are their own
// class; the others repeat with the node's position in its cell.
__device__ __forceinline__ int row_class(int g, int n1, int k, int left, int right0, int periodic) {
  if (!periodic) return g;
  if (g < left) return g;
  if (g >= right0) return left + (n1 - 1 - g);
  return 2 * left + g % k;
}

// Boundary type of the vertex patch at vertex v in [1, N-1] along one axis.
__device__ __forceinline__ int variant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap the (x, y) tile index so that XCD c walks one contiguous band
// of tiles (row-major): neighbouring tiles, whose halos overlap, then share
// that XCD's L2.  A bijection for any grid size.
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int gx = gridDim.x, T = gx * gridDim.y;
  const int L = blockIdx.x + blockIdx.y * gx;
  const int c = L & 7, q = L >> 3;
  const int logical = c * (T >> 3) + min(c, T & 7) + q;
  bx = logical % gx;
  by = logical / gx;
}

// Structural band of a row at position p in its cell (p = 0: vertex node)
// for the three 1D factors, OP = 0 (M), 1 (L), 2 (B): M and L couple the
// nodes of the one (p > 0) or two (p = 0) cells containing the row; B
// reaches one cell further on each side through the point terms.
template <int OP, int K>
struct Band {
  static constexpr int lo(int p) { return OP == 2 ? (p == 0 ? -2 * K : -K - p) : (p == 0 ? -K : -p); }
  static constexpr int hi(int p) { return OP == 2 ? (p == 0 ? 2 * K : 2 * K - p) : (p == 0 ? K : K - p); }
  static constexpr int width(int p) { return hi(p) - lo(p) + 1; }
  // input window (relative to the cell's first node minus 2K) of rows p0..K-1
  static constexpr int win_lo(int p0) { return 2 * K + (p0 == 0 ? lo(0) : lo(1) + 1); }
  static constexpr int win_hi() { return 2 * K + (OP == 2 ? 2 * K : K); }
};

}  // namespace tile
}  // namespace c0ip
