// Vector kernels of the flexible conjugate-gradient solve (internal to
// libc0ip; plain pointers).  Scalars live in a small device array sc[]:
//   sc[kZQ] = z . q_old, sc[kPQ] = p . q, sc[kRP] = r . p, sc[kRR] = r . r,
//   sc[kPQOLD] = the previous p . q, sc[kBETA], sc[kALPHA].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace c0ip {
namespace cg {

enum Slot { kZQ = 0, kPQ = 1, kRP = 2, kRR = 3, kPQOLD = 4, kBETA = 5, kALPHA = 6, kSlots = 8 };

int blocks(int64_t n);
// partial[b] = block b's share of z . q  (z float32 or float64)
template <typename Tz>
hipError_t launch_dot(int64_t n, const Tz* z, const double* q, double* partial, int nblk, hipStream_t s);
// partial[b], partial[nblk + b] = block b's shares of p . q and r . p
hipError_t launch_dot2(int64_t n, const double* p, const double* q, const double* r, double* partial, int nblk,
                       hipStream_t s);
// sc[slot + j] = sum of partial row j (j < m); then, by stage:
//   stage 1 (after z . q_old): beta = zq / pq_old;
//   stage 2 (after p . q, r . p): alpha = rp / pq, pq_old = pq;  stage 0: nothing.
hipError_t launch_reduce(int m, int nblk, const double* partial, double* sc, int slot, int stage, hipStream_t s);
// p = z - beta p  (beta = sc[kBETA]; first = 1: p = z)
template <typename Tz>
hipError_t launch_update_p(int64_t n, const Tz* z, const double* sc, double* p, int first, hipStream_t s);
// x += alpha p, r -= alpha q (alpha = sc[kALPHA]); partial[b] = block b's share of r . r;
// r32: NULL, or receives (float) of the new r (the next float32 V-cycle's input)
hipError_t launch_update_xr(int64_t n, const double* sc, const double* p, const double* q, double* x, double* r,
                            double* partial, int nblk, hipStream_t s, float* r32 = nullptr);

}  // namespace cg
}  // namespace c0ip
