// Exact local solvers: vertex-patch smoothers whose local solve is the
// dense inverse of the exact patch matrix A_v = R_v A R_v^T (internal to
// libc0ip; plain pointers).  Aex holds one inverse per patch type:
// Aex[(ty * 4 + tx) * NN * NN + i * NN + j], NN = (2k-1)^2, type = the
// patch's boundary variant along x and y (tile::variant).
#pragma once

#include <hip/hip_runtime.h>

namespace c0ip {

// x_out = x_in + omega * sum_v R_v^T A_v^{-1} R_v r (x_in == nullptr: 0);
// owner computes over tiles (x_out may equal x_in).
template <typename T>
hipError_t launch_patch2d_exact(int k, int N, const T* Aex, const T* r, const T* xin, T* xout, T omega,
                                hipStream_t s);
// One colour of the multiplicative smoother with exact local solves: launch_mvs2d_colour_exact (kernels.h).

}  // namespace c0ip
