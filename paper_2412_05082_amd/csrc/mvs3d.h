// One colour of the coloured multiplicative smoother on a 3D mesh (internal
// to libc0ip; plain pointers).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace c0ip {

// x += omega * sum over colour c's patches of R_v^T A~_v^{-1} R_v r, in
// place (16 colours; the colour's patches are disjoint and A-orthogonal).
template <typename T>
hipError_t launch_mvs3d_colour(int k, int N, int colour, const LevelEig<T>& e, const T* r, T* x, T omega,
                               hipStream_t s);

}  // namespace c0ip
