// The fused first pre-smoothing step and residual of a 2D V-cycle level
// (internal to libc0ip; plain pointers).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace c0ip {

// x1 = S(0, b) and r = b - A x1 on level N in one launch (owner computes).
// Returns hipErrorNotSupported for k > 3 (the patch solves are in registers).
template <typename T>
hipError_t launch_pre2d(int k, int N, const LevelCoef<T>& c, const LevelEig<T>& e, const T* b, T* x1, T* r, T omega,
                        hipStream_t s);
// Largest level (cells per direction) on which the V-cycle uses it.
constexpr int kPre2dMaxN = 128;

}  // namespace c0ip
