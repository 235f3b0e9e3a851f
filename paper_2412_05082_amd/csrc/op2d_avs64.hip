// Instantiations of the fused 2D smoother step in float64 (Sec. 3; the kernel is in op2d_impl.h).
#include "op2d_impl.h"
#include "pre2d.h"

namespace c0ip {

template hipError_t launch_avs2d<double>(int, int, const LevelCoef<double>&, const LevelEig<double>&, const double*,
                                         const double*, double*, double, hipStream_t, int, int64_t, const int*, int,
                                         const double*, const double*, int64_t);
template hipError_t launch_pre2d<double>(int, int, const LevelCoef<double>&, const LevelEig<double>&, const double*,
                                        double*, double*, double, hipStream_t);

}  // namespace c0ip
