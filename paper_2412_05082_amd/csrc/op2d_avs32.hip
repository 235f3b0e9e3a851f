// Instantiations of the fused 2D smoother step in float32 (Sec. 3; the kernel is in op2d_impl.h).
#include "op2d_impl.h"
#include "pre2d.h"

namespace c0ip {

template hipError_t launch_avs2d<float>(int, int, const LevelCoef<float>&, const LevelEig<float>&, const float*,
                                        const float*, float*, float, hipStream_t, int, int64_t, const int*, int,
                                        const float*, const float*, int64_t);
template hipError_t launch_pre2d<float>(int, int, const LevelCoef<float>&, const LevelEig<float>&, const float*,
                                        float*, float*, float, hipStream_t);

}  // namespace c0ip
