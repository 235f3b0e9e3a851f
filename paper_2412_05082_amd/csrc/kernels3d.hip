// 3D kernels (operator and smoother): not yet provided in this build.
#include "kernels.h"

namespace c0ip {

template <typename Tin, typename T>
hipError_t launch_apply3d(int, int, const LevelCoef<T>&, const Tin*, const T*, T*, hipStream_t) {
  return hipErrorNotSupported;
}
template <typename T>
hipError_t launch_patch3d(int, int, const LevelEig<T>&, const T*, const T*, T*, T, hipStream_t) {
  return hipErrorNotSupported;
}

template hipError_t launch_apply3d<double, double>(int, int, const LevelCoef<double>&, const double*,
                                                   const double*, double*, hipStream_t);
template hipError_t launch_apply3d<float, double>(int, int, const LevelCoef<double>&, const float*,
                                                  const double*, double*, hipStream_t);
template hipError_t launch_apply3d<float, float>(int, int, const LevelCoef<float>&, const float*, const float*,
                                                 float*, hipStream_t);
template hipError_t launch_patch3d<double>(int, int, const LevelEig<double>&, const double*, const double*,
                                           double*, double, hipStream_t);
template hipError_t launch_patch3d<float>(int, int, const LevelEig<float>&, const float*, const float*, float*,
                                          float, hipStream_t);

}  // namespace c0ip
