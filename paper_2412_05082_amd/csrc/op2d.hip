// Instantiations of the 2D operator kernels (eq. c0iptensorvp; the kernels are in op2d_impl.h).
#include "op2d_impl.h"

namespace c0ip {

int avs2d_variants(int k) {
  switch (k) {
    case 2: return FusedTiles<2>::n;
    case 3: return FusedTiles<3>::n;
    case 4: return FusedTiles<4>::n;
    case 5: return FusedTiles<5>::n;
    case 6: return FusedTiles<6>::n;
    case 7: return FusedTiles<7>::n;
    default: return 1;
  }
}
template hipError_t launch_apply2d<double, double>(int, int, const LevelCoef<double>&, const double*,
                                                   const double*, double*, hipStream_t, int, int64_t, const int*,
                                                   double*);
template hipError_t launch_apply2d<float, double>(int, int, const LevelCoef<double>&, const float*,
                                                  const double*, double*, hipStream_t, int, int64_t, const int*,
                                                  float*);
template hipError_t launch_apply2d<float, float>(int, int, const LevelCoef<float>&, const float*, const float*,
                                                 float*, hipStream_t, int, int64_t, const int*, float*);

}  // namespace c0ip
