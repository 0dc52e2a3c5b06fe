// Launch shapes of the level step with two groups per 512-thread workgroup
// (the kernel is in mhm_level.h; a translation unit of its own so that these
// instantiations compile in parallel with the others).

#include "mhm_level.h"

namespace gh {

template <typename T, bool kCfl, typename Off>
void launch_level_shape_g2(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                           const double* dt_dev, double dx, int first_order, int ws, int* n_bad, const CflOut& cfl,
                           int variant, int64_t blocks, int order, hipStream_t stream) {
  if (variant & 8)
    launch_level_lds<T, kCfl, Off, 1, 2>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                         variant, blocks, order, stream);
  else
    launch_level_lds<T, kCfl, Off, 0, 2>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                         variant, blocks, order, stream);
}

#define GH_G2(T, C, O)                                                                                           \
  template void launch_level_shape_g2<T, C, O>(const T*, T*, const LevelGeom&, const Gas<T>&, const double*,     \
                                               double, int, int, int*, const CflOut&, int, int64_t, int,         \
                                               hipStream_t);
GH_G2(double, true, unsigned int)
GH_G2(double, false, unsigned int)
GH_G2(double, true, int64_t)
GH_G2(double, false, int64_t)
GH_G2(float, true, unsigned int)
GH_G2(float, false, unsigned int)
GH_G2(float, true, int64_t)
GH_G2(float, false, int64_t)
#undef GH_G2

}  // namespace gh
