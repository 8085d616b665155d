// Kernels of the fused 3-D push/deposit for 8x8x8-cell tiles.
#include "push3d_impl.h"

namespace apt {

template hipError_t launch3d_tile<float, 8, 8, 8>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch3d_tile<double, 8, 8, 8>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
