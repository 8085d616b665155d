// 2-D push/deposit kernels with 16 x 16 tiles fixed at compile time.
#include "push2d_impl.h"

namespace apt {

template hipError_t launch2d_tile<float, 16, 16>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch2d_tile<double, 16, 16>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
