// Launcher of the fused 2-D push/deposit kernel (push2d_impl.h): dispatch on
// the tile shape.  The common shapes run kernels with the shape fixed at
// compile time (their own translation units); any other shape runs the
// kernel that reads it at run time.
#include "push2d_impl.h"

namespace apt {

template <typename T, int CTX, int CTZ>
hipError_t launch2d_tile(int pulse, const PushArgs<T> &a, int threads, hipStream_t s);

template <typename T> hipError_t launch_push_deposit_2d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    if (a.tile[0] == 16 && a.tile[2] == 8) return launch2d_tile<T, 16, 8>(pulse, a, threads, s);
    if (a.tile[0] == 32 && a.tile[2] == 8) return launch2d_tile<T, 32, 8>(pulse, a, threads, s);
    if (a.tile[0] == 16 && a.tile[2] == 16) return launch2d_tile<T, 16, 16>(pulse, a, threads, s);
    return launch2d_tile<T, 0, 0>(pulse, a, threads, s);
}

template hipError_t launch2d_tile<float, 0, 0>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch2d_tile<double, 0, 0>(int, const PushArgs<double> &, int, hipStream_t);
template hipError_t launch_push_deposit_2d<float>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch_push_deposit_2d<double>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
