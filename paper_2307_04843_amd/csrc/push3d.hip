// Launcher of the fused 3-D push/deposit kernel (push3d_impl.h): dispatch on
// the tile shape, whose kernels are compiled in their own translation units.
#include "kernels.h"

namespace apt {

template <typename T, int TX, int TY, int TZ>
hipError_t launch3d_tile(int pulse, const PushArgs<T> &a, int threads, hipStream_t s);

template <typename T> hipError_t launch_push_deposit_3d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    if (a.tile[0] == 8 && a.tile[1] == 4 && a.tile[2] == 4) return launch3d_tile<T, 8, 4, 4>(pulse, a, threads, s);
    if (a.tile[0] == 8 && a.tile[1] == 8 && a.tile[2] == 4) return launch3d_tile<T, 8, 8, 4>(pulse, a, threads, s);
    if (a.tile[0] == 8 && a.tile[1] == 8 && a.tile[2] == 8) return launch3d_tile<T, 8, 8, 8>(pulse, a, threads, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_push_deposit_3d<float>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch_push_deposit_3d<double>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
