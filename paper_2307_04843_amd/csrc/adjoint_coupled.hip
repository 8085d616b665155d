// Launchers of the reverse step in the fully coupled reading of gridded runs
// (the deposit and the gather differentiated too; see adjoint_impl.h).  A
// translation unit of its own, so that its kernel variants compile in
// parallel with the others.
#include "adjoint_impl.h"

namespace apt {

template <typename T, int PT, int GD> static void launch_cpl_gd(const AdjointArgs<T> &a, int np, hipStream_t s) {
    const int per_block = 256 * (GD >= 2 ? kAdjPpt : 1);
    const dim3 grid((a.n + per_block - 1) / per_block), block(256);
    const bool px = a.lam_proxy != nullptr;
    if constexpr (GD == 1) {
        if (np <= 2) {
            if (px) hipLaunchKernelGGL((k_adjoint_step<PT, 5, GD, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_adjoint_step<PT, 5, GD, false, true>), grid, block, 0, s, a);
        } else {
            if (px) hipLaunchKernelGGL((k_adjoint_step<PT, 7, GD, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_adjoint_step<PT, 7, GD, false, true>), grid, block, 0, s, a);
        }
    } else {
        // 2-D and 3-D: the current's adjoint (LDS copy of the grid adjoint it
        // reads), the rest, then the gather's adjoint (LDS accumulation)
        const size_t shj = (size_t)adj_lds_j<GD>() * sizeof(double);
        const int cap = a.scatter_cap > 0 ? a.scatter_cap : adj_lds_scatter<GD>();
        const size_t shs = (size_t)cap * sizeof(double);
        hipLaunchKernelGGL((k_adjoint_current<PT, GD, T>), grid, block, shj, s, a);
        if constexpr (GD == 3) {
            if (np <= 2) {
                if (px) hipLaunchKernelGGL((k_adjoint_step_rest3<PT, 5, true, T>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_adjoint_step_rest3<PT, 5, false, T>), grid, block, 0, s, a);
            } else {
                if (px) hipLaunchKernelGGL((k_adjoint_step_rest3<PT, 7, true, T>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_adjoint_step_rest3<PT, 7, false, T>), grid, block, 0, s, a);
            }
        } else if (np <= 2) {
            if (px) hipLaunchKernelGGL((k_adjoint_step_rest<PT, 5, GD, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_adjoint_step_rest<PT, 5, GD, false>), grid, block, 0, s, a);
        } else {
            if (px) hipLaunchKernelGGL((k_adjoint_step_rest<PT, 7, GD, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_adjoint_step_rest<PT, 7, GD, false>), grid, block, 0, s, a);
        }
        const dim3 grid3(a.tile_start ? (unsigned)a.ntile : (unsigned)((a.n + 255) / 256));
        hipLaunchKernelGGL((k_adjoint_gather_scatter<GD>), grid3, block, shs, s, a);
    }
}

template <typename T, int PT> static hipError_t launch_cpl(const AdjointArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    int np = 0;
    for (int k = 0; k < 4; ++k) np += a.slot[k] >= 0 ? 1 : 0;
    switch (a.dim) {
    case 1: launch_cpl_gd<T, PT, 1>(a, np, s); break;
    case 2: launch_cpl_gd<T, PT, 2>(a, np, s); break;
    case 3: launch_cpl_gd<T, PT, 3>(a, np, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T> hipError_t launch_adjoint_step_coupled(int pulse, const AdjointArgs<T> &a, hipStream_t s) {
    switch (pulse) {
    case PT_PLANE: return launch_cpl<T, PT_PLANE>(a, s);
    case PT_GAUSS: return launch_cpl<T, PT_GAUSS>(a, s);
    case PT_LG: return launch_cpl<T, PT_LG>(a, s);
    case PT_FF: return launch_cpl<T, PT_FF>(a, s);
    case PT_NP: return launch_cpl<T, PT_NP>(a, s);
    default: return hipErrorInvalidValue;
    }
}
int adjoint_scatter_lds_entries(int dim) { return dim == 3 ? adj_lds_scatter<3>() : adj_lds_scatter<2>(); }

template hipError_t launch_adjoint_step_coupled<float>(int, const AdjointArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_step_coupled<double>(int, const AdjointArgs<double> &, hipStream_t);

}  // namespace apt
