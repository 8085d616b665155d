// Launchers of the reverse step (gridless runs and the frozen-grid reading of
// gridded runs; the fully coupled variants are in adjoint_coupled.hip), the
// adjoint-state initialisation and the particle-id check.
#include "adjoint_impl.h"

namespace apt {

template <typename T, int PT, int GD> static void launch_adj_gd(const AdjointArgs<T> &a, int np, hipStream_t s) {
    const dim3 grid((a.n + 255) / 256), block(256);
    // parameter tangents padded to 2 or 4 (unused slots are -1 and stay zero)
    const bool px = a.lam_proxy != nullptr;
    if (np <= 2) {
        if (px) hipLaunchKernelGGL((k_adjoint_step<PT, 5, GD, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_step<PT, 5, GD, false, false>), grid, block, 0, s, a);
    } else {
        if (px) hipLaunchKernelGGL((k_adjoint_step<PT, 7, GD, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_adjoint_step<PT, 7, GD, false, false>), grid, block, 0, s, a);
    }
}

template <typename T, int PT> static hipError_t launch_adj(const AdjointArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    int np = 0;
    for (int k = 0; k < 4; ++k) np += a.slot[k] >= 0 ? 1 : 0;
    switch (a.dim) {
    case 0: launch_adj_gd<T, PT, 0>(a, np, s); break;
    case 1: launch_adj_gd<T, PT, 1>(a, np, s); break;
    case 2: launch_adj_gd<T, PT, 2>(a, np, s); break;
    case 3: launch_adj_gd<T, PT, 3>(a, np, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T> hipError_t launch_adjoint_step(int pulse, const AdjointArgs<T> &a, hipStream_t s) {
    if (a.lJ[0]) return launch_adjoint_step_coupled<T>(pulse, a, s);
    switch (pulse) {
    case PT_PLANE: return launch_adj<T, PT_PLANE>(a, s);
    case PT_GAUSS: return launch_adj<T, PT_GAUSS>(a, s);
    case PT_LG: return launch_adj<T, PT_LG>(a, s);
    case PT_FF: return launch_adj<T, PT_FF>(a, s);
    case PT_NP: return launch_adj<T, PT_NP>(a, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_adjoint_step<float>(int, const AdjointArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_step<double>(int, const AdjointArgs<double> &, hipStream_t);

// lam[0..2] = 0, lam[3..5] = dL/du (as FP64), partial = 0
template <typename T>
__global__ void k_adjoint_init(double *lam0, double *lam1, double *lam2, double *lam3, double *lam4, double *lam5,
                               const T *dl_du, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    lam0[p] = 0.0;
    lam1[p] = 0.0;
    lam2[p] = 0.0;
    lam3[p] = (double)dl_du[p];
    lam4[p] = (double)dl_du[n + p];
    lam5[p] = (double)dl_du[2 * n + p];
}
template <typename T> hipError_t launch_adjoint_init(double *const lam[6], const T *dl_du, int n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_adjoint_init<T>), dim3((n + 255) / 256), dim3(256), 0, s, lam[0], lam[1], lam[2], lam[3],
                       lam[4], lam[5], dl_du, n);
    return hipGetLastError();
}
template hipError_t launch_adjoint_init<float>(double *const[6], const float *, int, hipStream_t);

__global__ void k_check_ids(const int32_t *id, int n, int32_t *seen, unsigned long long *bad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int v = id[p];
    bool b = v < 0 || v >= n;
    if (!b) b = atomicAdd(&seen[v], 1) != 0;
    if (b) atomicAdd(bad, 1ull);
}
hipError_t launch_check_ids(const int32_t *id, int n, int32_t *seen, unsigned long long *bad, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_ids, dim3((n + 255) / 256), dim3(256), 0, s, id, n, seen, bad);
    return hipGetLastError();
}
template hipError_t launch_adjoint_init<double>(double *const[6], const double *, int, hipStream_t);

}  // namespace apt
