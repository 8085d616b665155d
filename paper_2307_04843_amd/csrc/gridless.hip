// Gridless test-particle step: analytic E1, B1 at the particle, relativistic
// Boris push, move, and the optional emission-proxy accumulation.  No grid
// (E2 = B2 = 0), so particles are independent: one thread per particle.
// Positions are per-axis (virtual cell, FP32 offset); the FP64 position
// x_min + (i + off) dx feeds the analytic phase.
#include "current_dev.h"
#include "kernels.h"

namespace apt {

template <typename T, int PT> __global__ __launch_bounds__(256) void k_gridless(GridlessArgs<T> a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    int ic[3];
    T of[3];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ic[c] = a.icell[c][p];
        of[c] = a.off[c][p];
        ok = ok && of[c] >= T(0) && of[c] < T(1);
    }
    T ux = a.u[0][p], uy = a.u[1][p], uz = a.u[2][p];
    ok = ok && finite_state(ux, uy, uz, T(0));
    if (!ok) {
        atomicAdd(a.n_bad, 1ull);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a.icell_out[c][p] = ic[c];
            a.off_out[c][p] = of[c];
        }
        a.u_out[0][p] = ux; a.u_out[1][p] = uy; a.u_out[2][p] = uz;
        return;
    }
    const double X = a.x_min[0] + ((double)ic[0] + (double)of[0]) * a.dx[0];
    const double Y = a.x_min[1] + ((double)ic[1] + (double)of[1]) * a.dx[1];
    const double Z = a.x_min[2] + ((double)ic[2] + (double)of[2]) * a.dx[2];
    T E[3], B[3];
    analytic_field<PT, T>(a.W, X, Y, Z, E, B);

    const T kap = T(0.5 * a.q_over_m * a.dt);
    const T u0x = ux, u0y = uy, u0z = uz;
    const T umx = ux + kap * E[0], umy = uy + kap * E[1], umz = uz + kap * E[2];
    const T ig = rsqrt_r<T>(T(1) + umx * umx + umy * umy + umz * umz);
    const T tx = kap * B[0] * ig, ty = kap * B[1] * ig, tz = kap * B[2] * ig;
    const T sf = T(2) / (T(1) + tx * tx + ty * ty + tz * tz);
    const T upx = umx + (umy * tz - umz * ty);
    const T upy = umy + (umz * tx - umx * tz);
    const T upz = umz + (umx * ty - umy * tx);
    ux = umx + sf * (upy * tz - upz * ty) + kap * E[0];
    uy = umy + sf * (upz * tx - upx * tz) + kap * E[1];
    uz = umz + sf * (upx * ty - upy * tx) + kap * E[2];

    if (a.proxy) {
        const T u0[3] = {u0x, u0y, u0z}, u1[3] = {ux, uy, uz};
        proxy_accumulate<T>(a.proxy + 2 * p, a.proxy + 2 * p, u0, u1, E, B, T(a.dt));
    }

    const T ign = rsqrt_r<T>(T(1) + ux * ux + uy * uy + uz * uz);
    const T uu[3] = {ux, uy, uz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T d = uu[c] * ign * T(a.dt / a.dx[c]);
        T no = of[c] + d;
        const T fl = floor_r<T>(no);
        int sh = (int)fl;
        no -= fl;
        if (no >= T(1)) { no -= T(1); sh += 1; }
        a.icell_out[c][p] = ic[c] + sh;
        a.off_out[c][p] = no;
    }
    a.u_out[0][p] = ux;
    a.u_out[1][p] = uy;
    a.u_out[2][p] = uz;
}

template <typename T, int PT> static hipError_t launch_gl(const GridlessArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_gridless<T, PT>), dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_gridless(int pulse, const GridlessArgs<T> &a, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch_gl<T, PT_NONE>(a, s);
    case PT_PLANE: return launch_gl<T, PT_PLANE>(a, s);
    case PT_GAUSS: return launch_gl<T, PT_GAUSS>(a, s);
    case PT_LG: return launch_gl<T, PT_LG>(a, s);
    case PT_FF: return launch_gl<T, PT_FF>(a, s);
    case PT_NP: return launch_gl<T, PT_NP>(a, s);
    default: return hipErrorInvalidValue;
    }
}
// E1, B1 at arbitrary lab points (internal units), component-major outputs;
// fd_delta != 0: B1 with the finite-duration correction of an analytic current.
template <typename T, int PT>
__global__ __launch_bounds__(256) void k_eval_pulse(PulseVar<T> W, double fd_delta, int64_t n, const double *xyz,
                                                    T *E, T *B) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    T e[3], b[3];
    const double L = 6.283185307179586;   // positions arrive in lambda units
    const double X = xyz[i] * L, Y = xyz[n + i] * L, Z = xyz[2 * n + i] * L;
    if (fd_delta != 0.0) field_fd<PT, T>(W, quadrature_vars(W), T(fd_delta), X, Y, Z, e, b);
    else analytic_field<PT, T>(W, X, Y, Z, e, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        E[c * n + i] = e[c];
        B[c * n + i] = b[c];
    }
}

template <typename T, int PT>
static hipError_t launch_ev(const PulseVar<T> &W, double fd_delta, int64_t n, const double *xyz, T *E, T *B,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_eval_pulse<T, PT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, fd_delta, n,
                       xyz, E, B);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_eval_pulse(int pulse, const PulseVar<T> &W, double fd_delta, int64_t n, const double *xyz, T *E,
                             T *B, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch_ev<T, PT_NONE>(W, 0.0, n, xyz, E, B, s);
    case PT_PLANE: return launch_ev<T, PT_PLANE>(W, fd_delta, n, xyz, E, B, s);
    case PT_GAUSS: return launch_ev<T, PT_GAUSS>(W, fd_delta, n, xyz, E, B, s);
    case PT_LG: return launch_ev<T, PT_LG>(W, fd_delta, n, xyz, E, B, s);
    case PT_FF: return launch_ev<T, PT_FF>(W, fd_delta, n, xyz, E, B, s);
    case PT_NP: return launch_ev<T, PT_NP>(W, 0.0, n, xyz, E, B, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_eval_pulse<float>(int, const PulseVar<float> &, double, int64_t, const double *, float *,
                                             float *, hipStream_t);
template hipError_t launch_eval_pulse<double>(int, const PulseVar<double> &, double, int64_t, const double *,
                                              double *, double *, hipStream_t);

template hipError_t launch_gridless<float>(int, const GridlessArgs<float> &, hipStream_t);
template hipError_t launch_gridless<double>(int, const GridlessArgs<double> &, hipStream_t);

}  // namespace apt
