// E1, B1 sampled on the Yee grid (the literal loop of Fig. 1): every
// component is evaluated at its own staggered node at time t^n and added to
// the internal field, so that the push gathers E1 + E2, B1 + B2 through the
// particle shape.  One thread per cell writes the six sums.  With an
// analytic current (Sec. IV) B1 carries its finite-duration correction, and
// k_analytic_current subtracts J1 at the half step from the deposited J.
// k_boundary_source drives the incoming-wave boundary of open-x rows.
#include <algorithm>

#include "current_dev.h"
#include "kernels.h"

namespace apt {

template <typename T, int PT> __global__ __launch_bounds__(256) void k_sample_pulse(SampleArgs<T> a) {
    const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < ncell; g += (size_t)gridDim.x * blockDim.x) {
        const uint32_t row = a.fnx.div((uint32_t)g);
        const int i = (int)(g - (size_t)row * a.n[0]);
        int j = 0, k = (int)row;
        if (a.dim == 3) {
            k = (int)a.fnxy.div((uint32_t)g);
            j = (int)(row - (uint32_t)k * a.n[1]);
        }
        // node and half-node coordinates per axis (lab, internal units)
        const double xn = a.x_min[0] + (double)win_col(i, a.xo, a.n[0]) * a.dx[0], xh = xn + 0.5 * a.dx[0];
        // 1-D rows: no stagger across rows (every component sits at the row's z)
        const double zn = a.x_min[2] + (double)k * a.dx[2], zh = a.dim == 1 ? zn : zn + 0.5 * a.dx[2];
        const double yn = a.dim == 3 ? a.x_min[1] + (double)j * a.dx[1] : a.q_slice;
        const double yh = a.dim == 3 ? yn + 0.5 * a.dx[1] : a.q_slice;
        T e[3], b[3], out[6];
        const PulseVar<T> Wq = quadrature_vars(a.W);
        const T delta = T(a.fd_delta);
        auto ev = [&](double x, double y, double z) {
            if (a.fd_b) field_fd<PT, T>(a.W, Wq, delta, x, y, z, e, b);
            else analytic_field<PT, T>(a.W, x, y, z, e, b);
        };
        // Ex (h, n, n), Bz (h, h, n): in 2-D both at (xh, zn)
        ev(xh, yn, zn);
        out[0] = e[0];
        if (a.dim < 3) out[5] = b[2];
        // Ey (n, h, n)
        ev(xn, yh, zn);
        out[1] = e[1];
        // Ez (n, n, h), Bx (n, h, h): in 2-D both at (xn, zh)
        ev(xn, yn, zh);
        out[2] = e[2];
        if (a.dim < 3) out[3] = b[0];
        // By (h, n, h)
        ev(xh, yn, zh);
        out[4] = b[1];
        if (a.dim == 3) {
            ev(xn, yh, zh);   // Bx (n, h, h)
            out[3] = b[0];
            ev(xh, yh, zn);   // Bz (h, h, n)
            out[5] = b[2];
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) a.S[c][g] = a.F[c][g] + out[c];
    }
}

template <typename T, int PT> static hipError_t launch_sp(const SampleArgs<T> &a, hipStream_t s) {
    const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
    if (ncell == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((ncell + 255) / 256, 65536);   // grid-stride beyond
    hipLaunchKernelGGL((k_sample_pulse<T, PT>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_sample_pulse(int pulse, const SampleArgs<T> &a, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch_sp<T, PT_NONE>(a, s);
    case PT_PLANE: return launch_sp<T, PT_PLANE>(a, s);
    case PT_GAUSS: return launch_sp<T, PT_GAUSS>(a, s);
    case PT_LG: return launch_sp<T, PT_LG>(a, s);
    case PT_FF: return launch_sp<T, PT_FF>(a, s);
    case PT_NP: return launch_sp<T, PT_NP>(a, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_sample_pulse<float>(int, const SampleArgs<float> &, hipStream_t);
template hipError_t launch_sample_pulse<double>(int, const SampleArgs<double> &, hipStream_t);

// J -= J1(t^{n+1/2}), each component on its E node.  One thread per cell.
template <typename T, int PT> __global__ __launch_bounds__(256) void k_analytic_current(CurrentArgs<T> a) {
    const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
    const PulseVar<T> Wq = quadrature_vars(a.W);
    const T wp2z = T(a.wp2z);
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < ncell; g += (size_t)gridDim.x * blockDim.x) {
        const uint32_t row = a.fnx.div((uint32_t)g);
        const int i = (int)(g - (size_t)row * a.n[0]);
        int j = 0, k = (int)row;
        if (a.dim == 3) {
            k = (int)a.fnxy.div((uint32_t)g);
            j = (int)(row - (uint32_t)k * a.n[1]);
        }
        const double xn = a.x_min[0] + (double)win_col(i, a.xo, a.n[0]) * a.dx[0], xh = xn + 0.5 * a.dx[0];
        // 1-D rows: no stagger across rows (every component sits at the row's z)
        const double zn = a.x_min[2] + (double)k * a.dx[2], zh = a.dim == 1 ? zn : zn + 0.5 * a.dx[2];
        const double yn = a.dim == 3 ? a.x_min[1] + (double)j * a.dx[1] : a.q_slice;
        const double yh = a.dim == 3 ? yn + 0.5 * a.dx[1] : a.q_slice;
        T j1[3];
        current_at<PT, T>(a.W, Wq, wp2z, a.fd, xh, yn, zn, j1);   // Jx (h, n, n)
        a.J[0][g] -= j1[0];
        current_at<PT, T>(a.W, Wq, wp2z, a.fd, xn, yh, zn, j1);   // Jy (n, h, n)
        a.J[1][g] -= j1[1];
        current_at<PT, T>(a.W, Wq, wp2z, a.fd, xn, yn, zh, j1);   // Jz (n, n, h)
        a.J[2][g] -= j1[2];
    }
}

template <typename T, int PT> static hipError_t launch_ac(const CurrentArgs<T> &a, hipStream_t s) {
    const size_t ncell = (size_t)a.n[0] * a.n[1] * a.n[2];
    if (ncell == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((ncell + 255) / 256, 65536);
    hipLaunchKernelGGL((k_analytic_current<T, PT>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_analytic_current(int pulse, const CurrentArgs<T> &a, hipStream_t s) {
    switch (pulse) {
    case PT_PLANE: return launch_ac<T, PT_PLANE>(a, s);
    case PT_GAUSS: return launch_ac<T, PT_GAUSS>(a, s);
    case PT_LG: return launch_ac<T, PT_LG>(a, s);
    case PT_FF: return launch_ac<T, PT_FF>(a, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_analytic_current<float>(int, const CurrentArgs<float> &, hipStream_t);
template hipError_t launch_analytic_current<double>(int, const CurrentArgs<double> &, hipStream_t);

// Incoming-wave boundary source (App. B): one thread per row evaluates the
// pulse at (x_min, row) at the half step; S = (S0/E0) E1_{y,z}.
template <typename T, int PT> __global__ __launch_bounds__(64) void k_boundary_source(BoundaryArgs<T> a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.rows) return;
    T e[3], b[3];
    const int j = r % a.ny, k = r / a.ny;
    const double y = a.ny > 1 ? a.x_min[1] + (double)j * a.dx[1] : a.q_slice;
    analytic_field<PT, T>(a.W, a.x_min[0], y, a.x_min[2] + (double)k * a.dx[2], e, b);
    a.S[2 * r] = T(a.s0) * e[1];
    a.S[2 * r + 1] = T(a.s0) * e[2];
}

template <typename T> hipError_t launch_boundary_source(int pulse, const BoundaryArgs<T> &a, hipStream_t s) {
    if (pulse != PT_PLANE) return hipErrorInvalidValue;   // the S0 amplitude is a plane-wave result
    if (a.rows <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_boundary_source<T, PT_PLANE>), dim3((unsigned)((a.rows + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_boundary_source<float>(int, const BoundaryArgs<float> &, hipStream_t);
template hipError_t launch_boundary_source<double>(int, const BoundaryArgs<double> &, hipStream_t);

}  // namespace apt
