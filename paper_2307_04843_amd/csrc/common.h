// Shared device/host helpers of the HIP path (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AP_HD __host__ __device__ __forceinline__
#define AP_D __device__ __forceinline__

namespace apt {

constexpr int kMaxSpecies = 4;
constexpr int kWave = 64;

// Unsigned division by a run-time constant d >= 1 for dividends < 2^31
// (Granlund-Montgomery "round-up" method with the add fix-up):
//   q = (umulhi(n, m) + n) >> s,  s = ceil(log2 d),  m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
    FastDiv() : d(1), m(1), s(0) {}
    explicit FastDiv(uint32_t d_) : d(d_) {
        uint32_t sh = 0;
        while ((1ull << sh) < d_) ++sh;
        s = sh;
        uint64_t two_s = 1ull << sh;
        m = (uint32_t)(((two_s - d_) << 32) / d_ + 1);
        if (d_ == 1) { m = 0; s = 0; }
    }
    AP_HD uint32_t div(uint32_t n) const {
#if defined(__HIP_DEVICE_COMPILE__)
        uint32_t hi = __umulhi(n, m);
#else
        uint32_t hi = (uint32_t)(((uint64_t)n * m) >> 32);
#endif
        return (hi + n) >> s;
    }
    AP_HD uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

template <typename T> struct Cx {
    T re, im;
    AP_HD Cx() : re(0), im(0) {}
    AP_HD Cx(T r, T i) : re(r), im(i) {}
};
template <typename T> AP_HD Cx<T> operator+(Cx<T> a, Cx<T> b) { return Cx<T>(a.re + b.re, a.im + b.im); }
template <typename T> AP_HD Cx<T> operator-(Cx<T> a, Cx<T> b) { return Cx<T>(a.re - b.re, a.im - b.im); }
template <typename T> AP_HD Cx<T> operator*(Cx<T> a, Cx<T> b) {
    return Cx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> AP_HD Cx<T> operator*(T s, Cx<T> a) { return Cx<T>(s * a.re, s * a.im); }

// Atomic add into LDS or coarse-grained global memory (hipMalloc / torch
// allocations) for float and double: the hardware float atomics, not a CAS loop.
AP_D void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
AP_D void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// LDS sub-buffer offsets are kept 16-byte aligned.
AP_HD size_t align_lds(size_t bytes) { return (bytes + 15) / 16 * 16; }

template <typename T> AP_D T floor_r(T x);
template <> AP_D float floor_r<float>(float x) { return floorf(x); }
template <> AP_D double floor_r<double>(double x) { return floor(x); }

template <typename T> AP_D T sqrt_r(T x);
template <> AP_D float sqrt_r<float>(float x) { return sqrtf(x); }
template <> AP_D double sqrt_r<double>(double x) { return sqrt(x); }

template <typename T> AP_D T rsqrt_r(T x);
template <> AP_D float rsqrt_r<float>(float x) { return rsqrtf(x); }
template <> AP_D double rsqrt_r<double>(double x) { return rsqrt(x); }

template <typename T> AP_D T exp_r(T x);
template <> AP_D float exp_r<float>(float x) { return expf(x); }
template <> AP_D double exp_r<double>(double x) { return exp(x); }

// sin(pi x), cos(pi x)
template <typename T> AP_D void sincospi_r(T x, T *s, T *c);
template <> AP_D void sincospi_r<float>(float x, float *s, float *c) { sincospif(x, s, c); }
template <> AP_D void sincospi_r<double>(double x, double *s, double *c) { sincospi(x, s, c); }

template <typename T> AP_D void sincos_r(T x, T *s, T *c);
template <> AP_D void sincos_r<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <> AP_D void sincos_r<double>(double x, double *s, double *c) { sincos(x, s, c); }

// Block-wide sum of doubles (blockDim.x a multiple of 64, <= 1024).
AP_D double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace apt
