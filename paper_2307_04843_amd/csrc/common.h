// Shared device/host helpers of the HIP path (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AP_HD __host__ __device__ __forceinline__
#define AP_D __device__ __forceinline__

namespace apt {

// Two-lane vector of a scalar type (LDS pairs).
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// Underlying scalar of a number type (the type itself for float and double;
// dual numbers specialise it): constants multiply through it at scalar cost.
template <typename R> struct ScalarOf { using type = R; };

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

// Accumulator of the LDS current tile.  FP64 runs add FP64.  FP32 runs add
// int64 fixed point with a power-of-two scale chosen per block (every
// contribution below 2^50 units, the node sums below 2^62): integer LDS
// atomics run faster than FP64 ones, and the tile's sums are exact and
// independent of the order of the atomics; the quantum is 2^-50 of the
// block's largest |q w| dx/dt, far below FP32 rounding.
template <typename T> struct JTile { using type = double; };
template <> struct JTile<float> { using type = unsigned long long; };

AP_D void lds_add(double *p, double c, double a) { atomic_add(p, c * a); }
AP_D void lds_add(unsigned long long *p, double c, double a) {
    // |c a| < 2^51: adding 1.5 * 2^52 leaves round(c a) in the low mantissa bits
    const double t = fma(c, a, 6755399441055744.0);
    atomicAdd(p, (unsigned long long)(__double_as_longlong(t) - 0x4338000000000000LL));
}
AP_D double lds_value(double v, double) { return v; }
AP_D double lds_value(unsigned long long v, double inv_scale) { return (double)(long long)v * inv_scale; }

// LDS sub-buffer offsets are kept 16-byte aligned.
AP_HD size_t align_lds(size_t bytes) { return (bytes + 15) / 16 * 16; }

template <typename T> AP_D T floor_r(T x);
template <> AP_D float floor_r<float>(float x) { return floorf(x); }
template <> AP_D double floor_r<double>(double x) { return floor(x); }

template <typename T> AP_D T sqrt_r(T x);
template <> AP_D float sqrt_r<float>(float x) { return sqrtf(x); }
template <> AP_D double sqrt_r<double>(double x) { return sqrt(x); }

// FP32: the hardware reciprocal square root, reciprocal and base-2 exponential
// (about 1 ulp); FP64: the correctly rounded library forms.
template <typename T> AP_D T rsqrt_r(T x);
template <> AP_D float rsqrt_r<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> AP_D double rsqrt_r<double>(double x) { return rsqrt(x); }

template <typename T> AP_D T rcp_r(T x);
template <> AP_D float rcp_r<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> AP_D double rcp_r<double>(double x) { return 1.0 / x; }

template <typename T> AP_D T exp_r(T x);
template <> AP_D float exp_r<float>(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
template <> AP_D double exp_r<double>(double x) { return exp(x); }

// sin(pi x), cos(pi x)
template <typename T> AP_D void sincospi_r(T x, T *s, T *c);
// FP32 sin(pi x), cos(pi x) for moderate |x| (here |x| <= ~2): reduce by
// quarter turns q = rint(2x), r = x - q/2 in [-1/4, 1/4] (exact), then the
// Taylor series of sin(pi r) to r^9 and cos(pi r) to r^10 (truncation below
// 1e-9 on the reduced range), then rotate by q quarter turns.
template <> AP_D void sincospi_r<float>(float x, float *s, float *c) {
    const float q = rintf(2.0f * x);
    const float r = fmaf(-0.5f, q, x);
    const float r2 = r * r;
    float ps = 0.08214588661112823f;                  // pi^9/9!
    ps = fmaf(ps, r2, -0.5992645293207921f);          // -pi^7/7!
    ps = fmaf(ps, r2, 2.5501640398773455f);           // pi^5/5!
    ps = fmaf(ps, r2, -5.16771278004997f);            // -pi^3/3!
    ps = fmaf(ps, r2, 3.141592653589793f);            // pi
    const float sr = ps * r;
    float pc = -0.025806891390014062f;                // -pi^10/10!
    pc = fmaf(pc, r2, 0.2353306303588932f);           // pi^8/8!
    pc = fmaf(pc, r2, -1.3352627688545893f);          // -pi^6/6!
    pc = fmaf(pc, r2, 4.058712126416768f);            // pi^4/4!
    pc = fmaf(pc, r2, -4.934802200544679f);           // -pi^2/2!
    const float cr = fmaf(pc, r2, 1.0f);
    const int k = (int)q & 3;
    const float ss = (k & 1) ? cr : sr;
    const float cc = (k & 1) ? sr : cr;
    *s = (k & 2) ? -ss : ss;
    *c = ((k + 1) & 2) ? -cc : cc;
}
template <> AP_D void sincospi_r<double>(double x, double *s, double *c) { sincospi(x, s, c); }

template <typename T> AP_D void sincos_r(T x, T *s, T *c);
template <> AP_D void sincos_r<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <> AP_D void sincos_r<double>(double x, double *s, double *c) { sincos(x, s, c); }

// Block-wide sum of doubles (blockDim.x a multiple of 64, <= 1024).
// Add the number of lanes of the wave with pred set to *counter (one atomic).
AP_D void wave_count(unsigned long long *counter, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m != 0ull && (int)(threadIdx.x & 63) == __ffsll((long long)__ballot(1)) - 1)
        atomicAdd(counter, (unsigned long long)__popcll(m));
}

AP_D double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Emission proxy of one push (Lienard power without its 2 r_e/3 constant):
// gamma^2 [ |E + beta x B|^2 - (beta . E)^2 ] dt with u_bar = (u0 + u1)/2,
// added to a compensated pair (sum, compensation) read from src[0..1] and
// written to dst[0..1].
template <typename T>
AP_D void proxy_accumulate(const T *src, T *dst, const T u0[3], const T u1[3], const T E[3], const T B[3], T dt) {
    const T bx = T(0.5) * (u0[0] + u1[0]), by = T(0.5) * (u0[1] + u1[1]), bz = T(0.5) * (u0[2] + u1[2]);
    const T gb = sqrt_r<T>(T(1) + bx * bx + by * by + bz * bz);
    const T igb = T(1) / gb;
    const T vx = bx * igb, vy = by * igb, vz = bz * igb;
    const T fx = E[0] + (vy * B[2] - vz * B[1]);
    const T fy = E[1] + (vz * B[0] - vx * B[2]);
    const T fz = E[2] + (vx * B[1] - vy * B[0]);
    const T ve = vx * E[0] + vy * E[1] + vz * E[2];
    const T inc = gb * gb * (fx * fx + fy * fy + fz * fz - ve * ve) * dt;
    const T s = src[0];
    T cmp = src[1];
    const T y = inc - cmp;
    const T tsum = s + y;
    cmp = (tsum - s) - y;
    dst[0] = tsum;
    dst[1] = cmp;
}

}  // namespace apt
