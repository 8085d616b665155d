// Forward-mode dual numbers for the adjoint kernels.
//
// Dual<T, N>  : value and N tangents of type T (the kernel's arithmetic type).
// DualD<T, N> : FP64 value with T tangents, for the FP64 island quantities
//               (positions, carrier phase, envelope argument, focal offset):
//               their values need FP64, their derivatives do not.
#pragma once

#include "common.h"

namespace apt {

template <typename T, int N> struct Dual {
    using scalar = T;
    T v;
    T d[N];
    AP_HD Dual() : v(T(0)) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
    AP_HD Dual(double x) : v(T(x)) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
    AP_HD Dual(float x) : v(T(x)) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
    AP_HD Dual(int x) : v(T(x)) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
    AP_HD static Dual var(T x, int slot) {
        Dual r(x);
        r.d[slot] = T(1);
        return r;
    }
};

template <typename T, int N> struct DualD {
    double v;
    T d[N];
    AP_HD DualD() : v(0.0) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
    AP_HD DualD(double x) : v(x) {
        for (int i = 0; i < N; ++i) d[i] = T(0);
    }
};

// ---- Dual arithmetic
#define AP_DUAL_T template <typename T, int N>
AP_DUAL_T AP_HD Dual<T, N> operator+(const Dual<T, N> &a, const Dual<T, N> &b) {
    Dual<T, N> r; r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
AP_DUAL_T AP_HD Dual<T, N> operator-(const Dual<T, N> &a, const Dual<T, N> &b) {
    Dual<T, N> r; r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
AP_DUAL_T AP_HD Dual<T, N> operator-(const Dual<T, N> &a) {
    Dual<T, N> r; r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
AP_DUAL_T AP_HD Dual<T, N> operator*(const Dual<T, N> &a, const Dual<T, N> &b) {
    Dual<T, N> r; r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
AP_DUAL_T AP_HD Dual<T, N> operator/(const Dual<T, N> &a, const Dual<T, N> &b) {
    Dual<T, N> r;
    const T ib = T(1) / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
// scalar (non-deduced) times dual: no product rule work on a constant
AP_DUAL_T AP_HD Dual<T, N> operator*(typename Dual<T, N>::scalar s, const Dual<T, N> &a) {
    Dual<T, N> r; r.v = s * a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i];
    return r;
}
AP_DUAL_T AP_HD Dual<T, N> operator*(const Dual<T, N> &a, typename Dual<T, N>::scalar s) { return s * a; }
AP_DUAL_T AP_HD Dual<T, N> &operator+=(Dual<T, N> &a, const Dual<T, N> &b) { a = a + b; return a; }
AP_DUAL_T AP_HD Dual<T, N> &operator-=(Dual<T, N> &a, const Dual<T, N> &b) { a = a - b; return a; }
AP_DUAL_T AP_HD bool operator>=(const Dual<T, N> &a, const Dual<T, N> &b) { return a.v >= b.v; }
AP_DUAL_T AP_HD bool operator<(const Dual<T, N> &a, const Dual<T, N> &b) { return a.v < b.v; }

template <typename T, int N> AP_D Dual<T, N> sqrt_r(Dual<T, N> a) {
    Dual<T, N> r; r.v = sqrt_r<T>(a.v);
    const T h = T(0.5) / r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
    return r;
}
template <typename T, int N> AP_D Dual<T, N> rsqrt_r(Dual<T, N> a) {
    Dual<T, N> r; r.v = rsqrt_r<T>(a.v);
    const T h = T(-0.5) * r.v * r.v * r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
    return r;
}
template <typename T, int N> AP_D Dual<T, N> rcp_r(Dual<T, N> a) {
    Dual<T, N> r; r.v = rcp_r<T>(a.v);
    const T h = -r.v * r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
    return r;
}
template <typename T, int N> AP_D Dual<T, N> exp_r(Dual<T, N> a) {
    Dual<T, N> r; r.v = exp_r<T>(a.v);
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * r.v;
    return r;
}
template <typename T, int N> AP_D void sincospi_r(Dual<T, N> a, Dual<T, N> *s, Dual<T, N> *c) {
    T sv, cv;
    sincospi_r<T>(a.v, &sv, &cv);
    s->v = sv; c->v = cv;
    const T pi = T(3.141592653589793);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        s->d[i] = pi * cv * a.d[i];
        c->d[i] = -pi * sv * a.d[i];
    }
}

template <typename T, int N> struct ScalarOf<Dual<T, N>> { using type = T; };

// ---- FP64-island helpers
AP_DUAL_T AP_HD DualD<T, N> operator+(const DualD<T, N> &a, const DualD<T, N> &b) {
    DualD<T, N> r; r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
AP_DUAL_T AP_HD DualD<T, N> operator-(const DualD<T, N> &a, const DualD<T, N> &b) {
    DualD<T, N> r; r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
AP_DUAL_T AP_HD DualD<T, N> operator*(const DualD<T, N> &a, const DualD<T, N> &b) {
    DualD<T, N> r; r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * T(b.v) + T(a.v) * b.d[i];
    return r;
}

// ---- type maps used by the generic pulse code
// island value, rounding to the working type, and constants
template <typename R> struct NumTraits;
template <> struct NumTraits<float> {
    using island = double;
    AP_HD static float from_island(double x) { return float(x); }
    AP_HD static double island_value(double x) { return x; }
};
template <> struct NumTraits<double> {
    using island = double;
    AP_HD static double from_island(double x) { return x; }
    AP_HD static double island_value(double x) { return x; }
};
template <typename T, int N> struct NumTraits<Dual<T, N>> {
    using island = DualD<T, N>;
    AP_HD static Dual<T, N> from_island(const DualD<T, N> &x) {
        Dual<T, N> r; r.v = T(x.v);
#pragma unroll
        for (int i = 0; i < N; ++i) r.d[i] = x.d[i];
        return r;
    }
    AP_HD static double island_value(const DualD<T, N> &x) { return x.v; }
};

// value part of a (possibly dual) number
AP_HD float val(float x) { return x; }
AP_HD double val(double x) { return x; }
template <typename T, int N> AP_HD T val(const Dual<T, N> &x) { return x.v; }
AP_HD double ival(double x) { return x; }
template <typename T, int N> AP_HD double ival(const DualD<T, N> &x) { return x.v; }

// subtract a constant from an island quantity (derivative unchanged)
AP_HD double island_shift(double x, double c) { return x - c; }
template <typename T, int N> AP_HD DualD<T, N> island_shift(DualD<T, N> x, double c) { x.v -= c; return x; }
AP_HD double island_scale(double x, double c) { return x * c; }
template <typename T, int N> AP_HD DualD<T, N> island_scale(DualD<T, N> x, double c) {
    x.v *= c;
#pragma unroll
    for (int i = 0; i < N; ++i) x.d[i] = x.d[i] * T(c);
    return x;
}

}  // namespace apt
