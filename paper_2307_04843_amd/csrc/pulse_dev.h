// Analytic vacuum fields E1, B1 evaluated at a particle (device code).
//
// The laser part of the field split E = E1 + E2, B = B1 + B2 (Eqs. (3)-(4)).
// Every pulse is written as the real part of an analytic signal
//     E_p = Re{ Gamma(eta) U(x, p, q) exp(i Theta) },   B_q = (B0/E0) E_p
// (Eqs. (15), (17) and the separable paraxial beam of Sec. III.A), with
// secondary components from the divergence relations of Sec. III.A:
//     E_x = Re{ -i (v_phi/omega) dU/dp Gamma e^{i Theta} },
//     B_x = Re{ -i (c/omega) (B0/E0) dU/dq Gamma e^{i Theta} }.
//
// The transverse profile uses the complex beam parameter
//     f = 1 / (1 + i s / x_R),   s = x_f - x,
// for which Eq. (21) reads U = f^{(D-1)/2} exp(-f r^2 / w0^2): |f| = w0/w,
// arg f = -atan(s/x_R) (Gouy phase) and Im(-f r^2/w0^2) = k r^2/(2R).
// No atan or explicit w, R are needed, and dU/dp = U (-2 f p / w0^2).
//
// Precision: the carrier phase k.x - omega t reaches 10^3 rad, so it is
// formed in FP64 from the FP64 position x_min + (i + off) dx and reduced to
// [-1/2, 1/2] revolutions before the FP32 sincos; the envelope argument
// eta and the focal offset s are FP64 differences rounded to T afterwards.
#pragma once

#include "common.h"
#include "nonparaxial_gen.h"

namespace apt {

enum PulseType : int32_t { PT_NONE = 0, PT_PLANE = 1, PT_GAUSS = 2, PT_LG = 3, PT_FF = 4, PT_NP = 5 };

constexpr int kNpTerms = 24;   // nonparaxial polynomial table entries per field

// Derived pulse constants, internal units (c = omega = 1).  Built on the
// host in FP64 by ap_set_pulse.
struct PulseDev {
    int32_t type, pol, d_f, lg_l, lg_p, np_order;
    double a0, tau, inv_tau, half_tau;
    double t_ref, x_ref, phi0, b_half;     // chirp: Phi = b_half (eta - tau/2)^2
    double k, inv_vg, v_phi, b_over_e;
    double x_f, inv_xr, inv_w0sq, y_c, z_c, q_slice;
    double beta_f, x0_ff, t0_ff;
    double lg_pref;                        // N (sqrt(2)/w0)^|l|
    double eps;                            // nonparaxial expansion parameter w0/x_R
    double np_e2, np_e4;                   // eps^2, eps^4 weights of the truncated potential
    double w0, x_r, inv_w0;
};

// Generalised Laguerre L_n^a(x) and its derivative (-L_{n-1}^{a+1}).
template <typename T> AP_D void laguerre(int n, int a, T x, T *L, T *dL) {
    T l0 = T(1), l1 = T(1 + a) - x;
    T m0 = T(1), m1 = T(2 + a) - x;   // the a+1 family for the derivative
    if (n == 0) { *L = T(1); *dL = T(0); return; }
    if (n == 1) { *L = l1; *dL = T(-1); return; }
    for (int m = 1; m < n; ++m) {
        T l2 = ((T(2 * m + 1 + a) - x) * l1 - T(m + a) * l0) / T(m + 1);
        l0 = l1; l1 = l2;
    }
    for (int m = 1; m < n - 1; ++m) {
        T m2 = ((T(2 * m + 2 + a) - x) * m1 - T(m + a + 1) * m0) / T(m + 1);
        m0 = m1; m1 = m2;
    }
    *L = l1;
    *dL = (n - 1 == 0) ? T(-1) : -m1;
}

// Field at lab point (X, Y, Z), time t.  Output in lab components.
// Returns false (fields zero) outside the envelope support.
template <int PT, typename T>
AP_D bool analytic_field(const PulseDev &P, double t, double X, double Y, double Z,
                         T E[3], T B[3]) {
    E[0] = E[1] = E[2] = T(0);
    B[0] = B[1] = B[2] = T(0);
    if constexpr (PT == PT_NONE) {
        return false;
    } else {
        // envelope argument: eta = (t - t_ref) - (x - x_ref)/v_g + tau/2  (FP64)
        const double eta = (t - P.t_ref) - (X - P.x_ref) * P.inv_vg + P.half_tau;
        if (!(eta > 0.0 && eta < P.tau)) return false;
        T se, ce;
        sincospi_r<T>(T(eta * P.inv_tau), &se, &ce);
        const T gam = T(P.a0) * se * se;
        // carrier + chirp phase, FP64, reduced to revolutions
        const double de = eta - P.half_tau;
        const double theta = (t - P.t_ref) - P.k * (X - P.x_ref) + P.phi0 + P.b_half * de * de;
        double rev = theta * 0.15915494309189535;   // 1/(2 pi)
        rev -= rint(rev);
        const T ang_pi = T(2.0 * rev);               // Theta / pi in [-1, 1]

        T ep, ex, bx;   // pulse-frame E_p, E_x, B_x; B_q = (B0/E0) E_p
        if constexpr (PT == PT_PLANE) {
            T s, c;
            sincospi_r<T>(ang_pi, &s, &c);
            ep = gam * c;
            ex = T(0);
            bx = T(0);
        } else {
            // pulse-frame transverse coordinates
            T p, q;
            if (P.pol == 0) { p = T(Y - P.y_c); q = T(Z - P.z_c); }
            else            { p = T(Z - P.z_c); q = T(-(Y - P.y_c)); }
            double s_d;
            if constexpr (PT == PT_FF) s_d = P.x0_ff + P.beta_f * (t - P.t0_ff) - X;
            else                       s_d = P.x_f - X;
            const T zeta = T(s_d * P.inv_xr);
            const T den = T(1) / (T(1) + zeta * zeta);          // |f|^2 = (w0/w)^2
            const Cx<T> f(den, -zeta * den);
            const T iw2 = T(P.inv_w0sq);
            T r2, hp, hq;   // r^2 and (1/2) d r^2 / dp, (1/2) d r^2 / dq
            if (PT == PT_LG || PT == PT_NP || P.d_f == 3) { r2 = p * p + q * q; hp = p; hq = q; }
            else if (P.pol == 1)           { r2 = p * p; hp = p; hq = T(0); }
            else                           { r2 = q * q; hp = T(0); hq = q; }
            const T rho2 = r2 * iw2;
            // exp(-f rho2) = exp(-den rho2) * exp(i zeta den rho2)
            const T amp = gam * exp_r<T>(-den * rho2);
            T s, c;
            sincospi_r<T>(ang_pi + zeta * den * rho2 * T(0.3183098861837907), &s, &c);
            Cx<T> V(amp * c, amp * s);                   // Gamma exp(-f rho2) e^{i Theta}
            if constexpr (PT == PT_NP) {
                // Gaussian beam beyond the paraxial approximation: fields derived
                // exactly from the eps^4-truncated vector potential (conjugated
                // polynomials from nonparaxial_gen.h; explicit i's conjugated here).
                const NpPoly<T> Q = np_polys<T>(f, rho2, T(1), T(P.np_e2), T(P.np_e4));
                const T eps = T(P.eps), e2 = eps * eps;
                const T xi = p * T(P.inv_w0), et = q * T(P.inv_w0);
                V = f * V;                                   // conj(psi0) Gamma e^{i Theta}
                const Cx<T> yEp = Q.G + (T(0.25) * e2) * (T(2) * Q.H + (T(4) * xi * xi) * Q.K);
                const Cx<T> yEq = (e2 * xi * et) * Q.K;
                const Cx<T> yEx = xi * (Cx<T>(T(0), -eps) * Q.H + (T(0.5) * e2 * eps) * Q.N);
                const Cx<T> yBq = Q.G + Cx<T>(T(0), T(0.5) * e2) * Q.M;
                const Cx<T> yBx = Cx<T>(T(0), -eps * et) * Q.H;
                ep = (yEp * V).re;
                ex = (yEx * V).re;
                bx = (yBx * V).re;
                const T eq = (yEq * V).re;
                const T bq = (yBq * V).re;
                E[0] = ex;
                B[0] = bx;
                if (P.pol == 0) { E[1] = ep; E[2] = eq; B[2] = bq; }      // p = y, q = z
                else            { E[2] = ep; E[1] = -eq; B[1] = -bq; }    // p = z, q = -y
                return true;
            } else if constexpr (PT == PT_LG) {
                const int la = P.lg_l >= 0 ? P.lg_l : -P.lg_l;
                const T sig = P.lg_l >= 0 ? T(1) : T(-1);
                // f^{|l|+1} (f / conj f)^{p}
                Cx<T> fp = f;
                for (int m = 0; m < la; ++m) fp = fp * f;
                if (P.lg_p > 0) {
                    const Cx<T> ratio = (T(1) / den) * (f * f);
                    for (int m = 0; m < P.lg_p; ++m) fp = fp * ratio;
                }
                V = T(P.lg_pref) * (fp * V);
                const Cx<T> pq(p, sig * q);
                Cx<T> pw(T(1), T(0)), pwm1(T(1), T(0));
                for (int m = 0; m < la; ++m) { pwm1 = pw; pw = pw * pq; }
                T Lg, dLg;
                laguerre<T>(P.lg_p, la, T(2) * rho2 * den, &Lg, &dLg);
                const T la_t = T(la);
                // U/V-factor A = pq^|l| L; dA/dp and dA/dq including the Gaussian factor
                const Cx<T> A = Lg * pw;
                const Cx<T> g2p = (T(-2) * iw2 * p) * f;   // d/dp of (-f r^2/w0^2)
                const Cx<T> g2q = (T(-2) * iw2 * q) * f;
                const T lp = T(4) * p * den * iw2 * dLg;
                const T lq = T(4) * q * den * iw2 * dLg;
                const Cx<T> Ap = (la_t * Lg) * pwm1 + lp * pw + g2p * A;
                const Cx<T> Aq = Cx<T>(T(0), sig * la_t * Lg) * pwm1 + lq * pw + g2q * A;
                const Cx<T> eV = A * V, pV = Ap * V, qV = Aq * V;
                ep = eV.re;
                ex = T(P.v_phi) * pV.im;            // Re{-i z} = Im z
                bx = T(P.b_over_e) * qV.im;
            } else {
                Cx<T> fV;
                if (P.d_f == 3) {
                    V = f * V;
                } else {
                    // principal sqrt(f) for Re f > 0, in the form without cancellation
                    // near focus: sr = sqrt((|f| + Re f)/2), si = Im f / (2 sr)
                    const T mod = sqrt_r<T>(den);      // |f| = sqrt(den)
                    const T sr = sqrt_r<T>(T(0.5) * (mod + f.re));
                    const T si = f.im / (T(2) * sr);
                    V = Cx<T>(sr, si) * V;
                }
                fV = f * V;
                ep = V.re;
                ex = T(P.v_phi) * (T(-2) * iw2 * hp) * fV.im;
                bx = T(P.b_over_e) * (T(-2) * iw2 * hq) * fV.im;
            }
        }
        const T bq = T(P.b_over_e) * ep;
        E[0] = ex;
        B[0] = bx;
        if (P.pol == 0) { E[1] = ep; B[2] = bq; }          // p = y, q = z
        else            { E[2] = ep; B[1] = -bq; }         // p = z, q = -y
        return true;
    }
}

}  // namespace apt
