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
#include "dual.h"
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
    int32_t envelope, sg_order;            // AP_ENV_*, super-Gaussian order g
    double inv_tau_g;                      // 1/tau_g of the super-Gaussian
    int32_t sampling;                      // AP_SAMPLE_* (host sequencing only)
    int32_t current, fd;                   // analytic current J1 on; finite-duration terms kept
    double wp2z;                           // omega_p^2 zeta / omega of J1
    double fd_delta;                       // 1 - v_phi / v_g (B1's finite-duration factor)
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

// Pulse constants of one time step.  R is the working number type (float,
// double or a dual number); I the matching FP64-island type.  The host builds
// the plain version per step in FP64 (so the kernels hold few live scalars);
// the adjoint builds a dual version with tangents on the parameters.
//     eta   = eta0 - X / v_g                      (envelope argument)
//     theta = th0 - k X + b_half (eta - tau/2)^2  (carrier + chirp phase)
//     s     = s0 - X                              (distance to focus)
template <typename R> struct PulseVar {
    using I = typename NumTraits<R>::island;
    double eta0, inv_vg, th0, k;
    double tau, inv_tau, half_tau;
    double y_c, z_c;
    I s0, b_half;
    R a0, inv_xr, inv_w0sq, inv_w0, eps, np_e2, np_e4, lg_pref, v_phi, b_over_e;
    int32_t pol, d_f, lg_l, lg_p;
    int32_t envelope, sg_order;
    double inv_tau_g;
};

template <typename R> AP_HD void fill_step_constants(const PulseDev &P, double t, PulseVar<R> &V) {
    V.eta0 = (t - P.t_ref) + P.half_tau + P.x_ref * P.inv_vg;
    V.inv_vg = P.inv_vg;
    V.th0 = (t - P.t_ref) + P.phi0 + P.k * P.x_ref;
    V.k = P.k;
    V.tau = P.tau;
    V.inv_tau = P.inv_tau;
    V.half_tau = P.half_tau;
    V.y_c = P.y_c;
    V.z_c = P.z_c;
    V.pol = P.pol;
    V.d_f = P.d_f;
    V.lg_l = P.lg_l;
    V.lg_p = P.lg_p;
    V.envelope = P.envelope;
    V.sg_order = P.sg_order;
    V.inv_tau_g = P.inv_tau_g;
}

// Plain constants of the step at time t (host or device).
template <typename R> AP_HD PulseVar<R> plain_vars(const PulseDev &P, double t) {
    PulseVar<R> V;
    fill_step_constants(P, t, V);
    V.s0 = P.type == PT_FF ? P.x0_ff + P.beta_f * (t - P.t0_ff) : P.x_f;
    V.b_half = P.b_half;
    V.a0 = R(P.a0);
    V.inv_xr = R(P.inv_xr);
    V.inv_w0sq = R(P.inv_w0sq);
    V.inv_w0 = R(P.inv_w0);
    V.eps = R(P.eps);
    V.np_e2 = R(P.np_e2);
    V.np_e4 = R(P.np_e4);
    V.lg_pref = R(P.lg_pref);
    V.v_phi = R(P.v_phi);
    V.b_over_e = R(P.b_over_e);
    return V;
}

// Field at lab point (X, Y, Z) (FP64 island numbers), time t.  Output in lab
// components.  Returns false (fields zero) outside the envelope support.
template <int PT, typename R, typename I>
AP_D bool analytic_field_g(const PulseVar<R> &W, const I &X, const I &Y, const I &Z, R E[3], R B[3]) {
    using NT = NumTraits<R>;
    E[0] = E[1] = E[2] = R(0.0);
    B[0] = B[1] = B[2] = R(0.0);
    if constexpr (PT == PT_NONE) {
        return false;
    } else {
        // envelope argument eta = eta0 - X/v_g (FP64 island)
        const I eta = island_shift(island_scale(X, -W.inv_vg), -W.eta0);
        const double eta_v = ival(eta);
        if (!(eta_v > 0.0 && eta_v < W.tau)) return false;
        R gam;
        if (W.envelope == 1) {
            // super-Gaussian exp(-x^(2g)), x = (eta - tau/2) / tau_g
            const R xg = NT::from_island(island_scale(island_shift(eta, W.half_tau), W.inv_tau_g));
            const R x2 = xg * xg;
            R pw = x2;
            for (int m = 1; m < W.sg_order; ++m) pw = pw * x2;
            gam = W.a0 * exp_r(-pw);
        } else {
            R se, ce;
            sincospi_r(NT::from_island(island_scale(eta, W.inv_tau)), &se, &ce);
            gam = W.a0 * se * se;
        }
        // carrier + chirp phase, FP64, reduced to revolutions
        const I de = island_shift(eta, W.half_tau);
        const I theta = island_shift(island_scale(X, -W.k), -W.th0) + W.b_half * de * de;
        I rev = island_scale(theta, 0.15915494309189535);   // 1/(2 pi)
        rev = island_shift(rev, rint(ival(rev)));
        const R ang_pi = NT::from_island(island_scale(rev, 2.0));   // Theta / pi in [-1, 1]

        R ep, ex, bx;   // pulse-frame E_p, E_x, B_x; B_q = (B0/E0) E_p
        if constexpr (PT == PT_PLANE) {
            R s, c;
            sincospi_r(ang_pi, &s, &c);
            ep = gam * c;
            ex = R(0.0);
            bx = R(0.0);
        } else {
            // pulse-frame transverse coordinates
            // (both offsets first, then a per-value select: selecting between the
            // Y and Z operands themselves would make the compiler address them
            // through scratch memory in the dual-number instantiations)
            const R dy = NT::from_island(island_shift(Y, W.y_c));
            const R dz = NT::from_island(island_shift(Z, W.z_c));
            const bool pol0 = W.pol == 0;
            const R p = pol0 ? dy : dz;
            const R q = pol0 ? dz : -dy;
            const I s_d = W.s0 - X;
            const R zeta = NT::from_island(s_d) * W.inv_xr;
            const R den = rcp_r(R(1.0) + zeta * zeta);          // |f|^2 = (w0/w)^2
            const Cx<R> f(den, -zeta * den);
            const R iw2 = W.inv_w0sq;
            R r2, hp, hq;   // r^2 and (1/2) d r^2 / dp, (1/2) d r^2 / dq
            if (PT == PT_LG || PT == PT_NP || W.d_f == 3) { r2 = p * p + q * q; hp = p; hq = q; }
            else if (W.pol == 1)                          { r2 = p * p; hp = p; hq = R(0.0); }
            else                                          { r2 = q * q; hp = R(0.0); hq = q; }
            const R rho2 = r2 * iw2;
            // exp(-f rho2) = exp(-den rho2) * exp(i zeta den rho2)
            const R amp = gam * exp_r(-(den * rho2));
            R s, c;
            sincospi_r(ang_pi + zeta * den * rho2 * R(0.3183098861837907), &s, &c);
            Cx<R> V(amp * c, amp * s);                   // Gamma exp(-f rho2) e^{i Theta}
            if constexpr (PT == PT_NP) {
                // Gaussian beam beyond the paraxial approximation: fields derived
                // exactly from the eps^4-truncated vector potential (conjugated
                // polynomials from nonparaxial_gen.h; explicit i's conjugated here).
                const NpPoly<R> Q = np_polys<R>(f, rho2, W.np_e2, W.np_e4);
                const R eps = W.eps, e2 = eps * eps;
                const R xi = p * W.inv_w0, et = q * W.inv_w0;
                V = f * V;                                   // conj(psi0) Gamma e^{i Theta}
                const Cx<R> yEp = Q.G + (R(0.25) * e2) * (R(2.0) * Q.H + (R(4.0) * xi * xi) * Q.K);
                const Cx<R> yEq = (e2 * xi * et) * Q.K;
                const Cx<R> yEx = xi * (Cx<R>(R(0.0), -eps) * Q.H + (R(0.5) * e2 * eps) * Q.N);
                const Cx<R> yBq = Q.G + Cx<R>(R(0.0), R(0.5) * e2) * Q.M;
                const Cx<R> yBx = Cx<R>(R(0.0), -(eps * et)) * Q.H;
                ep = (yEp * V).re;
                ex = (yEx * V).re;
                bx = (yBx * V).re;
                const R eq = (yEq * V).re;
                const R bq = (yBq * V).re;
                E[0] = ex;
                B[0] = bx;
                if (W.pol == 0) { E[1] = ep; E[2] = eq; B[2] = bq; }      // p = y, q = z
                else            { E[2] = ep; E[1] = -eq; B[1] = -bq; }    // p = z, q = -y
                return true;
            } else if constexpr (PT == PT_LG) {
                const int la = W.lg_l >= 0 ? W.lg_l : -W.lg_l;
                const R sig = W.lg_l >= 0 ? R(1.0) : R(-1.0);
                // f^{|l|+1} (f / conj f)^{p}
                Cx<R> fp = f;
                for (int m = 0; m < la; ++m) fp = fp * f;
                if (W.lg_p > 0) {
                    const Cx<R> ratio = rcp_r(den) * (f * f);
                    for (int m = 0; m < W.lg_p; ++m) fp = fp * ratio;
                }
                V = W.lg_pref * (fp * V);
                const Cx<R> pq(p, sig * q);
                Cx<R> pw(R(1.0), R(0.0)), pwm1(R(1.0), R(0.0));
                for (int m = 0; m < la; ++m) { pwm1 = pw; pw = pw * pq; }
                R Lg, dLg;
                laguerre<R>(W.lg_p, la, R(2.0) * rho2 * den, &Lg, &dLg);
                const R la_t = R(double(la));
                // U/V-factor A = pq^|l| L; dA/dp and dA/dq including the Gaussian factor
                const Cx<R> A = Lg * pw;
                const Cx<R> g2p = (R(-2.0) * iw2 * p) * f;   // d/dp of (-f r^2/w0^2)
                const Cx<R> g2q = (R(-2.0) * iw2 * q) * f;
                const R lp = R(4.0) * p * den * iw2 * dLg;
                const R lq = R(4.0) * q * den * iw2 * dLg;
                const Cx<R> Ap = (la_t * Lg) * pwm1 + lp * pw + g2p * A;
                const Cx<R> Aq = Cx<R>(R(0.0), sig * la_t * Lg) * pwm1 + lq * pw + g2q * A;
                const Cx<R> eV = A * V, pV = Ap * V, qV = Aq * V;
                ep = eV.re;
                ex = W.v_phi * pV.im;            // Re{-i z} = Im z
                bx = W.b_over_e * qV.im;
            } else {
                if (W.d_f == 3) {
                    V = f * V;
                } else {
                    // principal sqrt(f) for Re f > 0, in the form without cancellation
                    // near focus: sr = sqrt((|f| + Re f)/2), si = Im f / (2 sr)
                    const R mod = sqrt_r(den);      // |f| = sqrt(den)
                    const R sr = sqrt_r(R(0.5) * (mod + f.re));
                    const R si = R(0.5) * f.im * rcp_r(sr);
                    V = Cx<R>(sr, si) * V;
                }
                const Cx<R> fV = f * V;
                ep = V.re;
                ex = W.v_phi * (R(-2.0) * iw2 * hp) * fV.im;
                bx = W.b_over_e * (R(-2.0) * iw2 * hq) * fV.im;
            }
        }
        const R bq = W.b_over_e * ep;
        E[0] = ex;
        B[0] = bx;
        if (W.pol == 0) { E[1] = ep; B[2] = bq; }          // p = y, q = z
        else            { E[2] = ep; B[1] = -bq; }         // p = z, q = -y
        return true;
    }
}

// Plain (non-differentiated) evaluation used by the forward kernels.
template <int PT, typename T>
AP_D bool analytic_field(const PulseVar<T> &W, double X, double Y, double Z, T E[3], T B[3]) {
    return analytic_field_g<PT, T, double>(W, X, Y, Z, E, B);
}

}  // namespace apt
