// Analytic current J1 and the finite-duration correction of B1 (Sec. IV).
//
// With an analytic current the pulse is a wave of the plasma-filled Yee grid:
// E1 keeps the form Re{G Gamma e^{i(Theta + Phi)}}, J1 is the linear response
// dJ1/dt = omega_p^2 zeta E1, and B1 follows from Faraday's law.  Integrating
// over a finite-duration envelope multiplies the analytic signal by
//     C = A e^{i psi},
//     A   = 1 - delta Gamma''/Gamma + (delta Gamma'/Gamma)^2 / 2 - delta Phi' + delta Phi'^2,
//     psi = delta Gamma'/Gamma - delta Phi'' - 2 delta (Gamma'/Gamma) Phi'
// (omega = 1; ' = d/dt at fixed x), the lowest-order terms of the series:
// delta = 1 - v_phi/v_g for B1, delta = 1 for J1.  So
//     B1 = Re{C S_B},   J1 = wp2 zeta Re{-i C S_E},
// with S the analytic signals whose real parts the vacuum evaluation
// returns.  Their imaginary parts are the same evaluation a quarter period
// earlier in carrier phase (Re{S e^{-i pi/2}} = Im S), so the generic
// analytic_field code serves both without change.
#pragma once

#include "pulse_dev.h"

namespace apt {

// Gamma'/Gamma, Gamma''/Gamma, Phi', Phi'' at lab x (false outside the support).
template <typename T>
AP_D bool envelope_rates(const PulseVar<T> &W, double X, T &g1, T &g2, T &p1, T &p2) {
    const double eta = W.eta0 - X * W.inv_vg;
    if (!(eta > 0.0 && eta < W.tau)) return false;
    if (W.envelope == 1) {
        const T x = T((eta - W.half_tau) * W.inv_tau_g);
        const T itg = T(W.inv_tau_g);
        const int g = W.sg_order;
        T pw = T(1);                       // x^(2g-2)
        for (int m = 1; m < g; ++m) pw = pw * x * x;
        g1 = T(-2 * g) * pw * x * itg;
        g2 = g1 * g1 - T(2 * g * (2 * g - 1)) * pw * itg * itg;
    } else {
        T s, c;
        sincospi_r(T(eta * W.inv_tau), &s, &c);
        const T a = T(3.141592653589793 * W.inv_tau);
        const T is = T(1) / s;
        g1 = T(2) * a * c * is;
        g2 = T(2) * a * a * (c * c - s * s) * is * is;
    }
    const T b = T(2.0 * W.b_half);
    p1 = b * T(eta - W.half_tau);
    p2 = b;
    return true;
}

// C = A e^{i psi} of the lowest-order finite-duration terms for factor delta.
template <typename T> AP_D void fd_factor(T g1, T g2, T p1, T p2, T delta, T &cr, T &ci) {
    const T amp = T(1) - delta * g2 + T(0.5) * (delta * g1) * (delta * g1) - delta * p1 + delta * p1 * p1;
    const T psi = delta * g1 - delta * p2 - T(2) * delta * g1 * p1;
    T s, c;
    sincospi_r(psi * T(0.3183098861837907), &s, &c);
    cr = amp * c;
    ci = amp * s;
}

// The step's constants a quarter period earlier in carrier phase.
template <typename T> AP_D PulseVar<T> quadrature_vars(const PulseVar<T> &W) {
    PulseVar<T> Q = W;
    Q.th0 -= 1.5707963267948966;
    return Q;
}

// E1, B1 at a point with B1's finite-duration correction (delta = 1 - v_phi/v_g).
template <int PT, typename T>
AP_D void field_fd(const PulseVar<T> &W, const PulseVar<T> &Wq, T delta, double X, double Y, double Z, T E[3],
                   T B[3]) {
    if (!analytic_field<PT, T>(W, X, Y, Z, E, B)) return;
    T eq[3], bq[3], g1, g2, p1, p2, cr, ci;
    analytic_field<PT, T>(Wq, X, Y, Z, eq, bq);
    envelope_rates(W, X, g1, g2, p1, p2);
    fd_factor(g1, g2, p1, p2, delta, cr, ci);
#pragma unroll
    for (int c = 0; c < 3; ++c) B[c] = cr * B[c] - ci * bq[c];
}

// J1 at a point (W, Wq: constants of the half step t^{n+1/2}).
template <int PT, typename T>
AP_D void current_at(const PulseVar<T> &W, const PulseVar<T> &Wq, T wp2z, int fd, double X, double Y, double Z,
                     T J[3]) {
    T e0[3], b0[3], eq[3], bq[3];
    J[0] = J[1] = J[2] = T(0);
    if (!analytic_field<PT, T>(W, X, Y, Z, e0, b0)) return;
    analytic_field<PT, T>(Wq, X, Y, Z, eq, bq);
    T cr = T(1), ci = T(0);
    if (fd) {
        T g1, g2, p1, p2;
        envelope_rates(W, X, g1, g2, p1, p2);
        fd_factor(g1, g2, p1, p2, T(1), cr, ci);
    }
    // Re{-i C S} = Im{C S} = Re C Im S + Im C Re S
#pragma unroll
    for (int c = 0; c < 3; ++c) J[c] = wp2z * (cr * eq[c] + ci * e0[c]);
}

}  // namespace apt
