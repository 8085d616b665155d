// Adjoint of the gridless step (analytic field + Boris push + move + emission
// proxy) for gradients of particle observables with respect to the pulse
// parameters.  The same reverse step serves gridded runs in the frozen-grid
// reading: the E2, B2 each push gathered are a recorded external field, so
// E = E1(x; theta) + gather(E2)(x) and dE/dx gains the gradient of the
// quadratic-shape gather; the adjoint state is indexed by particle id, since
// re-sorts permute the particle arrays between steps.
//
// Forward step n (per particle):  E, B = field(x^n, t^n; theta)
//     u^{n+1/2} = Boris(u^{n-1/2}, E, B),   x^{n+1} = x^n + dt u^{n+1/2}/gamma,
//     proxy += P(u^{n-1/2}, u^{n+1/2}, E, B).
// Reverse step n, with lx = dL/dx^{n+1}, lu = dL/du^{n+1/2}, lp = dL/dproxy:
//     lu1 = lu + dt (lx - v (v . lx))/gamma + lp dP/du1
//     lu0 = J_u^T lu1 + lp dP/du0,  lE = J_E^T lu1 + lp dP/dE,  lB = J_B^T lu1 + lp dP/dB
//     lx <- lx + (dE/dx)^T lE + (dB/dx)^T lB,   g_theta += (dE/dtheta)^T lE + (dB/dtheta)^T lB
//     lu <- lu0.
// The field Jacobians come from forward-mode dual numbers through the same
// generic pulse code the forward kernels use, with NT tangents: x, y, z and
// one per requested parameter among w0, focal position, beta_f and chirp.
// The amplitude needs no tangent: every pulse field is proportional to a0,
// so dF/da0 = F / a0 (evaluated at a0 = 1 when a0 = 0).  9 tangents run
// through the Boris rotation and 12 through the proxy.  Adjoint state and
// gradient partials are FP64.
//
// Fully coupled reading of gridded runs (CPL): the particles also drive E2,
// B2 through their current J(x^n, x^{n+1}, u^{n+1/2}), and the gather reads
// E2^n, B2^n.  With lJ = dL/dJ^{n+1/2} on the E nodes (from the reverse Yee
// step, outside this kernel), each particle adds
//     lx^{n+1} += (dJ/dx^{n+1})^T lJ,   lx^n += (dJ/dx^n)^T lJ,
//     lu1 += (dv/du1)^T (dJ/dv)^T lJ   (out-of-plane components only),
// and scatters its field adjoint back through the gather weights,
//     lE2^n[node] += S(node) lE,   lB2^n[node] += S(node) lB.
#pragma once
#include "kernels.h"

namespace apt {

// Tangent k >= 3 carries parameter slot[k - 3]: set it to dv where that is `param`.
template <int NT, typename T> AP_D void seed_tangent(T (&d)[NT], const int32_t (&slot)[4], int param, double dv) {
#pragma unroll
    for (int k = 0; k < NT - 3; ++k)
        if (slot[k] == param) d[3 + k] = T(dv);
}

// Per-step pulse variables as duals; the amplitude is a0_eff (a0, or 1 when
// a0 = 0), without a tangent.
template <typename T, int NT>
AP_D PulseVar<Dual<T, NT>> adjoint_vars(const PulseDev &P, double t, const int32_t (&slot)[4], double a0_eff) {
    using DN = Dual<T, NT>;
    using IN = DualD<T, NT>;
    PulseVar<DN> V;
    fill_step_constants(P, t, V);
    V.a0 = DN(T(a0_eff));
    const double w0 = P.w0 > 0.0 ? P.w0 : 1.0;
    auto wd = [&](double v, double dv) {
        DN r(v);
        seed_tangent(r.d, slot, 1, dv);
        return r;
    };
    V.inv_xr = wd(P.inv_xr, -2.0 * P.inv_xr / w0);
    if (P.type == PT_FF) seed_tangent(V.inv_xr.d, slot, 3, P.inv_xr / (1.0 - P.beta_f));
    V.inv_w0sq = wd(P.inv_w0sq, -2.0 * P.inv_w0sq / w0);
    V.inv_w0 = wd(P.inv_w0, -P.inv_w0 / w0);
    V.eps = wd(P.eps, -P.eps / w0);
    V.np_e2 = wd(P.np_e2, -2.0 * P.np_e2 / w0);
    V.np_e4 = wd(P.np_e4, -4.0 * P.np_e4 / w0);
    const int la = P.lg_l < 0 ? -P.lg_l : P.lg_l;
    V.lg_pref = wd(P.lg_pref, -la * P.lg_pref / w0);
    V.v_phi = DN(P.v_phi);
    V.b_over_e = DN(P.b_over_e);
    // s0 = x_f, or x0_ff + beta_f (t - t0_ff) for the flying focus
    IN s0(P.type == PT_FF ? P.x0_ff + P.beta_f * (t - P.t0_ff) : P.x_f);
    seed_tangent(s0.d, slot, 2, 1.0);
    if (P.type == PT_FF) seed_tangent(s0.d, slot, 3, t - P.t0_ff);
    V.s0 = s0;
    IN bh(P.b_half);
    seed_tangent(bh.d, slot, 4, 0.5 / P.tau);
    V.b_half = bh;
    return V;
}

template <typename R>
AP_D void boris_g(const R u0[3], const R E[3], const R B[3], R kap, R u1[3]) {
    const R umx = u0[0] + kap * E[0], umy = u0[1] + kap * E[1], umz = u0[2] + kap * E[2];
    const R ig = rsqrt_r(R(1.0) + umx * umx + umy * umy + umz * umz);
    const R tx = kap * B[0] * ig, ty = kap * B[1] * ig, tz = kap * B[2] * ig;
    const R sf = R(2.0) / (R(1.0) + tx * tx + ty * ty + tz * tz);
    const R upx = umx + (umy * tz - umz * ty);
    const R upy = umy + (umz * tx - umx * tz);
    const R upz = umz + (umx * ty - umy * tx);
    u1[0] = umx + sf * (upy * tz - upz * ty) + kap * E[0];
    u1[1] = umy + sf * (upz * tx - upx * tz) + kap * E[1];
    u1[2] = umz + sf * (upx * ty - upy * tx) + kap * E[2];
}

template <typename R>
AP_D R proxy_g(const R u0[3], const R u1[3], const R E[3], const R B[3], R dt) {
    const R bx = R(0.5) * (u0[0] + u1[0]), by = R(0.5) * (u0[1] + u1[1]), bz = R(0.5) * (u0[2] + u1[2]);
    const R gb = sqrt_r(R(1.0) + bx * bx + by * by + bz * bz);
    const R igb = R(1.0) / gb;
    const R vx = bx * igb, vy = by * igb, vz = bz * igb;
    const R fx = E[0] + (vy * B[2] - vz * B[1]);
    const R fy = E[1] + (vz * B[0] - vx * B[2]);
    const R fz = E[2] + (vx * B[1] - vy * B[0]);
    const R ve = vx * E[0] + vy * E[1] + vz * E[2];
    return gb * gb * (fx * fx + fy * fy + fz * fz - ve * ve) * dt;
}

// Quadratic B-spline weights of nodes -1, 0, +1 at offset d and their d-derivatives.
template <typename T> AP_D void tsc3_d(T d, T w[3], T dw[3]) {
    const T lo = T(0.5) - d, hi = T(0.5) + d;
    w[0] = T(0.5) * lo * lo;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * hi * hi;
    dw[0] = -lo;
    dw[1] = T(-2) * d;
    dw[2] = hi;
}

// Three-node stencil of one axis for a component on nodes or half a cell up.
template <typename T> struct AxisStencil {
    int idx[3];
    T w[3], dw[3];
};
template <typename T> AP_D void axis_stencil(int i, T off, bool half, int n, AxisStencil<T> &st) {
    int c;
    T d;
    if (half) {
        c = i;
        d = off - T(0.5);
    } else {
        const int up = off >= T(0.5) ? 1 : 0;
        c = i + up;
        d = off - T(up);
    }
    tsc3_d(d, st.w, st.dw);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int v = c - 1 + m;
        st.idx[m] = v < 0 ? v + n : (v >= n ? v - n : v);
    }
}

// Gathered value and its gradient in cell units (x, y, z; y only in 3-D).
template <typename T, int GD>
AP_D void gather_grad(const T *F, const AxisStencil<T> &sx, const AxisStencil<T> &sy, const AxisStencil<T> &sz,
                      int nx, int ny, T &v, T (&gr)[3]) {
    v = T(0);
    gr[0] = gr[1] = gr[2] = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T pv = T(0), px = T(0), py = T(0);
#pragma unroll
        for (int q = 0; q < (GD == 3 ? 3 : 1); ++q) {
            const T *row = F + ((size_t)sz.idx[b] * ny + (GD == 3 ? sy.idx[q] : 0)) * nx;
            T r = T(0), rd = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const T f = row[sx.idx[m]];
                r += sx.w[m] * f;
                rd += sx.dw[m] * f;
            }
            const T wy = GD == 3 ? sy.w[q] : T(1);
            pv += wy * r;
            px += wy * rd;
            if (GD == 3) py += sy.dw[q] * r;
        }
        v += sz.w[b] * pv;
        gr[0] += sz.w[b] * px;
        gr[1] += sz.w[b] * py;
        gr[2] += sz.dw[b] * pv;
    }
}

// Quadratic B-spline of a node at distance d (cell units) and its d-derivative.
template <typename T> AP_D void tsc_vd(T d, T &v, T &dv) {
    const T ad = fabs(d);
    if (ad <= T(0.5)) {
        v = T(0.75) - d * d;
        dv = T(-2) * d;
    } else if (ad <= T(1.5)) {
        const T e = T(1.5) - ad;
        v = T(0.5) * e * e;
        dv = d > T(0) ? -e : e;
    } else {
        v = T(0);
        dv = T(0);
    }
}

AP_D __forceinline__ int wrap_idx(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Adjoint of one particle's charge-conserving current.  The current is that
// of the forward deposit: per active axis A, J_A(m + 1/2) = -q w (dx_A/dt)
// sum_{m' <= m} W_A(m') with W_A the shape-change weights, and the current
// along an axis without motion is q w v S_avg.  With lJ = -dt lE~ (lE~ the
// E adjoint after the first half of the reverse Yee step, read from lE_t)
//     G = sum over the 5-node window of lJ . J
// is differentiated in x^n, x^{n+1} (cell units, forward-mode tangents) and
// in v (out-of-plane components).  ov: offsets at x^n; dl: the step's
// displacement in cells; returns the cell-unit gradients and dG/dv.
// Readers of the grid adjoint lE~ at unwrapped node coordinates: from global
// memory (periodic wrap), or from a block's LDS copy of the box it needs.
struct AdjGlobalRd {
    const double *const *F;
    int n[3];
    AP_D double operator()(int c, int x, int y, int z) const {
        return F[c][((size_t)wrap_idx(z, n[2]) * n[1] + wrap_idx(y, n[1])) * n[0] + wrap_idx(x, n[0])];
    }
};
struct AdjLdsRd {
    const double *L;
    int lo[3], ext[3];
    AP_D double operator()(int c, int x, int y, int z) const {
        return L[(((size_t)c * ext[2] + (z - lo[2])) * ext[1] + (y - lo[1])) * ext[0] + (x - lo[0])];
    }
};

template <typename T, int GD, class RD>
AP_D void deposit_adjoint(const RD &rd, const int32_t n[3], const int ic[3], const T ov[3],
                          const T dl[3], const T v[3], double qw, double dt, const double dx[3], double gx0[3],
                          double gx1[3], double gv[3]) {
    constexpr int NA = GD == 3 ? 3 : (GD == 2 ? 2 : 1);
    const int ax[3] = {0, GD == 3 ? 1 : 2, 2};
    // per active slot: window start (node c - 2, unwrapped) and the positions
    // before / after the step relative to the window centre c
    T x0[NA], x1[NA];
    int cb[NA];
#pragma unroll
    for (int s = 0; s < NA; ++s) {
        const int A = ax[s];
        const int up = ov[A] >= T(0.5) ? 1 : 0;
        cb[s] = ic[A] + up - 2;
        x0[s] = ov[A] - T(up);
        x1[s] = x0[s] + dl[A];
    }
    (void)n;
    // shapes of window node m (0..4) on slot s, and their derivatives in x0, x1
    auto shp = [&](int s, int m, T &a0, T &d0, T &a1, T &d1) {
        tsc_vd(x0[s] - T(m - 2), a0, d0);
        tsc_vd(x1[s] - T(m - 2), a1, d1);
    };
    const double T3 = 1.0 / 3.0, T6 = 1.0 / 6.0;
    if constexpr (GD == 1) {
        // a row: J_x from the x shapes; y and z carry q w v times the mean shape
        double suf = 0.0, g0 = 0.0, g1 = 0.0, sy = 0.0, sz = 0.0, y0 = 0.0, y1 = 0.0, z0 = 0.0, z1 = 0.0;
#pragma unroll
        for (int m = 4; m >= 0; --m) {
            T a0, d0, a1, d1;
            shp(0, m, a0, d0, a1, d1);
            const double lx = rd(0, cb[0] + m, 0, ic[2]), ly = rd(1, cb[0] + m, 0, ic[2]);
            const double lz = rd(2, cb[0] + m, 0, ic[2]);
            suf += lx;
            g0 -= (double)d0 * suf;
            g1 += (double)d1 * suf;
            const double mean = 0.5 * ((double)a0 + (double)a1);
            sy += mean * ly;
            sz += mean * lz;
            y0 += 0.5 * (double)d0 * ly;
            y1 += 0.5 * (double)d1 * ly;
            z0 += 0.5 * (double)d0 * lz;
            z1 += 0.5 * (double)d1 * lz;
        }
        const double cj = qw * dx[0], cy = -dt * qw;
        gx0[0] = cj * g0 + cy * ((double)v[1] * y0 + (double)v[2] * z0);
        gx1[0] = cj * g1 + cy * ((double)v[1] * y1 + (double)v[2] * z1);
        gv[1] = cy * sy;
        gv[2] = cy * sz;
    } else if constexpr (GD == 2) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};   // d/d(x0, z0, x1, z1)
        const double cx = qw * dx[0], cz = qw * dx[2], cy = -dt * qw * (double)v[1];
        double sy = 0.0;
        // J_x: per z node, suffix sums of lE~_x along x
#pragma unroll 1
        for (int k = 0; k < 5; ++k) {
            T za0, zd0, za1, zd1;
            shp(1, k, za0, zd0, za1, zd1);
            double suf = 0.0, av = 0.0, a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int m = 4; m >= 0; --m) {
                T xa0, xd0, xa1, xd1;
                shp(0, m, xa0, xd0, xa1, xd1);
                suf += rd(0, cb[0] + m, 0, cb[1] + k);
                av += (double)(xa1 - xa0) * suf;
                a0 -= (double)xd0 * suf;
                a1 += (double)xd1 * suf;
            }
            const double zm = 0.5 * ((double)za0 + (double)za1);
            g[0] += cx * zm * a0;
            g[2] += cx * zm * a1;
            g[1] += cx * 0.5 * (double)zd0 * av;
            g[3] += cx * 0.5 * (double)zd1 * av;
        }
        // J_z: per x node, suffix sums along z; J_y: q w v_y times the mean shape product
#pragma unroll 1
        for (int m = 0; m < 5; ++m) {
            T xa0, xd0, xa1, xd1;
            shp(0, m, xa0, xd0, xa1, xd1);
            double suf = 0.0, av = 0.0, a0 = 0.0, a1 = 0.0;
            double p0 = 0.0, p1 = 0.0, r0 = 0.0, r1 = 0.0;   // sums over z for J_y
#pragma unroll
            for (int k = 4; k >= 0; --k) {
                T za0, zd0, za1, zd1;
                shp(1, k, za0, zd0, za1, zd1);
                suf += rd(2, cb[0] + m, 0, cb[1] + k);
                av += (double)(za1 - za0) * suf;
                a0 -= (double)zd0 * suf;
                a1 += (double)zd1 * suf;
                const double ly = rd(1, cb[0] + m, 0, cb[1] + k);
                p0 += ly * (T3 * (double)za0 + T6 * (double)za1);   // pairs with X0
                p1 += ly * (T6 * (double)za0 + T3 * (double)za1);   // pairs with X1
                r0 += ly * (double)zd0;
                r1 += ly * (double)zd1;
            }
            const double xm = 0.5 * ((double)xa0 + (double)xa1);
            g[1] += cz * xm * a0;
            g[3] += cz * xm * a1;
            g[0] += cz * 0.5 * (double)xd0 * av;
            g[2] += cz * 0.5 * (double)xd1 * av;
            sy += (double)xa0 * p0 + (double)xa1 * p1;
            g[0] += cy * (double)xd0 * p0;
            g[2] += cy * (double)xd1 * p1;
            g[1] += cy * r0 * (T3 * (double)xa0 + T6 * (double)xa1);
            g[3] += cy * r1 * (T6 * (double)xa0 + T3 * (double)xa1);
        }
        gx0[0] = g[0];
        gx0[2] = g[1];
        gx1[0] = g[2];
        gx1[2] = g[3];
        gv[1] = -dt * qw * sy;
    } else {
        // 3-D: W_A = DS_A tr(P, Q), tr = 1/3 (P0 Q0 + P1 Q1) + 1/6 (P1 Q0 + P0 Q1) over the
        // other two axes; per (b, c) the suffix-weighted sum along A carries the
        // two A tangents, tr the four others
        double gd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int s1 = s == 0 ? 1 : 0, s2 = s == 2 ? 1 : 2;   // the two other axes
            const double coef = qw * dx[s];
#pragma unroll 1
            for (int b = 0; b < 5; ++b) {
                T p0, dp0, p1, dp1;
                shp(s1, b, p0, dp0, p1, dp1);
                const int i1 = cb[s1] + b;
#pragma unroll 1
                for (int c = 0; c < 5; ++c) {
                    T q0, dq0, q1, dq1;
                    shp(s2, c, q0, dq0, q1, dq1);
                    const double tr = T3 * ((double)p0 * q0 + (double)p1 * q1) + T6 * ((double)p1 * q0 + (double)p0 * q1);
                    int id3[3];
                    id3[s1] = i1;
                    id3[s2] = cb[s2] + c;
                    double suf = 0.0, av = 0.0, a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int m = 4; m >= 0; --m) {
                        T sa0, sd0, sa1, sd1;
                        shp(s, m, sa0, sd0, sa1, sd1);
                        id3[s] = cb[s] + m;
                        suf += rd(s, id3[0], id3[1], id3[2]);
                        av += (double)(sa1 - sa0) * suf;
                        a0 -= (double)sd0 * suf;
                        a1 += (double)sd1 * suf;
                    }
                    gd[s] += coef * tr * a0;
                    gd[3 + s] += coef * tr * a1;
                    gd[s1] += coef * av * (double)dp0 * (T3 * (double)q0 + T6 * (double)q1);
                    gd[3 + s1] += coef * av * (double)dp1 * (T3 * (double)q1 + T6 * (double)q0);
                    gd[s2] += coef * av * (double)dq0 * (T3 * (double)p0 + T6 * (double)p1);
                    gd[3 + s2] += coef * av * (double)dq1 * (T3 * (double)p1 + T6 * (double)p0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            gx0[k] = gd[k];
            gx1[k] = gd[3 + k];
        }
    }
}

// The gather's adjoint: val spread to the nodes of the stencil with the
// gather's weights (FP64 atomics).
template <typename T, int GD>
AP_D void scatter_adjoint(double *F, const AxisStencil<T> &sx, const AxisStencil<T> &sy, const AxisStencil<T> &sz,
                          int nx, int ny, double val) {
#pragma unroll
    for (int b = 0; b < (GD == 1 ? 1 : 3); ++b) {
#pragma unroll
        for (int q = 0; q < (GD == 3 ? 3 : 1); ++q) {
            const double wzy = (double)sz.w[b] * (GD == 3 ? (double)sy.w[q] : 1.0) * val;
            double *row = F + ((size_t)sz.idx[b] * ny + (GD == 3 ? sy.idx[q] : 0)) * nx;
#pragma unroll
            for (int m = 0; m < 3; ++m) atomicAdd(row + sx.idx[m], (double)sx.w[m] * wzy);
        }
    }
}

// LDS staging of the gather's adjoint (coupled 2-D/3-D): a block's particles
// are nearly tile-sorted, so their stencils cover a small box of nodes; the
// block accumulates there and flushes each node once.
// LDS of a coupled block, in doubles: the gather's adjoint (six components)
// and the grid adjoint lE~ the current's adjoint reads (three components)
template <int GD> constexpr int adj_lds_scatter() { return GD == 3 ? 8192 : 3072; }
template <int GD> constexpr int adj_lds_j() { return GD == 3 ? 6144 : 3072; }
constexpr int kAdjPpt = 1;             // particles per thread in those blocks (4 measured slower)
struct AdjRegion {
    int lo[3], ext[3], n[3];
    AP_D int local(int ax, int idx) const {
        int l = idx - lo[ax];
        if (l < 0) l += n[ax];
        else if (l >= n[ax]) l -= n[ax];
        return l;
    }
};
// LDS accumulator L: FP64, or int64 fixed point with scale `scale` (lds_add).
template <typename T, int GD, typename JA>
AP_D void scatter_adjoint_lds(JA *L, int comp, const AdjRegion &R, const AxisStencil<T> &sx,
                              const AxisStencil<T> &sy, const AxisStencil<T> &sz, double val, double scale = 1.0) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int q = 0; q < (GD == 3 ? 3 : 1); ++q) {
            const double wzy = (double)sz.w[b] * (GD == 3 ? (double)sy.w[q] : 1.0) * val;
            const int l2 = R.local(2, sz.idx[b]), l1 = GD == 3 ? R.local(1, sy.idx[q]) : 0;
            JA *row = L + (((size_t)comp * R.ext[2] + l2) * R.ext[1] + l1) * R.ext[0];
#pragma unroll
            for (int m = 0; m < 3; ++m) lds_add(row + R.local(0, sx.idx[m]), (double)sx.w[m] * wzy, scale);
        }
    }
}

template <typename T, int GD> AP_D void grid_stencils(const int ic[3], const T ov[3], const int32_t n[3],
                                                     AxisStencil<T> sn[3], AxisStencil<T> sh[3]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (GD <= 2 && ax == 1) continue;
        if (GD == 1 && ax == 2) {
            // 1-D rows: the particle's own row, weight one, no gradient
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                sn[2].idx[m] = ic[2];
                sn[2].w[m] = T(m == 0 ? 1 : 0);
                sn[2].dw[m] = T(0);
            }
            sh[2] = sn[2];
            continue;
        }
        axis_stencil(ic[ax], ov[ax], false, n[ax], sn[ax]);
        axis_stencil(ic[ax], ov[ax], true, n[ax], sh[ax]);
    }
}

// PASS (coupled reading): 0 = the whole reverse step; 1 = the current's
// adjoint only (a value-only forward pass, then d/dx^{n+1} and the
// out-of-plane d/dv folded into the particle's adjoint state, d/dx^n kept in
// a.gx0[0..3)); 2 = the rest but the gather's adjoint, reading d/dx^n and
// leaving the adjoints of the gathered E, B in a.gx0[0..6); the gather's
// adjoint is then k_adjoint_gather_scatter.  The passes split the working
// set of one fused kernel (and its two LDS boxes) over three launches.
template <typename T, int PT, int NT, int GD, bool PX, bool CPL, int PASS = 0>
AP_D __forceinline__ void adjoint_step_body(const AdjointArgs<T> &a) {
    static_assert(PASS == 0 || (CPL && GD > 0), "the passes split the coupled reverse step");
    // particles per thread: the coupled 2-D/3-D blocks take a tile's worth, so
    // that their LDS region is flushed once for more particles
    constexpr int PPT = (CPL && GD >= 2) ? kAdjPpt : 1;
    const int base = blockIdx.x * blockDim.x * PPT + threadIdx.x;
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    auto load = [&](int p, int &lid, bool &ok, int ic[3], T ov[3]) {
        lid = p;          // index of the particle's adjoint state
        ok = p < a.n;
        ic[0] = ic[1] = ic[2] = 0;
        ov[0] = ov[1] = ov[2] = T(0);
        if (GD > 0 && ok) {
            // grid state: linear cell + offsets on the active axes; particles the
            // push skipped (invalid cell or offset) keep their adjoint state
            const int cell = a.G.cell[p];
            lid = a.G.id[p];
            ov[0] = a.off[0][p];
            if (GD >= 2) ov[2] = a.off[2][p];
            if (GD == 3) ov[1] = a.off[1][p];
            const int nx = a.G.n[0], nxy = a.G.n[0] * a.G.n[1];
            ok = (unsigned)cell < (unsigned)nxy * (unsigned)a.G.n[2] && ov[0] >= T(0) && ov[0] < T(1) &&
                 ov[1] >= T(0) && ov[1] < T(1) && ov[2] >= T(0) && ov[2] < T(1) && (unsigned)lid < (unsigned)a.n;
            const int k = (int)a.G.fnxy.div((unsigned)cell);
            const int r = cell - k * nxy;
            const int j = (int)a.G.fnx.div((unsigned)r);
            ic[0] = r - j * nx;
            ic[1] = j;
            ic[2] = k;
        }
    };
    // coupled 2-D/3-D: the block's bounding box of cells fixes its LDS region
    AdjRegion R{};
    AdjLdsRd JR{};
    bool use_lds = false, use_ldsj = false;
    int vol = 0;
    double *lds_adj = nullptr;
    if constexpr (CPL && GD >= 2 && PASS != 2) {
        extern __shared__ double adj_dyn[];
        lds_adj = adj_dyn;
        __shared__ int bbox[6];
        if (threadIdx.x < 3) {
            bbox[threadIdx.x] = 0x7fffffff;
            bbox[3 + threadIdx.x] = -0x7fffffff;
        }
        __syncthreads();
        for (int kk = 0; kk < PPT; ++kk) {
            int lid, ic[3];
            bool ok;
            T ov[3];
            load(base + kk * (int)blockDim.x, lid, ok, ic, ov);
            if (ok) {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    atomicMin(&bbox[ax], ic[ax]);
                    atomicMax(&bbox[3 + ax], ic[ax]);
                }
            }
        }
        __syncthreads();
        bool fits = true;
        vol = 6;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            R.n[ax] = a.G.n[ax];
            if (GD == 2 && ax == 1) {
                R.lo[1] = 0;
                R.ext[1] = 1;
                continue;
            }
            // stencil nodes reach one below the lowest cell and two above the highest
            R.lo[ax] = bbox[ax] - 1;
            R.ext[ax] = bbox[3 + ax] - bbox[ax] + 4;
            fits = fits && bbox[ax] <= bbox[3 + ax] && R.ext[ax] <= R.n[ax];
            vol *= R.ext[ax];
        }
        use_lds = PASS != 1 && fits && vol <= adj_lds_scatter<GD>();
        if (use_lds)
            for (int i = threadIdx.x; i < vol; i += blockDim.x) lds_adj[i] = 0.0;
        // the current's window reaches two nodes below the lowest cell and three above the highest
        constexpr int joff = PASS == 1 ? 0 : adj_lds_scatter<GD>();
        JR.L = lds_adj + joff;
        int volj = 3;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (GD == 2 && ax == 1) {
                JR.lo[1] = 0;
                JR.ext[1] = 1;
                continue;
            }
            JR.lo[ax] = bbox[ax] - 2;
            JR.ext[ax] = bbox[3 + ax] - bbox[ax] + 6;
            volj *= JR.ext[ax];
        }
        use_ldsj = PASS != 2 && bbox[0] <= bbox[3] && volj <= adj_lds_j<GD>();
        if (use_ldsj) {
            double *L = lds_adj + joff;
            const int per = JR.ext[0] * JR.ext[1] * JR.ext[2];
            for (int i = threadIdx.x; i < volj; i += blockDim.x) {
                const int comp = i / per;
                int r = i - comp * per;
                const int l2 = r / (JR.ext[0] * JR.ext[1]);
                r -= l2 * JR.ext[0] * JR.ext[1];
                const int l1 = r / JR.ext[0], l0 = r - l1 * JR.ext[0];
                const int gx = wrap_idx(JR.lo[0] + l0, a.G.n[0]), gy = wrap_idx(JR.lo[1] + l1, a.G.n[1]);
                const int gz = wrap_idx(JR.lo[2] + l2, a.G.n[2]);
                L[i] = a.lJ[comp][((size_t)gz * a.G.n[1] + gy) * a.G.n[0] + gx];
            }
        }
        __syncthreads();
    }
    for (int kk = 0; kk < PPT; ++kk) {
    const int p = base + kk * (int)blockDim.x;
    int lid, ic[3];
    bool ok;
    T ov[3];
    load(p, lid, ok, ic, ov);
    if (ok) {
        using DN = Dual<T, NT>;
        using IN = DualD<T, NT>;
        IN Xd[3];
        T u0v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (GD == 0) Xd[c] = IN(a.x_min[c] + ((double)a.icell[c][p] + (double)a.off[c][p]) * a.dx[c]);
            else if (GD <= 2 && c == 1) Xd[c] = IN(a.G.q_slice);
            else Xd[c] = IN(a.x_min[c] + ((double)(c == 0 ? win_col(ic[0], a.xo, a.G.n[0]) : ic[c]) + (double)ov[c]) * a.dx[c]);
            Xd[c].d[c] = T(1);
            u0v[c] = a.u[c][p];
        }
        // coupled reading: the current's adjoint first, from a value-only pass
        // (push and move as the forward step takes them), so that its working
        // set does not overlap the dual-number one below
        double gx0[3] = {0.0, 0.0, 0.0}, gx1[3] = {0.0, 0.0, 0.0}, gv[3] = {0.0, 0.0, 0.0};
        if constexpr (PASS == 2) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gx0[c] = a.gx0[(size_t)c * a.n + p];
        }
        if constexpr (CPL && GD > 0 && PASS != 2) {
            T ev[3], bv[3];
            analytic_field<PT, T>(plain_vars<T>(a.P, a.t), Xd[0].v, Xd[1].v, Xd[2].v, ev, bv);
            {
                AxisStencil<T> sn[3], sh[3];
                grid_stencils<T, GD>(ic, ov, a.G.n, sn, sh);
                T gr[3], gvv;
                const int nx = a.G.n[0], ny = a.G.n[1];
                gather_grad<T, GD>(a.G.F[0], sh[0], sn[1], sn[2], nx, ny, gvv, gr); ev[0] += gvv;
                gather_grad<T, GD>(a.G.F[1], sn[0], sh[1], sn[2], nx, ny, gvv, gr); ev[1] += gvv;
                gather_grad<T, GD>(a.G.F[2], sn[0], sn[1], sh[2], nx, ny, gvv, gr); ev[2] += gvv;
                gather_grad<T, GD>(a.G.F[3], sn[0], sh[1], sh[2], nx, ny, gvv, gr); bv[0] += gvv;
                gather_grad<T, GD>(a.G.F[4], sh[0], sn[1], sh[2], nx, ny, gvv, gr); bv[1] += gvv;
                gather_grad<T, GD>(a.G.F[5], sh[0], sh[1], sn[2], nx, ny, gvv, gr); bv[2] += gvv;
            }
            T u1p[3];
            boris_g<T>(u0v, ev, bv, T(0.5 * a.q_over_m * a.dt), u1p);
            const T ig = rsqrt_r<T>(T(1) + u1p[0] * u1p[0] + u1p[1] * u1p[1] + u1p[2] * u1p[2]);
            const T vt[3] = {u1p[0] * ig, u1p[1] * ig, u1p[2] * ig};
            T dl[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c == 0 || GD == 3 || (GD == 2 && c == 2)) {
                    const T d = vt[c] * T(a.dt / a.dx[c]);
                    dl[c] = fabs(d) < T(1) ? d : T(0);   // the forward push holds a too-fast move
                }
            }
            const double qw = a.q * (double)a.w[p];
            if (GD >= 2 && use_ldsj) {
                deposit_adjoint<T, GD>(JR, a.G.n, ic, ov, dl, vt, qw, a.dt, a.dx, gx0, gx1, gv);
            } else {
                const AdjGlobalRd gr{a.lJ, {a.G.n[0], a.G.n[1], a.G.n[2]}};
                deposit_adjoint<T, GD>(gr, a.G.n, ic, ov, dl, vt, qw, a.dt, a.dx, gx0, gx1, gv);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c == 0 || GD == 3 || (GD == 2 && c == 2)) {
                    gx1[c] /= a.dx[c];
                    gx0[c] /= a.dx[c];
                }
            }
            if constexpr (PASS == 1) {
                // d/dx^{n+1} joins the adjoint of x^{n+1}; the move takes d/dv
                // to the adjoint of u^{n+1/2} (velocity v = u ig, gamma = 1/ig)
                const double vg = (double)vt[0] * gv[0] + (double)vt[1] * gv[1] + (double)vt[2] * gv[2];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (c == 0 || GD == 3 || (GD == 2 && c == 2)) a.lam[c][lid] += gx1[c];
                    if (gv[c] != 0.0 || vg != 0.0) a.lam[3 + c][lid] += (gv[c] - (double)vt[c] * vg) * (double)ig;
                    a.gx0[(size_t)c * a.n + p] = gx0[c];
                }
                continue;
            }
        }
        const double a0_eff = a.P.a0 != 0.0 ? a.P.a0 : 1.0;
        const PulseVar<DN> W = adjoint_vars<T, NT>(a.P, a.t, a.slot, a0_eff);
        DN E8[3], B8[3];
        analytic_field_g<PT, DN, IN>(W, Xd[0], Xd[1], Xd[2], E8, B8);
        // fields per unit amplitude (dF/da0), then at the actual amplitude
        T Fu[6];
        const T ascale = T(a.P.a0 / a0_eff), ia0 = T(1.0 / a0_eff);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Fu[c] = E8[c].v * ia0;
            Fu[3 + c] = B8[c].v * ia0;
            E8[c].v *= ascale;
            B8[c].v *= ascale;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                E8[c].d[k] *= ascale;
                B8[c].d[k] *= ascale;
            }
        }
        if (GD > 0) {
            // recorded E2, B2: E_c sits half a cell up on axis c, B_c on
            // nodes along c and half a cell up on the other axes
            AxisStencil<T> sn[3], sh[3];
            grid_stencils<T, GD>(ic, ov, a.G.n, sn, sh);
            const T idx_[3] = {T(1.0 / a.dx[0]), T(1.0 / a.dx[1]), T(1.0 / a.dx[2])};
            // each field with its own stencils, written out so that no stencil
            // is selected at run time (that selection put them in scratch memory)
            auto add = [&](DN &F8, const T *F, const AxisStencil<T> &sx, const AxisStencil<T> &sy,
                           const AxisStencil<T> &sz) {
                T v, gr[3];
                gather_grad<T, GD>(F, sx, sy, sz, a.G.n[0], a.G.n[1], v, gr);
                F8.v += v;
                F8.d[0] += gr[0] * idx_[0];
                if (GD == 3) F8.d[1] += gr[1] * idx_[1];
                if (GD >= 2) F8.d[2] += gr[2] * idx_[2];
            };
            add(E8[0], a.G.F[0], sh[0], sn[1], sn[2]);
            add(E8[1], a.G.F[1], sn[0], sh[1], sn[2]);
            add(E8[2], a.G.F[2], sn[0], sn[1], sh[2]);
            add(B8[0], a.G.F[3], sn[0], sh[1], sh[2]);
            add(B8[1], a.G.F[4], sh[0], sn[1], sh[2]);
            add(B8[2], a.G.F[5], sh[0], sh[1], sn[2]);
        }

        // Boris Jacobian: tangents over (u0, E, B)
        using D9 = Dual<T, 9>;
        D9 uu[3], ee[3], bb[3], u1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uu[c] = D9::var(u0v[c], c);
            ee[c] = D9::var(E8[c].v, 3 + c);
            bb[c] = D9::var(B8[c].v, 6 + c);
        }
        boris_g<D9>(uu, ee, bb, D9(0.5 * a.q_over_m * a.dt), u1);

        double lx[3], lu1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lx[c] = a.lam[c][lid];
            lu1[c] = a.lam[3 + c][lid];
        }
        // the current depends on x^{n+1}
#pragma unroll
        for (int c = 0; c < 3; ++c) lx[c] += gx1[c];
        // move: x^{n+1} = x^n + dt u1/gamma1 (and v of the out-of-plane current)
        {
            const double v1[3] = {(double)u1[0].v, (double)u1[1].v, (double)u1[2].v};
            const double g1 = sqrt(1.0 + v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2]);
            const double vv[3] = {v1[0] / g1, v1[1] / g1, v1[2] / g1};
            const double vl = vv[0] * lx[0] + vv[1] * lx[1] + vv[2] * lx[2];
            const double vg = vv[0] * gv[0] + vv[1] * gv[1] + vv[2] * gv[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) lu1[c] += (a.dt * (lx[c] - vv[c] * vl) + (gv[c] - vv[c] * vg)) / g1;
        }
        double lu0[3] = {0.0, 0.0, 0.0}, lE[3] = {0.0, 0.0, 0.0}, lB[3] = {0.0, 0.0, 0.0};
        if (PX && a.lam_proxy) {
            const double lp = (double)a.lam_proxy[lid];
            if (lp != 0.0) {
                using D12 = Dual<T, 12>;
                D12 q0[3], q1[3], qe[3], qb[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q0[c] = D12::var(u0v[c], c);
                    q1[c] = D12::var(u1[c].v, 3 + c);
                    qe[c] = D12::var(E8[c].v, 6 + c);
                    qb[c] = D12::var(B8[c].v, 9 + c);
                }
                const D12 P12 = proxy_g<D12>(q0, q1, qe, qb, D12(a.dt));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    lu0[c] += lp * (double)P12.d[c];
                    lu1[c] += lp * (double)P12.d[3 + c];
                    lE[c] += lp * (double)P12.d[6 + c];
                    lB[c] += lp * (double)P12.d[9 + c];
                }
            }
        }
        // Boris adjoint
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lu0[c] += lu1[r] * (double)u1[r].d[c];
                lE[c] += lu1[r] * (double)u1[r].d[3 + c];
                lB[c] += lu1[r] * (double)u1[r].d[6 + c];
            }
        }
        if constexpr (PASS == 2) {
            // the adjoints of the gathered E, B for the scatter pass
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a.gx0[(size_t)c * a.n + p] = lE[c];
                a.gx0[(size_t)(3 + c) * a.n + p] = lB[c];
            }
        }
        if constexpr (CPL && GD > 0 && PASS != 2) {
            // the gather's adjoint into the grid adjoints of E2^n, B2^n
            AxisStencil<T> sn[3], sh[3];
            grid_stencils<T, GD>(ic, ov, a.G.n, sn, sh);
            const int nx = a.G.n[0], ny = a.G.n[1];
            if (GD >= 2 && use_lds) {
                scatter_adjoint_lds<T, GD>(lds_adj, 0, R, sh[0], sn[1], sn[2], lE[0]);
                scatter_adjoint_lds<T, GD>(lds_adj, 1, R, sn[0], sh[1], sn[2], lE[1]);
                scatter_adjoint_lds<T, GD>(lds_adj, 2, R, sn[0], sn[1], sh[2], lE[2]);
                scatter_adjoint_lds<T, GD>(lds_adj, 3, R, sn[0], sh[1], sh[2], lB[0]);
                scatter_adjoint_lds<T, GD>(lds_adj, 4, R, sh[0], sn[1], sh[2], lB[1]);
                scatter_adjoint_lds<T, GD>(lds_adj, 5, R, sh[0], sh[1], sn[2], lB[2]);
            } else {
            scatter_adjoint<T, GD>(a.lEg[0], sh[0], sn[1], sn[2], nx, ny, lE[0]);
            scatter_adjoint<T, GD>(a.lEg[1], sn[0], sh[1], sn[2], nx, ny, lE[1]);
            scatter_adjoint<T, GD>(a.lEg[2], sn[0], sn[1], sh[2], nx, ny, lE[2]);
            scatter_adjoint<T, GD>(a.lBg[0], sn[0], sh[1], sh[2], nx, ny, lB[0]);
            scatter_adjoint<T, GD>(a.lBg[1], sh[0], sn[1], sh[2], nx, ny, lB[1]);
            scatter_adjoint<T, GD>(a.lBg[2], sh[0], sh[1], sn[2], nx, ny, lB[2]);
            }
        }
        // field adjoint
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = lx[c] + gx0[c];
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += lE[k] * (double)E8[k].d[c] + lB[k] * (double)B8[k].d[c];
            // an (x, z) grid does not move y, 1-D rows move x only: those adjoints stay zero
            if (GD == 0 || GD == 3 || c == 0 || (GD == 2 && c == 2)) a.lam[c][lid] = acc;
            a.lam[3 + c][lid] = lu0[c];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) g[0] += lE[k] * (double)Fu[k] + lB[k] * (double)Fu[3 + k];
#pragma unroll
        for (int j = 0; j < NT - 3; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += lE[k] * (double)E8[k].d[3 + j] + lB[k] * (double)B8[k].d[3 + j];
#pragma unroll
            for (int q = 1; q < 5; ++q)
                if (a.slot[j] == q) g[q] += acc;
        }
    }
    }   // particles of this thread
    if constexpr (CPL && GD >= 2 && PASS != 2) {
        if (use_lds) {
            // flush: each node of the region once (zero sums skipped)
            __syncthreads();
            const int per = R.ext[0] * R.ext[1] * R.ext[2];
            for (int i = threadIdx.x; i < vol; i += blockDim.x) {
                const double v = lds_adj[i];
                if (v == 0.0) continue;
                const int comp = i / per;
                int r = i - comp * per;
                const int l2 = r / (R.ext[0] * R.ext[1]);
                r -= l2 * R.ext[0] * R.ext[1];
                const int l1 = r / R.ext[0], l0 = r - l1 * R.ext[0];
                int g[3] = {R.lo[0] + l0, R.lo[1] + l1, R.lo[2] + l2};
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) g[ax] = wrap_idx(g[ax], R.n[ax]);
                const size_t node = ((size_t)g[2] * R.n[1] + g[1]) * R.n[0] + g[0];
                atomicAdd(comp < 3 ? a.lEg[comp] + node : a.lBg[comp - 3] + node, v);
            }
        }
    }
    if constexpr (PASS == 1) return;
    // per-block FP64 sum, accumulated into this block's slot (no atomics)
    __shared__ double red[5][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const double s = wave_sum(g[j]);
        if (lane == 0) red[j][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[threadIdx.x][w];
        a.partial[(size_t)blockIdx.x * 5 + threadIdx.x] += s;
    }
}

// The gather's adjoint of the coupled reverse step (after PASS 2): each
// particle's adjoints of its gathered E, B (a.gx0, [6][n]) spread to the
// grid adjoints lEg, lBg with the gather's weights, accumulated in an LDS
// box and flushed once per node.  With a.tile_start a block takes the slots
// of one tile and its box is the tile's, widened by a.tile_margin cells (a
// tile-sorted state that has moved by up to that many cells since its sort
// stays inside); a particle whose stencil leaves the box adds its terms
// with global FP64 atomics.  Without it a block takes 256 consecutive slots
// and the box is their cells' bounding box (global atomics for the whole
// block when that box does not fit).  A block works through its slots in
// runs of at most kScatterRun, each with its own scale and flush.  The
// sums do not depend on the order of the state.
constexpr int kScatterRun = 4096;
template <typename T, int GD> AP_D __forceinline__ void adjoint_gather_scatter_body(const AdjointArgs<T> &a) {
    // FP32 runs accumulate in int64 fixed point (JTile) with a power-of-two
    // scale from the run's largest |value|: every term lies below 2^B units,
    // B = min(50, 58 - ceil(log2(run length))), and a node takes at most one
    // term per particle of the run, so its sum stays below 2^58.  Integer LDS
    // atomics run faster than FP64 ones, and the sums do not depend on the
    // order of the atomics
    using JA = typename JTile<T>::type;
    extern __shared__ double adj_dyn_raw[];
    JA *adj_dyn = reinterpret_cast<JA *>(adj_dyn_raw);
    __shared__ int bbox[6];
    __shared__ double s_max[4];
    const int nx = a.G.n[0], ny = a.G.n[1], nxy = a.G.n[0] * a.G.n[1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const bool by_tile = a.tile_start != nullptr;
    const int cap = a.scatter_cap > 0 ? a.scatter_cap : adj_lds_scatter<GD>();
    int r0, r1;
    AdjRegion R{};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) R.n[ax] = a.G.n[ax];
    if (by_tile) {
        r0 = a.tile_start[blockIdx.x];
        r1 = a.tile_start[blockIdx.x + 1];
        const int t[3] = {(int)blockIdx.x % a.tile_n[0], ((int)blockIdx.x / a.tile_n[0]) % a.tile_n[1],
                          (int)blockIdx.x / (a.tile_n[0] * a.tile_n[1])};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int ext = a.tile_dim[ax] + 3 + 2 * a.tile_margin;
            if ((GD == 2 && ax == 1) || ext >= R.n[ax]) {
                R.lo[ax] = 0;   // the whole axis
                R.ext[ax] = R.n[ax];
            } else {
                R.lo[ax] = wrap_idx(t[ax] * a.tile_dim[ax] - 1 - a.tile_margin, R.n[ax]);
                R.ext[ax] = ext;
            }
        }
    } else {
        r0 = blockIdx.x * 256;
        r1 = min(r0 + 256, a.n);
    }
    r0 = max(r0, 0);
    r1 = min(r1, a.n);
    // slot p: its cell (ic) and offsets (ov), false for a particle outside
    // the grid or with an id out of range (it adds nothing)
    auto load = [&](int p, int ic[3], T ov[3]) -> bool {
        const int cell = a.G.cell[p];
        ov[0] = a.off[0][p];
        ov[1] = GD == 3 ? a.off[1][p] : T(0);
        ov[2] = a.off[2][p];
        const bool ok = (unsigned)cell < (unsigned)nxy * (unsigned)a.G.n[2] && ov[0] >= T(0) && ov[0] < T(1) &&
                        ov[1] >= T(0) && ov[1] < T(1) && ov[2] >= T(0) && ov[2] < T(1) &&
                        (unsigned)a.G.id[p] < (unsigned)a.n;
        const int k = (int)a.G.fnxy.div((unsigned)cell);
        const int r = cell - k * nxy;
        const int j = (int)a.G.fnx.div((unsigned)r);
        ic[0] = r - j * nx;
        ic[1] = j;
        ic[2] = k;
        return ok;
    };
    // the stencil of a particle in cell ic covers nodes ic - 1 .. ic + 2 per axis
    auto in_box = [&](const int ic[3]) -> bool {
        bool in = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (R.ext[ax] == R.n[ax]) continue;
            int d = ic[ax] - (R.lo[ax] + 1);
            if (d < 0) d += R.n[ax];
            else if (d >= R.n[ax]) d -= R.n[ax];
            in = in && d <= R.ext[ax] - 4;
        }
        return in;
    };
    for (int c0 = r0; c0 < r1; c0 += kScatterRun) {
        const int c1 = min(c0 + kScatterRun, r1);
        if (threadIdx.x < 3) {
            bbox[threadIdx.x] = 0x7fffffff;
            bbox[3 + threadIdx.x] = -0x7fffffff;
        }
        // the run's box of cells (256-slot blocks) and (FP32) its largest |value|
        int mn[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, mx[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
        double m = 0.0;
        // thread t takes the run's slots t*k .. t*k + k - 1: a wave's lanes
        // then lie k slots apart, in distinct cells also where the state
        // holds a cell's particles next to each other (their LDS adds do not
        // collide), and each thread's reads stay contiguous
        const int k_per = (c1 - c0 + (int)blockDim.x - 1) / (int)blockDim.x;
        const int t0 = c0 + (int)threadIdx.x * k_per, t1 = min(t0 + k_per, c1);
        if (!by_tile || std::is_same<T, float>::value) {
            for (int p = t0; p < t1; ++p) {
                int ic[3];
                T ov[3];
                if (!load(p, ic, ov)) continue;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    mn[ax] = min(mn[ax], ic[ax]);
                    mx[ax] = max(mx[ax], ic[ax]);
                }
                if constexpr (std::is_same<T, float>::value) {
                    double mp = 0.0;
#pragma unroll
                    for (int c = 0; c < 6; ++c) mp = fmax(mp, fabs(a.gx0[(size_t)c * a.n + p]));
                    if (__builtin_isfinite(mp)) m = fmax(m, mp);   // a non-finite value goes to the global path
                }
            }
        }
        for (int d = 32; d > 0; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
        if (lane == 0) s_max[wid] = m;
        if (!by_tile) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                for (int d = 32; d > 0; d >>= 1) {
                    mn[ax] = min(mn[ax], __shfl_xor(mn[ax], d, 64));
                    mx[ax] = max(mx[ax], __shfl_xor(mx[ax], d, 64));
                }
        }
        __syncthreads();
        if (!by_tile && lane == 0) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                atomicMin(&bbox[ax], mn[ax]);
                atomicMax(&bbox[3 + ax], mx[ax]);
            }
        }
        __syncthreads();
        bool use_lds = true;
        if (!by_tile) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (GD == 2 && ax == 1) {
                    R.lo[1] = 0;
                    R.ext[1] = 1;
                    continue;
                }
                R.lo[ax] = bbox[ax] - 1;
                R.ext[ax] = bbox[3 + ax] - bbox[ax] + 4;
                use_lds = use_lds && bbox[ax] <= bbox[3 + ax] && R.ext[ax] <= R.n[ax];
            }
        }
        const int per = R.ext[0] * R.ext[1] * R.ext[2], vol = 6 * per;
        use_lds = use_lds && vol <= cap;
        if (use_lds)
            for (int i = threadIdx.x; i < vol; i += blockDim.x) adj_dyn[i] = JA(0);
        double scale = 1.0, inv_scale = 1.0;
        if constexpr (std::is_same<T, float>::value) {
            m = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
            if (m > 0.0) {
                int e, lb = 0;
                frexp(m, &e);   // every term (a value times stencil weights <= 1) lies below 2^e
                e = e < -960 ? -960 : e;   // keeps the scale finite; smaller terms round to zero
                while ((1 << lb) < c1 - c0) ++lb;
                const int bits = min(50, 58 - lb);
                scale = ldexp(1.0, bits - e);
                inv_scale = ldexp(1.0, e - bits);
            }
        }
        __syncthreads();
        for (int p = t0; p < t1; ++p) {
            int ic[3];
            T ov[3];
            if (!load(p, ic, ov)) continue;
            double lE[3], lB[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lE[c] = a.gx0[(size_t)c * a.n + p];
                lB[c] = a.gx0[(size_t)(3 + c) * a.n + p];
            }
            AxisStencil<T> sn[3], sh[3];
            grid_stencils<T, GD>(ic, ov, a.G.n, sn, sh);
            bool fin = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) fin = fin && __builtin_isfinite(lE[c]) && __builtin_isfinite(lB[c]);
            if (use_lds && fin && (!by_tile || in_box(ic))) {
                scatter_adjoint_lds<T, GD>(adj_dyn, 0, R, sh[0], sn[1], sn[2], lE[0], scale);
                scatter_adjoint_lds<T, GD>(adj_dyn, 1, R, sn[0], sh[1], sn[2], lE[1], scale);
                scatter_adjoint_lds<T, GD>(adj_dyn, 2, R, sn[0], sn[1], sh[2], lE[2], scale);
                scatter_adjoint_lds<T, GD>(adj_dyn, 3, R, sn[0], sh[1], sh[2], lB[0], scale);
                scatter_adjoint_lds<T, GD>(adj_dyn, 4, R, sh[0], sn[1], sh[2], lB[1], scale);
                scatter_adjoint_lds<T, GD>(adj_dyn, 5, R, sh[0], sh[1], sn[2], lB[2], scale);
            } else {
                scatter_adjoint<T, GD>(a.lEg[0], sh[0], sn[1], sn[2], nx, ny, lE[0]);
                scatter_adjoint<T, GD>(a.lEg[1], sn[0], sh[1], sn[2], nx, ny, lE[1]);
                scatter_adjoint<T, GD>(a.lEg[2], sn[0], sn[1], sh[2], nx, ny, lE[2]);
                scatter_adjoint<T, GD>(a.lBg[0], sn[0], sh[1], sh[2], nx, ny, lB[0]);
                scatter_adjoint<T, GD>(a.lBg[1], sh[0], sn[1], sh[2], nx, ny, lB[1]);
                scatter_adjoint<T, GD>(a.lBg[2], sh[0], sh[1], sn[2], nx, ny, lB[2]);
            }
        }
        if (!use_lds) continue;   // uniform over the block
        __syncthreads();
        for (int i = threadIdx.x; i < vol; i += blockDim.x) {
            const JA raw = adj_dyn[i];
            if (raw == JA(0)) continue;
            const double v = lds_value(raw, inv_scale);
            const int comp = i / per;
            int r = i - comp * per;
            const int l2 = r / (R.ext[0] * R.ext[1]);
            r -= l2 * R.ext[0] * R.ext[1];
            const int l1 = r / R.ext[0], l0 = r - l1 * R.ext[0];
            int g[3] = {R.lo[0] + l0, R.lo[1] + l1, R.lo[2] + l2};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) g[ax] = wrap_idx(g[ax], R.n[ax]);
            const size_t node = ((size_t)g[2] * R.n[1] + g[1]) * R.n[0] + g[0];
            atomicAdd(comp < 3 ? a.lEg[comp] + node : a.lBg[comp - 3] + node, v);
        }
        __syncthreads();   // the next run reuses bbox, s_max and the LDS box
    }
}
// FP32 (int64 LDS sums): three waves per SIMD, with a few spills, measured
// faster than two; FP64 at three would spill some 45 registers.
template <int GD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_adjoint_gather_scatter(
    AdjointArgs<float> a) {
    adjoint_gather_scatter_body<float, GD>(a);
}
template <int GD> __global__ __launch_bounds__(256) void k_adjoint_gather_scatter(AdjointArgs<double> a) {
    adjoint_gather_scatter_body<double, GD>(a);
}

// FP32: two waves per SIMD (the compiler keeps the dual-number working set
// in 256 registers with a few spills), measured faster than one wave without
// spills.  FP64 needs twice the registers and runs best at one wave.  The
// proxy term (PX) is a kernel of its own: its 12-tangent Jacobian would
// otherwise raise the register demand of every launch.
// (3-D with 5 tangents also fits three waves without spills, 158 VGPRs for
// the flying focus, but ran 57 ms against 47 at two.)
template <int PT, int NT, int GD, bool PX, bool CPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint_step(AdjointArgs<float> a) {
    adjoint_step_body<float, PT, NT, GD, PX, CPL>(a);
}
template <int PT, int NT, int GD, bool PX, bool CPL>
__global__ __launch_bounds__(256) void k_adjoint_step(AdjointArgs<double> a) {
    adjoint_step_body<double, PT, NT, GD, PX, CPL>(a);
}
// The coupled 2-D/3-D reverse step in three launches (see adjoint_step_body's
// PASS): the current's adjoint (159 VGPRs in 3-D FP32, three waves per
// SIMD), the rest, then k_adjoint_gather_scatter.
template <int PT, int GD, typename T>
__global__ __launch_bounds__(256) void k_adjoint_current(AdjointArgs<T> a) {
    adjoint_step_body<T, PT, 5, GD, false, true, 1>(a);
}
// The rest: (x, z) grids at two waves per SIMD (FP32).  In 3-D the
// dual-number working set and the 27-point gather gradients take 161-203
// VGPRs in FP32 without the proxy term (two waves); the proxy term, the
// nonparaxial pulse and FP64 need more (one wave: at two they spilled up to
// ~1000 words).
template <int PT, int NT, int GD, bool PX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adjoint_step_rest(
    AdjointArgs<float> a) {
    adjoint_step_body<float, PT, NT, GD, PX, true, 2>(a);
}
template <int PT, int NT, int GD, bool PX>
__global__ __launch_bounds__(256) void k_adjoint_step_rest(AdjointArgs<double> a) {
    adjoint_step_body<double, PT, NT, GD, PX, true, 2>(a);
}
// Waves per SIMD of the 3-D pass 2: two where its working set fits 256
// registers without spills (FP32 without the proxy term, pulses but the
// nonparaxial one: 161-203 VGPRs), else one.
template <int PT, bool PX, typename T> struct Rest3Waves {
    static constexpr int v = (std::is_same<T, float>::value && !PX && PT != PT_NP) ? 2 : 1;
};
template <int PT, int NT, bool PX, typename T>
__global__ __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(Rest3Waves<PT, PX, T>::v, Rest3Waves<PT, PX, T>::v))) void k_adjoint_step_rest3(AdjointArgs<T> a) {
    adjoint_step_body<T, PT, NT, 3, PX, true, 2>(a);
}

}  // namespace apt
