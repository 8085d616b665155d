// Fused per-particle kernel for (x, z) grids: gather E2, B2 (LDS-staged tile),
// analytic E1, B1 at the particle, relativistic Boris push, move, and
// charge-conserving quadratic-shape (Esirkepov) deposition of J into an
// LDS-private tile that is flushed to the global grid with atomics.
//
// One workgroup owns one particle tile (or 1/splits of it).  Tiles are
// TX x TZ cells; the LDS region adds kHaloLo cells below and kHaloHi above
// on each axis.  Particles whose stencil leaves the region (they drifted
// more than kDrift cells since the last re-sort) take the global path
// (direct loads and global atomics), so correctness never depends on how
// fresh the sort is.
#pragma once
#include "kernels.h"

namespace apt {

template <typename T> AP_D void tsc3(T d, T w[3]) {
    // quadratic B-spline weights of nodes -1, 0, +1 for offset d in [-1/2, 1/2]
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
}

// Place 3 weights of a stencil that starts o (0 or 1) nodes into a 4-node window.
template <typename T> AP_D void place4(int o, const T w[3], T out[4]) {
    const bool z = (o == 0);
    out[0] = z ? w[0] : T(0);
    out[1] = z ? w[1] : w[0];
    out[2] = z ? w[2] : w[1];
    out[3] = z ? T(0) : w[2];
}

AP_D int wrap_idx(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Esirkepov deposition of one particle into the LDS current tile on a WX x WZ
// node window (rows of RX nodes; window origin x0, z0).  A 3-node axis is
// exact when the stencil keeps its nearest node on that axis: the fourth
// weight is then zero before and after the move, and so is every current
// term that involves it.  In a 4-node window the lanes that kept their node
// skip those zero terms (fewer active lanes per LDS atomic).
template <int WX, int WZ, typename T, typename JA>
AP_D void deposit_window(JA *sJ, int RC, int RX, int x0, int z0, const T S0x[4], const T DSx[4],
                         const T S0z[4], const T DSz[4], T fx, T fy, T fz, double scale) {
    JA *Jx = sJ, *Jy = sJ + RC, *Jz = sJ + 2 * RC;
    const T third = T(1.0 / 3.0);
    auto atomic_add = [scale](JA *p, double v) {
        if ((WX == 3 && WZ == 3) || v != 0.0) lds_add(p, v, scale);
    };
#pragma unroll
    for (int b = 0; b < WZ; ++b) {
        const T cz = S0z[b] + T(0.5) * DSz[b];
        T cum = T(0);
#pragma unroll
        for (int m = 0; m < WX - 1; ++m) {
            cum += DSx[m] * cz;
            atomic_add(&Jx[(z0 + b) * RX + x0 + m], (double)(fx * cum));
        }
    }
#pragma unroll
    for (int m = 0; m < WX; ++m) {
        const T cx = S0x[m] + T(0.5) * DSx[m];
        T cum = T(0);
#pragma unroll
        for (int b = 0; b < WZ - 1; ++b) {
            cum += DSz[b] * cx;
            atomic_add(&Jz[(z0 + b) * RX + x0 + m], (double)(fz * cum));
        }
    }
#pragma unroll
    for (int b = 0; b < WZ; ++b)
#pragma unroll
        for (int m = 0; m < WX; ++m) {
            const T wy = S0x[m] * S0z[b] + T(0.5) * DSx[m] * S0z[b] + T(0.5) * S0x[m] * DSz[b] +
                         third * DSx[m] * DSz[b];
            atomic_add(&Jy[(z0 + b) * RX + x0 + m], (double)(fy * wy));
        }
}

// CTX, CTZ: the tile shape at compile time (LDS offsets become immediates),
// or 0, 0: the run's tile shape at run time.
// Blocks per CU the registers are budgeted for: five in FP32 runs (LDS holds
// five 32 x 8 tile blocks), three in FP64 runs (two with the eps^4 pulse,
// which would spill at three).
template <typename T, int PT, bool INPLACE, bool PROXY, int CTX, int CTZ>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 5 : (PT == PT_NP ? 2 : 3)) void k_push_deposit_2d(PushArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int TXv = CTX ? CTX : a.tile[0], TZv = CTZ ? CTZ : a.tile[2];
    const int RX = CTX ? CTX + kHaloLo + kHaloHi : a.reg[0];
    const int RZ = CTZ ? CTZ + kHaloLo + kHaloHi : a.reg[2];
    const int RC = RX * RZ;
    // Staged fields, on the region's inner box (nodes 1 .. R - 2 per axis:
    // the gather of a particle within the drift margin reads one node below
    // its cell and two above; the J tile keeps the whole region): 30.8 KB
    // per 32 x 8 tile block in FP32 runs, so five blocks share a CU.
    // Components that share a stencil window are stored as pairs, (Ex, Bz) on
    // (half, node) and (Ez, Bx) on (node, half), so one LDS read serves both;
    // Ey (node, node) and By (half, half) alone.
    const int IX = RX - 2, IC = IX * (RZ - 2);
    using T2 = typename Vec2<T>::type;
    T2 *sP = reinterpret_cast<T2 *>(smem_raw);               // [2][IC] pairs
    T *sS = reinterpret_cast<T *>(sP + 2 * IC);              // [2][IC] Ey, By
    // The current tile: FP64 in FP64 runs, int64 fixed point in FP32 runs
    // (JTile; ds_add_f64 measured several times faster than ds_add_f32 here,
    // ds_add_u64 faster again).
    using A = typename JTile<T>::type;
    A *sJ = reinterpret_cast<A *>(smem_raw + align_lds(6 * IC * sizeof(T)));   // Jx Jy Jz
    __shared__ float s_red[4];

    // XCD-aware mapping: consecutive hardware block ids go round-robin to
    // the 8 XCDs; give each XCD a contiguous run of logical tiles so that
    // halo re-reads of neighbouring tiles hit the same L2.
    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int logical = (bid & 7) * (nb >> 3) + (bid >> 3);
    if (logical >= a.n_logical) return;
    const int tile = logical / a.splits;
    const int split = logical - tile * a.splits;
    const int tx = tile % a.ntile[0];
    const int tz = tile / a.ntile[0];
    const int nx = a.n[0], nz = a.n[2];
    const int X0 = tx * TXv, Z0 = tz * TZv;
    const int ox = X0 - kHaloLo, oz = Z0 - kHaloLo;

    for (int f = threadIdx.x; f < IC; f += blockDim.x) {
        const int lz = f / IX;
        const int lx = f - lz * IX;
        const int gx = ((ox + lx + 1) % nx + nx) % nx;
        const int gz = ((oz + lz + 1) % nz + nz) % nz;
        const size_t g = (size_t)gz * nx + gx;
        T2 p0, p1;
        p0.x = a.E[0][g]; p0.y = a.B[2][g];
        p1.x = a.E[2][g]; p1.y = a.B[0][g];
        sP[f] = p0;
        sP[IC + f] = p1;
        sS[f] = a.E[1][g];
        sS[IC + f] = a.B[1][g];
    }
    for (int e = threadIdx.x; e < RC; e += blockDim.x) {
        sJ[0 * RC + e] = A(0);
        sJ[1 * RC + e] = A(0);
        sJ[2 * RC + e] = A(0);
    }
    // fixed-point scale of the block's current tile (FP32 runs): every
    // contribution is below |q w| max(dx, dz) / dt (the running sums and
    // shape factors are at most 1, |v_y| < c < dx / dt); from the largest
    // |q w| of the block's particles (non-finite weights belong to skipped
    // particles) and their count
    double scale = 1.0, inv_scale = 1.0;
    if constexpr (std::is_same<T, float>::value) {
        float qw = 0.f;
        int count = 0;
        for (int s = 0; s < a.nsp; ++s) {
            const SpeciesIO<T> &S = a.sp[s];
            const int beg = S.tile_start[tile];
            const int cnt = S.tile_start[tile + 1] - beg;
            const int pb = beg + (int)(((long long)cnt * split) / a.splits);
            const int pe = beg + (int)(((long long)cnt * (split + 1)) / a.splits);
            count += pe - pb;
            const float qa = fabsf((float)S.q);
            const T *w_in = INPLACE ? S.w_out : S.w_in;
            for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
                const float v = qa * fabsf((float)w_in[p]);
                if (__builtin_isfinite(v)) qw = fmaxf(qw, v);
            }
        }
        for (int d = 32; d > 0; d >>= 1) qw = fmaxf(qw, __shfl_xor(qw, d, 64));
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = qw;
        __syncthreads();
        qw = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
        const double fbound = (double)qw * fmax(a.dx[0], a.dx[2]) / a.dt;
        if (fbound > 0.0) {
            int e, ec;
            frexp(fbound, &e);                              // fbound < 2^e
            frexp((double)(count > 0 ? count : 1), &ec);   // count < 2^ec
            const int k = min(50 - e, 62 - e - ec);
            scale = ldexp(1.0, k);
            inv_scale = ldexp(1.0, -k);
        }
    }
    __syncthreads();

    const T dtdx = T(a.dt / a.dx[0]);
    const T dtdz = T(a.dt / a.dx[2]);
    const int half_nx = nx >> 1, half_nz = nz >> 1;
    const unsigned ncell = (unsigned)nx * (unsigned)nz;

    for (int s = 0; s < a.nsp; ++s) {
        const SpeciesIO<T> &S = a.sp[s];
        // in-place steps read and write the same arrays (fewer live pointers)
        const int32_t *cell_in = INPLACE ? S.cell_out : S.cell_in;
        const T *off_in0 = INPLACE ? S.off_out[0] : S.off_in[0];
        const T *off_in1 = INPLACE ? S.off_out[1] : S.off_in[1];
        const T *off_in2 = INPLACE ? S.off_out[2] : S.off_in[2];
        const T *u_in0 = INPLACE ? S.u_out[0] : S.u_in[0];
        const T *u_in1 = INPLACE ? S.u_out[1] : S.u_in[1];
        const T *u_in2 = INPLACE ? S.u_out[2] : S.u_in[2];
        const T *w_in = INPLACE ? S.w_out : S.w_in;
        const int beg = S.tile_start[tile];
        const int cnt = S.tile_start[tile + 1] - beg;
        const int pb = beg + (int)(((long long)cnt * split) / a.splits);
        const int pe = beg + (int)(((long long)cnt * (split + 1)) / a.splits);
        const T kap = T(0.5 * S.q_over_m * a.dt);
        const T cjx = T(-S.q * a.dx[0] / a.dt);
        const T cjz = T(-S.q * a.dx[2] / a.dt);
        const T cjy = T(S.q);
        for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
            const int cell = cell_in[p];
            const T offx = off_in0[p];
            const T offz = off_in2[p];
            T ux = u_in0[p], uy = u_in1[p], uz = u_in2[p];
            const T w = w_in[p];
            const bool ok = (unsigned)cell < ncell && offx >= T(0) && offx < T(1) &&
                            offz >= T(0) && offz < T(1) && finite_state(ux, uy, uz, w);
            if (!ok) {
                count_skipped(a.n_bad, cell);
                S.cell_out[p] = cell;
                S.off_out[0][p] = offx;
                S.off_out[2][p] = offz;
                S.u_out[0][p] = ux; S.u_out[1][p] = uy; S.u_out[2][p] = uz;
                if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
                if (PROXY && !INPLACE && S.proxy_out) {
                    S.proxy_out[2 * p] = S.proxy_in[2 * p];
                    S.proxy_out[2 * p + 1] = S.proxy_in[2 * p + 1];
                }
                continue;
            }
            const int k = (int)a.fnx.div((unsigned)cell);
            const int i = cell - k * nx;
            int di = i - X0, dk = k - Z0;
            if (di < -half_nx) di += nx; else if (di >= nx - half_nx) di -= nx;
            if (dk < -half_nz) dk += nz; else if (dk >= nz - half_nz) dk -= nz;
            const int la = di + kHaloLo, lb = dk + kHaloLo;
            const bool in_lds = la >= 2 && la <= RX - 4 && lb >= 2 && lb <= RZ - 4;
            wave_count(a.n_offtile, !in_lds);

            // ---- gather E2, B2 (quadratic shape at each staggered location)
            const int nxn = offx >= T(0.5) ? 1 : 0;
            const int nzn = offz >= T(0.5) ? 1 : 0;
            T wxn[3], wxh[3], wzn[3], wzh[3];
            tsc3(offx - T(nxn), wxn);
            tsc3(offx - T(0.5), wxh);
            tsc3(offz - T(nzn), wzn);
            tsc3(offz - T(0.5), wzh);
            T e2[3], b2[3];
            if (in_lds) {
                // stencil starts in the inner box (region node - 1 per axis)
                const int xn = la + nxn - 2, xh = la - 2, zn = lb + nzn - 2, zh = lb - 2;
                auto G = [&](const T *F, int bx, const T *wx, int bz, const T *wz) {
                    T acc = T(0);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const T *row = F + (bz + b) * IX + bx;
                        acc += wz[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2]);
                    }
                    return acc;
                };
                auto G2 = [&](const T2 *F, int bx, const T *wx, int bz, const T *wz, T &o0, T &o1) {
                    T a0 = T(0), a1 = T(0);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const T2 *row = F + (bz + b) * IX + bx;
                        const T2 r0 = row[0], r1 = row[1], r2 = row[2];
                        a0 += wz[b] * (wx[0] * r0.x + wx[1] * r1.x + wx[2] * r2.x);
                        a1 += wz[b] * (wx[0] * r0.y + wx[1] * r1.y + wx[2] * r2.y);
                    }
                    o0 = a0;
                    o1 = a1;
                };
                G2(sP, xh, wxh, zn, wzn, e2[0], b2[2]);
                G2(sP + IC, xn, wxn, zh, wzh, e2[2], b2[0]);
                e2[1] = G(sS, xn, wxn, zn, wzn);
                b2[1] = G(sS + IC, xh, wxh, zh, wzh);
            } else {
                int gxn[3], gxh[3];
                size_t gzn[3], gzh[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    gxn[m] = wrap_idx(i + nxn - 1 + m, nx);
                    gxh[m] = wrap_idx(i - 1 + m, nx);
                    gzn[m] = (size_t)wrap_idx(k + nzn - 1 + m, nz) * nx;
                    gzh[m] = (size_t)wrap_idx(k - 1 + m, nz) * nx;
                }
                auto G = [&](const T *F, const int *gx, const T *wx, const size_t *gz, const T *wz) {
                    T acc = T(0);
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        acc += wz[b] * (wx[0] * F[gz[b] + gx[0]] + wx[1] * F[gz[b] + gx[1]] +
                                        wx[2] * F[gz[b] + gx[2]]);
                    return acc;
                };
                e2[0] = G(a.E[0], gxh, wxh, gzn, wzn);
                e2[1] = G(a.E[1], gxn, wxn, gzn, wzn);
                e2[2] = G(a.E[2], gxn, wxn, gzh, wzh);
                b2[0] = G(a.B[0], gxn, wxn, gzh, wzh);
                b2[1] = G(a.B[1], gxh, wxh, gzh, wzh);
                b2[2] = G(a.B[2], gxh, wxh, gzn, wzn);
            }

            // ---- analytic E1, B1 at the particle (FP64 position)
            T e1[3], b1[3];
            const double X = a.x_min[0] + ((double)win_col(i, a.xo, a.n[0]) + (double)offx) * a.dx[0];
            const double Z = a.x_min[2] + ((double)k + (double)offz) * a.dx[2];
            analytic_field<PT, T>(a.W, X, a.q_slice, Z, e1, b1);
            const T Ex = e1[0] + e2[0], Ey = e1[1] + e2[1], Ez = e1[2] + e2[2];
            const T Bx = b1[0] + b2[0], By = b1[1] + b2[1], Bz = b1[2] + b2[2];

            // ---- relativistic Boris push
            const T u0x = ux, u0y = uy, u0z = uz;
            const T umx = ux + kap * Ex, umy = uy + kap * Ey, umz = uz + kap * Ez;
            const T ig = rsqrt_r<T>(T(1) + umx * umx + umy * umy + umz * umz);
            const T tx_ = kap * Bx * ig, ty_ = kap * By * ig, tz_ = kap * Bz * ig;
            const T sf = T(2) / (T(1) + tx_ * tx_ + ty_ * ty_ + tz_ * tz_);
            const T upx = umx + (umy * tz_ - umz * ty_);
            const T upy = umy + (umz * tx_ - umx * tz_);
            const T upz = umz + (umx * ty_ - umy * tx_);
            ux = umx + sf * (upy * tz_ - upz * ty_) + kap * Ex;
            uy = umy + sf * (upz * tx_ - upx * tz_) + kap * Ey;
            uz = umz + sf * (upx * ty_ - upy * tx_) + kap * Ez;
            if constexpr (PROXY) {
                if (S.proxy_out) {
                    const T uv0[3] = {u0x, u0y, u0z}, uv1[3] = {ux, uy, uz};
                    const T Ev[3] = {Ex, Ey, Ez}, Bv[3] = {Bx, By, Bz};
                    proxy_accumulate<T>((INPLACE ? S.proxy_out : S.proxy_in) + 2 * p, S.proxy_out + 2 * p, uv0, uv1,
                                        Ev, Bv, T(a.dt));
                }
            }

            // ---- move in (cell, offset) form
            const T ign = rsqrt_r<T>(T(1) + ux * ux + uy * uy + uz * uz);
            T ddx = ux * ign * dtdx, ddz = uz * ign * dtdz;
            if (!push_move_ok(ign, ddx) || !push_move_ok(ign, ddz)) {
                atomicAdd(a.n_fast, 1ull);
                if (!push_move_ok(ign, ddx)) ddx = T(0);
                if (!push_move_ok(ign, ddz)) ddz = T(0);
            }
            T nox = offx + ddx, noz = offz + ddz;
            int sx = (int)floor_r<T>(nox), sz = (int)floor_r<T>(noz);
            nox -= T(sx); noz -= T(sz);
            if (nox >= T(1)) { nox -= T(1); sx += 1; }
            if (noz >= T(1)) { noz -= T(1); sz += 1; }

            // ---- Esirkepov deposition on a 4 x 4 node window (relative to i, k)
            const int n1x = sx + (nox >= T(0.5) ? 1 : 0);
            const int n1z = sz + (noz >= T(0.5) ? 1 : 0);
            T w1x[3], w1z[3];
            tsc3(nox - T(n1x - sx), w1x);
            tsc3(noz - T(n1z - sz), w1z);
            const int bx = min(nxn, n1x) - 1, bz = min(nzn, n1z) - 1;
            T S0x[4], S1x[4], S0z[4], S1z[4], DSx[4], DSz[4];
            place4(nxn - 1 - bx, wxn, S0x);
            place4(n1x - 1 - bx, w1x, S1x);
            place4(nzn - 1 - bz, wzn, S0z);
            place4(n1z - 1 - bz, w1z, S1z);
#pragma unroll
            for (int m = 0; m < 4; ++m) { DSx[m] = S1x[m] - S0x[m]; DSz[m] = S1z[m] - S0z[m]; }
            const T fx = cjx * w, fz = cjz * w, fy = cjy * w * uy * ign;
            const T third = T(1.0 / 3.0);
            if (in_lds) {
                // window width per axis, uniform over the wave
                const bool wx4 = __any(nxn != n1x), wz4 = __any(nzn != n1z);
                const int x0 = la + bx, z0 = lb + bz;
                if (wx4 && wz4) deposit_window<4, 4>(sJ, RC, RX, x0, z0, S0x, DSx, S0z, DSz, fx, fy, fz, scale);
                else if (wx4) deposit_window<4, 3>(sJ, RC, RX, x0, z0, S0x, DSx, S0z, DSz, fx, fy, fz, scale);
                else if (wz4) deposit_window<3, 4>(sJ, RC, RX, x0, z0, S0x, DSx, S0z, DSz, fx, fy, fz, scale);
                else deposit_window<3, 3>(sJ, RC, RX, x0, z0, S0x, DSx, S0z, DSz, fx, fy, fz, scale);
            } else {
                int gx[4];
                size_t gz[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    gx[m] = wrap_idx(wrap_idx(i + bx + m, nx), nx);
                    gz[m] = (size_t)wrap_idx(wrap_idx(k + bz + m, nz), nz) * nx;
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T cz = S0z[b] + T(0.5) * DSz[b];
                    T cum = T(0);
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        cum += DSx[m] * cz;
                        atomic_add(&a.Jacc[0][gz[b] + gx[m]], (double)(fx * cum));
                    }
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const T cx = S0x[m] + T(0.5) * DSx[m];
                    T cum = T(0);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        cum += DSz[b] * cx;
                        atomic_add(&a.Jacc[2][gz[b] + gx[m]], (double)(fz * cum));
                    }
                }
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const T wy = S0x[m] * S0z[b] + T(0.5) * DSx[m] * S0z[b] +
                                     T(0.5) * S0x[m] * DSz[b] + third * DSx[m] * DSz[b];
                        atomic_add(&a.Jacc[1][gz[b] + gx[m]], (double)(fy * wy));
                    }
            }

            // ---- write back
            const int i1 = wrap_idx(i + sx, nx), k1 = wrap_idx(k + sz, nz);
            S.cell_out[p] = i1 + k1 * nx;
            S.off_out[0][p] = nox;
            S.off_out[2][p] = noz;
            S.u_out[0][p] = ux;
            S.u_out[1][p] = uy;
            S.u_out[2][p] = uz;
            if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
        }
    }
    __syncthreads();

    for (int e = threadIdx.x; e < RC; e += blockDim.x) {
        const int lz = e / RX;
        const int lx = e - lz * RX;
        const int gx = ((ox + lx) % nx + nx) % nx;
        const int gz = ((oz + lz) % nz + nz) % nz;
        const size_t g = (size_t)gz * nx + gx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const A v = sJ[c * RC + e];
            if (v != A(0)) atomic_add(&a.Jacc[c][g], lds_value(v, inv_scale));
        }
    }
}

template <typename T, int PT, int CTX, int CTZ>
hipError_t launch2d(const PushArgs<T> &a, int threads, hipStream_t s) {
    const size_t rc = (size_t)a.reg[0] * a.reg[2];
    const size_t ic = (size_t)(a.reg[0] - 2) * (a.reg[2] - 2);
    const size_t lds = align_lds(6 * ic * sizeof(T)) + 3 * rc * sizeof(double);
    const int blocks = ((a.n_logical + 7) / 8) * 8;
    if (blocks == 0) return hipSuccess;
    bool proxy = false;
    for (int k = 0; k < a.nsp; ++k) proxy = proxy || a.sp[k].proxy_out != nullptr;
    const bool inplace = a.sp[0].copy_static == 0;
    if (inplace && !proxy)
        hipLaunchKernelGGL((k_push_deposit_2d<T, PT, true, false, CTX, CTZ>), dim3(blocks), dim3(threads), lds, s, a);
    else if (!proxy)
        hipLaunchKernelGGL((k_push_deposit_2d<T, PT, false, false, CTX, CTZ>), dim3(blocks), dim3(threads), lds, s,
                           a);
    else if (inplace)
        hipLaunchKernelGGL((k_push_deposit_2d<T, PT, true, true, CTX, CTZ>), dim3(blocks), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_push_deposit_2d<T, PT, false, true, CTX, CTZ>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// Every pulse family of one tile shape (instantiated per shape in its own
// translation unit).
template <typename T, int CTX, int CTZ>
hipError_t launch2d_tile(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch2d<T, PT_NONE, CTX, CTZ>(a, threads, s);
    case PT_PLANE: return launch2d<T, PT_PLANE, CTX, CTZ>(a, threads, s);
    case PT_GAUSS: return launch2d<T, PT_GAUSS, CTX, CTZ>(a, threads, s);
    case PT_LG: return launch2d<T, PT_LG, CTX, CTZ>(a, threads, s);
    case PT_FF: return launch2d<T, PT_FF, CTX, CTZ>(a, threads, s);
    case PT_NP: return launch2d<T, PT_NP, CTX, CTZ>(a, threads, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace apt
