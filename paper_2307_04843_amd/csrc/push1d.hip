// Fused per-particle kernel for rows of independent 1-D grids (the
// reduced-dimensionality series of Sec. III.B: each row is a 1D-3V
// simulation along x at its own transverse lab position).  Per particle:
// gather E2, B2 on the 3-node quadratic stencil along x (LDS-staged row
// segment), analytic E1, B1 at (x, the pulse's y slice, the row's z),
// relativistic Boris push (three velocity components), move along x, and
// charge-conserving deposition: J_x from the change of the quadratic shape
// (Esirkepov in 1-D), J_y and J_z as q w v times the time-averaged shape.
//
// One workgroup owns one tile (TX cells of one row, or 1/splits of it) with
// a halo of kHaloLo / kHaloHi nodes; pushes whose stencil leaves the staged
// segment use global memory, as in the 2-D kernel.
#include "kernels.h"

namespace apt {

template <typename T> AP_D void tsc3_1d(T d, T w[3]) {
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
}

template <typename T> AP_D void place4_1d(int o, const T w[3], T out[4]) {
    const bool z = (o == 0);
    out[0] = z ? w[0] : T(0);
    out[1] = z ? w[1] : w[0];
    out[2] = z ? w[2] : w[1];
    out[3] = z ? T(0) : w[2];
}

AP_D int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <typename T, int PT, bool INPLACE, bool PROXY>
__global__ __launch_bounds__(256) void k_push_deposit_1d(PushArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int RX = a.reg[0];
    T *sF = reinterpret_cast<T *>(smem_raw);                                   // [6][RX]
    double *sJ = reinterpret_cast<double *>(smem_raw + align_lds(6 * RX * sizeof(T)));   // [3][RX]

    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int logical = (bid & 7) * (nb >> 3) + (bid >> 3);
    if (logical >= a.n_logical) return;
    const int tile = logical / a.splits;
    const int split = logical - tile * a.splits;
    const int tx = tile % a.ntile[0];
    const int row = tile / a.ntile[0];
    const int nx = a.n[0];
    const int X0 = tx * a.tile[0];
    const int ox = X0 - kHaloLo;
    const size_t row0 = (size_t)row * nx;

    for (int e = threadIdx.x; e < RX; e += blockDim.x) {
        const size_t g = row0 + ((ox + e) % nx + nx) % nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sF[c * RX + e] = a.E[c][g];
            sF[(3 + c) * RX + e] = a.B[c][g];
            sJ[c * RX + e] = 0.0;
        }
    }
    __syncthreads();

    const T dtdx = T(a.dt / a.dx[0]);
    const int half_nx = nx >> 1;
    const unsigned ncell = (unsigned)nx * (unsigned)a.n[2];
    const double Zrow = a.x_min[2] + (double)row * a.dx[2];

    for (int s = 0; s < a.nsp; ++s) {
        const SpeciesIO<T> &S = a.sp[s];
        const int32_t *cell_in = INPLACE ? S.cell_out : S.cell_in;
        const T *off_in0 = INPLACE ? S.off_out[0] : S.off_in[0];
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
        const T cjt = T(S.q);
        for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
            const int cell = cell_in[p];
            const T offx = off_in0[p];
            T ux = u_in0[p], uy = u_in1[p], uz = u_in2[p];
            const T w = w_in[p];
            const int prow = (int)a.fnx.div((unsigned)cell);
            // a particle belongs to its tile's row; anything else is invalid state
            const bool ok = (unsigned)cell < ncell && prow == row && offx >= T(0) && offx < T(1) &&
                            finite_state(ux, uy, uz, w);
            if (!ok) {
                count_skipped(a.n_bad, cell);
                S.cell_out[p] = cell;
                S.off_out[0][p] = offx;
                S.u_out[0][p] = ux; S.u_out[1][p] = uy; S.u_out[2][p] = uz;
                if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
                if (PROXY && !INPLACE && S.proxy_out) {
                    S.proxy_out[2 * p] = S.proxy_in[2 * p];
                    S.proxy_out[2 * p + 1] = S.proxy_in[2 * p + 1];
                }
                continue;
            }
            const int i = cell - prow * nx;
            int di = i - X0;
            if (di < -half_nx) di += nx; else if (di >= nx - half_nx) di -= nx;
            const int la = di + kHaloLo;
            const bool in_lds = la >= 2 && la <= RX - 4;
            wave_count(a.n_offtile, !in_lds);

            // ---- gather: Ex, By, Bz half a cell up in x; Ey, Ez, Bx on nodes
            const int nxn = offx >= T(0.5) ? 1 : 0;
            T wn[3], wh[3];
            tsc3_1d(offx - T(nxn), wn);
            tsc3_1d(offx - T(0.5), wh);
            T f[6];
            if (in_lds) {
                const int bn = la + nxn - 1, bh = la - 1;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const bool half = (c == 0 || c == 4 || c == 5);
                    const T *F = sF + c * RX + (half ? bh : bn);
                    const T *wt = half ? wh : wn;
                    f[c] = wt[0] * F[0] + wt[1] * F[1] + wt[2] * F[2];
                }
            } else {
                int gn[3], gh[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    gn[m] = wrap1(i + nxn - 1 + m, nx);
                    gh[m] = wrap1(i - 1 + m, nx);
                }
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const bool half = (c == 0 || c == 4 || c == 5);
                    const T *F = (c < 3 ? a.E[c] : a.B[c - 3]) + row0;
                    const int *gi = half ? gh : gn;
                    const T *wt = half ? wh : wn;
                    f[c] = wt[0] * F[gi[0]] + wt[1] * F[gi[1]] + wt[2] * F[gi[2]];
                }
            }

            // ---- analytic E1, B1 at the particle (FP64 position)
            T e1[3], b1[3];
            const double X = a.x_min[0] + ((double)win_col(i, a.xo, a.n[0]) + (double)offx) * a.dx[0];
            analytic_field<PT, T>(a.W, X, a.q_slice, Zrow, e1, b1);
            const T Ex = e1[0] + f[0], Ey = e1[1] + f[1], Ez = e1[2] + f[2];
            const T Bx = b1[0] + f[3], By = b1[1] + f[4], Bz = b1[2] + f[5];

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

            // ---- move along x
            const T ign = rsqrt_r<T>(T(1) + ux * ux + uy * uy + uz * uz);
            T ddx = ux * ign * dtdx;
            if (!push_move_ok(ign, ddx)) {
                atomicAdd(a.n_fast, 1ull);
                ddx = T(0);
            }
            T nox = offx + ddx;
            int sx = (int)floor_r<T>(nox);
            nox -= T(sx);
            if (nox >= T(1)) { nox -= T(1); sx += 1; }

            // ---- deposition on a 4-node window relative to i
            const int n1x = sx + (nox >= T(0.5) ? 1 : 0);
            T w1[3];
            tsc3_1d(nox - T(n1x - sx), w1);
            const int bx = min(nxn, n1x) - 1;
            T S0[4], S1[4], DS[4];
            place4_1d(nxn - 1 - bx, wn, S0);
            place4_1d(n1x - 1 - bx, w1, S1);
#pragma unroll
            for (int m = 0; m < 4; ++m) DS[m] = S1[m] - S0[m];
            const T fx = cjx * w, fy = cjt * w * uy * ign, fz = cjt * w * uz * ign;
            if (in_lds) {
                double *Jx = sJ, *Jy = sJ + RX, *Jz = sJ + 2 * RX;
                const int x0 = la + bx;
                T cum = T(0);
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    cum += DS[m];
                    const T v = fx * cum;
                    if (v != T(0)) atomic_add(&Jx[x0 + m], (double)v);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const T sa = S0[m] + T(0.5) * DS[m];
                    if (sa != T(0)) {
                        atomic_add(&Jy[x0 + m], (double)(fy * sa));
                        atomic_add(&Jz[x0 + m], (double)(fz * sa));
                    }
                }
            } else {
                T cum = T(0);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const size_t g = row0 + wrap1(wrap1(i + bx + m, nx), nx);
                    if (m < 3) {
                        cum += DS[m];
                        const T v = fx * cum;
                        if (v != T(0)) atomic_add(&a.Jacc[0][g], (double)v);
                    }
                    const T sa = S0[m] + T(0.5) * DS[m];
                    if (sa != T(0)) {
                        atomic_add(&a.Jacc[1][g], (double)(fy * sa));
                        atomic_add(&a.Jacc[2][g], (double)(fz * sa));
                    }
                }
            }

            // ---- write back
            S.cell_out[p] = (int)row0 + wrap1(i + sx, nx);
            S.off_out[0][p] = nox;
            S.u_out[0][p] = ux;
            S.u_out[1][p] = uy;
            S.u_out[2][p] = uz;
            if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
        }
    }
    __syncthreads();

    for (int e = threadIdx.x; e < RX; e += blockDim.x) {
        const size_t g = row0 + ((ox + e) % nx + nx) % nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = sJ[c * RX + e];
            if (v != 0.0) atomic_add(&a.Jacc[c][g], v);
        }
    }
}

template <typename T, int PT>
static hipError_t launch1d(const PushArgs<T> &a, int threads, hipStream_t s) {
    const size_t rx = (size_t)a.reg[0];
    const size_t lds = align_lds(6 * rx * sizeof(T)) + 3 * rx * sizeof(double);
    const int blocks = ((a.n_logical + 7) / 8) * 8;
    if (blocks == 0) return hipSuccess;
    bool proxy = false;
    for (int k = 0; k < a.nsp; ++k) proxy = proxy || a.sp[k].proxy_out != nullptr;
    const bool inplace = a.sp[0].copy_static == 0;
    if (inplace && !proxy)
        hipLaunchKernelGGL((k_push_deposit_1d<T, PT, true, false>), dim3(blocks), dim3(threads), lds, s, a);
    else if (!proxy)
        hipLaunchKernelGGL((k_push_deposit_1d<T, PT, false, false>), dim3(blocks), dim3(threads), lds, s, a);
    else if (inplace)
        hipLaunchKernelGGL((k_push_deposit_1d<T, PT, true, true>), dim3(blocks), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_push_deposit_1d<T, PT, false, true>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_push_deposit_1d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch1d<T, PT_NONE>(a, threads, s);
    case PT_PLANE: return launch1d<T, PT_PLANE>(a, threads, s);
    case PT_GAUSS: return launch1d<T, PT_GAUSS>(a, threads, s);
    case PT_LG: return launch1d<T, PT_LG>(a, threads, s);
    case PT_FF: return launch1d<T, PT_FF>(a, threads, s);
    case PT_NP: return launch1d<T, PT_NP>(a, threads, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_push_deposit_1d<float>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch_push_deposit_1d<double>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
