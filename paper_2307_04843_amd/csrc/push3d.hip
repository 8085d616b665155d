// Fused per-particle kernel for 3-D grids: LDS-staged gather of E2, B2 on a
// 3 x 3 x 3 quadratic stencil per staggered component, analytic E1, B1 at the
// particle, relativistic Boris push, move, and Esirkepov deposition on a
// 4 x 4 x 4 node window into an LDS-private J tile flushed with atomics.
// Particles whose stencil leaves the staged region use global memory.
#include "kernels.h"

namespace apt {

constexpr int kLo3 = 2;   // 3-D halo: no drift margin (LDS budget), sort often
constexpr int kHi3 = 3;

template <typename T> AP_D void tsc3w(T d, T w[3]) {
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
}

template <typename T> AP_D void place4w(int o, const T w[3], T out[4]) {
    const bool z = (o == 0);
    out[0] = z ? w[0] : T(0);
    out[1] = z ? w[1] : w[0];
    out[2] = z ? w[2] : w[1];
    out[3] = z ? T(0) : w[2];
}

AP_D int wrap3(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Esirkepov deposition of one particle into the LDS current tile on a W^3 node
// window with origin (o0, o1, o2).  W = 3 is exact when no axis changes its
// nearest node during the move (the fourth weight is zero before and after).
// In the 4-node window a lane whose node did not change on an axis has a zero
// slice there; its zero contributions are skipped, which takes their LDS
// traffic off the shared atomic pipe (measured 1.3x on the whole kernel).
template <int W, typename T>
AP_D void deposit_window3(double *sJ, int RC, int RXY, int RX, int o0, int o1, int o2, const T (&S0)[3][4],
                          const T (&DS)[3][4], const T (&fj)[3]) {
    const T third = T(1.0 / 3.0);
    auto at = [&](int comp, int i4, int j4, int k4) {
        return sJ + comp * RC + (o2 + k4) * RXY + (o1 + j4) * RX + o0 + i4;
    };
    auto atomic_add = [](double *p, double v) {
        if (W == 3 || v != 0.0) apt::atomic_add(p, v);
    };
    // Jx: cumulative along x of Wx = DSx (S0y S0z + DSy S0z/2 + S0y DSz/2 + DSy DSz/3)
#pragma unroll
    for (int k4 = 0; k4 < W; ++k4)
#pragma unroll
        for (int j4 = 0; j4 < W; ++j4) {
            const T cyz = S0[1][j4] * S0[2][k4] + T(0.5) * DS[1][j4] * S0[2][k4] +
                          T(0.5) * S0[1][j4] * DS[2][k4] + third * DS[1][j4] * DS[2][k4];
            T cum = T(0);
#pragma unroll
            for (int i4 = 0; i4 < W - 1; ++i4) {
                cum += DS[0][i4] * cyz;
                atomic_add(at(0, i4, j4, k4), (double)(fj[0] * cum));
            }
        }
#pragma unroll
    for (int k4 = 0; k4 < W; ++k4)
#pragma unroll
        for (int i4 = 0; i4 < W; ++i4) {
            const T cxz = S0[0][i4] * S0[2][k4] + T(0.5) * DS[0][i4] * S0[2][k4] +
                          T(0.5) * S0[0][i4] * DS[2][k4] + third * DS[0][i4] * DS[2][k4];
            T cum = T(0);
#pragma unroll
            for (int j4 = 0; j4 < W - 1; ++j4) {
                cum += DS[1][j4] * cxz;
                atomic_add(at(1, i4, j4, k4), (double)(fj[1] * cum));
            }
        }
#pragma unroll
    for (int j4 = 0; j4 < W; ++j4)
#pragma unroll
        for (int i4 = 0; i4 < W; ++i4) {
            const T cxy = S0[0][i4] * S0[1][j4] + T(0.5) * DS[0][i4] * S0[1][j4] +
                          T(0.5) * S0[0][i4] * DS[1][j4] + third * DS[0][i4] * DS[1][j4];
            T cum = T(0);
#pragma unroll
            for (int k4 = 0; k4 < W - 1; ++k4) {
                cum += DS[2][k4] * cxy;
                atomic_add(at(2, i4, j4, k4), (double)(fj[2] * cum));
            }
        }
}

template <typename T, int PT, bool INPLACE, bool PROXY>
__global__ __launch_bounds__(256) void k_push_deposit_3d(PushArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int RX = a.reg[0], RY = a.reg[1], RZ = a.reg[2];
    const int RXY = RX * RY;
    const int RC = RXY * RZ;
    T *sF = sm;
    double *sJ = reinterpret_cast<double *>(smem_raw + align_lds(6 * RC * sizeof(T)));

    const int nb = gridDim.x;
    const int bid = blockIdx.x;
    const int logical = (bid & 7) * (nb >> 3) + (bid >> 3);
    if (logical >= a.n_logical) return;
    const int tile = logical / a.splits;
    const int split = logical - tile * a.splits;
    const int tx = tile % a.ntile[0];
    const int tyz = tile / a.ntile[0];
    const int ty = tyz % a.ntile[1];
    const int tz = tyz / a.ntile[1];
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int X0 = tx * a.tile[0], Y0 = ty * a.tile[1], Z0 = tz * a.tile[2];
    const int ox = X0 - kLo3, oy = Y0 - kLo3, oz = Z0 - kLo3;

    for (int e = threadIdx.x; e < RC; e += blockDim.x) {
        const int lz = e / RXY;
        const int r = e - lz * RXY;
        const int ly = r / RX;
        const int lx = r - ly * RX;
        const int gx = ((ox + lx) % nx + nx) % nx;
        const int gy = ((oy + ly) % ny + ny) % ny;
        const int gz = ((oz + lz) % nz + nz) % nz;
        const size_t g = (size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sF[c * RC + e] = a.E[c][g];
            sF[(3 + c) * RC + e] = a.B[c][g];
            sJ[c * RC + e] = 0.0;
        }
    }
    __syncthreads();

    const T dtd[3] = {T(a.dt / a.dx[0]), T(a.dt / a.dx[1]), T(a.dt / a.dx[2])};
    const int nn[3] = {nx, ny, nz};
    const int org[3] = {X0, Y0, Z0};
    const int reg[3] = {RX, RY, RZ};
    const unsigned ncell = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    // stagger of each component per axis: 1 = half node
    // Ex(h,n,n) Ey(n,h,n) Ez(n,n,h) Bx(n,h,h) By(h,n,h) Bz(h,h,n)
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
        const T cj[3] = {T(-S.q * a.dx[0] / a.dt), T(-S.q * a.dx[1] / a.dt), T(-S.q * a.dx[2] / a.dt)};
        for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
            const int cell = cell_in[p];
            T off[3];
            bool ok = (unsigned)cell < ncell;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                off[c] = (c == 0 ? off_in0 : (c == 1 ? off_in1 : off_in2))[p];
                ok = ok && off[c] >= T(0) && off[c] < T(1);
            }
            T ux = u_in0[p], uy = u_in1[p], uz = u_in2[p];
            const T w = w_in[p];
            if (!ok) {
                atomicAdd(a.n_bad, 1ull);
                S.cell_out[p] = cell;
#pragma unroll
                for (int c = 0; c < 3; ++c) S.off_out[c][p] = off[c];
                S.u_out[0][p] = ux; S.u_out[1][p] = uy; S.u_out[2][p] = uz;
                if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
                if (PROXY && !INPLACE && S.proxy_out) {
                    S.proxy_out[2 * p] = S.proxy_in[2 * p];
                    S.proxy_out[2 * p + 1] = S.proxy_in[2 * p + 1];
                }
                continue;
            }
            const int row = (int)a.fnx.div((unsigned)cell);
            const int kk = (int)a.fnxy.div((unsigned)cell);
            int idx[3];
            idx[0] = cell - row * nx;
            idx[1] = row - kk * ny;
            idx[2] = kk;
            int loc[3];
            bool in_lds = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int d = idx[c] - org[c];
                const int h = nn[c] >> 1;
                if (d < -h) d += nn[c]; else if (d >= nn[c] - h) d -= nn[c];
                loc[c] = d + kLo3;
                in_lds = in_lds && loc[c] >= 2 && loc[c] <= reg[c] - 4;
            }
            wave_count(a.n_offtile, !in_lds);
            // weights: node (n) and half-node (h) per axis
            int nod[3];
            T wn[3][3], wh[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                nod[c] = off[c] >= T(0.5) ? 1 : 0;
                tsc3w(off[c] - T(nod[c]), wn[c]);
                tsc3w(off[c] - T(0.5), wh[c]);
            }
            // gather one component with staggers (sx, sy, sz)
            auto gath = [&](int comp, int sx, int sy, int sz) {
                const T *wx = sx ? wh[0] : wn[0];
                const T *wy = sy ? wh[1] : wn[1];
                const T *wz = sz ? wh[2] : wn[2];
                const int bx = sx ? -1 : nod[0] - 1;
                const int by = sy ? -1 : nod[1] - 1;
                const int bz = sz ? -1 : nod[2] - 1;
                T acc = T(0);
                if (in_lds) {
                    const T *F = sF + comp * RC;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const T *row_ = F + (loc[2] + bz + c) * RXY + (loc[1] + by + b) * RX + loc[0] + bx;
                            acc += wz[c] * wy[b] * (wx[0] * row_[0] + wx[1] * row_[1] + wx[2] * row_[2]);
                        }
                } else {
                    const T *F = comp < 3 ? a.E[comp] : a.B[comp - 3];
                    int gx[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) gx[m] = wrap3(idx[0] + bx + m, nx);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const size_t gz = (size_t)wrap3(idx[2] + bz + c, nz) * ny;
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const size_t rbase = (gz + (size_t)wrap3(idx[1] + by + b, ny)) * nx;
                            acc += wz[c] * wy[b] * (wx[0] * F[rbase + gx[0]] + wx[1] * F[rbase + gx[1]] +
                                                    wx[2] * F[rbase + gx[2]]);
                        }
                    }
                }
                return acc;
            };
            T e2[3], b2[3];
            e2[0] = gath(0, 1, 0, 0);
            e2[1] = gath(1, 0, 1, 0);
            e2[2] = gath(2, 0, 0, 1);
            b2[0] = gath(3, 0, 1, 1);
            b2[1] = gath(4, 1, 0, 1);
            b2[2] = gath(5, 1, 1, 0);

            T e1[3], b1[3];
            const double X = a.x_min[0] + ((double)idx[0] + (double)off[0]) * a.dx[0];
            const double Y = a.x_min[1] + ((double)idx[1] + (double)off[1]) * a.dx[1];
            const double Z = a.x_min[2] + ((double)idx[2] + (double)off[2]) * a.dx[2];
            analytic_field<PT, T>(a.W, X, Y, Z, e1, b1);
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

            const T ign = rsqrt_r<T>(T(1) + ux * ux + uy * uy + uz * uz);
            const T uu[3] = {ux, uy, uz};
            T nof[3];
            int sh[3];
            bool fast = false;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T d = uu[c] * ign * dtd[c];
                if (!(fabs(d) < T(1))) { d = T(0); fast = true; }
                T no = off[c] + d;
                int sc = (int)floor_r<T>(no);
                no -= T(sc);
                if (no >= T(1)) { no -= T(1); sc += 1; }
                nof[c] = no;
                sh[c] = sc;
            }
            if (fast) atomicAdd(a.n_fast, 1ull);

            // Esirkepov on the 4x4x4 window relative to the old cell
            T S0[3][4], DS[3][4];
            int base[3];
            bool moved_node = false;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int n1 = sh[c] + (nof[c] >= T(0.5) ? 1 : 0);
                moved_node = moved_node || (n1 != nod[c]);
                T w1[3];
                tsc3w(nof[c] - T(n1 - sh[c]), w1);
                base[c] = min(nod[c], n1) - 1;
                T s1[4];
                place4w(nod[c] - 1 - base[c], wn[c], S0[c]);
                place4w(n1 - 1 - base[c], w1, s1);
#pragma unroll
                for (int m = 0; m < 4; ++m) DS[c][m] = s1[m] - S0[c][m];
            }
            const T fj[3] = {cj[0] * w, cj[1] * w, cj[2] * w};
            if (in_lds) {
                // window width uniform over the wave
                const int o0 = loc[0] + base[0], o1 = loc[1] + base[1], o2 = loc[2] + base[2];
                if (__any(moved_node)) deposit_window3<4>(sJ, RC, RXY, RX, o0, o1, o2, S0, DS, fj);
                else deposit_window3<3>(sJ, RC, RXY, RX, o0, o1, o2, S0, DS, fj);
            } else {
                const T third = T(1.0 / 3.0);
                auto addJ = [&](int comp, int i4, int j4, int k4, T v) {
                    if (v == T(0)) return;
                    const int gx = wrap3(idx[0] + base[0] + i4, nx);
                    const int gy = wrap3(idx[1] + base[1] + j4, ny);
                    const int gz = wrap3(idx[2] + base[2] + k4, nz);
                    atomic_add(&a.Jacc[comp][(size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz)], (double)v);
                };
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                    for (int j4 = 0; j4 < 4; ++j4) {
                        const T cyz = S0[1][j4] * S0[2][k4] + T(0.5) * DS[1][j4] * S0[2][k4] +
                                      T(0.5) * S0[1][j4] * DS[2][k4] + third * DS[1][j4] * DS[2][k4];
                        T cum = T(0);
#pragma unroll
                        for (int i4 = 0; i4 < 3; ++i4) {
                            cum += DS[0][i4] * cyz;
                            addJ(0, i4, j4, k4, fj[0] * cum);
                        }
                    }
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                    for (int i4 = 0; i4 < 4; ++i4) {
                        const T cxz = S0[0][i4] * S0[2][k4] + T(0.5) * DS[0][i4] * S0[2][k4] +
                                      T(0.5) * S0[0][i4] * DS[2][k4] + third * DS[0][i4] * DS[2][k4];
                        T cum = T(0);
#pragma unroll
                        for (int j4 = 0; j4 < 3; ++j4) {
                            cum += DS[1][j4] * cxz;
                            addJ(1, i4, j4, k4, fj[1] * cum);
                        }
                    }
#pragma unroll
                for (int j4 = 0; j4 < 4; ++j4)
#pragma unroll
                    for (int i4 = 0; i4 < 4; ++i4) {
                        const T cxy = S0[0][i4] * S0[1][j4] + T(0.5) * DS[0][i4] * S0[1][j4] +
                                      T(0.5) * S0[0][i4] * DS[1][j4] + third * DS[0][i4] * DS[1][j4];
                        T cum = T(0);
#pragma unroll
                        for (int k4 = 0; k4 < 3; ++k4) {
                            cum += DS[2][k4] * cxy;
                            addJ(2, i4, j4, k4, fj[2] * cum);
                        }
                    }
            }

            int ni[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) ni[c] = wrap3(idx[c] + sh[c], nn[c]);
            S.cell_out[p] = ni[0] + nx * (ni[1] + ny * ni[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) S.off_out[c][p] = nof[c];
            S.u_out[0][p] = ux;
            S.u_out[1][p] = uy;
            S.u_out[2][p] = uz;
            if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[p]; }
        }
    }
    __syncthreads();

    for (int e = threadIdx.x; e < RC; e += blockDim.x) {
        const int lz = e / RXY;
        const int r = e - lz * RXY;
        const int ly = r / RX;
        const int lx = r - ly * RX;
        const int gx = ((ox + lx) % nx + nx) % nx;
        const int gy = ((oy + ly) % ny + ny) % ny;
        const int gz = ((oz + lz) % nz + nz) % nz;
        const size_t g = (size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = sJ[c * RC + e];
            if (v != 0.0) atomic_add(&a.Jacc[c][g], v);
        }
    }
}

template <typename T, int PT>
static hipError_t launch3d(const PushArgs<T> &a0, int threads, hipStream_t s) {
    const bool inplace = a0.sp[0].copy_static == 0;
    PushArgs<T> a = a0;
    for (int c = 0; c < 3; ++c) a.reg[c] = a.tile[c] + kLo3 + kHi3;
    const size_t rc = (size_t)a.reg[0] * a.reg[1] * a.reg[2];
    const size_t lds = align_lds(6 * rc * sizeof(T)) + 3 * rc * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    const int blocks = ((a.n_logical + 7) / 8) * 8;
    if (blocks == 0) return hipSuccess;
    bool proxy = false;
    for (int k = 0; k < a.nsp; ++k) proxy = proxy || a.sp[k].proxy_out != nullptr;
    if (inplace && !proxy)
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, true, false>), dim3(blocks), dim3(threads), lds, s, a);
    else if (!proxy)
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, false, false>), dim3(blocks), dim3(threads), lds, s, a);
    else if (inplace)
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, true, true>), dim3(blocks), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, false, true>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_push_deposit_3d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch3d<T, PT_NONE>(a, threads, s);
    case PT_PLANE: return launch3d<T, PT_PLANE>(a, threads, s);
    case PT_GAUSS: return launch3d<T, PT_GAUSS>(a, threads, s);
    case PT_LG: return launch3d<T, PT_LG>(a, threads, s);
    case PT_FF: return launch3d<T, PT_FF>(a, threads, s);
    case PT_NP: return launch3d<T, PT_NP>(a, threads, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_push_deposit_3d<float>(int, const PushArgs<float> &, int, hipStream_t);
template hipError_t launch_push_deposit_3d<double>(int, const PushArgs<double> &, int, hipStream_t);

}  // namespace apt
