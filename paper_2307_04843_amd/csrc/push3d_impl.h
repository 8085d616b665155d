// Fused per-particle kernel for 3-D grids (implementation; the launcher
// dispatching on the tile shape is in push3d.hip): LDS-staged gather of E2, B2 on a
// 3 x 3 x 3 quadratic stencil per staggered component, analytic E1, B1 at the
// particle, relativistic Boris push, move, and Esirkepov deposition on a
// window of 3 or 4 nodes per axis into an LDS-private FP64 J tile flushed
// with atomics.  Particles whose stencil leaves the staged region use
// global memory.
//
// The tile shape (TX, TY, TZ) is a compile-time parameter: the staged region
// (tile + 2 nodes below + 3 above per axis) then has constant strides, so
// every gather read and every deposit atomic of a particle addresses LDS as
// one per-particle base plus an immediate offset, and the staging and flush
// loops decompose node indices with constant divisors.
#pragma once

#include <type_traits>

#include "kernels.h"

namespace apt {

constexpr int kLo3 = 2;   // 3-D halo: no drift margin (LDS budget), sort often
constexpr int kHi3 = 3;

template <int TX, int TY, int TZ> struct Region3 {
    static constexpr int RX = TX + kLo3 + kHi3, RY = TY + kLo3 + kHi3, RZ = TZ + kLo3 + kHi3;
    static constexpr int RXY = RX * RY;
    static constexpr int RC = RXY * RZ;
    // the gather's inner box (nodes 1 .. R - 2 per axis), where E2, B2 are staged
    static constexpr int IX = RX - 2, IXY = IX * (RY - 2), IC = IXY * (RZ - 2);
};


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

// Periodic image of a staged node coordinate (v >= -kLo3): one subtraction
// on grids wider than the region, repeated on tiny grids.
AP_D int wrap_node(int v, int n) {
    v = v < 0 ? v + n : v;
    v = v >= n ? v - n : v;
    if (v >= n) v %= n;   // grids narrower than the staged region only
    return v;
}

// 27-point quadratic gather of one component from its LDS block at base
// (x fastest; rows RX apart, planes RXY apart: constant offsets).
template <int RX, int RXY, typename T>
AP_D T gather27(const T *F, int base, const T wx[3], const T wy[3], const T wz[3]) {
    const T *f = F + base;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T pl = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T *r = f + c * RXY + b * RX;
            pl += wy[b] * (wx[0] * r[0] + wx[1] * r[1] + wx[2] * r[2]);
        }
        acc += wz[c] * pl;
    }
    return acc;
}

// Esirkepov deposition of one particle on a WX x WY x WZ node window whose
// origin is at LDS index o (constant strides).  An axis of width 3 is exact
// when no lane of the wave changed its nearest node on it: the fourth
// weight is zero before and after the move, and so is every current term
// that involves it.  Esirkepov's W in product form,
//     W_x(i,j,k) = DS_x[i] A_x(j,k),  A_x = p_y[j] S0_z[k] + q_y[j] DS_z[k],
//     p = S0 + DS/2,  q = S0/2 + DS/3,
// makes J_x(i,j,k) = -q w dx/dt sum_{i' <= i} W_x(i',j,k) = C_x[i] A_x(j,k),
// with C_x the running sum of DS_x (scaled by -q w dx/dt) along x: one FP64
// product per node.  Likewise J_y, J_z.  In a 4-node window, a lane whose
// nearest node did not change on that axis has zero terms on the window's
// rim (last running-sum node along the flux axis, fourth node across it):
// those atomics run under the mask of the lanes that moved (`wide`).
template <int RX, int RXY, int RC, int WX, int WY, int WZ, typename T, typename JA>
AP_D void deposit3(JA *sJ, int o, const T (&S0)[3][4], const T (&DS)[3][4], const T (&fj)[3], double scale,
                   const bool (&wide)[3]) {
    constexpr int W[3] = {WX, WY, WZ};
    // running sums of DS along each axis, scaled, in FP64
    double C[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            acc += (double)DS[c][m];
            C[c][m] = acc * ((double)fj[c] * scale);
        }
    }
    JA *J = sJ + o;
    // component c (flux axis c) with transverse axes (t1, t2): node (a1, a2)
    // across, m along; strides of the flux and transverse axes
    auto comp = [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int t1 = c == 0 ? 1 : 0, t2 = c == 2 ? 1 : 2;
        constexpr int st[3] = {1, RX, RXY};
        JA *Jc = J + c * RC;
#pragma unroll
        for (int a2 = 0; a2 < W[t2]; ++a2)
#pragma unroll
            for (int a1 = 0; a1 < W[t1]; ++a1) {
                const bool rim_t = (W[t1] == 4 && a1 == 3) || (W[t2] == 4 && a2 == 3);
                if (rim_t && !((W[t1] == 4 && a1 == 3 ? wide[t1] : true) && (W[t2] == 4 && a2 == 3 ? wide[t2] : true)))
                    continue;
                const T pa = S0[t1][a1] + T(0.5) * DS[t1][a1];
                const T qa = T(0.5) * S0[t1][a1] + T(1.0 / 3.0) * DS[t1][a1];
                const double A = (double)(pa * S0[t2][a2] + qa * DS[t2][a2]);
                JA *row = Jc + a2 * st[t2] + a1 * st[t1];
#pragma unroll
                for (int m = 0; m < W[c] - 1; ++m) {
                    if (W[c] == 4 && m == 2 && !wide[c]) continue;
                    lds_add(row + m * st[c], C[c][m], A);
                }
            }
    };
    comp(std::integral_constant<int, 0>());
    comp(std::integral_constant<int, 1>());
    comp(std::integral_constant<int, 2>());
}

template <typename T, int PT, bool INPLACE, bool PROXY, int TX, int TY, int TZ>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 3 : 2) void k_push_deposit_3d(PushArgs<T> a) {
    using R = Region3<TX, TY, TZ>;
    constexpr int RX = R::RX, RXY = R::RXY, RC = R::RC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sF = reinterpret_cast<T *>(smem_raw);
    using JA = typename JTile<T>::type;
    JA *sJ = reinterpret_cast<JA *>(smem_raw + align_lds(6 * R::IC * sizeof(T)));
    __shared__ float s_red[4];
    __shared__ int s_stay[kMaxSpecies];   // fused re-sort: particles of each species staying in the tile

    // Block -> tile: the hardware hands consecutive block ids to the 8 XCDs
    // in turn.  Runs of `xcd_chunk` consecutive tiles along x go to one XCD
    // and the XCDs take neighbouring runs, so the whole chip sweeps the domain
    // together (a z-slab of tiles at a time, whose staged data stays in the
    // shared last-level cache) while each XCD keeps x- and y-neighbour tiles
    // in its own L2.
    const int bid = blockIdx.x;
    const int chunk = a.xcd_chunk;
    const int grp = (bid >> 3) / chunk, rem = (bid >> 3) - grp * chunk;
    const int logical = grp * 8 * chunk + (bid & 7) * chunk + rem;
    if (logical >= a.n_logical) return;
    const int tile = logical / a.splits;
    const int split = logical - tile * a.splits;
    const int tyz = (int)a.fntx.div((unsigned)tile);
    const int tx = tile - tyz * a.ntile[0];
    const int tz = (int)a.fntxy.div((unsigned)tile);
    const int ty = tyz - tz * a.ntile[1];
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int X0 = tx * TX, Y0 = ty * TY, Z0 = tz * TZ;
    const int ox = X0 - kLo3, oy = Y0 - kLo3, oz = Z0 - kLo3;

    // staged node e -> global node: no periodic wrap for tiles whose region
    // lies inside the grid (uniform over the block)
    const bool interior = ox >= 0 && oy >= 0 && oz >= 0 && ox + R::RX <= nx && oy + R::RY <= ny && oz + R::RZ <= nz;
    const unsigned nxy = (unsigned)nx * (unsigned)ny;
    const size_t g0 = (size_t)ox + (size_t)nx * ((size_t)oy + (size_t)ny * (size_t)oz);
    auto global_node = [&](int e) -> size_t {
        const int lz = e / RXY;
        const int rr = e - lz * RXY;
        const int ly = rr / RX;
        const int lx = rr - ly * RX;
        if (interior) return g0 + (size_t)((unsigned)lz * nxy + (unsigned)ly * (unsigned)nx + (unsigned)lx);
        return (size_t)wrap_node(ox + lx, nx) +
               (size_t)nx * ((size_t)wrap_node(oy + ly, ny) + (size_t)ny * (size_t)wrap_node(oz + lz, nz));
    };
    if (threadIdx.x < kMaxSpecies) s_stay[threadIdx.x] = 0;
    auto block_range = [&](int s, int &pb, int &pe) {
        const int beg = a.sp[s].tile_start[tile];
        const int cnt = a.sp[s].tile_start[tile + 1] - beg;
        pb = beg + (int)(((long long)cnt * split) / a.splits);
        pe = beg + (int)(((long long)cnt * (split + 1)) / a.splits);
    };
    // Latency: the record (cell, offsets, momenta, weight) of this thread's
    // first particle of species 0, the permutation entry of its first
    // particle of species 1 and the staged fields are all loaded before the
    // first wait -- permutation entries first, then the fields, then the
    // record -- and only then written to LDS.
    struct Rec {
        int q, cell;
        T off[3], u[3], w;
    };
    auto load_rec = [&](const SpeciesIO<T> &S, int q) {
        Rec r;
        r.q = q;
        r.cell = (INPLACE ? S.cell_out : S.cell_in)[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r.off[c] = (INPLACE ? S.off_out[c] : S.off_in[c])[q];
            r.u[c] = (INPLACE ? S.u_out[c] : S.u_in[c])[q];
        }
        r.w = (INPLACE ? S.w_out : S.w_in)[q];
        return r;
    };
    auto first_slot = [&](int s, int &q) {
        int pb, pe;
        block_range(s, pb, pe);
        const int p = pb + (int)threadIdx.x;
        if (p >= pe) return false;
        q = (INPLACE || !a.sp[s].perm) ? p : a.sp[s].perm[p];
        return true;
    };
    // (FP32 runs: the FP64 kernels have no registers to spare for it)
    constexpr bool PREFETCH = std::is_same<T, float>::value;
    int q0 = 0, q1 = 0;
    const bool has0 = PREFETCH && a.nsp > 0 && first_slot(0, q0);
    const bool has1 = PREFETCH && a.nsp > 1 && first_slot(1, q1);
    // E2, B2 are staged on the region's inner box only (nodes 1 .. R - 2 per
    // axis): the gather of a particle in the tile reads one node below its
    // cell and two above, while the deposit's window (the J tile, the whole
    // region) reaches one further on each side
    constexpr int IX = R::IX, IXY = R::IXY, IC = R::IC;
    constexpr int NIT = (IC + 255) / 256;   // launched with 256 threads
    auto inner_node = [&](int f) {
        const int fz = f / IXY;
        const int fr = f - fz * IXY;
        const int fy = fr / IX;
        return (fz + 1) * RXY + (fy + 1) * RX + (fr - fy * IX + 1);
    };
    T sv[NIT][6];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int f = (int)threadIdx.x + 256 * k;
        if (f < IC) {
            const size_t g = global_node(inner_node(f));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sv[k][c] = a.E[c][g];
                sv[k][3 + c] = a.B[c][g];
            }
        }
    }
    Rec pre0{};
    if (has0) pre0 = load_rec(a.sp[0], q0);
    Rec pre1{};
    if (has1) pre1 = load_rec(a.sp[1], q1);
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int f = (int)threadIdx.x + 256 * k;
        if (f < IC) {
#pragma unroll
            for (int c = 0; c < 6; ++c) sF[c * IC + f] = sv[k][c];
        }
    }
    for (int e = (int)threadIdx.x; e < RC; e += 256) {
#pragma unroll
        for (int c = 0; c < 3; ++c) sJ[c * RC + e] = JA(0);
    }
    // fixed-point scale of the block's current tile (FP32 runs): from the
    // largest |q w| of its particles (non-finite weights belong to skipped
    // particles) and its particle count
    double scale = 1.0, inv_scale = 1.0;
    if constexpr (std::is_same<T, float>::value) {
        float qw = 0.f;
        int count = 0;
        for (int s = 0; s < a.nsp; ++s) {
            int pb, pe;
            block_range(s, pb, pe);
            count += pe - pb;
            const float qa = fabsf((float)a.sp[s].q);
            const T *w_in = INPLACE ? a.sp[s].w_out : a.sp[s].w_in;
            const int32_t *perm = INPLACE ? nullptr : a.sp[s].perm;
            for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
                const bool first = PREFETCH && p == pb + (int)threadIdx.x;
                const T wv = first && s == 0 ? pre0.w : (first && s == 1 ? pre1.w : w_in[perm ? perm[p] : p]);
                const float v = qa * fabsf((float)wv);
                if (__builtin_isfinite(v)) qw = fmaxf(qw, v);
            }
        }
        for (int d = 32; d > 0; d >>= 1) qw = fmaxf(qw, __shfl_xor(qw, d, 64));
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = qw;
        __syncthreads();
        qw = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
        const double fbound = (double)qw * fmax(a.dx[0], fmax(a.dx[1], a.dx[2])) / a.dt;
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

    const T dtd[3] = {T(a.dt / a.dx[0]), T(a.dt / a.dx[1]), T(a.dt / a.dx[2])};
    const int nn[3] = {nx, ny, nz};
    const int org[3] = {X0, Y0, Z0};
    constexpr int reg[3] = {R::RX, R::RY, R::RZ};
    const unsigned ncell = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    // stagger of each component per axis (1 = half node):
    // Ex(h,n,n) Ey(n,h,n) Ez(n,n,h) Bx(n,h,h) By(h,n,h) Bz(h,h,n)
    for (int s = 0; s < a.nsp; ++s) {
        const SpeciesIO<T> &S = a.sp[s];
        int pb, pe;
        block_range(s, pb, pe);
        const T kap = T(0.5 * S.q_over_m * a.dt);
        const T cj[3] = {T(-S.q * a.dx[0] / a.dt), T(-S.q * a.dx[1] / a.dt), T(-S.q * a.dx[2] / a.dt)};
        // fused re-sort: rank of the particle in the tile of its new cell,
        // stayers of this block counted per wave (their order is kept); the
        // others are only counted in the tile they enter
        auto emit_key = [&](int p, int tnew) {
            const int lane = (int)(threadIdx.x & 63);
            const bool st = tnew == tile;
            const unsigned long long act = __ballot(1);
            const unsigned long long m = __ballot(st);
            const int leader = __ffsll((long long)act) - 1;
            int base = 0;
            if (lane == leader && m != 0ull) base = atomicAdd(&s_stay[s], (int)__popcll(m));
            base = __shfl(base, leader, 64);
            int key = -1;   // a particle changing tile takes its rank in the permutation kernel
            if (st) key = base + (int)__popcll(m & ((1ull << lane) - 1ull));
            else atomicAdd(&S.mcount[tnew], 1);   // no return value: the wave does not wait for it
            S.key_out[p] = key;
        };
        auto tile_of3 = [&](int i, int j, int k) { return i / TX + a.ntile[0] * (j / TY + a.ntile[1] * (k / TZ)); };
        // p: output slot; q: input slot (the previous order through perm)
        for (int p = pb + (int)threadIdx.x; p < pe; p += blockDim.x) {
            const bool first = PREFETCH && p == pb + (int)threadIdx.x;
            const Rec r = first && s == 0 ? pre0 : (first && s == 1 ? pre1 : load_rec(S, INPLACE || !S.perm ? p : S.perm[p]));
            const int q = r.q;
            const int cell = r.cell;
            T off[3];
            bool ok = (unsigned)cell < ncell;
            off[0] = r.off[0];
            off[1] = r.off[1];
            off[2] = r.off[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) ok = ok && off[c] >= T(0) && off[c] < T(1);
            T ux = r.u[0], uy = r.u[1], uz = r.u[2];
            const T w = r.w;
            ok = ok && finite_state(ux, uy, uz, w);
            if (!ok) {
                count_skipped(a.n_bad, cell);
                S.cell_out[p] = cell;
#pragma unroll
                for (int c = 0; c < 3; ++c) S.off_out[c][p] = off[c];
                S.u_out[0][p] = ux; S.u_out[1][p] = uy; S.u_out[2][p] = uz;
                if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[q]; }
                if (PROXY && !INPLACE && S.proxy_out) {
                    S.proxy_out[2 * p] = S.proxy_in[2 * q];
                    S.proxy_out[2 * p + 1] = S.proxy_in[2 * q + 1];
                }
                if (!INPLACE && S.key_out) {
                    int tnew = dead_tile(p, a.ntile[0] * a.ntile[1] * a.ntile[2]);
                    if ((unsigned)cell < ncell) {
                        const int r = (int)a.fnx.div((unsigned)cell), k = (int)a.fnxy.div((unsigned)cell);
                        tnew = tile_of3(cell - r * nx, r - k * ny, k);
                    }
                    emit_key(p, tnew);
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
            T e2[3], b2[3];
            if (in_lds) {
                // stencil starts on the node (n) and half-node (h) lattice of each axis
                // stencil starts in the inner box (region node - 1 per axis)
                const int xn = loc[0] + nod[0] - 2, xh = loc[0] - 2;
                const int yn = (loc[1] + nod[1] - 2) * IX, yh = (loc[1] - 2) * IX;
                const int zn = (loc[2] + nod[2] - 2) * IXY, zh = (loc[2] - 2) * IXY;
                e2[0] = gather27<IX, IXY>(sF + 0 * IC, xh + yn + zn, wh[0], wn[1], wn[2]);
                e2[1] = gather27<IX, IXY>(sF + 1 * IC, xn + yh + zn, wn[0], wh[1], wn[2]);
                e2[2] = gather27<IX, IXY>(sF + 2 * IC, xn + yn + zh, wn[0], wn[1], wh[2]);
                b2[0] = gather27<IX, IXY>(sF + 3 * IC, xn + yh + zh, wn[0], wh[1], wh[2]);
                b2[1] = gather27<IX, IXY>(sF + 4 * IC, xh + yn + zh, wh[0], wn[1], wh[2]);
                b2[2] = gather27<IX, IXY>(sF + 5 * IC, xh + yh + zn, wh[0], wh[1], wn[2]);
            } else {
                auto gath = [&](int comp, int sx, int sy, int sz) {
                    const T *wx = sx ? wh[0] : wn[0];
                    const T *wy = sy ? wh[1] : wn[1];
                    const T *wz = sz ? wh[2] : wn[2];
                    const int bx = sx ? -1 : nod[0] - 1;
                    const int by = sy ? -1 : nod[1] - 1;
                    const int bz = sz ? -1 : nod[2] - 1;
                    const T *F = comp < 3 ? a.E[comp] : a.B[comp - 3];
                    int gx[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) gx[m] = wrap3(idx[0] + bx + m, nx);
                    T acc = T(0);
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
                    return acc;
                };
                e2[0] = gath(0, 1, 0, 0);
                e2[1] = gath(1, 0, 1, 0);
                e2[2] = gath(2, 0, 0, 1);
                b2[0] = gath(3, 0, 1, 1);
                b2[1] = gath(4, 1, 0, 1);
                b2[2] = gath(5, 1, 1, 0);
            }

            T e1[3], b1[3];
            const double X = a.x_min[0] + ((double)win_col(idx[0], a.xo, a.n[0]) + (double)off[0]) * a.dx[0];
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
                    proxy_accumulate<T>((INPLACE ? S.proxy_out : S.proxy_in) + 2 * q, S.proxy_out + 2 * p, uv0, uv1,
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
                if (!push_move_ok(ign, d)) { d = T(0); fast = true; }
                T no = off[c] + d;
                int sc = (int)floor_r<T>(no);
                no -= T(sc);
                if (no >= T(1)) { no -= T(1); sc += 1; }
                nof[c] = no;
                sh[c] = sc;
            }
            if (fast) atomicAdd(a.n_fast, 1ull);

            // Esirkepov on a window relative to the old cell
            T S0[3][4], DS[3][4];
            int base[3];
            bool wide[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int n1 = sh[c] + (nof[c] >= T(0.5) ? 1 : 0);
                wide[c] = n1 != nod[c];
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
                // window width per axis, uniform over the wave
                const int o = (loc[2] + base[2]) * RXY + (loc[1] + base[1]) * RX + loc[0] + base[0];
                const int wmask = (__any(wide[0]) ? 1 : 0) | (__any(wide[1]) ? 2 : 0) | (__any(wide[2]) ? 4 : 0);
                switch (wmask) {
                case 0: deposit3<RX, RXY, RC, 3, 3, 3>(sJ, o, S0, DS, fj, scale, wide); break;
                case 1: deposit3<RX, RXY, RC, 4, 3, 3>(sJ, o, S0, DS, fj, scale, wide); break;
                case 2: deposit3<RX, RXY, RC, 3, 4, 3>(sJ, o, S0, DS, fj, scale, wide); break;
                case 3: deposit3<RX, RXY, RC, 4, 4, 3>(sJ, o, S0, DS, fj, scale, wide); break;
                case 4: deposit3<RX, RXY, RC, 3, 3, 4>(sJ, o, S0, DS, fj, scale, wide); break;
                case 5: deposit3<RX, RXY, RC, 4, 3, 4>(sJ, o, S0, DS, fj, scale, wide); break;
                case 6: deposit3<RX, RXY, RC, 3, 4, 4>(sJ, o, S0, DS, fj, scale, wide); break;
                default: deposit3<RX, RXY, RC, 4, 4, 4>(sJ, o, S0, DS, fj, scale, wide); break;
                }
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
            if (!INPLACE) { S.w_out[p] = w; S.id_out[p] = S.id_in[q]; }
            if (!INPLACE && S.key_out) emit_key(p, tile_of3(ni[0], ni[1], ni[2]));
        }
    }
    __syncthreads();
    if (!INPLACE && (int)threadIdx.x < a.nsp && a.sp[threadIdx.x].key_out) a.sp[threadIdx.x].stay[tile] = s_stay[threadIdx.x];

    for (int e = threadIdx.x; e < RC; e += blockDim.x) {
        const size_t g = global_node(e);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = lds_value(sJ[c * RC + e], inv_scale);
            if (v != 0.0) atomic_add(&a.Jacc[c][g], v);
        }
    }
}

template <int TX, int TY, int TZ> constexpr size_t lds3(size_t real) {
    return align_lds(6 * (size_t)Region3<TX, TY, TZ>::IC * real) +
           3 * (size_t)Region3<TX, TY, TZ>::RC * sizeof(double);
}

template <typename T, int PT, int TX, int TY, int TZ>
hipError_t launch3d_shape(const PushArgs<T> &a, int threads, hipStream_t s) {
    if (a.n_logical == 0) return hipSuccess;
    if (threads != 256) return hipErrorInvalidValue;   // the block reductions assume four waves
    const size_t lds = lds3<TX, TY, TZ>(sizeof(T));
    const int per = 8 * a.xcd_chunk;
    const int blocks = ((a.n_logical + per - 1) / per) * per;
    // every 3-D push reads a freshly sorted copy or goes through the
    // re-sort permutation: the in-place instantiation is not needed (an
    // in-place call is still correct: each slot is read and written by one thread)
    bool proxy = false;
    for (int k = 0; k < a.nsp; ++k) proxy = proxy || a.sp[k].proxy_out != nullptr;
    if (!proxy)
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, false, false, TX, TY, TZ>), dim3(blocks), dim3(threads), lds, s,
                           a);
    else
        hipLaunchKernelGGL((k_push_deposit_3d<T, PT, false, true, TX, TY, TZ>), dim3(blocks), dim3(threads), lds, s,
                           a);
    return hipGetLastError();
}

// Every pulse family of one tile shape (instantiated per shape in its own
// translation unit: push3d_t844.hip, push3d_t884.hip, push3d_t888.hip).
template <typename T, int TX, int TY, int TZ>
hipError_t launch3d_tile(int pulse, const PushArgs<T> &a, int threads, hipStream_t s) {
    switch (pulse) {
    case PT_NONE: return launch3d_shape<T, PT_NONE, TX, TY, TZ>(a, threads, s);
    case PT_PLANE: return launch3d_shape<T, PT_PLANE, TX, TY, TZ>(a, threads, s);
    case PT_GAUSS: return launch3d_shape<T, PT_GAUSS, TX, TY, TZ>(a, threads, s);
    case PT_LG: return launch3d_shape<T, PT_LG, TX, TY, TZ>(a, threads, s);
    case PT_FF: return launch3d_shape<T, PT_FF, TX, TY, TZ>(a, threads, s);
    case PT_NP: return launch3d_shape<T, PT_NP, TX, TY, TZ>(a, threads, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace apt
