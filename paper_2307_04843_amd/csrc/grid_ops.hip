// Grid-side kernels: Yee update of E2, B2 only, J clear, tile sort,
// FP64 diagnostics (moments, energies, charge density, continuity residual).
#include <algorithm>
#include <climits>
#include <cstdint>

#include "kernels.h"

namespace apt {

// ---------------------------------------------------------------------------
// Yee update (Sec. II.A, Eqs. (7)-(9) generalised to 2-D/3-D; Eq. (4): the
// update acts on the internal fields only, driven by the particle current).
// Split step: B <- B - (dt/2) curl E; E <- E + dt (curl B - J); B <- B - (dt/2) curl E.
// Component order in F: Ex Ey Ez Bx By Bz Jx Jy Jz, each nx*ny*nz, x fastest.
// ---------------------------------------------------------------------------
struct YeeIdx {
    int nx, ny, nz;
    FastDiv fnx, fny;
};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_yee_b(T *__restrict__ Ex, T *__restrict__ Ey, T *__restrict__ Ez,
                                              T *__restrict__ Bx, T *__restrict__ By, T *__restrict__ Bz,
                                              YeeIdx g, T hx, T hy, T hz, size_t ncell, int open_x) {
    // hx = (dt/2)/dx etc.
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < ncell; c += (size_t)gridDim.x * blockDim.x) {
        const uint32_t cc = (uint32_t)c;
        const uint32_t row = g.fnx.div(cc);
        const int i = (int)(cc - row * g.nx);
        const int ip = (i + 1 == g.nx) ? -(g.nx - 1) : 1;
        int j = 0, k, jp = 0;
        if (DIM == 3) {
            const uint32_t kk = g.fny.div(row);
            j = (int)(row - kk * g.ny);
            k = (int)kk;
            jp = (j + 1 == g.ny) ? -(g.ny - 1) * g.nx : g.nx;
        } else {
            k = (int)row;
        }
        const long slab = (long)g.nx * g.ny;
        const long kp = (k + 1 == g.nz) ? -(long)(g.nz - 1) * slab : slab;
        const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
        // curl E at the B locations (forward differences)
        T cx = -(Ey[c + kp] - ey) * hz;
        T cy = (Ex[c + kp] - ex) * hz - (Ez[c + ip] - ez) * hx;
        T cz = (Ey[c + ip] - ey) * hx;
        if (DIM == 3) {
            cx += (Ez[c + jp] - ez) * hy;
            cz -= (Ex[c + jp] - ex) * hy;
        }
        Bx[c] -= cx;
        // open x ends: the transverse B nodes at nx - 1/2 lie outside the domain
        const bool ghost = open_x && i == g.nx - 1;
        By[c] = ghost ? T(0) : By[c] - cy;
        Bz[c] = ghost ? T(0) : Bz[c] - cz;
        (void)j;
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_yee_e(T *__restrict__ Ex, T *__restrict__ Ey, T *__restrict__ Ez,
                                              const T *__restrict__ Bx, const T *__restrict__ By,
                                              const T *__restrict__ Bz, const T *__restrict__ Jx,
                                              const T *__restrict__ Jy, const T *__restrict__ Jz,
                                              YeeIdx g, T cx_, T cy_, T cz_, T dt, size_t ncell,
                                              int open_x, const T *__restrict__ src, T r) {
    // c*_ = dt/dx etc.; r = dx/dt
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < ncell; c += (size_t)gridDim.x * blockDim.x) {
        const uint32_t cc = (uint32_t)c;
        const uint32_t row = g.fnx.div(cc);
        const int i = (int)(cc - row * g.nx);
        const int im = (i == 0) ? (g.nx - 1) : -1;
        int k, jm = 0;
        if (DIM == 3) {
            const uint32_t kk = g.fny.div(row);
            const int j = (int)(row - kk * g.ny);
            k = (int)kk;
            jm = (j == 0) ? (g.ny - 1) * g.nx : -g.nx;
        } else {
            k = (int)row;
        }
        const long slab = (long)g.nx * g.ny;
        const long km = (k == 0) ? (long)(g.nz - 1) * slab : -slab;
        const T bx = Bx[c], by = By[c], bz = Bz[c];
        // curl B at the E locations (backward differences)
        T qx = -(by - By[c + km]) * cz_;
        T qy = (bx - Bx[c + km]) * cz_ - (bz - Bz[c + im]) * cx_;
        T qz = (by - By[c + im]) * cx_;
        if (DIM == 3) {
            qx += (bz - Bz[c + jm]) * cy_;
            qz -= (bx - Bx[c + jm]) * cy_;
        }
        const T ey = Ey[c], ez = Ez[c];
        T ny = ey + (qy - dt * Jy[c]), nz = ez + (qz - dt * Jz[c]);
        if (open_x && (i == 0 || i == g.nx - 1)) {
            // App. B: Ampere's law with the outside B node and the step-averaged
            // incoming-wave condition (x_min: E_y + B_z = 2 S_y, E_z - B_y = 2 S_z;
            // x_max: no incoming wave), solved for the new boundary E; J is not
            // applied at the boundary nodes
            const T ir = T(1) / (T(1) + r), rm = r - T(1);
            if (i == 0) {
                // one source pair per row of x nodes (the row index is j + ny k)
                const T sy = src ? src[2 * row] : T(0), sz = src ? src[2 * row + 1] : T(0);
                ny = (T(4) * sy - T(2) * bz + rm * ey) * ir;
                nz = (T(4) * sz + T(2) * by + rm * ez) * ir;
            } else {
                ny = (T(2) * Bz[c - 1] + rm * ey) * ir;
                nz = (rm * ez - T(2) * By[c - 1]) * ir;
            }
        }
        Ex[c] += qx - dt * Jx[c];
        Ey[c] = ny;
        Ez[c] = nz;
    }
}

static int grid_blocks(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (int)(b == 0 ? 1 : b);
}
// One thread per cell for the Yee stencils (their grid-stride loops run
// once): more loads in flight than a capped grid whose threads stride over
// the cells, measured 26 % faster on 268M cells.
static int cell_blocks(size_t n) {
    const size_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 0x7fffffff ? 0x7fffffff : b));
}

template <typename T>
hipError_t launch_yee(int dim, T *const F[9], const YeeArgsBase &a, int no_yee, hipStream_t s) {
    if (no_yee) return hipSuccess;
    YeeIdx g;
    g.nx = a.n[0];
    g.ny = dim == 3 ? a.n[1] : 1;
    g.nz = a.n[2];
    g.fnx = FastDiv((uint32_t)g.nx);
    g.fny = FastDiv((uint32_t)g.ny);
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    const int blocks = cell_blocks(ncell);
    // 1-D rows: the (x, z) kernels with no z derivative, so rows do not couple
    const T hx = T(0.5 * a.dt / a.dx[0]), hy = T(0.5 * a.dt / a.dx[1]);
    const T hz = dim == 1 ? T(0) : T(0.5 * a.dt / a.dx[2]);
    const T cx = T(a.dt / a.dx[0]), cy = T(a.dt / a.dx[1]);
    const T cz = dim == 1 ? T(0) : T(a.dt / a.dx[2]);
    const int ox = a.open_x ? 1 : 0;
    const T *src = static_cast<const T *>(a.src);
    const T r = T(a.dx[0] / a.dt);
    if (dim == 3) {
        hipLaunchKernelGGL((k_yee_b<T, 3>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], g, hx, hy, hz, ncell, ox);
        hipLaunchKernelGGL((k_yee_e<T, 3>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], F[6], F[7], F[8], g, cx, cy, cz, T(a.dt), ncell, ox, src, r);
        hipLaunchKernelGGL((k_yee_b<T, 3>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], g, hx, hy, hz, ncell, ox);
    } else {
        hipLaunchKernelGGL((k_yee_b<T, 2>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], g, hx, hy, hz, ncell, ox);
        hipLaunchKernelGGL((k_yee_e<T, 2>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], F[6], F[7], F[8], g, cx, cy, cz, T(a.dt), ncell, ox, src, r);
        hipLaunchKernelGGL((k_yee_b<T, 2>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], g, hx, hy, hz, ncell, ox);
    }
    return hipGetLastError();
}
template hipError_t launch_yee<float>(int, float *const[9], const YeeArgsBase &, int, hipStream_t);
template hipError_t launch_yee<double>(int, double *const[9], const YeeArgsBase &, int, hipStream_t);

// Reverse of the split Yee step (B half, E full, B half) for the adjoints
// (lE, lB) of (E, B).  The discrete curls are transposes of each other
// (C_B = C_E^T on a periodic Yee grid), so the transposed step is
//     lE <- lE - (dt/2) C_B lB;   lJt = lE;   lB <- lB + dt C_E lE;   lE <- lE - (dt/2) C_B lB
// with dL/dJ^{n+1/2} = -dt lJt.  The forward kernels run it with negated
// coefficients (k_yee_e adds c C_B B - dt J: here c = -(dt/2)/dx and no J;
// k_yee_b subtracts h C_E E: here h = -dt/dx).
hipError_t launch_yee_adjoint(int dim, double *lE, double *lB, double *lJt, const YeeArgsBase &a, hipStream_t s) {
    YeeIdx g;
    g.nx = a.n[0];
    g.ny = dim == 3 ? a.n[1] : 1;
    g.nz = a.n[2];
    g.fnx = FastDiv((uint32_t)g.nx);
    g.fny = FastDiv((uint32_t)g.ny);
    const size_t nc = (size_t)g.nx * g.ny * g.nz;
    const int blocks = cell_blocks(nc);
    double *E0 = lE, *E1 = lE + nc, *E2 = lE + 2 * nc, *B0 = lB, *B1 = lB + nc, *B2 = lB + 2 * nc;
    const double ex = -0.5 * a.dt / a.dx[0], ey = -0.5 * a.dt / a.dx[1], ez = dim == 1 ? 0.0 : -0.5 * a.dt / a.dx[2];
    const double bx = -a.dt / a.dx[0], by = -a.dt / a.dx[1], bz = dim == 1 ? 0.0 : -a.dt / a.dx[2];
    if (dim == 3) {
        hipLaunchKernelGGL((k_yee_e<double, 3>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, lJt, lJt + nc, lJt + 2 * nc, g, ex, ey, ez, 0.0, nc, 0, (const double *)nullptr, 1.0);
    } else {
        hipLaunchKernelGGL((k_yee_e<double, 2>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, lJt, lJt + nc, lJt + 2 * nc, g, ex, ey, ez, 0.0, nc, 0, (const double *)nullptr, 1.0);
    }
    hipError_t e = hipMemcpyAsync(lJt, lE, 3 * nc * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if (dim == 3) {
        hipLaunchKernelGGL((k_yee_b<double, 3>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, g, bx, by, bz, nc, 0);
        hipLaunchKernelGGL((k_yee_e<double, 3>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, lJt, lJt + nc, lJt + 2 * nc, g, ex, ey, ez, 0.0, nc, 0, (const double *)nullptr, 1.0);
    } else {
        hipLaunchKernelGGL((k_yee_b<double, 2>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, g, bx, by, bz, nc, 0);
        hipLaunchKernelGGL((k_yee_e<double, 2>), dim3(blocks), dim3(256), 0, s, E0, E1, E2, B0, B1, B2, lJt, lJt + nc, lJt + 2 * nc, g, ex, ey, ez, 0.0, nc, 0, (const double *)nullptr, 1.0);
    }
    return hipGetLastError();
}

template <typename T> __global__ void k_fill_zero(T *p, size_t n) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        p[c] = T(0);
}
template <typename T> hipError_t launch_fill_zero(T *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(grid_blocks(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
template hipError_t launch_fill_zero<float>(float *, size_t, hipStream_t);
template hipError_t launch_fill_zero<double>(double *, size_t, hipStream_t);
template hipError_t launch_fill_zero<int32_t>(int32_t *, size_t, hipStream_t);
template hipError_t launch_fill_zero<unsigned long long>(unsigned long long *, size_t, hipStream_t);
template hipError_t launch_fill_zero<uint32_t>(uint32_t *, size_t, hipStream_t);

// Emission proxy of each particle: its compensated pair (sum s, compensation
// c) read out as the FP64 value s - c, in slot order.
template <typename T> __global__ void k_proxy_value(const T *pair, double *out, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[p] = (double)pair[2 * p] - (double)pair[2 * p + 1];
}
template <typename T> hipError_t launch_proxy_value(const T *pair, double *out, int n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_proxy_value<T>), dim3((n + 255) / 256), dim3(256), 0, s, pair, out, n);
    return hipGetLastError();
}
template hipError_t launch_proxy_value<float>(const float *, double *, int, hipStream_t);
template hipError_t launch_proxy_value<double>(const double *, double *, int, hipStream_t);

template <typename T> __global__ void k_round_current(const double *jacc, T *J, size_t n) {
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x)
        J[c] = T(jacc[c]);
}
template <typename T> hipError_t launch_round_current(const double *jacc, T *J, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_round_current<T>), dim3(grid_blocks(n)), dim3(256), 0, s, jacc, J, n);
    return hipGetLastError();
}
template hipError_t launch_round_current<float>(const double *, float *, size_t, hipStream_t);
template hipError_t launch_round_current<double>(const double *, double *, size_t, hipStream_t);

// ---------------------------------------------------------------------------
// Tile sort: counting sort of particles by tile id (rank from a wave-
// aggregated atomic, exclusive scan of the counts, scatter).
// ---------------------------------------------------------------------------
AP_D int tile_of(int cell, int dim, const FastDiv &fnx, const FastDiv &fnxy, const FastDiv &ftx,
                 const FastDiv &fty, const FastDiv &ftz, const int32_t *ntile) {
    const uint32_t c = (uint32_t)cell;
    const uint32_t row = fnx.div(c);
    const uint32_t i = c - row * fnx.d;
    uint32_t j = 0, k = row;
    if (dim == 3) {
        k = fnxy.div(c);
        j = row - k * (fnxy.d / fnx.d);
    }
    const int tx = (int)ftx.div(i), tz = (int)ftz.div(k);
    const int ty = dim == 3 ? (int)fty.div(j) : 0;
    return tx + ntile[0] * (ty + ntile[1] * tz);
}

// Tile histogram and each particle's rank within its tile.  Lanes of a wave
// with equal tiles are grouped (ballot); the block's four waves then combine
// their groups per tile in LDS, so that one global atomic per (block, tile)
// hands out the block's slots (sorted input puts a block in one to three
// tiles).  Tiles more than kAggSlots above the block's smallest take a global
// atomic per wave group.  Within a block the ranks follow wave then lane order.
constexpr int kAggSlots = 32;

__global__ __launch_bounds__(256) void k_tile_count(SortArgs a) {
    __shared__ int s_cnt[4][kAggSlots];
    __shared__ int s_base[kAggSlots];
    __shared__ int s_min[4];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int key = -1;
    if (p < a.n) {
        const int cell = a.cell[p];
        key = (unsigned)cell < a.ncell ? tile_of(cell, a.dim, a.fnx, a.fnxy, a.ftx, a.fty, a.ftz, a.ntile)
                                       : dead_tile(p, a.ntile[0] * a.ntile[1] * a.ntile[2]);
    }
    int km = key >= 0 ? key : INT_MAX;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) km = min(km, __shfl_xor(km, off, 64));
    if (lane == 0) s_min[wid] = km;
    for (int e = threadIdx.x; e < 4 * kAggSlots; e += blockDim.x) s_cnt[e / kAggSlots][e % kAggSlots] = 0;
    __syncthreads();
    const int key0 = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
    int slot = -1, local = 0;
    unsigned long long active = __ballot(key >= 0);
    while (active) {
        const int leader = __ffsll((long long)active) - 1;
        const int lkey = __shfl(key, leader, 64);
        const unsigned long long match = __ballot(key == lkey) & active;
        const bool mine = key == lkey && ((match >> lane) & 1ull);
        const int below = __popcll(match & ((1ull << lane) - 1ull));
        const int sl = lkey - key0;
        if (sl < kAggSlots) {
            if (lane == leader) s_cnt[wid][sl] = __popcll(match);
            if (mine) {
                slot = sl;
                local = below;
            }
        } else {
            int base = 0;
            if (lane == leader) base = atomicAdd(&a.count[lkey], __popcll(match));
            base = __shfl(base, leader, 64);
            if (mine) a.rank[p] = base + below;
        }
        active &= ~match;
    }
    __syncthreads();
    if (threadIdx.x < kAggSlots) {
        const int sl = threadIdx.x;
        int run = 0;
        for (int w = 0; w < 4; ++w) {
            const int c = s_cnt[w][sl];
            s_cnt[w][sl] = run;
            run += c;
        }
        s_base[sl] = run > 0 ? atomicAdd(&a.count[key0 + sl], run) : 0;
    }
    __syncthreads();
    if (slot >= 0) a.rank[p] = s_base[slot] + s_cnt[wid][slot] + local;
}

hipError_t launch_tile_count(const SortArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_count, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Exclusive scan of n counts into start[0..n] by one workgroup of 1024
// threads, each owning a contiguous chunk (the top level of launch_scan).
__global__ __launch_bounds__(1024) void k_scan(const int32_t *count, int32_t *start, int32_t n) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = t * chunk;
    const int e = min(n, b + chunk);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += count[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
    for (int i = b; i < e; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == 1023) start[n] = part[1023];
}

// Two-level scan for many tiles: each block of 1024 threads owns kScanChunk
// consecutive counts (4 per thread).
constexpr int kScanChunk = 4096;

// Exclusive scan of one int per thread over a 1024-thread block; returns the
// block total through *total.
AP_D int block_exclusive_scan(int v, int *sh, int *total) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int w = 0; w < 16; ++w) {
            const int c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[16] = run;
    }
    __syncthreads();
    const int out = sh[wid] + x - v;
    *total = sh[16];
    return out;
}

__global__ __launch_bounds__(1024) void k_scan_part(const int32_t *count, int32_t n, int32_t *part) {
    __shared__ int sh[17];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * 4;
    int v = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (base + m < n) v += count[base + m];
    int total;
    block_exclusive_scan(v, sh, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_final(const int32_t *count, int32_t n, const int32_t *part_start,
                                                     int32_t *start) {
    __shared__ int sh[17];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * 4;
    int c[4], v = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c[m] = base + m < n ? count[base + m] : 0;
        v += c[m];
    }
    int total;
    int run = part_start[blockIdx.x] + block_exclusive_scan(v, sh, &total);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (base + m < n) start[base + m] = run;
        run += c[m];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) start[n] = part_start[gridDim.x];
}

int32_t scan_part_len(int32_t n_tiles) { return (n_tiles + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_scan(const int32_t *count, int32_t *start, int32_t n_tiles, int32_t *part, hipStream_t s) {
    if (n_tiles <= kScanChunk) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, count, start, n_tiles);
        return hipGetLastError();
    }
    // part: [nb] block totals, then [nb + 1] their exclusive scan
    const int nb = (n_tiles + kScanChunk - 1) / kScanChunk;
    int32_t *part_start = part + nb;
    hipLaunchKernelGGL(k_scan_part, dim3(nb), dim3(1024), 0, s, count, n_tiles, part);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, part, part_start, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(1024), 0, s, count, n_tiles, part_start, start);
    return hipGetLastError();
}

// ---- moving window (Sec. III.C): ring along x, a shift moves the origin

template <typename T> AP_D bool window_leaves(const WindowArgs<T> &a, int cell) {
    return (unsigned)cell < a.ncell && cell - (int)a.fnx.div((uint32_t)cell) * a.nx == a.col;
}

// Wave-aggregated count of the lanes where f holds.
AP_D void wave_count(bool f, unsigned long long *count) {
    const unsigned long long b = __ballot(f);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

template <typename T> __global__ __launch_bounds__(256) void k_window_init(WindowArgs<T> a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false, free_slot = false;
    if (p < a.n) {
        const int id = a.id[p];
        bad = (unsigned)id >= (unsigned)a.n;
        free_slot = !bad && a.cell[p] == kDeadCell;
        if (free_slot) {
            atomicOr(&a.freemap[id >> 5], 1u << (id & 31));
            a.free_slot[id] = p;
        }
    }
    wave_count(bad, a.count);
    wave_count(free_slot, a.count_free);
}

template <typename T> __global__ __launch_bounds__(256) void k_window_check_inject(WindowArgs<T> a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_inj) return;
    const int cell = a.in_cell[r];
    bool ok = (unsigned)cell < a.ncell && cell - (int)a.fnx.div((uint32_t)cell) * a.nx == a.in_col;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (a.in_off[k]) ok = ok && a.in_off[k][r] >= T(0) && a.in_off[k][r] < T(1);
    if (!ok) atomicAdd(a.count, 1ull);
}

template <typename T> __global__ __launch_bounds__(256) void k_window_count_leavers(WindowArgs<T> a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    wave_count(p < a.n && window_leaves(a, a.cell[p]), a.count);
}

// A particle in the leaving column falls behind the window: its slot is
// freed (state zeroed), its id joins the free ids and records the slot.
template <typename T> AP_D void window_free(const WindowArgs<T> &a, int p) {
    a.cell[p] = kDeadCell;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (a.off[k]) a.off[k][p] = T(0);
        a.u[k][p] = T(0);
    }
    a.w[p] = T(0);
    if (a.proxy) {
        a.proxy[2 * p] = T(0);
        a.proxy[2 * p + 1] = T(0);
    }
    const int id = a.id[p];
    atomicOr(&a.freemap[id >> 5], 1u << (id & 31));
    a.free_slot[id] = p;
}

// Grid-stride pass over the cells, four per 16-byte load when the array is
// 16-byte aligned (leavers are rare: one column of the window).
template <typename T> __global__ __launch_bounds__(256) void k_window_leave(WindowArgs<T> a, int vec) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    int cnt = 0;
    int done = 0;
    if (vec) {
        const int nq = a.n >> 2;
        const int4 *c4 = reinterpret_cast<const int4 *>(a.cell);
        for (int q = g; q < nq; q += stride) {
            const int4 c = c4[q];
            const int p = q << 2;
            if (window_leaves(a, c.x)) { window_free(a, p); ++cnt; }
            if (window_leaves(a, c.y)) { window_free(a, p + 1); ++cnt; }
            if (window_leaves(a, c.z)) { window_free(a, p + 2); ++cnt; }
            if (window_leaves(a, c.w)) { window_free(a, p + 3); ++cnt; }
        }
        done = nq << 2;
    }
    for (int p = done + g; p < a.n; p += stride)
        if (window_leaves(a, a.cell[p])) { window_free(a, p); ++cnt; }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(a.count, (unsigned long long)cnt);
}

__global__ __launch_bounds__(256) void k_window_popcount(const uint32_t *freemap, int32_t words, int32_t *pop) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < words) pop[w] = __popc(freemap[w]);
}

// One slot reached twice (a listed slot inside a scanned tile, or listed
// twice) is freed once: the thread that swaps its cell to the dead value.
template <typename T> AP_D bool window_free_once(const WindowArgs<T> &a, int p, int cell) {
    if (atomicCAS(&a.cell[p], cell, kDeadCell) != cell) return false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (a.off[k]) a.off[k][p] = T(0);
        a.u[k][p] = T(0);
    }
    a.w[p] = T(0);
    if (a.proxy) {
        a.proxy[2 * p] = T(0);
        a.proxy[2 * p + 1] = T(0);
    }
    const int id = a.id[p];
    atomicOr(&a.freemap[id >> 5], 1u << (id & 31));
    a.free_slot[id] = p;
    return true;
}

// Blocks [0, ncols * ntile_z): one tile each, a pass over its slot range;
// the remaining blocks: the listed slots, 256 each.
template <typename T> __global__ __launch_bounds__(256) void k_window_leave_tiles(WindowArgs<T> a, LeaveTiles lt) {
    const int b = blockIdx.x;
    const int ntb = lt.ncols * lt.ntile_z;
    int cnt = 0;
    if (b < ntb) {
        const int tz = b / lt.ncols;
        const int tx = (lt.tx0 + (b - tz * lt.ncols)) % lt.ntile_x;
        const int t = tx + lt.ntile_x * tz;
        const int end = lt.start[t + 1];
        for (int p = lt.start[t] + (int)threadIdx.x; p < end; p += blockDim.x) {
            const int c = a.cell[p];
            if (window_leaves(a, c) && window_free_once(a, p, c)) ++cnt;
        }
    } else {
        const int j = (b - ntb) * (int)blockDim.x + (int)threadIdx.x;
        if (j < lt.list_n) {
            const int p = lt.list[j];
            if ((unsigned)p < (unsigned)a.n) {
                const int c = a.cell[p];
                if (window_leaves(a, c) && window_free_once(a, p, c)) ++cnt;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(a.count, (unsigned long long)cnt);
}

template <typename T> AP_D void window_put(const WindowArgs<T> &a, int p, int r) {
    if (a.inj_list) a.inj_list[r] = p;
    const int ic = a.in_cell[r];
    const int row = (int)a.fnx.div((uint32_t)ic);
    a.cell[p] = row * a.nx + a.col;   // the entering column is the storage column that left
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (a.off[k]) a.off[k][p] = a.in_off[k][r];
        a.u[k][p] = a.in_u[k][r];
    }
    a.w[p] = a.in_w[r];
}

// Injected particle r takes the r-th smallest free id (the word holding it by
// binary search of the popcount scan, then the bit) and that id's slot, when
// the slot hint is still right.
template <typename T> __global__ __launch_bounds__(256) void k_window_fill_hint(WindowArgs<T> a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_inj) return;
    int lo = 0, hi = a.words - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.frank[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    uint32_t bits = a.freemap[lo];
    for (int k = r - a.frank[lo]; k > 0 && bits; --k) bits &= bits - 1u;
    const int id = (lo << 5) + __ffs(bits) - 1;
    const int p = (bits && id < a.n) ? a.free_slot[id] : -1;
    if ((unsigned)p < (unsigned)a.n && a.cell[p] == kDeadCell && a.id[p] == id) window_put(a, p, r);
    else atomicAdd(a.miss, 1ull);
}

// The rest (only when a hint was stale): every free slot whose id ranks
// below n_inj takes its particle; slots filled above are no longer free.
template <typename T> __global__ __launch_bounds__(256) void k_window_fill_scan(WindowArgs<T> a) {
    if (*a.miss == 0) return;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
        if (a.cell[p] != kDeadCell) continue;
        const int id = a.id[p];
        const uint32_t bits = a.freemap[id >> 5];
        const int r = a.frank[id >> 5] + __popc(bits & ((1u << (id & 31)) - 1u));
        if (r < a.n_inj) window_put(a, p, r);
    }
}

// Clears the bits of the ids ranked below n_inj: in word w, the first
// n_inj - frank[w] set bits.
__global__ __launch_bounds__(256) void k_window_clear(uint32_t *freemap, const int32_t *frank, int32_t words,
                                                      int32_t n_inj) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= words) return;
    int take = n_inj - frank[w];
    if (take <= 0) return;
    uint32_t bits = freemap[w];
    while (take > 0 && bits) {
        bits &= bits - 1u;   // clear the lowest set bit
        --take;
    }
    freemap[w] = bits;
}

template <typename T>
__global__ __launch_bounds__(256) void k_window_column(T *F0, T *F1, T *F2, T *F3, T *F4, T *F5, int32_t col,
                                                       int32_t nx, size_t rows) {
    for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < rows; r += (size_t)gridDim.x * blockDim.x) {
        const size_t c = r * (size_t)nx + (size_t)col;
        F0[c] = T(0); F1[c] = T(0); F2[c] = T(0);
        F3[c] = T(0); F4[c] = T(0); F5[c] = T(0);
    }
}

template <typename T> hipError_t launch_window_init(const WindowArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_window_init<T>), dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_window_check_inject(const WindowArgs<T> &a, hipStream_t s) {
    if (a.n_inj == 0) return hipSuccess;
    hipLaunchKernelGGL((k_window_check_inject<T>), dim3((a.n_inj + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_window_count_leavers(const WindowArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_window_count_leavers<T>), dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
template <typename T> hipError_t launch_window_leave(const WindowArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const int vec = (reinterpret_cast<uintptr_t>(a.cell) & 15u) == 0 ? 1 : 0;
    const int items = vec ? (a.n + 3) / 4 : a.n;
    const int blocks = std::min((items + 255) / 256, 4096);
    hipLaunchKernelGGL((k_window_leave<T>), dim3(blocks), dim3(256), 0, s, a, vec);
    return hipGetLastError();
}
template <typename T> hipError_t launch_window_leave_tiles(const WindowArgs<T> &a, const LeaveTiles &lt, hipStream_t s) {
    const int blocks = lt.ncols * lt.ntile_z + (lt.list_n + 255) / 256;
    if (a.n == 0 || blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_window_leave_tiles<T>), dim3(blocks), dim3(256), 0, s, a, lt);
    return hipGetLastError();
}
hipError_t launch_window_popcount(const uint32_t *freemap, int32_t words, int32_t *pop, hipStream_t s) {
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_window_popcount, dim3((words + 255) / 256), dim3(256), 0, s, freemap, words, pop);
    return hipGetLastError();
}
template <typename T> hipError_t launch_window_fill(const WindowArgs<T> &a, hipStream_t s) {
    if (a.n == 0 || a.n_inj == 0) return hipSuccess;
    hipLaunchKernelGGL((k_window_fill_hint<T>), dim3((a.n_inj + 255) / 256), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_window_fill_scan<T>), dim3(std::min((a.n + 255) / 256, 2048)), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_window_clear(uint32_t *freemap, const int32_t *frank, int32_t words, int32_t n_inj,
                               hipStream_t s) {
    if (words == 0 || n_inj == 0) return hipSuccess;
    hipLaunchKernelGGL(k_window_clear, dim3((words + 255) / 256), dim3(256), 0, s, freemap, frank, words, n_inj);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_window_column(T *const F[6], int32_t col, int32_t nx, size_t ncell, hipStream_t s) {
    const size_t rows = ncell / (size_t)nx;
    hipLaunchKernelGGL((k_window_column<T>), dim3(grid_blocks(rows)), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4],
                       F[5], col, nx, rows);
    return hipGetLastError();
}
template hipError_t launch_window_init<float>(const WindowArgs<float> &, hipStream_t);
template hipError_t launch_window_init<double>(const WindowArgs<double> &, hipStream_t);
template hipError_t launch_window_check_inject<float>(const WindowArgs<float> &, hipStream_t);
template hipError_t launch_window_check_inject<double>(const WindowArgs<double> &, hipStream_t);
template hipError_t launch_window_count_leavers<float>(const WindowArgs<float> &, hipStream_t);
template hipError_t launch_window_count_leavers<double>(const WindowArgs<double> &, hipStream_t);
template hipError_t launch_window_leave<float>(const WindowArgs<float> &, hipStream_t);
template hipError_t launch_window_leave<double>(const WindowArgs<double> &, hipStream_t);
template hipError_t launch_window_leave_tiles<float>(const WindowArgs<float> &, const LeaveTiles &, hipStream_t);
template hipError_t launch_window_leave_tiles<double>(const WindowArgs<double> &, const LeaveTiles &, hipStream_t);
template hipError_t launch_window_fill<float>(const WindowArgs<float> &, hipStream_t);
template hipError_t launch_window_fill<double>(const WindowArgs<double> &, hipStream_t);
template hipError_t launch_window_column<float>(float *const[6], int32_t, int32_t, size_t, hipStream_t);
template hipError_t launch_window_column<double>(double *const[6], int32_t, int32_t, size_t, hipStream_t);

template <typename T> __global__ __launch_bounds__(256) void k_scatter(ScatterArgs<T> a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int cell = a.cell_src[p];
    const int tile = (unsigned)cell < a.ncell ? tile_of(cell, a.dim, a.fnx, a.fnxy, a.ftx, a.fty, a.ftz, a.ntile)
                                              : dead_tile(p, a.ntile[0] * a.ntile[1] * a.ntile[2]);
    // Place the particle at its tile slot.  Ranks follow the previous order
    // (a wave's lanes rank in lane order).  When that order is cell-major
    // (about M particles per cell), a ragged transpose of the tile's rank
    // sequence with stride M puts consecutive slots in different cells, so the
    // 64 lanes of a wave update distinct current nodes in the push kernel's
    // LDS atomics; M = 1 keeps the previous order.
    const int base = a.start[tile];
    const int cnt = a.start[tile + 1] - base;
    const int r = a.rank[p];
    int slot = r;
    const int M = a.interleave;
    if (M > 1 && cnt > M) {
        const int q0 = cnt / M, rem = cnt - q0 * M;
        const int q = r / M, m = r - q * M;
        slot = m * q0 + (m < rem ? m : rem) + q;
    }
    const int d = base + slot;
    a.cell_dst[d] = cell;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (a.off_src[c]) a.off_dst[c][d] = a.off_src[c][p];
        a.u_dst[c][d] = a.u_src[c][p];
    }
    a.w_dst[d] = a.w_src[p];
    a.id_dst[d] = a.id_src[p];
    if (a.free_slot && cell == kDeadCell) a.free_slot[a.id_src[p]] = d;
    if (a.proxy_src) {
        a.proxy_dst[2 * d] = a.proxy_src[2 * p];
        a.proxy_dst[2 * d + 1] = a.proxy_src[2 * p + 1];
    }
}

template <typename T> hipError_t launch_scatter(const ScatterArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_scatter<T>), dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_scatter<float>(const ScatterArgs<float> &, hipStream_t);
template hipError_t launch_scatter<double>(const ScatterArgs<double> &, hipStream_t);

__global__ __launch_bounds__(256) void k_resort_counts(const int32_t *stay, const int32_t *mcount, int32_t *count,
                                                        int32_t n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) count[t] = stay[t] + mcount[t];
}

hipError_t launch_resort_counts(const int32_t *stay, const int32_t *mcount, int32_t *count, int32_t n_tiles,
                                hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resort_counts, dim3((n_tiles + 255) / 256), dim3(256), 0, s, stay, mcount, count, n_tiles);
    return hipGetLastError();
}

// Particles changing tile take their ranks after the tile's stayers.  The
// lanes of a wave (consecutive slots of one old tile) enter few distinct
// tiles: one counter atomic per distinct tile, its lanes ranked in lane order.
constexpr int kPermPpt = 8;   // particles per thread: independent load chains in flight
__global__ __launch_bounds__(256) void k_resort_perm(PermArgs a) {
    const int p0 = blockIdx.x * blockDim.x * kPermPpt + threadIdx.x;
    int t[kPermPpt], k[kPermPpt], cell[kPermPpt];
#pragma unroll
    for (int u = 0; u < kPermPpt; ++u) {
        const int p = p0 + u * (int)blockDim.x;
        cell[u] = p < a.n ? a.cell[p] : -1;
        k[u] = p < a.n ? a.key[p] : 0;
    }
#pragma unroll
    for (int u = 0; u < kPermPpt; ++u) {
        const int p = p0 + u * (int)blockDim.x;
        t[u] = (unsigned)cell[u] < a.ncell ? tile_of(cell[u], a.dim, a.fnx, a.fnxy, a.ftx, a.fty, a.ftz, a.ntile)
                                           : dead_tile(p, a.ntile[0] * a.ntile[1] * a.ntile[2]);
    }
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int u = 0; u < kPermPpt; ++u) {
        const int p = p0 + u * (int)blockDim.x;
        const bool live = p < a.n;
        unsigned long long todo = __ballot(live && k[u] < 0);
        int slot = k[u];
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int tl = __shfl(t[u], leader, 64);
            const unsigned long long m = __ballot(live && k[u] < 0 && t[u] == tl);
            int base = 0;
            if (lane == leader) base = atomicAdd(&a.mrank[tl], (int)__popcll(m));
            base = __shfl(base, leader, 64);
            if ((m >> lane) & 1ull) slot = a.stay[tl] + base + (int)__popcll(m & ((1ull << lane) - 1ull));
            todo &= ~m;
        }
        if (live) a.perm[a.start[t[u]] + slot] = p;
    }
}

hipError_t launch_resort_perm(const PermArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const int per = 256 * kPermPpt;
    hipLaunchKernelGGL(k_resort_perm, dim3((a.n + per - 1) / per), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 diagnostics
// ---------------------------------------------------------------------------
template <int NV> AP_D void block_reduce_store(double (&v)[NV], double *out) {
    __shared__ double red[NV][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const double s = wave_sum(v[m]);
        if (lane == 0) red[m][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

template <typename T> __global__ __launch_bounds__(256) void k_diag_particles(DiagArgs<T> a) {
    double v[kDiagVals];
#pragma unroll
    for (int m = 0; m < kDiagVals; ++m) v[m] = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n; p += gridDim.x * blockDim.x) {
        const int32_t cell = a.cell ? a.cell[p] : 0;
        if (a.cell && cell == kDeadCell) continue;   // free slot of a moving window
        const double ux = a.u[0][p], uy = a.u[1][p], uz = a.u[2][p];
        const double w = a.w[p];
        // a valid particle: finite momentum and weight, cell on the grid, offsets in [0, 1)
        bool fin = isfinite(ux) && isfinite(uy) && isfinite(uz) && isfinite(w);
        if (a.cell) fin = fin && (uint32_t)cell < a.ncell;
        for (int c = 0; c < 3; ++c)
            if (a.off[c]) {
                const double o = a.off[c][p];
                fin = fin && o >= 0.0 && o < 1.0;
            }
        const double uu = ux * ux + uy * uy + uz * uz;
        const double g = sqrt(1.0 + uu);
        if (!fin || !isfinite(g)) { v[10] += 1.0; continue; }
        v[0] += w;
        v[1] += w * ux; v[2] += w * uy; v[3] += w * uz;
        v[4] += w * ux * ux; v[5] += w * uy * uy; v[6] += w * uz * uz;
        v[7] += w * g;
        v[8] += w * (uu / (g + 1.0));   // gamma - 1 without cancellation
        // compensated pair: the sum carries the compensation's error with the opposite sign
        if (a.proxy) v[9] += (double)a.proxy[2 * p] - (double)a.proxy[2 * p + 1];
    }
    block_reduce_store<kDiagVals>(v, a.partial + (size_t)blockIdx.x * kDiagVals);
}

template <typename T> hipError_t launch_diag_particles(const DiagArgs<T> &a, hipStream_t s) {
    hipLaunchKernelGGL((k_diag_particles<T>), dim3(a.blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_diag_particles<float>(const DiagArgs<float> &, hipStream_t);
template hipError_t launch_diag_particles<double>(const DiagArgs<double> &, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_diag_fields(const T *E0, const T *E1, const T *E2, const T *B0,
                                                     const T *B1, const T *B2, size_t n, double *partial) {
    double v[1] = {0.0};
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
        const double a0 = E0[c], a1 = E1[c], a2 = E2[c], b0 = B0[c], b1 = B1[c], b2 = B2[c];
        v[0] += a0 * a0 + a1 * a1 + a2 * a2 + b0 * b0 + b1 * b1 + b2 * b2;
    }
    block_reduce_store<1>(v, partial + blockIdx.x);
}

template <typename T>
hipError_t launch_diag_fields(T *const F[6], size_t ncell, double *partial, int blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_diag_fields<T>), dim3(blocks), dim3(256), 0, s, F[0], F[1], F[2], F[3], F[4], F[5], ncell, partial);
    return hipGetLastError();
}
template hipError_t launch_diag_fields<float>(float *const[6], size_t, double *, int, hipStream_t);
template hipError_t launch_diag_fields<double>(double *const[6], size_t, double *, int, hipStream_t);

// out[m] = sum over rows b of partial[b][m], m < nvals <= 16: one workgroup,
// each thread sums a strided set of rows for every m, then a fixed-order
// tree in LDS (deterministic for a given row count).
__global__ __launch_bounds__(1024) void k_sum_partials(const double *partial, int blocks, int nvals, double *out) {
    __shared__ double red[16][1024 / 64];
    double s[16];
    for (int m = 0; m < 16; ++m) s[m] = 0.0;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x)
        for (int m = 0; m < nvals && m < 16; ++m) s[m] += partial[(size_t)b * nvals + m];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int m = 0; m < nvals && m < 16; ++m) {
        const double w = wave_sum(s[m]);
        if (lane == 0) red[m][wid] = w;
    }
    __syncthreads();
    if ((int)threadIdx.x < nvals && threadIdx.x < 16) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
}

hipError_t launch_sum_partials(const double *partial, int blocks, int nvals, double *out, hipStream_t s) {
    if (nvals > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, partial, blocks, nvals, out);
    return hipGetLastError();
}

// Charge density at the nodes, quadratic shape, FP64 atomics.
template <typename T> __global__ __launch_bounds__(256) void k_rho(RhoArgs<T> a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int cell = a.cell[p];
    if ((unsigned)cell >= (unsigned)a.nn[0] * (unsigned)a.nn[1] * (unsigned)a.nn[2]) return;
    const uint32_t row = a.fnx.div((uint32_t)cell);
    int idx[3];
    idx[0] = cell - (int)row * a.nn[0];
    if (a.dim == 3) {
        const uint32_t k = a.fnxy.div((uint32_t)cell);
        idx[1] = (int)(row - k * a.nn[1]);
        idx[2] = (int)k;
    } else {
        idx[1] = 0;
        idx[2] = (int)row;
    }
    int base[3];
    double wt[3][3];
    for (int ax = 0; ax < 3; ++ax) {
        if (!a.off[ax] || (a.dim <= 2 && ax == 1) || (a.dim == 1 && ax == 2)) {
            base[ax] = idx[ax];   // inactive axis: the node of the particle's own row
            wt[ax][0] = 1.0; wt[ax][1] = 0.0; wt[ax][2] = 0.0;
            continue;
        }
        const double o = (double)a.off[ax][p];
        const int nn = o >= 0.5 ? 1 : 0;
        const double d = o - nn;
        base[ax] = idx[ax] + nn - 1;
        wt[ax][0] = 0.5 * (0.5 - d) * (0.5 - d);
        wt[ax][1] = 0.75 - d * d;
        wt[ax][2] = 0.5 * (0.5 + d) * (0.5 + d);
    }
    const double qw = a.q * (double)a.w[p];
    const int ny_loop = (a.dim == 3) ? 3 : 1;
    for (int c = 0; c < 3; ++c) {
        const int gz = (base[2] + c + a.nn[2]) % a.nn[2];
        for (int b = 0; b < ny_loop; ++b) {
            const int gy = (a.dim == 3) ? (base[1] + b + a.nn[1]) % a.nn[1] : 0;
            for (int m = 0; m < 3; ++m) {
                const int gx = (base[0] + m + a.nn[0]) % a.nn[0];
                const size_t g = (size_t)gx + (size_t)a.nn[0] * ((size_t)gy + (size_t)a.nn[1] * gz);
                atomicAdd(&a.rho[g], qw * wt[0][m] * wt[1][b] * wt[2][c]);
            }
        }
    }
}

template <typename T> hipError_t launch_rho(const RhoArgs<T> &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_rho<T>), dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_rho<float>(const RhoArgs<float> &, hipStream_t);
template hipError_t launch_rho<double>(const RhoArgs<double> &, hipStream_t);

// max |(rho1 - rho0)/dt + div J| and max |J| (non-negative doubles compare
// like their bit patterns, so an integer atomicMax orders them).
template <typename T>
__global__ __launch_bounds__(256) void k_continuity(YeeIdx g, int dim, double idx, double idy, double idz,
                                                    double idt, const double *rho0, const double *rho1,
                                                    const T *Jx, const T *Jy, const T *Jz, size_t ncell,
                                                    unsigned long long *res_max, unsigned long long *j_max) {
    double rmax = 0.0, jm = 0.0;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < ncell; c += (size_t)gridDim.x * blockDim.x) {
        const uint32_t cc = (uint32_t)c;
        const uint32_t row = g.fnx.div(cc);
        const int i = (int)(cc - row * g.nx);
        const long im = (i == 0) ? (g.nx - 1) : -1;
        int k;
        long jmo = 0;
        if (dim == 3) {
            const uint32_t kk = g.fny.div(row);
            const int j = (int)(row - kk * g.ny);
            k = (int)kk;
            jmo = (j == 0) ? (long)(g.ny - 1) * g.nx : -(long)g.nx;
        } else {
            k = (int)row;
        }
        const long slab = (long)g.nx * g.ny;
        const long km = (k == 0) ? (long)(g.nz - 1) * slab : -slab;
        double div = ((double)Jx[c] - (double)Jx[c + im]) * idx + ((double)Jz[c] - (double)Jz[c + km]) * idz;
        if (dim == 3) div += ((double)Jy[c] - (double)Jy[c + jmo]) * idy;
        const double r = (rho1[c] - rho0[c]) * idt + div;
        rmax = fmax(rmax, fabs(r));
        jm = fmax(jm, fmax(fabs((double)Jx[c]), fmax(fabs((double)Jy[c]), fabs((double)Jz[c]))));
    }
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
        jm = fmax(jm, __shfl_xor(jm, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(res_max, (unsigned long long)__double_as_longlong(rmax));
        atomicMax(j_max, (unsigned long long)__double_as_longlong(jm));
    }
}

template <typename T>
hipError_t launch_continuity(int dim, const int32_t n[3], const double dx[3], double dt, const double *rho0,
                             const double *rho1, T *const J[3], unsigned long long *res_max,
                             unsigned long long *j_max, hipStream_t s) {
    YeeIdx g;
    g.nx = n[0];
    g.ny = dim == 3 ? n[1] : 1;
    g.nz = n[2];
    g.fnx = FastDiv((uint32_t)g.nx);
    g.fny = FastDiv((uint32_t)g.ny);
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((k_continuity<T>), dim3(grid_blocks(ncell)), dim3(256), 0, s, g, dim, 1.0 / dx[0],
                       1.0 / dx[1], dim == 1 ? 0.0 : 1.0 / dx[2], 1.0 / dt, rho0, rho1, J[0], J[1], J[2], ncell,
                       res_max, j_max);
    return hipGetLastError();
}
template hipError_t launch_continuity<float>(int, const int32_t[3], const double[3], double, const double *,
                                             const double *, float *const[3], unsigned long long *,
                                             unsigned long long *, hipStream_t);
template hipError_t launch_continuity<double>(int, const int32_t[3], const double[3], double, const double *,
                                              const double *, double *const[3], unsigned long long *,
                                              unsigned long long *, hipStream_t);

}  // namespace apt
