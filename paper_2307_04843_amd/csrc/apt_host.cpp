// Host runtime of the C ABI declared in include/apt.h: validation, workspace
// layout, FP64 pulse constants, per-step kernel sequencing on the caller's
// stream, diagnostics and per-kernel event timing.
#include "apt.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <optional>
#include <string>
#include <vector>

#include "kernels.h"

using namespace apt;

namespace {

thread_local std::string g_err;

ap_status fail(ap_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

const double kTwoPi = 6.283185307179586;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Normalised run description (internal units: c = omega = 1).
struct RunShape {
    int dim = 0, prec = 0, nsp = 0;
    int n[3] = {1, 1, 1};
    int tile[3] = {1, 1, 1};
    int ntile[3] = {1, 1, 1};
    int64_t ncell = 0, ntiles = 0;
    double dx[3] = {0, 0, 0};
    double x_min[3] = {0, 0, 0};
    double dt = 0, t0 = 0;
    int sort_every = 8;
    int splits = 1;
    int options = 0;
    size_t real = 4;
    int64_t np[kMaxSpecies] = {0, 0, 0, 0};
    double q[kMaxSpecies] = {0, 0, 0, 0};
    double m[kMaxSpecies] = {1, 1, 1, 1};
    bool has_proxy[kMaxSpecies] = {false, false, false, false};   // gridded: species carries a proxy
    int xo = 0;                     // moving window: storage column of the window's first column
    int adj_mode = AP_ADJ_FROZEN;   // reading of the gridded adjoint (fixes the checkpoint layout)
};

struct WorkLayout {
    size_t counters = 0, sums = 0, partial = 0, rho0 = 0, rho1 = 0, jacc = 0, esamp = 0, scan_part = 0, bsrc = 0,
           total = 0;
    // moving window: per species the free-id bit map; popcounts of its words,
    // their scan, scan scratch and counters, shared by the species
    size_t wmap[kMaxSpecies] = {}, wslot[kMaxSpecies] = {}, wpop = 0, wfrank = 0, wpart = 0, wcnt = 0;
    // slots of the particles injected since the last full sort (2-D windows)
    size_t winj[kMaxSpecies] = {};
    int64_t winj_cap[kMaxSpecies] = {};
    size_t lam[6] = {}, adj_partial = 0;   // gridless adjoint state and gradient partials
    int adj_blocks = 0;
    size_t slot_bytes = 0;                 // one checkpoint slot (all species), gridless
    size_t slot_off[kMaxSpecies] = {};     // species block offsets inside a slot
    size_t count[kMaxSpecies] = {}, start[kMaxSpecies] = {}, rank[kMaxSpecies] = {};
    size_t alt_cell[kMaxSpecies] = {}, alt_off[kMaxSpecies][3] = {}, alt_u[kMaxSpecies][3] = {};
    size_t alt_w[kMaxSpecies] = {}, alt_id[kMaxSpecies] = {}, alt_proxy[kMaxSpecies] = {};
    // fused re-sort (3-D): re-sort keys written by the push, the permutation
    // the next push reads through, entering and staying counts per tile
    size_t key[kMaxSpecies] = {}, perm[kMaxSpecies] = {}, mcount[kMaxSpecies] = {}, stay[kMaxSpecies] = {};
};

constexpr int kDiagBlocks = 512;
constexpr int kCounters = 8;   // n_fast, n_bad, res_max, j_max, n_offtile, ...
// moving-window counters: [0] bad ids / injected particles, [1 + i] free slots
// at ap_init and leavers of the last shift, [1 + kMaxSpecies + i] leavers
// counted ahead, [1 + 2 kMaxSpecies + i] stale slot hints of the last fill
constexpr int kWinCounters = 1 + 3 * kMaxSpecies;

// Axes with dynamics (derivatives, motion, stagger).  dim 1: rows of
// independent lines along x; the z index is the row.
bool axis_active(int dim, int ax) { return dim == 3 || dim == 0 || (dim == 2 && ax != 1) || ax == 0; }

ap_status make_shape(const ap_grid_desc *g, const ap_species_desc *sp, int32_t nsp, RunShape *out) {
    if (!g) return fail(AP_E_ARG, "grid description is NULL");
    if (!sp) return fail(AP_E_ARG, "species description is NULL");
    if (g->dim < 0 || g->dim > 3) return fail(AP_E_ARG, "dim must be 0, 1, 2 or 3");
    if (g->precision != AP_F32 && g->precision != AP_F64) return fail(AP_E_ARG, "precision must be AP_F32 or AP_F64");
    if (nsp < 1 || nsp > kMaxSpecies) return fail(AP_E_ARG, "n_species must be 1..4");
    RunShape s;
    s.dim = g->dim;
    s.prec = g->precision;
    s.nsp = nsp;
    s.real = g->precision == AP_F64 ? 8 : 4;
    for (int ax = 0; ax < 3; ++ax) {
        const bool act = axis_active(s.dim, ax);
        if (act && !finite_pos(g->dx[ax])) return fail(AP_E_ARG, "dx must be finite and > 0 on every active axis");
        if (!std::isfinite(g->x_min[ax])) return fail(AP_E_ARG, "x_min must be finite");
        s.dx[ax] = act ? g->dx[ax] * kTwoPi : 1.0;
        s.x_min[ax] = g->x_min[ax] * kTwoPi;
        if (s.dim > 0) {
            if (act) {
                if (g->n[ax] < 4) return fail(AP_E_ARG, "need at least 4 cells on every active axis");
                s.n[ax] = g->n[ax];
            } else if (s.dim == 1 && ax == 2) {
                // rows of a 1-D run: row k sits at lab z = x_min[2] + k dx[2]
                if (g->n[2] < 1) return fail(AP_E_ARG, "a 1-D run needs n[2] >= 1 rows");
                if (!std::isfinite(g->dx[2]) || g->dx[2] < 0.0) return fail(AP_E_ARG, "row spacing dx[2] must be >= 0");
                s.n[2] = g->n[2];
                s.dx[2] = g->dx[2] * kTwoPi;
            } else {
                s.n[ax] = 1;
            }
        }
    }
    if (!std::isfinite(g->t0)) return fail(AP_E_ARG, "t0 must be finite");
    if (!std::isfinite(g->dt) || g->dt < 0.0) return fail(AP_E_ARG, "dt must be finite and >= 0");
    s.t0 = g->t0 * kTwoPi;
    if (s.dim > 0) {
        s.ncell = (int64_t)s.n[0] * s.n[1] * s.n[2];
        if (s.ncell >= (int64_t)1 << 31) return fail(AP_E_ARG, "grid too large: cell count must be < 2^31");
        double inv2 = 0.0, dmin = 1e300;
        for (int ax = 0; ax < 3; ++ax)
            if (axis_active(s.dim, ax)) { inv2 += 1.0 / (s.dx[ax] * s.dx[ax]); dmin = std::fmin(dmin, s.dx[ax]); }
        s.dt = g->dt > 0.0 ? g->dt * kTwoPi : 0.95 / std::sqrt((double)s.dim) * dmin;
        if (!(s.dt < 1.0 / std::sqrt(inv2))) return fail(AP_E_ARG, "dt exceeds the Yee stability limit");
        const int def1[3] = {32, 1, 1}, def2[3] = {32, 1, 8}, def3[3] = {8, 4, 4};
        for (int ax = 0; ax < 3; ++ax) {
            int t = g->tile[ax] > 0 ? g->tile[ax] : (s.dim == 3 ? def3[ax] : (s.dim == 2 ? def2[ax] : def1[ax]));
            if (!axis_active(s.dim, ax)) t = 1;
            // 3-D tile shapes are compiled into the push kernel (constant LDS
            // strides; 2-D: 16x8, 32x8 and 16x16 are, others read at run
            // time); a tile wider than a tiny grid covers its periodic images
            if (s.dim != 3 && t > s.n[ax]) t = s.n[ax];
            if (t > 64) return fail(AP_E_ARG, "tile extent must be <= 64 cells");
            s.tile[ax] = t;
            s.ntile[ax] = (s.n[ax] + t - 1) / t;
        }
        if (s.dim == 3 && !(s.tile[0] == 8 && ((s.tile[1] == 4 && s.tile[2] == 4) ||
                                               (s.tile[1] == 8 && (s.tile[2] == 4 || s.tile[2] == 8)))))
            return fail(AP_E_ARG, "3-D tiles must be 8x4x4, 8x8x4 or 8x8x8 cells");
        s.ntiles = (int64_t)s.ntile[0] * s.ntile[1] * s.ntile[2];
        // LDS of the push kernel: 9 components on the tile plus its halo
        size_t region = 1;
        for (int ax = 0; ax < 3; ++ax)
            if (axis_active(s.dim, ax)) region *= (size_t)(s.tile[ax] + (s.dim == 3 ? 5 : kHaloLo + kHaloHi));
        if (align_lds(region * 6 * s.real) + region * 3 * 8 > 160 * 1024)
            return fail(AP_E_ARG, "tile too large for LDS (reduce tile extents)");
    } else {
        if (!(g->dt > 0.0)) return fail(AP_E_ARG, "gridless runs need dt > 0");
        s.dt = g->dt * kTwoPi;
    }
    if (g->sort_every < 0) return fail(AP_E_ARG, "sort_every must be >= 0");
    if (g->options & ~(AP_GRID_PULSE_ON_GRID | AP_GRID_PROXY | AP_GRID_OPEN_X | AP_GRID_MOVING_WINDOW))
        return fail(AP_E_ARG, "unknown grid option bits");
    if ((g->options & AP_GRID_MOVING_WINDOW) && s.dim == 0) return fail(AP_E_ARG, "a moving window needs a grid");
    if ((g->options & AP_GRID_OPEN_X) && s.dim == 0) return fail(AP_E_ARG, "AP_GRID_OPEN_X needs a grid");
    if ((g->options & AP_GRID_OPEN_X) && (g->options & AP_GRID_MOVING_WINDOW))
        return fail(AP_E_ARG, "AP_GRID_OPEN_X and AP_GRID_MOVING_WINDOW exclude each other");
    if ((g->options & AP_GRID_PULSE_ON_GRID) && s.dim == 0)
        return fail(AP_E_ARG, "AP_GRID_PULSE_ON_GRID needs a grid");
    if ((g->options & AP_GRID_PROXY) && s.dim == 0)
        return fail(AP_E_ARG, "AP_GRID_PROXY needs a grid (gridless runs always accept a proxy)");
    s.options = g->options;
    // default re-sort interval: 2-D tiles carry a two-cell drift margin; 3-D
    // tiles none (LDS budget), so 3-D re-sorts every step (a push that leaves
    // the staged region takes the global path, which measured costlier than
    // the sort)
    s.sort_every = g->sort_every > 0 ? g->sort_every : (s.dim == 3 ? 1 : 8);
    int64_t total = 0;
    for (int i = 0; i < nsp; ++i) {
        if (!finite_pos(sp[i].m)) return fail(AP_E_ARG, "species mass must be finite and > 0");
        if (!std::isfinite(sp[i].q)) return fail(AP_E_ARG, "species charge must be finite");
        if (sp[i].n < 0 || sp[i].n >= ((int64_t)1 << 31)) return fail(AP_E_ARG, "species count must be in [0, 2^31)");
        s.np[i] = sp[i].n;
        s.q[i] = sp[i].q;
        s.m[i] = sp[i].m;
        total += sp[i].n;
    }
    if (s.dim > 0) {
        const double avg = (double)total / (double)s.ntiles;
        double target = (double)total / 4096.0;
        if (target < 512.0) target = 512.0;
        if (target > 8192.0) target = 8192.0;
        int sp_ = (int)std::ceil(avg / target);
        if (sp_ < 1) sp_ = 1;
        if (sp_ > 64) sp_ = 64;
        // 3-D: one workgroup per tile (the fused re-sort counts a tile's
        // staying particles in its workgroup)
        s.splits = s.dim == 3 ? 1 : sp_;
    }
    *out = s;
    return AP_OK;
}

WorkLayout make_layout(const RunShape &s) {
    WorkLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = align_up(off, 256);
        off = o + bytes;
        return o;
    };
    L.counters = take(kCounters * 8);
    L.sums = take((size_t)kDiagVals * 8 * (kMaxSpecies + 1));
    L.partial = take((size_t)kDiagBlocks * kDiagVals * 8);
    if (s.dim > 0) {
        L.rho0 = take((size_t)s.ncell * 8);
        L.rho1 = take((size_t)s.ncell * 8);
        // FP64 accumulator of the step's current (FP32 runs; FP64 runs use J)
        if (s.prec == AP_F32) L.jacc = take((size_t)s.ncell * 3 * 8);
        // E2 + E1 and B2 + B1 with E1, B1 sampled on the grid (AP_SAMPLE_GRID)
        if (s.options & AP_GRID_PULSE_ON_GRID) L.esamp = take((size_t)s.ncell * 6 * s.real);
        L.scan_part = take((size_t)2 * scan_part_len((int32_t)s.ntiles) * 4);
        // boundary source S_y, S_z per row (incoming-wave x_min of open rows)
        if (s.options & AP_GRID_OPEN_X) L.bsrc = take((size_t)s.n[1] * s.n[2] * 2 * s.real);
        if (s.options & AP_GRID_MOVING_WINDOW) {
            int64_t wmax = 1;
            for (int i = 0; i < s.nsp; ++i) {
                const int64_t words = (s.np[i] + 31) / 32;
                wmax = words > wmax ? words : wmax;
                L.wmap[i] = take((size_t)words * 4);
                L.wslot[i] = take((size_t)(s.np[i] > 0 ? s.np[i] : 1) * 4);
                if (s.dim == 2) {
                    L.winj_cap[i] = s.np[i] / 16 > 4096 ? s.np[i] / 16 : 4096;
                    L.winj[i] = take((size_t)L.winj_cap[i] * 4);
                }
            }
            L.wpop = take((size_t)wmax * 4);
            L.wfrank = take((size_t)(wmax + 1) * 4);
            L.wpart = take((size_t)2 * scan_part_len((int32_t)wmax) * 4);
            L.wcnt = take((size_t)kWinCounters * 8);
        }
        for (int i = 0; i < s.nsp; ++i) {
            const size_t N = (size_t)s.np[i];
            L.count[i] = take((size_t)s.ntiles * 4);
            L.start[i] = take((size_t)(s.ntiles + 1) * 4);
            L.rank[i] = take(N * 4);
            L.alt_cell[i] = take(N * 4);
            for (int c = 0; c < 3; ++c) {
                if (axis_active(s.dim, c)) L.alt_off[i][c] = take(N * s.real);
                L.alt_u[i][c] = take(N * s.real);
            }
            L.alt_w[i] = take(N * s.real);
            L.alt_id[i] = take(N * 4);
            // the proxy's (sum, compensation) pair follows its particle through re-sorts
            if (s.options & AP_GRID_PROXY) L.alt_proxy[i] = take(N * 2 * s.real);
            if (s.dim == 3) {
                L.key[i] = take(N * 4);
                L.perm[i] = take(N * 4);
                L.mcount[i] = take((size_t)s.ntiles * 4);
                L.stay[i] = take((size_t)s.ntiles * 4);
            }
        }
    }
    if (s.dim == 0) {
        int64_t nmax = 0;
        for (int i = 0; i < s.nsp; ++i) nmax = s.np[i] > nmax ? s.np[i] : nmax;
        for (int c = 0; c < 6; ++c) L.lam[c] = take((size_t)nmax * 8);
        L.adj_blocks = (int)((nmax + 255) / 256);
        if (L.adj_blocks < 1) L.adj_blocks = 1;
        L.adj_partial = take((size_t)L.adj_blocks * 5 * 8);
        size_t so = 0;
        for (int i = 0; i < s.nsp; ++i) {
            L.slot_off[i] = so;
            so += align_up((size_t)s.np[i] * (12 + 6 * s.real), 256);
        }
        L.slot_bytes = so;
    }
    L.total = align_up(off, 256);
    return L;
}

// Checkpoint buffer of a gridded run (frozen-grid adjoint):
//   [adjoint state: 6 x n_max FP64][gradient partials]
//   [final-state slot][ceil(n/K) checkpoint slots][K replay slots]
// A checkpoint slot holds every species (cell, id, offsets, u, w, and the
// proxy pair of a species that carries one) and E2, B2; a replay slot holds
// E2, B2 and the species being differentiated (no w, no proxy: the proxy
// enters no step, so its adjoint is constant).
struct GridCkpt {
    size_t lam[6] = {}, partial = 0, fixed = 0;
    size_t lam_sp[kMaxSpecies][6] = {};   // coupled: adjoint state of every species
    size_t lgrid = 0;                     // coupled: FP64 adjoints lE, lB, lJt (3 x ncell each)
    size_t gx0 = 0;                       // coupled: [6][n] per-particle values between the reverse passes
    int blocks = 0;
    size_t outer = 0, inner = 0;
    size_t sp_off[kMaxSpecies] = {};   // species blocks inside a checkpoint slot
    size_t fields = 0;                 // E2, B2 inside a checkpoint slot (at 0 in a replay slot)
    size_t inner_sp = 0;               // frozen: the differentiated species' block inside a replay slot
    size_t inner_off[kMaxSpecies] = {};   // coupled: every species' block (with w) inside a replay slot
};

size_t sp_block_bytes(const RunShape &s, int i, bool with_w, bool with_proxy) {
    const size_t N = (size_t)s.np[i];
    const size_t nact = s.dim == 3 ? 3 : 2;
    const size_t npr = (with_proxy && s.has_proxy[i]) ? 2 : 0;
    return align_up(N * 8 + N * s.real * (nact + 3 + (with_w ? 1 : 0) + npr), 256);
}

GridCkpt grid_ckpt(const RunShape &s) {
    GridCkpt G;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = align_up(off, 256);
        off = o + bytes;
        return o;
    };
    int64_t nmax = 0;
    for (int i = 0; i < s.nsp; ++i) nmax = s.np[i] > nmax ? s.np[i] : nmax;
    const bool cpl = s.adj_mode == AP_ADJ_COUPLED;
    if (cpl) {
        for (int i = 0; i < s.nsp; ++i)
            for (int c = 0; c < 6; ++c) G.lam_sp[i][c] = take((size_t)s.np[i] * 8);
        G.lgrid = take((size_t)9 * (size_t)s.ncell * 8);
        G.gx0 = take((size_t)6 * (size_t)(nmax > 0 ? nmax : 1) * 8);
    } else {
        for (int c = 0; c < 6; ++c) G.lam[c] = take((size_t)nmax * 8);
    }
    G.blocks = (int)((nmax + 255) / 256);
    if (G.blocks < 1) G.blocks = 1;
    G.partial = take((size_t)G.blocks * 5 * 8);
    G.fixed = align_up(off, 256);
    const size_t fbytes = align_up((size_t)6 * (size_t)s.ncell * s.real, 256);
    size_t so = 0, mx = 0, io = fbytes;
    for (int i = 0; i < s.nsp; ++i) {
        G.sp_off[i] = so;
        so += sp_block_bytes(s, i, true, true);
        const size_t b = sp_block_bytes(s, i, false, false);
        mx = b > mx ? b : mx;
        G.inner_off[i] = io;
        io += sp_block_bytes(s, i, true, false);
    }
    G.fields = so;
    G.outer = so + fbytes;
    G.inner_sp = fbytes;
    G.inner = cpl ? io : fbytes + mx;
    return G;
}

// Bytes of checkpoint storage for recording n steps with segment K.
size_t ckpt_need(const RunShape &s, const WorkLayout &L, int64_t n, int64_t K) {
    const int64_t nseg = n > 0 ? (n + K - 1) / K : 1;
    if (s.dim == 0) {
        const int64_t slots = nseg + K > 2 ? nseg + K : 2;
        return (size_t)slots * L.slot_bytes;
    }
    const GridCkpt G = grid_ckpt(s);
    return G.fixed + (size_t)(1 + nseg) * G.outer + (size_t)K * G.inner;
}

// Bytes of the binomial schedule with S slots, whatever the number of steps:
// gridless, S slots plus a work slot; gridded, the fixed part, a copy of the
// final state and S whole states.
size_t revolve_need(const RunShape &s, const WorkLayout &L, int64_t S) {
    if (s.dim == 0) return (size_t)(S + 1) * L.slot_bytes;
    const GridCkpt G = grid_ckpt(s);
    return G.fixed + (size_t)(1 + S) * G.outer;
}

// Binomial checkpointing.  With the state at step l held in a slot and s
// further slots free, R(s, t) = C(s + t + 1, s + 1) steps can be reversed
// when every step is advanced at most t times: R(0, t) = t + 1 (re-advance
// from l for each step) and R(s, t) = R(s, t - 1) + R(s - 1, t) (a state
// stored d steps ahead splits the range into a left part reversed again from
// l and a right part with one slot less).  R(s, t) = 0 for t < 0.
int64_t revolve_capacity(int64_t s, int64_t t) {
    if (t < 0) return 0;
    unsigned __int128 v = 1;   // C(s + 1 + k, k) for k = 1..t
    for (int64_t k = 1; k <= t; ++k) {
        v = v * (unsigned __int128)(s + 1 + k) / (unsigned __int128)k;
        if (v > (unsigned __int128)INT64_MAX) return INT64_MAX;
    }
    return (int64_t)v;
}

// Fewest repetitions t with R(s, t) >= n.
int64_t revolve_repeats(int64_t n, int64_t s) {
    int64_t t = 0;
    while (revolve_capacity(s, t) < n) ++t;
    return t;
}

// Forward steps of reversing n steps with s free slots when every advance
// counts: t n - R(s + 1, t - 1) with t = revolve_repeats(n, s); the k-th step
// of the range costs revolve_repeats(k, s).
int64_t revolve_cost(int64_t n, int64_t s) {
    if (n <= 1) return 0;
    const int64_t t = revolve_repeats(n, s);
    return t * n - revolve_capacity(s + 1, t - 1);
}

// Split of n >= 2 steps with s >= 1 free slots that reaches revolve_cost:
// the smallest d with d <= R(s, t - 1) (left part, one repetition less) and
// n - d <= R(s - 1, t) (right part, one slot less) that is not below
// R(s, t - 2).
int64_t revolve_split(int64_t n, int64_t s) {
    const int64_t t = revolve_repeats(n, s);
    int64_t d = revolve_capacity(s, t - 2);
    const int64_t r = n - revolve_capacity(s - 1, t);
    if (r > d) d = r;
    if (d > n - 1) d = n - 1;
    return d < 1 ? 1 : d;
}

// States the recording sweep stores (relative steps, increasing), the
// recording being free: n steps fall into segments i = 0.. s with s - i free
// slots each, the k-th step of segment i costing revolve_repeats(k, s - i);
// filling every segment up to a common cost level tau minimises the total.
std::vector<int64_t> revolve_spine(int64_t n, int64_t s, int64_t *cost = nullptr) {
    int64_t tau = 0;
    for (;;) {
        int64_t cap = 0;
        for (int64_t i = 0; i <= s && cap < n; ++i) {
            const int64_t c = revolve_capacity(s - i, tau);
            cap = c > n ? n : cap + c;
        }
        if (cap >= n) break;
        ++tau;
    }
    std::vector<int64_t> size((size_t)s + 1, 0);
    int64_t left = n;
    for (int64_t i = 0; i <= s; ++i) {
        int64_t d = revolve_capacity(s - i, tau - 1);
        if (d > left) d = left;
        size[(size_t)i] = d;
        left -= d;
    }
    for (int64_t i = 0; i <= s && left > 0; ++i) {
        int64_t more = revolve_capacity(s - i, tau) - size[(size_t)i];
        if (more > left) more = left;
        size[(size_t)i] += more;
        left -= more;
    }
    std::vector<int64_t> pos;
    int64_t at = 0, total = 0;
    for (int64_t i = 0; i <= s; ++i) {
        total += revolve_cost(size[(size_t)i], s - i);
        at += size[(size_t)i];
        if (i < s && at < n && size[(size_t)i] > 0) pos.push_back(at);
    }
    if (cost) *cost = total;
    return pos;
}

PulseDev default_pulse() {
    PulseDev P;
    std::memset(&P, 0, sizeof(P));
    P.type = PT_NONE;
    P.tau = 1.0;
    P.inv_tau = 1.0;
    P.inv_vg = 1.0;
    P.v_phi = 1.0;
    P.b_over_e = 1.0;
    P.k = 1.0;
    return P;
}

struct TimedPair {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

// Library-held scratch of ap_gather_diag_static, for callers that cannot
// allocate device memory: the per-species sums, then the per-block partial
// sums of the diagnostics reductions (66,176 bytes, whatever the run's size).
// Each GPU holds its own copy until the process ends; host code reaches it
// only through the address resolved per device (static_scratch), never
// through the name.
constexpr size_t kStaticSums = (size_t)(kMaxSpecies + 1) * kDiagVals;
constexpr size_t kStaticDoubles = kStaticSums + (size_t)kDiagBlocks * kDiagVals;
static __device__ __align__(256) double scratch[kStaticDoubles];
static_assert(sizeof(scratch) == 66176, "the documented size of the static scratch");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Resolve the device address of `scratch` on device dev, once per device,
// with dev current (the caller's current device is restored).
hipError_t resolve_static_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double *>(ptr);
    return hipSuccess;
}

double *static_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

}  // namespace

struct ap_ctx {
    RunShape s;
    WorkLayout L;
    ap_buffers buf;
    hipStream_t stream = nullptr;
    int device = 0;              // device of the stream
    PulseDev P;
    int pulse_type = -1;
    double s0 = 1.0;             // S0/E0 of the incoming-wave boundary (AP_SAMPLE_BOUNDARY)
    // moving window: free slots per species, up to the leavers of the last
    // shift (counted on the device, added at the next shift)
    int64_t n_free[kMaxSpecies] = {0, 0, 0, 0};
    // 2-D moving window: the step of the last full sort, and the particles
    // injected since (their slots listed while the list holds them)
    int64_t sort_step = 0;
    int64_t inj_n[kMaxSpecies] = {0, 0, 0, 0};
    bool inj_overflow = false;
    int64_t step = 0;
    bool sorted_once = false;
    bool need_sort = false;      // re-sort before the next push (state restored from a checkpoint)
    // fused re-sort (3-D): within an ap_step call the particle state moves
    // between the caller's arrays and the workspace copy every step; it is
    // back in the caller's arrays when the call returns
    bool state_alt = false;      // the current state is in the workspace copy
    bool keys_valid = false;     // the last push wrote re-sort keys for the current state
    bool no_fuse = false;        // full re-sorts only (reverse-sweep replays)
    bool timing = false;
    std::vector<TimedPair> pending;
    std::vector<hipEvent_t> pool;
    double acc_ms[4] = {0, 0, 0, 0};
    int64_t acc_n[4] = {0, 0, 0, 0};
    int64_t acc_pushes = 0;
    int64_t push_since_read = 0;
    // adjoint checkpoints
    unsigned char *ckpt = nullptr;
    size_t ckpt_bytes = 0;
    int64_t segment = 0;
    int64_t rec_n = 0, rec_step0 = 0;
    // binomial schedule: slots of whole states (0: none, segments instead);
    // the recorded states besides step 0, as (relative step, slot)
    int32_t revolve = 0;
    std::vector<std::pair<int64_t, int32_t>> spine;

    unsigned char *work() const { return static_cast<unsigned char *>(buf.work); }
    template <typename X> X *wp(size_t off) const { return reinterpret_cast<X *>(work() + off); }
    unsigned long long *counters() const { return wp<unsigned long long>(L.counters); }
};

namespace {

hipError_t take_event(ap_ctx *c, hipEvent_t *e) {
    if (!c->pool.empty()) {
        *e = c->pool.back();
        c->pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

struct Timer {
    ap_ctx *c;
    int kind;
    hipEvent_t a = nullptr;
    Timer(ap_ctx *c_, int k) : c(c_), kind(k) {
        if (c->timing && take_event(c, &a) == hipSuccess) hipEventRecord(a, c->stream);
    }
    ~Timer() {
        if (!c->timing || !a) return;
        hipEvent_t b;
        if (take_event(c, &b) != hipSuccess) return;
        hipEventRecord(b, c->stream);
        c->pending.push_back({kind, a, b});
    }
};

// Full re-sorts only while a reverse sweep replays segments (its replay
// slots copy the caller's arrays at every step).
struct NoFuse {
    ap_ctx *c;
    explicit NoFuse(ap_ctx *c_) : c(c_) { c->no_fuse = true; }
    ~NoFuse() { c->no_fuse = false; }
};

ap_status hip_fail(hipError_t e, const char *where) {
    return fail(AP_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, where)                         \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hip_fail(_e, where); \
    } while (0)

template <typename T> ap_status step_gridded(ap_ctx *c, uint32_t flags);
template <typename T> ap_status restore_primary(ap_ctx *c);
template <typename T> ap_status shift_window_impl(ap_ctx *c, int32_t dir, const ap_inject *inject);
template <typename T> ap_status window_init(ap_ctx *c);
template <typename T> ap_status step_gridless(ap_ctx *c, uint32_t flags);
template <typename T>
ap_status backward_impl(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                        double *out);
template <typename T>
ap_status backward_grid(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                        double *out);
template <typename T>
ap_status backward_coupled(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                           double *out);

double laguerre_host(int n, int a, double x) {
    double l0 = 1.0, l1 = 1.0 + a - x;
    if (n == 0) return l0;
    for (int m = 1; m < n; ++m) {
        const double l2 = ((2 * m + 1 + a - x) * l1 - (m + a) * l0) / (m + 1);
        l0 = l1;
        l1 = l2;
    }
    return l1;
}

}  // namespace

extern "C" {

const char *ap_last_error(void) { return g_err.c_str(); }

ap_status ap_query_layout(const ap_grid_desc *grid, const ap_species_desc *species, int32_t n_species,
                          ap_layout *out) {
    try {
        if (!out) return fail(AP_E_ARG, "layout output is NULL");
        RunShape s;
        const ap_status st = make_shape(grid, species, n_species, &s);
        if (st != AP_OK) return st;
        const WorkLayout L = make_layout(s);
        out->grid_bytes = s.dim > 0 ? (size_t)9 * (size_t)s.ncell * s.real : 0;
        out->work_bytes = L.total;
        out->real_bytes = s.real;
        out->n_cells = s.ncell;
        out->n_tiles = s.ntiles;
        out->ckpt_slot_bytes = L.slot_bytes;
        return AP_OK;
    } catch (...) {
        return fail(AP_E_NOMEM, "host allocation failed");
    }
}

ap_status ap_init(const ap_grid_desc *grid, const ap_species_desc *species, int32_t n_species,
                  const ap_buffers *buffers, void *hip_stream, ap_ctx **out) {
    try {
        if (!out) return fail(AP_E_ARG, "context output is NULL");
        if (!buffers) return fail(AP_E_ARG, "buffers are NULL");
        RunShape s;
        const ap_status st = make_shape(grid, species, n_species, &s);
        if (st != AP_OK) return st;
        if (!buffers->work) return fail(AP_E_ARG, "work buffer is NULL");
        if (s.dim > 0 && !buffers->grid) return fail(AP_E_ARG, "grid buffer is NULL");
        for (int i = 0; i < n_species; ++i) {
            const ap_particles &p = buffers->sp[i];
            if (s.np[i] == 0) continue;
            bool okp = p.u[0] && p.u[1] && p.u[2] && p.w;
            if (s.dim == 0) {
                okp = okp && p.icell[0] && p.icell[1] && p.icell[2] && p.off[0] && p.off[1] && p.off[2];
            } else {
                okp = okp && p.cell && p.off[0] && p.id && (s.dim == 1 || p.off[2]) && (s.dim != 3 || p.off[1]);
            }
            if (!okp) return fail(AP_E_ARG, "species " + std::to_string(i) + ": a required particle array is NULL");
        }
        for (int i = 0; i < n_species; ++i) {
            if (s.dim == 0 || !buffers->sp[i].proxy) continue;
            if (!(s.options & AP_GRID_PROXY))
                return fail(AP_E_ARG, "species " + std::to_string(i) + ": a gridded proxy needs AP_GRID_PROXY");
            s.has_proxy[i] = s.np[i] > 0;
        }
        ap_ctx *c = new (std::nothrow) ap_ctx;
        if (!c) return fail(AP_E_NOMEM, "context allocation failed");
        c->s = s;
        c->L = make_layout(s);
        c->buf = *buffers;
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->P = default_pulse();
        // the stream's device; ap_gather_diag_static's scratch is resolved there
        hipError_t e = c->stream ? hipStreamGetDevice(c->stream, &c->device) : hipGetDevice(&c->device);
        if (e == hipSuccess) e = resolve_static_scratch(c->device);
        if (e == hipSuccess) e = launch_fill_zero<unsigned long long>(c->counters(), kCounters, c->stream);
        if (e == hipSuccess && s.dim > 0) {
            if (s.prec == AP_F64)
                e = launch_fill_zero<double>(static_cast<double *>(buffers->grid), (size_t)9 * s.ncell, c->stream);
            else
                e = launch_fill_zero<float>(static_cast<float *>(buffers->grid), (size_t)9 * s.ncell, c->stream);
        }
        if (e == hipSuccess && (s.options & AP_GRID_MOVING_WINDOW)) {
            const ap_status st = s.prec == AP_F64 ? window_init<double>(c) : window_init<float>(c);
            if (st != AP_OK) {
                delete c;
                return st;
            }
        }
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "ap_init");
        }
        *out = c;
        return AP_OK;
    } catch (...) {
        return fail(AP_E_NOMEM, "host allocation failed");
    }
}

ap_status ap_set_pulse(ap_ctx *c, int32_t type, const ap_pulse_params *prm) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (type < AP_PULSE_NONE || type > AP_PULSE_GAUSS_NP) return fail(AP_E_ARG, "unknown pulse type");
    PulseDev P = default_pulse();
    P.type = type;
    if (type == AP_PULSE_NONE) {
        c->P = P;
        c->pulse_type = type;
        return AP_OK;
    }
    if (!prm) return fail(AP_E_ARG, "pulse parameters are NULL");
    const double vals[] = {prm->a0, prm->tau, prm->t_ref, prm->x_ref, prm->phi0, prm->chirp, prm->x_f,
                           prm->w0, prm->y_c, prm->z_c, prm->q_slice, prm->beta_f, prm->x0_ff, prm->t0_ff,
                           prm->dx_prop, prm->dt_prop, prm->wp2, prm->zeta};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(AP_E_ARG, "pulse parameters must be finite");
    if (!(prm->tau > 0.0)) return fail(AP_E_ARG, "tau must be > 0");
    if (prm->pol != 0 && prm->pol != 1) return fail(AP_E_ARG, "pol must be 0 or 1");
    if (prm->dispersion < AP_DISP_PAPER2 || prm->dispersion > AP_DISP_PLASMA)
        return fail(AP_E_ARG, "unknown dispersion mode");
    const bool plasma = prm->dispersion == AP_DISP_PLASMA;
    if (plasma) {
        if (type == AP_PULSE_GAUSS_NP) return fail(AP_E_ARG, "the nonparaxial Gaussian is a vacuum solution");
        if (c->s.dim == 0) return fail(AP_E_ARG, "an analytic current needs a grid");
        if (prm->sampling != AP_SAMPLE_GRID)
            return fail(AP_E_UNSUPPORTED, "an analytic current needs the pulse sampled on the grid (AP_SAMPLE_GRID)");
        if (prm->wp2 < 0.0 || prm->zeta < 0.0) return fail(AP_E_ARG, "wp2 and zeta must be >= 0");
    }
    const bool focused = type != AP_PULSE_PLANE;
    if (focused && !(prm->w0 > 0.0)) return fail(AP_E_ARG, "w0 must be > 0");
    if (focused && type != AP_PULSE_GAUSS_NP && prm->d_f != 2 && prm->d_f != 3)
        return fail(AP_E_ARG, "d_f must be 2 or 3");
    if (type == AP_PULSE_LG) {
        if (prm->d_f != 3) return fail(AP_E_ARG, "Laguerre-Gaussian modes need d_f = 3");
        if (prm->lg_p < 0 || prm->lg_p > 8 || prm->lg_l < -8 || prm->lg_l > 8)
            return fail(AP_E_ARG, "LG indices must satisfy 0 <= p <= 8, |l| <= 8");
    }
    if (type == AP_PULSE_FF && prm->beta_f == 1.0) return fail(AP_E_ARG, "flying focus needs beta_f != 1");
    if (prm->envelope != AP_ENV_SIN2 && prm->envelope != AP_ENV_SGAUSS)
        return fail(AP_E_ARG, "unknown envelope");
    if (prm->envelope == AP_ENV_SGAUSS) {
        if (prm->sg_order < 1 || prm->sg_order > 32) return fail(AP_E_ARG, "sg_order must be 1..32");
        if (!std::isfinite(prm->fwhm) || !(prm->fwhm > 0.0)) return fail(AP_E_ARG, "fwhm must be > 0");
    }
    if (prm->sampling != AP_SAMPLE_PARTICLES && prm->sampling != AP_SAMPLE_GRID &&
        prm->sampling != AP_SAMPLE_BOUNDARY)
        return fail(AP_E_ARG, "unknown sampling mode");
    if (prm->sampling == AP_SAMPLE_BOUNDARY) {
        if (!(c->s.options & AP_GRID_OPEN_X))
            return fail(AP_E_STATE, "launching through the boundary needs a run created with AP_GRID_OPEN_X");
        if (type != AP_PULSE_PLANE) return fail(AP_E_ARG, "only a PLANE pulse is launched through the boundary");
    }
    if (prm->sampling == AP_SAMPLE_GRID && !(c->s.dim > 0 && (c->s.options & AP_GRID_PULSE_ON_GRID)))
        return fail(AP_E_STATE, "grid sampling needs a gridded run created with AP_GRID_PULSE_ON_GRID");
    if (type == AP_PULSE_GAUSS_NP) {
        if (prm->dispersion != AP_DISP_VACUUM)
            return fail(AP_E_ARG, "the nonparaxial Gaussian is a vacuum solution: use AP_DISP_VACUUM");
        if (prm->np_order != 0 && prm->np_order != 2 && prm->np_order != 4)
            return fail(AP_E_ARG, "np_order must be 0, 2 or 4");
    }
    const double L = kTwoPi;
    // numerical dispersion constants (Sec. II.A, Eqs. (10)-(14)), omega = 1
    double v_phi = 1.0, v_g = 1.0, boe = 1.0;
    if (prm->dispersion != AP_DISP_VACUUM) {
        const double dxp = (prm->dx_prop > 0.0 ? prm->dx_prop * L : c->s.dx[0]);
        const double dtp = (prm->dt_prop > 0.0 ? prm->dt_prop * L : c->s.dt);
        if (!(dxp > 0.0) || !(dtp > 0.0) || c->s.dim == 0 && !(prm->dx_prop > 0.0 && prm->dt_prop > 0.0))
            return fail(AP_E_ARG, "grid dispersion modes need dx_prop and dt_prop");
        const double cr = dtp / dxp;
        if (plasma) {
            // Sec. IV: sin^2(dt/2) - wp2 zeta (dt/2) sin(dt/2) = (dt/dx)^2 sin^2(k dx/2), omega = 1
            const double zeta = prm->zeta > 0.0 ? prm->zeta : 1.0;
            const double h = 0.5 * dtp, sh = std::sin(h), ch = std::cos(h);
            const double lhs = sh * sh - prm->wp2 * zeta * h * sh;
            if (!(lhs > 0.0) || !(std::sqrt(lhs) / cr < 1.0))
                return fail(AP_E_ARG, "no propagating Yee mode for this plasma density");
            const double kk = 2.0 / dxp * std::asin(std::sqrt(lhs) / cr);
            v_phi = 1.0 / kk;
            const double dlhs = sh * ch * dtp - prm->wp2 * zeta * h * (h * ch - sh);
            v_g = cr * cr * std::sin(0.5 * kk * dxp) * std::cos(0.5 * kk * dxp) * dxp / dlhs;
            boe = ch * std::sqrt(1.0 - prm->wp2 * zeta * h / sh);
            P.current = 1;
            P.fd = prm->no_fd ? 0 : 1;
            P.wp2z = prm->wp2 * zeta;
            P.fd_delta = 1.0 - v_phi / v_g;
        } else if (prm->dispersion == AP_DISP_PAPER2) {
            v_phi = 1.0 - (1.0 - cr * cr) * dxp * dxp / 24.0;
            v_g = 1.0 - (1.0 - cr * cr) * dxp * dxp / 8.0;
            boe = 1.0 - dtp * dtp / 8.0;
        } else {
            const double sarg = std::sin(0.5 * dtp) / cr;
            if (!(sarg < 1.0)) return fail(AP_E_ARG, "no propagating Yee mode at this resolution");
            const double kk = 2.0 / dxp * std::asin(sarg);
            v_phi = 1.0 / kk;
            v_g = std::cos(0.5 * kk * dxp) / std::cos(0.5 * dtp);
            boe = std::cos(0.5 * dtp);
        }
    }
    P.pol = prm->pol;
    P.d_f = (type == AP_PULSE_PLANE || type == AP_PULSE_GAUSS_NP) ? 3 : prm->d_f;
    P.lg_l = prm->lg_l;
    P.lg_p = prm->lg_p;
    P.np_order = prm->np_order;
    P.envelope = prm->envelope;
    P.sg_order = prm->envelope == AP_ENV_SGAUSS ? prm->sg_order : 1;
    // super-Gaussian: intensity exp(-2 x^(2g)) is 1/2 at x = (ln 2 / 2)^(1/(2g)),
    // so tau_g = FWHM / (2 (ln 2 / 2)^(1/(2g)))
    P.inv_tau_g = prm->envelope == AP_ENV_SGAUSS
                      ? 2.0 * std::pow(0.5 * std::log(2.0), 0.5 / prm->sg_order) / (prm->fwhm * L)
                      : 0.0;
    P.sampling = prm->sampling;
    P.a0 = prm->a0;
    P.tau = prm->tau * L;
    P.inv_tau = 1.0 / P.tau;
    P.half_tau = 0.5 * P.tau;
    P.t_ref = prm->t_ref * L;
    P.x_ref = prm->x_ref * L;
    P.phi0 = prm->phi0;
    P.b_half = 0.5 * prm->chirp / P.tau;
    P.k = 1.0 / v_phi;
    P.inv_vg = 1.0 / v_g;
    P.v_phi = v_phi;
    P.b_over_e = boe;
    P.x_f = prm->x_f * L;
    P.y_c = prm->y_c * L;
    P.z_c = prm->z_c * L;
    P.q_slice = prm->q_slice * L;
    P.beta_f = prm->beta_f;
    P.x0_ff = prm->x0_ff * L;
    P.t0_ff = prm->t0_ff * L;
    if (focused) {
        const double w0 = prm->w0 * L;
        P.w0 = w0;
        P.inv_w0sq = 1.0 / (w0 * w0);
        P.x_r = P.k * w0 * w0 / 2.0;
        double xr = P.x_r;
        if (type == AP_PULSE_FF) xr *= (1.0 - prm->beta_f);
        P.inv_xr = 1.0 / xr;
        P.eps = w0 / P.x_r;
        P.inv_w0 = 1.0 / w0;
        P.np_e2 = prm->np_order >= 2 ? P.eps * P.eps : 0.0;
        P.np_e4 = prm->np_order >= 4 ? P.eps * P.eps * P.eps * P.eps : 0.0;
    }
    if (type == AP_PULSE_LG) {
        const int la = prm->lg_l < 0 ? -prm->lg_l : prm->lg_l;
        // normalise the peak |U| at focus to one (a0 is the peak field)
        double norm;
        if (prm->lg_p == 0) {
            norm = la == 0 ? 1.0 : std::pow(std::exp(1.0) / la, 0.5 * la);
        } else {
            auto prof = [&](double x) {
                return std::pow(x, 0.5 * la) * std::fabs(laguerre_host(prm->lg_p, la, x)) * std::exp(-0.5 * x);
            };
            // bracket the maximum on a grid, then golden-section refinement
            const int ng = 60000;
            int ib = 0;
            double best = -1.0;
            for (int m = 0; m <= ng; ++m) {
                const double v = prof(60.0 * m / ng);
                if (v > best) { best = v; ib = m; }
            }
            double lo = 60.0 * (ib > 0 ? ib - 1 : 0) / ng, hi = 60.0 * (ib < ng ? ib + 1 : ng) / ng;
            const double gr = 0.6180339887498949;
            double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
            double f1 = prof(x1), f2 = prof(x2);
            for (int it = 0; it < 200 && hi - lo > 1e-14; ++it) {
                if (f1 < f2) { lo = x1; x1 = x2; f1 = f2; x2 = lo + gr * (hi - lo); f2 = prof(x2); }
                else { hi = x2; x2 = x1; f2 = f1; x1 = hi - gr * (hi - lo); f1 = prof(x1); }
            }
            double mx = std::fmax(best, prof(0.5 * (lo + hi)));
            norm = 1.0 / mx;
        }
        P.lg_pref = norm * std::pow(std::sqrt(2.0) / P.w0, (double)la);
    }
    double s0 = 1.0;
    if (prm->sampling == AP_SAMPLE_BOUNDARY) {
        // App. B, exact form: S0/E0 = [cos(dt/2) + r sin(dt/2) cos(k dx/2)/sin(k dx/2)]/2,
        // r = dx/dt, k the vacuum Yee wavenumber along x: sin(k dx/2) = r sin(dt/2)
        const double dx = c->s.dx[0], dt = c->s.dt, r = dx / dt, h = 0.5 * dt;
        const double sk = r * std::sin(h);
        if (!(sk > 0.0 && sk < 1.0)) return fail(AP_E_ARG, "no propagating Yee mode along x for this dx, dt");
        s0 = 0.5 * (std::cos(h) + r * std::sin(h) * std::cos(std::asin(sk)) / sk);
    }
    c->P = P;
    c->s0 = s0;
    c->pulse_type = type;
    c->rec_n = 0;   // a recording holds for the pulse it was made with
    return AP_OK;
}

ap_status ap_step(ap_ctx *c, int64_t n_steps, uint32_t flags) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (n_steps < 0) return fail(AP_E_ARG, "n_steps must be >= 0");
    if (c->pulse_type < 0) return fail(AP_E_STATE, "ap_set_pulse must be called before ap_step");
    if (flags & ~(AP_STEP_CONTINUITY | AP_STEP_NO_YEE | AP_STEP_RECORD)) return fail(AP_E_ARG, "unknown step flag");
    if (c->s.dim == 0 && (flags & (AP_STEP_CONTINUITY | AP_STEP_NO_YEE)))
        return fail(AP_E_ARG, "grid flags on a gridless run");
    if (flags & AP_STEP_RECORD) {
        if (!c->ckpt) return fail(AP_E_STATE, "ap_set_checkpoints must be called before recording");
        const size_t need = c->revolve > 0 ? revolve_need(c->s, c->L, c->revolve)
                                           : ckpt_need(c->s, c->L, n_steps, c->segment);
        if (need > c->ckpt_bytes)
            return fail(AP_E_ARG, "checkpoint buffer too small: need " + std::to_string(need) + " bytes");
        c->rec_n = n_steps;
        c->rec_step0 = c->step;
        // binomial schedule: the states its first descent stores (slot 0 holds step 0)
        c->spine.clear();
        if (c->revolve > 0) {
            int32_t next = 1;
            for (int64_t m : revolve_spine(n_steps, c->revolve - 1)) c->spine.push_back({m, next++});
        }
    } else {
        c->rec_n = 0;   // any unrecorded step invalidates the recording
    }
    try {
        ap_status st = AP_OK;
        for (int64_t k = 0; k < n_steps && st == AP_OK; ++k) {
            if (c->s.dim == 0)
                st = c->s.prec == AP_F64 ? step_gridless<double>(c, flags) : step_gridless<float>(c, flags);
            else
                st = c->s.prec == AP_F64 ? step_gridded<double>(c, flags) : step_gridded<float>(c, flags);
            if (st == AP_OK) c->step++;
        }
        // the caller's arrays hold the state when the call returns
        const ap_status sr = c->s.dim == 0 ? AP_OK
                                           : (c->s.prec == AP_F64 ? restore_primary<double>(c) : restore_primary<float>(c));
        return st != AP_OK ? st : sr;
    } catch (...) {
        return fail(AP_E_NOMEM, "host allocation failed");
    }
}

ap_status ap_get_time(const ap_ctx *c, double *t, int64_t *step) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (t) *t = (c->s.t0 + (double)c->step * c->s.dt) / kTwoPi;
    if (step) *step = c->step;
    return AP_OK;
}

namespace {

// The diagnostics reductions of ap_gather_diag and ap_gather_diag_static.
// sums: (kMaxSpecies + 1) x kDiagVals doubles, partial: kDiagBlocks x
// kDiagVals doubles, both device.  Every slot read back is written by this
// call (per-block rows by the reduction kernels, sums by k_sum_partials), so
// neither needs clearing.
static ap_status gather_diag(ap_ctx *c, uint32_t what, ap_diag *out, double *sums, double *partial, bool timed) {
    if (!out) return fail(AP_E_ARG, "diag output is NULL");
    if (what & ~(AP_DIAG_PARTICLES | AP_DIAG_FIELDS)) return fail(AP_E_ARG, "unknown diag mask");
    ap_diag d;
    std::memset(&d, 0, sizeof(d));
    const RunShape &s = c->s;
    double host[(kMaxSpecies + 1) * kDiagVals];
    std::memset(host, 0, sizeof(host));
    {
        std::optional<Timer> tm;
        if (timed) tm.emplace(c, 3);
        if (what & AP_DIAG_PARTICLES) {
            for (int i = 0; i < s.nsp; ++i) {
                const ap_particles &p = c->buf.sp[i];
                hipError_t e;
                if (s.prec == AP_F64) {
                    DiagArgs<double> a{};
                    for (int k = 0; k < 3; ++k) { a.u[k] = (const double *)p.u[k]; a.off[k] = (const double *)(axis_active(s.dim, k) ? p.off[k] : nullptr); }
                    a.w = (const double *)p.w; a.proxy = (const double *)p.proxy; a.n = (int)s.np[i]; a.dim = s.dim;
                    a.cell = s.dim > 0 ? p.cell : nullptr; a.ncell = (uint32_t)s.ncell;
                    a.partial = partial; a.blocks = kDiagBlocks;
                    e = launch_diag_particles<double>(a, c->stream);
                } else {
                    DiagArgs<float> a{};
                    for (int k = 0; k < 3; ++k) { a.u[k] = (const float *)p.u[k]; a.off[k] = (const float *)(axis_active(s.dim, k) ? p.off[k] : nullptr); }
                    a.w = (const float *)p.w; a.proxy = (const float *)p.proxy; a.n = (int)s.np[i]; a.dim = s.dim;
                    a.cell = s.dim > 0 ? p.cell : nullptr; a.ncell = (uint32_t)s.ncell;
                    a.partial = partial; a.blocks = kDiagBlocks;
                    e = launch_diag_particles<float>(a, c->stream);
                }
                if (e != hipSuccess) return hip_fail(e, "ap_gather_diag");
                HIPCHK(launch_sum_partials(partial, kDiagBlocks, kDiagVals, sums + (size_t)i * kDiagVals, c->stream), "ap_gather_diag");
            }
        }
        if ((what & AP_DIAG_FIELDS) && s.dim > 0) {
            hipError_t e;
            if (s.prec == AP_F64) {
                double *F[6];
                for (int k = 0; k < 6; ++k) F[k] = static_cast<double *>(c->buf.grid) + (size_t)k * s.ncell;
                e = launch_diag_fields<double>(F, (size_t)s.ncell, partial, kDiagBlocks, c->stream);
            } else {
                float *F[6];
                for (int k = 0; k < 6; ++k) F[k] = static_cast<float *>(c->buf.grid) + (size_t)k * s.ncell;
                e = launch_diag_fields<float>(F, (size_t)s.ncell, partial, kDiagBlocks, c->stream);
            }
            if (e != hipSuccess) return hip_fail(e, "ap_gather_diag");
            HIPCHK(launch_sum_partials(partial, kDiagBlocks, 1, sums + (size_t)kMaxSpecies * kDiagVals, c->stream), "ap_gather_diag");
        }
    }
    unsigned long long cnt[kCounters];
    HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, c->stream), "ap_gather_diag");
    HIPCHK(hipMemcpyAsync(cnt, c->counters(), sizeof(cnt), hipMemcpyDeviceToHost, c->stream), "ap_gather_diag");
    // the step counters (dropped moves, skipped pushes, continuity maxima,
    // off-tile pushes) cover the steps since the previous ap_gather_diag
    HIPCHK(launch_fill_zero<unsigned long long>(c->counters(), 5, c->stream), "ap_gather_diag");
    HIPCHK(hipStreamSynchronize(c->stream), "ap_gather_diag");
    d.t = (s.t0 + (double)c->step * s.dt) / kTwoPi;
    d.step = c->step;
    int64_t nonfinite = 0;
    if (what & AP_DIAG_PARTICLES) {
        for (int i = 0; i < s.nsp; ++i) {
            const double *v = host + (size_t)i * kDiagVals;
            const double sw = v[0];
            d.sum_w[i] = sw;
            const double inv = sw != 0.0 ? 1.0 / sw : 0.0;
            for (int k = 0; k < 3; ++k) {
                d.mean_u[i][k] = v[1 + k] * inv;
                d.mean_u2[i][k] = v[4 + k] * inv;
            }
            d.mean_gamma[i] = v[7] * inv;
            d.kinetic[i] = c->s.m[i] * v[8];
            d.proxy_sum[i] = v[9];
            nonfinite += (int64_t)v[10];
        }
    }
    if ((what & AP_DIAG_FIELDS) && s.dim > 0) {
        // per unit transverse length (2-D) or area (1-D)
        double vol = s.dx[0] * (s.dim >= 2 ? s.dx[2] : 1.0) * (s.dim == 3 ? s.dx[1] : 1.0);
        d.field_energy = 0.5 * host[(size_t)kMaxSpecies * kDiagVals] * vol;
    }
    double rmax, jmax;
    std::memcpy(&rmax, &cnt[2], 8);
    std::memcpy(&jmax, &cnt[3], 8);
    d.continuity_max = rmax;
    d.j_max = jmax;
    d.n_nonfinite = nonfinite;
    d.n_fast = (int64_t)cnt[0];
    d.n_offtile = (int64_t)cnt[4];
    d.n_skipped = (int64_t)cnt[1];
    *out = d;
    if (d.n_nonfinite > 0 || d.n_fast > 0 || d.n_skipped > 0)
        return fail(AP_E_NUMERIC, "invalid particle state (" + std::to_string(d.n_nonfinite) + " now, " +
                                      std::to_string(d.n_skipped) + " skipped pushes) or " +
                                      std::to_string(d.n_fast) + " dropped moves since the last diagnostics");
    return AP_OK;
}

}  // namespace

ap_status ap_gather_diag(ap_ctx *c, uint32_t what, ap_diag *out) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    return gather_diag(c, what, out, c->wp<double>(c->L.sums), c->wp<double>(c->L.partial), true);
}

ap_status ap_gather_diag_static(ap_ctx *c, uint32_t what, ap_diag *out) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    double *base = static_scratch(c->device);
    if (!base) return fail(AP_E_STATE, "static scratch not resolved for device " + std::to_string(c->device));
    // no event timing: the pool may have to create events
    return gather_diag(c, what, out, base, base + kStaticSums, false);
}

ap_status ap_eval_pulse(ap_ctx *c, int64_t n, const double *xyz, double t, void *E, void *B) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(AP_E_ARG, "n must be in [0, 2^31)");
    if (!std::isfinite(t)) return fail(AP_E_ARG, "t must be finite");
    if (n > 0 && (!xyz || !E || !B)) return fail(AP_E_ARG, "NULL buffer");
    if (c->pulse_type < 0) return fail(AP_E_STATE, "ap_set_pulse must be called before ap_eval_pulse");
    hipError_t e;
    // positions arrive in lambda units; the device function works in internal units
    if (n == 0) return AP_OK;
    const double fd_delta = (c->P.current && c->P.fd) ? c->P.fd_delta : 0.0;
    if (c->s.prec == AP_F64)
        e = launch_eval_pulse<double>(c->P.type, plain_vars<double>(c->P, t * kTwoPi), fd_delta, n, xyz,
                                      static_cast<double *>(E), static_cast<double *>(B), c->stream);
    else
        e = launch_eval_pulse<float>(c->P.type, plain_vars<float>(c->P, t * kTwoPi), fd_delta, n, xyz,
                                     static_cast<float *>(E), static_cast<float *>(B), c->stream);
    if (e != hipSuccess) return hip_fail(e, "ap_eval_pulse");
    return AP_OK;
}

ap_status ap_read_proxy(ap_ctx *c, int32_t species, double *dst) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (species < 0 || species >= c->s.nsp) return fail(AP_E_ARG, "species index out of range");
    const bool has = c->s.dim > 0 ? c->s.has_proxy[species] : c->buf.sp[species].proxy != nullptr;
    if (!has) return fail(AP_E_ARG, "the species carries no emission proxy");
    const int n = (int)c->s.np[species];
    if (n > 0 && !dst) return fail(AP_E_ARG, "destination is NULL");
    hipError_t e = c->s.prec == AP_F64
                       ? launch_proxy_value<double>(static_cast<const double *>(c->buf.sp[species].proxy), dst, n,
                                                    c->stream)
                       : launch_proxy_value<float>(static_cast<const float *>(c->buf.sp[species].proxy), dst, n,
                                                   c->stream);
    if (e != hipSuccess) return hip_fail(e, "ap_read_proxy");
    return AP_OK;
}

ap_status ap_set_checkpoints(ap_ctx *c, void *dev, size_t bytes, int32_t segment) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (segment < 1) return fail(AP_E_ARG, "segment must be >= 1");
    if (!dev || bytes < ckpt_need(c->s, c->L, 1, 1))
        return fail(AP_E_ARG, "checkpoint buffer NULL or smaller than one recorded step needs");
    c->ckpt = static_cast<unsigned char *>(dev);
    c->ckpt_bytes = bytes;
    c->segment = segment;
    c->revolve = 0;
    c->spine.clear();
    c->rec_n = 0;
    return AP_OK;
}

ap_status ap_set_revolve(ap_ctx *c, void *dev, size_t bytes, int32_t slots) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (slots < 1) return fail(AP_E_ARG, "slots must be >= 1");
    const size_t need = revolve_need(c->s, c->L, slots);
    if (!dev || bytes < need)
        return fail(AP_E_ARG, "checkpoint buffer NULL or smaller than " + std::to_string(need) + " bytes");
    c->ckpt = static_cast<unsigned char *>(dev);
    c->ckpt_bytes = bytes;
    c->segment = 1;
    c->revolve = slots;
    c->spine.clear();
    c->rec_n = 0;
    return AP_OK;
}

ap_status ap_revolve_bytes(const ap_ctx *c, int32_t slots, size_t *bytes) {
    if (!c || !bytes) return fail(AP_E_ARG, "NULL argument");
    if (slots < 1) return fail(AP_E_ARG, "slots must be >= 1");
    *bytes = revolve_need(c->s, c->L, slots);
    return AP_OK;
}

ap_status ap_revolve_plan(int64_t n_steps, int32_t slots, int64_t *repeats, int64_t *forward_steps) {
    if (n_steps < 1 || slots < 1) return fail(AP_E_ARG, "n_steps and slots must be >= 1");
    if (!repeats && !forward_steps) return fail(AP_E_ARG, "NULL argument");
    if (slots == 1 && n_steps > (int64_t)1 << 31)
        return fail(AP_E_ARG, "one slot: n_steps too large (quadratic re-advancing)");
    int64_t cost = 0;
    const std::vector<int64_t> pos = revolve_spine(n_steps, slots - 1, &cost);
    if (repeats) {
        // the most any step is re-advanced: the cost of each segment's last step
        int64_t t = 0, at = 0;
        for (size_t i = 0; i <= pos.size(); ++i) {
            const int64_t end = i < pos.size() ? pos[i] : n_steps;
            const int64_t ti = revolve_repeats(end - at, slots - 1 - (int64_t)i);
            t = ti > t ? ti : t;
            at = end;
        }
        *repeats = t;
    }
    if (forward_steps) *forward_steps = cost;
    return AP_OK;
}

ap_status ap_set_adjoint_mode(ap_ctx *c, int32_t mode) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (mode != AP_ADJ_FROZEN && mode != AP_ADJ_COUPLED) return fail(AP_E_ARG, "unknown adjoint mode");
    if (mode == AP_ADJ_COUPLED && c->s.dim == 0) return fail(AP_E_ARG, "the coupled reading needs a grid");
    if (mode == AP_ADJ_COUPLED && (c->s.options & AP_GRID_OPEN_X))
        return fail(AP_E_UNSUPPORTED, "the coupled adjoint is built for periodic grids");
    c->s.adj_mode = mode;
    // the checkpoint layout depends on the mode: a buffer must be set again
    c->ckpt = nullptr;
    c->ckpt_bytes = 0;
    c->segment = 0;
    c->revolve = 0;
    c->spine.clear();
    c->rec_n = 0;
    return AP_OK;
}

ap_status ap_checkpoint_bytes(const ap_ctx *c, int64_t n_steps, int32_t segment, size_t *bytes) {
    if (!c || !bytes) return fail(AP_E_ARG, "NULL argument");
    if (n_steps < 1 || segment < 1) return fail(AP_E_ARG, "n_steps and segment must be >= 1");
    *bytes = ckpt_need(c->s, c->L, n_steps, segment);
    return AP_OK;
}

ap_status ap_backward(ap_ctx *c, int32_t species, const void *dl_du, const void *dl_dproxy,
                      const int32_t *param_ids, int32_t n_params, double *out) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (c->s.dim > 0 && dl_dproxy && (species < 0 || species >= c->s.nsp || !c->s.has_proxy[species]))
        return fail(AP_E_ARG, "the species carries no emission proxy");
    if (c->s.dim > 0 && c->P.sampling != AP_SAMPLE_PARTICLES)
        return fail(AP_E_UNSUPPORTED, "the adjoint of gridded runs needs the pulse evaluated per particle");
    if (c->rec_n <= 0) return fail(AP_E_STATE, "no recorded forward run (step with AP_STEP_RECORD first)");
    if (c->step != c->rec_step0 + c->rec_n) return fail(AP_E_STATE, "the state moved past the recorded window");
    if (species < 0 || species >= c->s.nsp) return fail(AP_E_ARG, "species index out of range");
    if (!dl_du || !out || (n_params > 0 && !param_ids)) return fail(AP_E_ARG, "NULL argument");
    if (n_params < 0 || n_params > 5) return fail(AP_E_ARG, "n_params must be 0..5");
    for (int k = 0; k < n_params; ++k) {
        if (param_ids[k] < AP_PARAM_A0 || param_ids[k] > AP_PARAM_CHIRP) return fail(AP_E_ARG, "unknown parameter id");
        for (int j = 0; j < k; ++j)
            if (param_ids[j] == param_ids[k]) return fail(AP_E_ARG, "repeated parameter id");
    }
    if (c->P.type == PT_NONE) return fail(AP_E_STATE, "no pulse set");
    try {
        if (c->s.dim > 0 && c->s.adj_mode == AP_ADJ_COUPLED)
            return c->s.prec == AP_F64
                       ? backward_coupled<double>(c, species, dl_du, dl_dproxy, param_ids, n_params, out)
                       : backward_coupled<float>(c, species, dl_du, dl_dproxy, param_ids, n_params, out);
        if (c->s.dim > 0)
            return c->s.prec == AP_F64 ? backward_grid<double>(c, species, dl_du, dl_dproxy, param_ids, n_params, out)
                                       : backward_grid<float>(c, species, dl_du, dl_dproxy, param_ids, n_params, out);
        return c->s.prec == AP_F64 ? backward_impl<double>(c, species, dl_du, dl_dproxy, param_ids, n_params, out)
                                   : backward_impl<float>(c, species, dl_du, dl_dproxy, param_ids, n_params, out);
    } catch (...) {
        return fail(AP_E_NOMEM, "host allocation failed");
    }
}

ap_status ap_timing_enable(ap_ctx *c, int32_t enable) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    c->timing = enable != 0;
    return AP_OK;
}

ap_status ap_timing_read(ap_ctx *c, ap_timing *out, int32_t reset) {
    if (!c || !out) return fail(AP_E_ARG, "NULL argument");
    HIPCHK(hipStreamSynchronize(c->stream), "ap_timing_read");
    for (const TimedPair &tp : c->pending) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, tp.a, tp.b), "ap_timing_read");
        c->acc_ms[tp.kind] += ms;
        c->acc_n[tp.kind] += 1;
        c->pool.push_back(tp.a);
        c->pool.push_back(tp.b);
    }
    c->pending.clear();
    c->acc_pushes += c->push_since_read;
    c->push_since_read = 0;
    out->ms_push = c->acc_ms[0];
    out->ms_yee = c->acc_ms[1];
    out->ms_sort = c->acc_ms[2];
    out->ms_other = c->acc_ms[3];
    out->n_push = c->acc_n[0];
    out->n_yee = c->acc_n[1];
    out->n_sort = c->acc_n[2];
    out->n_other = c->acc_n[3];
    out->pushes = c->acc_pushes;
    if (reset) {
        for (int k = 0; k < 4; ++k) { c->acc_ms[k] = 0; c->acc_n[k] = 0; }
        c->acc_pushes = 0;
    }
    return AP_OK;
}

ap_status ap_shift_window(ap_ctx *c, int32_t dir, const ap_inject *inject) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (!(c->s.options & AP_GRID_MOVING_WINDOW))
        return fail(AP_E_STATE, "the run was not created with AP_GRID_MOVING_WINDOW");
    if (dir != 1 && dir != -1) return fail(AP_E_ARG, "dir must be +1 or -1");
    try {
        return c->s.prec == AP_F64 ? shift_window_impl<double>(c, dir, inject)
                                   : shift_window_impl<float>(c, dir, inject);
    } catch (...) {
        return fail(AP_E_NOMEM, "host allocation failed");
    }
}

ap_status ap_get_window(const ap_ctx *c, double *x_min, int32_t *origin) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (x_min) *x_min = c->s.x_min[0] / kTwoPi;
    if (origin) *origin = c->s.xo;
    return AP_OK;
}

ap_status ap_window_due(const ap_ctx *c, double beta, double x_ref, double t_ref, int32_t *dir) {
    if (!c) return fail(AP_E_ARG, "context is NULL");
    if (!dir) return fail(AP_E_ARG, "dir output is NULL");
    if (!std::isfinite(beta) || !std::isfinite(x_ref) || !std::isfinite(t_ref))
        return fail(AP_E_ARG, "beta, x_ref and t_ref must be finite");
    if (c->s.dim == 0) return fail(AP_E_ARG, "a moving window needs a grid");
    // internal units: lengths in lambda / 2 pi, times in 1 / omega
    const double t = c->s.t0 + (double)c->step * c->s.dt;
    const double target = x_ref * kTwoPi + beta * (t - t_ref * kTwoPi);
    const double d = (target - c->s.x_min[0]) / c->s.dx[0];
    // half-open interval [-1/2, 1/2): a tie never shifts back and forth
    *dir = d >= 0.5 ? 1 : (d < -0.5 ? -1 : 0);
    return AP_OK;
}

ap_status ap_destroy(ap_ctx *c) {
    if (!c) return AP_OK;
    (void)hipStreamSynchronize(c->stream);
    for (const TimedPair &tp : c->pending) { hipEventDestroy(tp.a); hipEventDestroy(tp.b); }
    for (hipEvent_t e : c->pool) hipEventDestroy(e);
    delete c;
    return AP_OK;
}

}  // extern "C"

namespace {

// Gridless arguments for species i reading from and writing to the given state.
template <typename T>
GridlessArgs<T> gridless_args(ap_ctx *c, int i, int32_t *const icell[3], T *const off[3], T *const u[3],
                              int32_t *const icell_out[3], T *const off_out[3], T *const u_out[3], T *proxy,
                              double t) {
    const RunShape &s = c->s;
    GridlessArgs<T> a{};
    for (int k = 0; k < 3; ++k) {
        a.icell[k] = icell[k];
        a.off[k] = off[k];
        a.u[k] = u[k];
        a.icell_out[k] = icell_out[k];
        a.off_out[k] = off_out[k];
        a.u_out[k] = u_out[k];
        a.dx[k] = s.dx[k];
        a.x_min[k] = s.x_min[k];
    }
    a.proxy = proxy;
    a.n = (int)s.np[i];
    a.q_over_m = s.q[i] / s.m[i];
    a.dt = s.dt;
    a.t = t;
    a.n_bad = c->counters() + 1;
    a.W = plain_vars<T>(c->P, t);
    return a;
}

// Pointers of species i inside checkpoint slot k.
template <typename T> void slot_ptrs(ap_ctx *c, int64_t k, int i, int32_t *icell[3], T *off[3], T *u[3]) {
    const size_t N = (size_t)c->s.np[i];
    unsigned char *base = c->ckpt + (size_t)k * c->L.slot_bytes + c->L.slot_off[i];
    for (int a = 0; a < 3; ++a) icell[a] = reinterpret_cast<int32_t *>(base) + a * N;
    T *r = reinterpret_cast<T *>(base + 12 * N);
    for (int a = 0; a < 3; ++a) {
        off[a] = r + a * N;
        u[a] = r + (3 + a) * N;
    }
}

// Reverse sweep of the binomial schedule over relative steps [l, r), the
// state of step l in slot_l and sfree slots free below it.  advance(from, l,
// d, to) leaves the state of step l + d in slot `to` (-1: the working state);
// leaf(j, slot) runs reverse step j from the state in `slot` (-1: working).
// The states the recording sweep stored (stored) are used where the
// recursion asks for them.
struct Revolve {
    std::function<ap_status(int32_t, int64_t, int64_t, int32_t)> advance;
    std::function<ap_status(int64_t, int32_t)> leaf;
    std::vector<std::pair<int64_t, int32_t>> stored;
    std::vector<int32_t> pool;

    ap_status run(int64_t l, int64_t r, int32_t slot_l, int64_t sfree) {
        const int64_t n = r - l;
        if (n == 1) return leaf(l, slot_l);
        if (sfree == 0) {
            // no slot left: each step again from l
            for (int64_t j = r - 1; j > l; --j) {
                ap_status st = advance(slot_l, l, j - l, -1);
                if (st != AP_OK) return st;
                st = leaf(j, -1);
                if (st != AP_OK) return st;
            }
            return leaf(l, slot_l);
        }
        // the next state of the recording's first descent, if it lies in (l, r), else the split
        int64_t m = l + revolve_split(n, sfree);
        int32_t slot_m = -1;
        for (size_t k = 0; k < stored.size(); ++k)
            if (stored[k].first > l && stored[k].first < r) {
                m = stored[k].first;
                slot_m = stored[k].second;
                stored.erase(stored.begin() + (std::ptrdiff_t)k);
                break;
            }
        if (slot_m < 0) {
            if (pool.empty()) return fail(AP_E_STATE, "binomial schedule ran out of slots");
            slot_m = pool.back();
            pool.pop_back();
            const ap_status st = advance(slot_l, l, m - l, slot_m);
            if (st != AP_OK) return st;
        }
        ap_status st = run(m, r, slot_m, sfree - 1);
        if (st != AP_OK) return st;
        pool.push_back(slot_m);
        return run(l, m, slot_l, sfree);
    }
};

// A Revolve over the context's recording: slot 0 holds step 0, the spine
// its stored states, the other slots start free.
Revolve make_revolve(const ap_ctx *c) {
    Revolve R;
    R.stored = c->spine;
    for (int32_t k = c->revolve - 1; k > (int32_t)c->spine.size(); --k) R.pool.push_back(k);
    return R;
}

// Slot that the recording sweep stores the state of relative step k in, or
// -1: every segment's first step (segments), or step 0 and the first
// descent of the binomial schedule.
int64_t record_slot(const ap_ctx *c, int64_t k) {
    if (c->revolve == 0) return k % c->segment == 0 ? k / c->segment : -1;
    if (k == 0) return 0;
    for (const auto &e : c->spine)
        if (e.first == k) return e.second;
    return -1;
}

template <typename T> ap_status copy_state_to_slot(ap_ctx *c, int64_t k) {
    for (int i = 0; i < c->s.nsp; ++i) {
        const size_t N = (size_t)c->s.np[i];
        if (N == 0) continue;
        int32_t *ic[3];
        T *off[3], *u[3];
        slot_ptrs<T>(c, k, i, ic, off, u);
        const ap_particles &p = c->buf.sp[i];
        for (int a = 0; a < 3; ++a) {
            HIPCHK(hipMemcpyAsync(ic[a], p.icell[a], N * 4, hipMemcpyDeviceToDevice, c->stream), "checkpoint");
            HIPCHK(hipMemcpyAsync(off[a], p.off[a], N * sizeof(T), hipMemcpyDeviceToDevice, c->stream), "checkpoint");
            HIPCHK(hipMemcpyAsync(u[a], p.u[a], N * sizeof(T), hipMemcpyDeviceToDevice, c->stream), "checkpoint");
        }
    }
    return AP_OK;
}

template <typename T> ap_status step_gridless(ap_ctx *c, uint32_t flags) {
    const RunShape &s = c->s;
    if (flags & AP_STEP_RECORD) {
        const int64_t k = c->step - c->rec_step0;
        const int64_t slot = record_slot(c, k);
        if (slot >= 0) {
            const ap_status st = copy_state_to_slot<T>(c, slot);
            if (st != AP_OK) return st;
        }
    }
    Timer tm(c, 0);
    for (int i = 0; i < s.nsp; ++i) {
        if (s.np[i] == 0) continue;
        const ap_particles &p = c->buf.sp[i];
        T *off[3] = {static_cast<T *>(p.off[0]), static_cast<T *>(p.off[1]), static_cast<T *>(p.off[2])};
        T *u[3] = {static_cast<T *>(p.u[0]), static_cast<T *>(p.u[1]), static_cast<T *>(p.u[2])};
        GridlessArgs<T> a = gridless_args<T>(c, i, p.icell, off, u, p.icell, off, u, static_cast<T *>(p.proxy),
                                             s.t0 + (double)c->step * s.dt);
        HIPCHK(launch_gridless<T>(c->P.type, a, c->stream), "gridless push");
        c->push_since_read += s.np[i];
    }
    return AP_OK;
}

template <typename T>
ap_status backward_impl(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                        double *out) {
    const RunShape &s = c->s;
    const WorkLayout &L = c->L;
    const int n = (int)s.np[sp];
    double *lam[6];
    for (int k = 0; k < 6; ++k) lam[k] = c->wp<double>(L.lam[k]);
    double *partial = c->wp<double>(L.adj_partial);
    // tangent slots of the requested parameters (the amplitude needs none)
    int32_t slot[4] = {-1, -1, -1, -1};
    int nslot = 0;
    for (int k = 0; k < np_; ++k)
        if (ids[k] != AP_PARAM_A0) slot[nslot++] = ids[k];
    HIPCHK(launch_fill_zero<double>(partial, (size_t)L.adj_blocks * 5, c->stream), "backward");
    HIPCHK(launch_adjoint_init<T>(lam, static_cast<const T *>(dl_du), n, c->stream), "backward");
    // reverse step j (relative) from the state in slot k
    auto leaf = [&](int64_t j, int64_t k) -> ap_status {
        int32_t *ic[3];
        T *of[3], *u[3];
        slot_ptrs<T>(c, k, sp, ic, of, u);
        AdjointArgs<T> a{};
        for (int q = 0; q < 3; ++q) {
            a.icell[q] = ic[q];
            a.off[q] = of[q];
            a.u[q] = u[q];
            a.dx[q] = s.dx[q];
            a.x_min[q] = s.x_min[q];
        }
        for (int q = 0; q < 6; ++q) a.lam[q] = lam[q];
        a.lam_proxy = static_cast<const T *>(dl_dproxy);
        a.partial = partial;
        for (int q = 0; q < 4; ++q) a.slot[q] = slot[q];
        a.n = n;
        a.q_over_m = s.q[sp] / s.m[sp];
        a.dt = s.dt;
        a.t = s.t0 + (double)(c->rec_step0 + j) * s.dt;
        a.P = c->P;
        a.dim = 0;
        HIPCHK(launch_adjoint_step<T>(c->P.type, a, c->stream), "backward step");
        return AP_OK;
    };
    // d forward steps of the species from slot `from` (relative step l) into slot `to`
    auto advance = [&](int64_t from, int64_t l, int64_t d, int64_t to) -> ap_status {
        for (int64_t k = 0; k < d; ++k) {
            int32_t *ic_i[3], *ic_o[3];
            T *of_i[3], *u_i[3], *of_o[3], *u_o[3];
            slot_ptrs<T>(c, k == 0 ? from : to, sp, ic_i, of_i, u_i);
            slot_ptrs<T>(c, to, sp, ic_o, of_o, u_o);
            const double t = s.t0 + (double)(c->rec_step0 + l + k) * s.dt;
            GridlessArgs<T> a = gridless_args<T>(c, sp, ic_i, of_i, u_i, ic_o, of_o, u_o, nullptr, t);
            HIPCHK(launch_gridless<T>(c->P.type, a, c->stream), "backward replay");
        }
        return AP_OK;
    };
    if (c->revolve > 0) {
        // binomial schedule; slot c->revolve is the working state
        const int64_t work = c->revolve;
        Revolve R = make_revolve(c);
        R.advance = [&](int32_t from, int64_t l, int64_t d, int32_t to) {
            return advance(from, l, d, to >= 0 ? to : work);
        };
        R.leaf = [&](int64_t j, int32_t k) { return leaf(j, k >= 0 ? k : work); };
        const ap_status st = R.run(0, c->rec_n, 0, c->revolve - 1);
        if (st != AP_OK) return st;
    } else {
        const int64_t K = c->segment;
        const int64_t nseg = (c->rec_n + K - 1) / K;
        const int64_t inner0 = nseg;   // first inner slot
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t s0 = seg * K;
            const int64_t len = (c->rec_n - s0) < K ? (c->rec_n - s0) : K;
            // replay the segment forward from its checkpoint into the inner slots
            for (int64_t j = 0; j + 1 < len; ++j) {
                const ap_status st = advance(j == 0 ? seg : inner0 + j, s0 + j, 1, inner0 + j + 1);
                if (st != AP_OK) return st;
            }
            for (int64_t j = len - 1; j >= 0; --j) {
                const ap_status st = leaf(s0 + j, j == 0 ? seg : inner0 + j);
                if (st != AP_OK) return st;
            }
        }
    }
    double *sums = c->wp<double>(L.sums);
    HIPCHK(launch_sum_partials(partial, L.adj_blocks, 5, sums, c->stream), "backward");
    double host[5];
    HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, c->stream), "backward");
    HIPCHK(hipStreamSynchronize(c->stream), "backward");
    // internal -> lambda units for the length parameters (w0, focal position)
    const double unit[5] = {1.0, kTwoPi, kTwoPi, 1.0, 1.0};
    for (int k = 0; k < np_; ++k) out[k] = host[ids[k]] * unit[ids[k]];
    return AP_OK;
}

// ---- gridded checkpoints

template <typename T> struct SpBlock {
    int32_t *cell, *id;
    T *off[3], *u[3], *w, *proxy;
};

// Species i's arrays inside a slot block that starts at base.
template <typename T>
SpBlock<T> sp_block(unsigned char *base, const RunShape &s, int i, bool with_w, bool with_proxy) {
    SpBlock<T> b{};
    const size_t N = (size_t)s.np[i];
    b.cell = reinterpret_cast<int32_t *>(base);
    b.id = b.cell + N;
    T *r = reinterpret_cast<T *>(base + 8 * N);
    for (int a = 0; a < 3; ++a) {
        b.off[a] = axis_active(s.dim, a) ? r : nullptr;
        if (b.off[a]) r += N;
    }
    for (int a = 0; a < 3; ++a) {
        b.u[a] = r;
        r += N;
    }
    b.w = with_w ? r : nullptr;
    if (b.w) r += N;
    b.proxy = (with_proxy && s.has_proxy[i]) ? r : nullptr;
    return b;
}

template <typename T> SpBlock<T> live_block(ap_ctx *c, int i) {
    const ap_particles &p = c->buf.sp[i];
    SpBlock<T> b{};
    b.cell = p.cell;
    b.id = p.id;
    for (int a = 0; a < 3; ++a) {
        b.off[a] = axis_active(c->s.dim, a) ? static_cast<T *>(p.off[a]) : nullptr;
        b.u[a] = static_cast<T *>(p.u[a]);
    }
    b.w = static_cast<T *>(p.w);
    b.proxy = c->s.has_proxy[i] ? static_cast<T *>(p.proxy) : nullptr;
    return b;
}

// The sort's workspace copy of species i, as a block.
template <typename T> SpBlock<T> alt_block(ap_ctx *c, int i) {
    const WorkLayout &L = c->L;
    SpBlock<T> b{};
    b.cell = c->wp<int32_t>(L.alt_cell[i]);
    b.id = c->wp<int32_t>(L.alt_id[i]);
    for (int a = 0; a < 3; ++a) {
        b.off[a] = axis_active(c->s.dim, a) ? c->wp<T>(L.alt_off[i][a]) : nullptr;
        b.u[a] = c->wp<T>(L.alt_u[i][a]);
    }
    b.w = c->wp<T>(L.alt_w[i]);
    b.proxy = c->s.has_proxy[i] ? c->wp<T>(L.alt_proxy[i]) : nullptr;
    return b;
}

// Counting sort of species i's records in src by tile into its workspace
// copy: tile histogram and ranks, exclusive scan into the tile starts
// (L.start[i]), scatter.  interleave: the within-tile transpose stride (1
// keeps the order); free_slot: moving-window slot hints to update, or null.
// src.proxy null leaves the proxies out.
template <typename T>
ap_status tile_sort_to_alt(ap_ctx *c, int i, const SpBlock<T> &src, int32_t interleave, int32_t *free_slot) {
    const RunShape &s = c->s;
    const WorkLayout &L = c->L;
    int32_t *count = c->wp<int32_t>(L.count[i]);
    int32_t *start = c->wp<int32_t>(L.start[i]);
    int32_t *rank = c->wp<int32_t>(L.rank[i]);
    HIPCHK(launch_fill_zero<int32_t>(count, (size_t)s.ntiles, c->stream), "sort");
    SortArgs sa{};
    sa.cell = src.cell;
    sa.ncell = (uint32_t)s.ncell;
    sa.n = (int)s.np[i];
    sa.dim = s.dim;
    sa.fnx = FastDiv((uint32_t)s.n[0]);
    sa.fnxy = FastDiv((uint32_t)(s.n[0] * s.n[1]));
    sa.ftx = FastDiv((uint32_t)s.tile[0]);
    sa.fty = FastDiv((uint32_t)s.tile[1]);
    sa.ftz = FastDiv((uint32_t)s.tile[2]);
    for (int k = 0; k < 3; ++k) sa.ntile[k] = s.ntile[k];
    sa.count = count;
    sa.rank = rank;
    if (s.np[i] > 0) HIPCHK(launch_tile_count(sa, c->stream), "tile count");
    HIPCHK(launch_scan(count, start, (int32_t)s.ntiles, c->wp<int32_t>(L.scan_part), c->stream), "tile scan");
    const SpBlock<T> dst = alt_block<T>(c, i);
    ScatterArgs<T> sc{};
    sc.cell_src = src.cell;
    sc.cell_dst = dst.cell;
    for (int k = 0; k < 3; ++k) {
        sc.off_src[k] = dst.off[k] ? src.off[k] : nullptr;
        sc.off_dst[k] = dst.off[k];
        sc.u_src[k] = src.u[k];
        sc.u_dst[k] = dst.u[k];
    }
    sc.w_src = src.w;
    sc.w_dst = dst.w;
    sc.id_src = src.id;
    sc.id_dst = dst.id;
    sc.free_slot = free_slot;
    sc.proxy_src = src.proxy && dst.proxy ? src.proxy : nullptr;
    sc.proxy_dst = src.proxy && dst.proxy ? dst.proxy : nullptr;
    sc.rank = rank;
    sc.start = start;
    sc.ncell = (uint32_t)s.ncell;
    sc.interleave = interleave;
    sc.n = (int)s.np[i];
    sc.dim = s.dim;
    sc.fnx = sa.fnx;
    sc.fnxy = sa.fnxy;
    sc.ftx = sa.ftx;
    sc.fty = sa.fty;
    sc.ftz = sa.ftz;
    for (int k = 0; k < 3; ++k) sc.ntile[k] = s.ntile[k];
    HIPCHK(launch_scatter<T>(sc, c->stream), "tile scatter");
    return AP_OK;
}

template <typename T> ap_status copy_block(ap_ctx *c, const SpBlock<T> &dst, const SpBlock<T> &src, size_t N, bool w) {
    if (N == 0) return AP_OK;
    HIPCHK(hipMemcpyAsync(dst.cell, src.cell, N * 4, hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
    HIPCHK(hipMemcpyAsync(dst.id, src.id, N * 4, hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
    for (int a = 0; a < 3; ++a) {
        if (dst.off[a]) HIPCHK(hipMemcpyAsync(dst.off[a], src.off[a], N * sizeof(T), hipMemcpyDeviceToDevice, c->stream),
                               "checkpoint copy");
        HIPCHK(hipMemcpyAsync(dst.u[a], src.u[a], N * sizeof(T), hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
    }
    if (w) HIPCHK(hipMemcpyAsync(dst.w, src.w, N * sizeof(T), hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
    if (w && dst.proxy && src.proxy)
        HIPCHK(hipMemcpyAsync(dst.proxy, src.proxy, 2 * N * sizeof(T), hipMemcpyDeviceToDevice, c->stream),
               "checkpoint copy");
    return AP_OK;
}

unsigned char *ckpt_final(ap_ctx *c) { return c->ckpt + grid_ckpt(c->s).fixed; }
unsigned char *ckpt_outer(ap_ctx *c, int64_t k) {
    const GridCkpt G = grid_ckpt(c->s);
    return c->ckpt + G.fixed + (size_t)(1 + k) * G.outer;
}
unsigned char *ckpt_inner(ap_ctx *c, int64_t j) {
    const GridCkpt G = grid_ckpt(c->s);
    const int64_t nseg = (c->rec_n + c->segment - 1) / c->segment;
    return c->ckpt + G.fixed + (size_t)(1 + nseg) * G.outer + (size_t)j * G.inner;
}

// Whole state (every species, E2, B2) to a checkpoint slot or back.
template <typename T> ap_status save_ckpt(ap_ctx *c, unsigned char *slot, bool restore = false) {
    const RunShape &s = c->s;
    const GridCkpt G = grid_ckpt(s);
    for (int i = 0; i < s.nsp; ++i) {
        const SpBlock<T> live = live_block<T>(c, i), blk = sp_block<T>(slot + G.sp_off[i], s, i, true, true);
        const ap_status st = restore ? copy_block<T>(c, live, blk, (size_t)s.np[i], true)
                                     : copy_block<T>(c, blk, live, (size_t)s.np[i], true);
        if (st != AP_OK) return st;
    }
    unsigned char *grid = static_cast<unsigned char *>(c->buf.grid);
    const size_t fb = (size_t)6 * (size_t)s.ncell * sizeof(T);
    HIPCHK(hipMemcpyAsync(restore ? grid : slot + G.fields, restore ? slot + G.fields : grid, fb,
                          hipMemcpyDeviceToDevice, c->stream), "checkpoint copy");
    return AP_OK;
}

// Replay slot: E2, B2 and species sp at the start of a step.
template <typename T> ap_status save_replay(ap_ctx *c, unsigned char *slot, int sp) {
    const RunShape &s = c->s;
    const GridCkpt G = grid_ckpt(s);
    HIPCHK(hipMemcpyAsync(slot, c->buf.grid, (size_t)6 * (size_t)s.ncell * sizeof(T), hipMemcpyDeviceToDevice,
                          c->stream), "replay copy");
    if (s.adj_mode == AP_ADJ_COUPLED) {
        // every species, with weights (they scale the current)
        for (int i = 0; i < s.nsp; ++i) {
            SpBlock<T> live = live_block<T>(c, i);
            live.proxy = nullptr;
            const ap_status st =
                copy_block<T>(c, sp_block<T>(slot + G.inner_off[i], s, i, true, false), live, (size_t)s.np[i], true);
            if (st != AP_OK) return st;
        }
        return AP_OK;
    }
    return copy_block<T>(c, sp_block<T>(slot + G.inner_sp, s, sp, false, false), live_block<T>(c, sp),
                         (size_t)s.np[sp], false);
}

// Binomial schedule, gridded runs: the whole state of relative step l from
// slot `from` into the caller's arrays and the grid, d steps of the full
// loop, then (to >= 0) the state into slot `to`.
template <typename T> ap_status revolve_advance_grid(ap_ctx *c, int32_t from, int64_t l, int64_t d, int32_t to) {
    ap_status st = save_ckpt<T>(c, ckpt_outer(c, from), true);
    if (st != AP_OK) return st;
    c->step = c->rec_step0 + l;
    c->need_sort = true;
    for (int64_t k = 0; k < d; ++k) {
        st = step_gridded<T>(c, 0);
        if (st != AP_OK) return st;
        c->step++;
    }
    return to >= 0 ? save_ckpt<T>(c, ckpt_outer(c, to)) : AP_OK;
}

// Reverse sweep of a recorded gridded run (frozen-grid reading).  Each
// segment is restored from its checkpoint and replayed with the full loop
// (push, deposit, field update), storing E2, B2 and the species at the start
// of every step; the adjoint steps then run backwards over those slots.  The
// state after the last recorded step is put back at the end.
template <typename T>
ap_status backward_grid(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                        double *out) {
    const NoFuse nf(c);
    const RunShape &s = c->s;
    const GridCkpt G = grid_ckpt(s);
    const int n = (int)s.np[sp];
    unsigned long long *cnt = c->counters();
    unsigned long long saved[kCounters];
    {
        // the adjoint state is indexed by particle id: ids must be 0..n-1, each once
        int32_t *seen = c->wp<int32_t>(c->L.rank[sp]);
        HIPCHK(launch_fill_zero<int32_t>(seen, (size_t)n, c->stream), "backward");
        HIPCHK(hipMemcpyAsync(saved, cnt, sizeof(saved), hipMemcpyDeviceToHost, c->stream), "backward");
        HIPCHK(launch_fill_zero<unsigned long long>(cnt + 5, 1, c->stream), "backward");
        HIPCHK(launch_check_ids(c->buf.sp[sp].id, n, seen, cnt + 5, c->stream), "backward");
        unsigned long long bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, cnt + 5, sizeof(bad), hipMemcpyDeviceToHost, c->stream), "backward");
        HIPCHK(hipStreamSynchronize(c->stream), "backward");
        if (bad != 0) return fail(AP_E_ARG, "particle ids of the species are not a permutation of 0..n-1");
    }
    double *lam[6];
    for (int k = 0; k < 6; ++k) lam[k] = reinterpret_cast<double *>(c->ckpt + G.lam[k]);
    double *partial = reinterpret_cast<double *>(c->ckpt + G.partial);
    int32_t slot[4] = {-1, -1, -1, -1};
    int nslot = 0;
    for (int k = 0; k < np_; ++k)
        if (ids[k] != AP_PARAM_A0) slot[nslot++] = ids[k];
    ap_status st = save_ckpt<T>(c, ckpt_final(c));
    if (st != AP_OK) return st;
    HIPCHK(launch_fill_zero<double>(partial, (size_t)G.blocks * 5, c->stream), "backward");
    HIPCHK(launch_adjoint_init<T>(lam, static_cast<const T *>(dl_du), n, c->stream), "backward");
    const FastDiv fnx((uint32_t)s.n[0]), fnxy((uint32_t)(s.n[0] * s.n[1]));
    // reverse step j (relative) from E2, B2 at F and the species' block b
    auto leaf = [&](int64_t j, const T *F, const SpBlock<T> &b) -> ap_status {
        AdjointArgs<T> a{};
        a.xo = s.xo;
        for (int k = 0; k < 3; ++k) {
            a.off[k] = b.off[k];
            a.u[k] = b.u[k];
            a.dx[k] = s.dx[k];
            a.x_min[k] = s.x_min[k];
            a.G.n[k] = s.n[k];
        }
        for (int k = 0; k < 6; ++k) {
            a.lam[k] = lam[k];
            a.G.F[k] = F + (size_t)k * (size_t)s.ncell;
        }
        a.G.cell = b.cell;
        a.G.id = b.id;
        a.G.fnx = fnx;
        a.G.fnxy = fnxy;
        a.G.q_slice = c->P.q_slice;
        a.dim = s.dim;
        a.lam_proxy = static_cast<const T *>(dl_dproxy);   // by particle id, like dl_du
        a.partial = partial;
        for (int k = 0; k < 4; ++k) a.slot[k] = slot[k];
        a.n = n;
        a.q_over_m = s.q[sp] / s.m[sp];
        a.dt = s.dt;
        a.t = s.t0 + (double)(c->rec_step0 + j) * s.dt;
        a.P = c->P;
        HIPCHK(launch_adjoint_step<T>(c->P.type, a, c->stream), "backward step");
        return AP_OK;
    };
    if (c->revolve > 0) {
        Revolve R = make_revolve(c);
        R.advance = [&](int32_t from, int64_t l, int64_t d, int32_t to) {
            return revolve_advance_grid<T>(c, from, l, d, to);
        };
        R.leaf = [&](int64_t j, int32_t k) -> ap_status {
            if (k < 0) return leaf(j, static_cast<const T *>(c->buf.grid), live_block<T>(c, sp));
            unsigned char *slot_k = ckpt_outer(c, k);
            return leaf(j, reinterpret_cast<const T *>(slot_k + G.fields),
                        sp_block<T>(slot_k + G.sp_off[sp], s, sp, true, true));
        };
        st = R.run(0, c->rec_n, 0, c->revolve - 1);
        if (st != AP_OK) return st;
    } else {
        const int64_t K = c->segment;
        const int64_t nseg = (c->rec_n + K - 1) / K;
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t s0 = seg * K;
            const int64_t len = (c->rec_n - s0) < K ? (c->rec_n - s0) : K;
            st = save_ckpt<T>(c, ckpt_outer(c, seg), true);
            if (st != AP_OK) return st;
            c->step = c->rec_step0 + s0;
            c->need_sort = true;
            for (int64_t j = 0; j < len; ++j) {
                st = save_replay<T>(c, ckpt_inner(c, j), sp);
                if (st != AP_OK) return st;
                if (j + 1 < len) {
                    st = step_gridded<T>(c, 0);
                    if (st != AP_OK) return st;
                    c->step++;
                }
            }
            for (int64_t j = len - 1; j >= 0; --j) {
                unsigned char *slot_j = ckpt_inner(c, j);
                st = leaf(s0 + j, reinterpret_cast<const T *>(slot_j),
                          sp_block<T>(slot_j + G.inner_sp, s, sp, false, false));
                if (st != AP_OK) return st;
            }
        }
    }
    st = save_ckpt<T>(c, ckpt_final(c), true);
    if (st != AP_OK) return st;
    c->step = c->rec_step0 + c->rec_n;
    c->need_sort = true;
    HIPCHK(hipMemcpyAsync(cnt, saved, sizeof(saved), hipMemcpyHostToDevice, c->stream), "backward");
    double *sums = c->wp<double>(c->L.sums);
    HIPCHK(launch_sum_partials(partial, G.blocks, 5, sums, c->stream), "backward");
    double host[5];
    HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, c->stream), "backward");
    HIPCHK(hipStreamSynchronize(c->stream), "backward");
    const double unit[5] = {1.0, kTwoPi, kTwoPi, 1.0, 1.0};
    for (int k = 0; k < np_; ++k) out[k] = host[ids[k]] * unit[ids[k]];
    return AP_OK;
}

// Reverse sweep in the fully coupled reading: every species' adjoint state and
// the FP64 grid adjoints of E2, B2 run backwards together.  Per reverse step:
// the transposed Yee step (leaving dL/dJ = -dt lJt), then for each species
// the particle adjoint, which reads lJt through its current and adds its
// gather's adjoint to lE, lB.  Replay slots hold every species with weights.
template <typename T>
ap_status backward_coupled(ap_ctx *c, int sp, const void *dl_du, const void *dl_dproxy, const int32_t *ids, int np_,
                           double *out) {
    const NoFuse nf(c);
    const RunShape &s = c->s;
    const GridCkpt G = grid_ckpt(s);
    const size_t nc = (size_t)s.ncell;
    unsigned long long *cnt = c->counters();
    unsigned long long saved[kCounters];
    HIPCHK(hipMemcpyAsync(saved, cnt, sizeof(saved), hipMemcpyDeviceToHost, c->stream), "backward");
    for (int i = 0; i < s.nsp; ++i) {
        // each adjoint state is indexed by particle id: ids must be 0..n-1, each once
        if (s.np[i] == 0) continue;
        int32_t *seen = c->wp<int32_t>(c->L.rank[i]);
        HIPCHK(launch_fill_zero<int32_t>(seen, (size_t)s.np[i], c->stream), "backward");
        HIPCHK(launch_fill_zero<unsigned long long>(cnt + 5, 1, c->stream), "backward");
        HIPCHK(launch_check_ids(c->buf.sp[i].id, (int)s.np[i], seen, cnt + 5, c->stream), "backward");
        unsigned long long bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, cnt + 5, sizeof(bad), hipMemcpyDeviceToHost, c->stream), "backward");
        HIPCHK(hipStreamSynchronize(c->stream), "backward");
        if (bad != 0) {
            HIPCHK(hipMemcpyAsync(cnt, saved, sizeof(saved), hipMemcpyHostToDevice, c->stream), "backward");
            return fail(AP_E_ARG, "particle ids of species " + std::to_string(i) + " are not a permutation of 0..n-1");
        }
    }
    double *lam[kMaxSpecies][6];
    for (int i = 0; i < s.nsp; ++i)
        for (int k = 0; k < 6; ++k) lam[i][k] = reinterpret_cast<double *>(c->ckpt + G.lam_sp[i][k]);
    double *lE = reinterpret_cast<double *>(c->ckpt + G.lgrid), *lB = lE + 3 * nc, *lJt = lE + 6 * nc;
    double *partial = reinterpret_cast<double *>(c->ckpt + G.partial);
    int32_t slot[4] = {-1, -1, -1, -1};
    int nslot = 0;
    for (int k = 0; k < np_; ++k)
        if (ids[k] != AP_PARAM_A0) slot[nslot++] = ids[k];
    ap_status st = save_ckpt<T>(c, ckpt_final(c));
    if (st != AP_OK) return st;
    HIPCHK(launch_fill_zero<double>(partial, (size_t)G.blocks * 5, c->stream), "backward");
    HIPCHK(launch_fill_zero<double>(lE, 9 * nc, c->stream), "backward");
    for (int i = 0; i < s.nsp; ++i) {
        if (i == sp) {
            HIPCHK(launch_adjoint_init<T>(lam[i], static_cast<const T *>(dl_du), (int)s.np[i], c->stream), "backward");
        } else {
            for (int k = 0; k < 6; ++k) HIPCHK(launch_fill_zero<double>(lam[i][k], (size_t)s.np[i], c->stream), "backward");
        }
    }
    YeeArgsBase yb{};
    for (int k = 0; k < 3; ++k) {
        yb.n[k] = s.n[k];
        yb.dx[k] = s.dx[k];
    }
    yb.dt = s.dt;
    const FastDiv fnx((uint32_t)s.n[0]), fnxy((uint32_t)(s.n[0] * s.n[1]));
    // Each reverse step tile-sorts its state into the sort's workspace copy
    // (free here: every replay starts with a full sort) when a tile's box
    // (the tile plus the stencil margin, or the whole axis where that would
    // cover it) fits the LDS of the gather's adjoint and the tiles hold 2048
    // particles or fewer on average.  The three passes then take the sorted
    // copy, and the gather's adjoint runs one block per tile with its LDS
    // sized to that box.
    bool tile_ranges = s.dim >= 2;
    int64_t tile_box = 6;
    for (int ax = 0; ax < 3; ++ax)
        if (axis_active(s.dim, ax)) tile_box *= std::min<int64_t>(s.tile[ax] + 3, s.n[ax]);
    tile_ranges = tile_ranges && tile_box <= adjoint_scatter_lds_entries(s.dim);
    for (int i = 0; i < s.nsp; ++i) tile_ranges = tile_ranges && s.np[i] <= 2048 * s.ntiles;
    // reverse step j (relative) from E2, B2 at F and every species' block
    auto leaf = [&](int64_t j, const T *F, const SpBlock<T> *blk) -> ap_status {
        HIPCHK(launch_yee_adjoint(s.dim, lE, lB, lJt, yb, c->stream), "backward yee");
        for (int i = 0; i < s.nsp; ++i) {
            if (s.np[i] == 0) continue;
            const SpBlock<T> &b = blk[i];
            AdjointArgs<T> a{};
            // the state, tile-sorted into the sort's workspace copy when the
            // tile ranges are in use (the adjoint state is indexed by particle
            // id, so the passes may take the particles in any order)
            SpBlock<T> sb = b;
            if (tile_ranges && b.cell != c->wp<int32_t>(c->L.alt_cell[i])) {
                SpBlock<T> src = b;
                src.proxy = nullptr;
                const ap_status sst = tile_sort_to_alt<T>(c, i, src, 1, nullptr);
                if (sst != AP_OK) return sst;
                sb = alt_block<T>(c, i);
                sb.proxy = nullptr;
                a.tile_start = c->wp<int32_t>(c->L.start[i]);
                a.ntile = (int32_t)s.ntiles;
                for (int k = 0; k < 3; ++k) {
                    a.tile_dim[k] = s.tile[k];
                    a.tile_n[k] = s.ntile[k];
                }
                a.tile_margin = 0;
                a.scatter_cap = (int32_t)tile_box;
            }
            a.xo = s.xo;
            for (int k = 0; k < 3; ++k) {
                a.off[k] = sb.off[k];
                a.u[k] = sb.u[k];
                a.dx[k] = s.dx[k];
                a.x_min[k] = s.x_min[k];
                a.G.n[k] = s.n[k];
                a.lJ[k] = lJt + (size_t)k * nc;
                a.lEg[k] = lE + (size_t)k * nc;
                a.lBg[k] = lB + (size_t)k * nc;
            }
            for (int k = 0; k < 6; ++k) {
                a.lam[k] = lam[i][k];
                a.G.F[k] = F + (size_t)k * nc;
            }
            a.G.cell = sb.cell;
            a.G.id = sb.id;
            a.G.fnx = fnx;
            a.G.fnxy = fnxy;
            a.G.q_slice = c->P.q_slice;
            a.w = sb.w;
            a.q = s.q[i];
            a.dim = s.dim;
            a.gx0 = reinterpret_cast<double *>(c->ckpt + G.gx0);
            a.lam_proxy = i == sp ? static_cast<const T *>(dl_dproxy) : nullptr;
            a.partial = partial;
            for (int k = 0; k < 4; ++k) a.slot[k] = slot[k];
            a.n = (int)s.np[i];
            a.q_over_m = s.q[i] / s.m[i];
            a.dt = s.dt;
            a.t = s.t0 + (double)(c->rec_step0 + j) * s.dt;
            a.P = c->P;
            HIPCHK(launch_adjoint_step<T>(c->P.type, a, c->stream), "backward step");
        }
        return AP_OK;
    };
    SpBlock<T> blk[kMaxSpecies];
    if (c->revolve > 0) {
        Revolve R = make_revolve(c);
        R.advance = [&](int32_t from, int64_t l, int64_t d, int32_t to) {
            return revolve_advance_grid<T>(c, from, l, d, to);
        };
        R.leaf = [&](int64_t j, int32_t k) -> ap_status {
            if (k < 0) {
                for (int i = 0; i < s.nsp; ++i) blk[i] = live_block<T>(c, i);
                return leaf(j, static_cast<const T *>(c->buf.grid), blk);
            }
            unsigned char *slot_k = ckpt_outer(c, k);
            for (int i = 0; i < s.nsp; ++i) blk[i] = sp_block<T>(slot_k + G.sp_off[i], s, i, true, true);
            return leaf(j, reinterpret_cast<const T *>(slot_k + G.fields), blk);
        };
        st = R.run(0, c->rec_n, 0, c->revolve - 1);
        if (st != AP_OK) return st;
    } else {
        const int64_t K = c->segment;
        const int64_t nseg = (c->rec_n + K - 1) / K;
        for (int64_t seg = nseg - 1; seg >= 0; --seg) {
            const int64_t s0 = seg * K;
            const int64_t len = (c->rec_n - s0) < K ? (c->rec_n - s0) : K;
            st = save_ckpt<T>(c, ckpt_outer(c, seg), true);
            if (st != AP_OK) return st;
            c->step = c->rec_step0 + s0;
            c->need_sort = true;
            for (int64_t j = 0; j < len; ++j) {
                st = save_replay<T>(c, ckpt_inner(c, j), sp);
                if (st != AP_OK) return st;
                if (j + 1 < len) {
                    st = step_gridded<T>(c, 0);
                    if (st != AP_OK) return st;
                    c->step++;
                }
            }
            for (int64_t j = len - 1; j >= 0; --j) {
                unsigned char *slot_j = ckpt_inner(c, j);
                for (int i = 0; i < s.nsp; ++i) blk[i] = sp_block<T>(slot_j + G.inner_off[i], s, i, true, false);
                st = leaf(s0 + j, reinterpret_cast<const T *>(slot_j), blk);
                if (st != AP_OK) return st;
            }
        }
    }
    st = save_ckpt<T>(c, ckpt_final(c), true);
    if (st != AP_OK) return st;
    c->step = c->rec_step0 + c->rec_n;
    c->need_sort = true;
    HIPCHK(hipMemcpyAsync(cnt, saved, sizeof(saved), hipMemcpyHostToDevice, c->stream), "backward");
    double *sums = c->wp<double>(c->L.sums);
    HIPCHK(launch_sum_partials(partial, G.blocks, 5, sums, c->stream), "backward");
    double host[5];
    HIPCHK(hipMemcpyAsync(host, sums, sizeof(host), hipMemcpyDeviceToHost, c->stream), "backward");
    HIPCHK(hipStreamSynchronize(c->stream), "backward");
    const double unit[5] = {1.0, kTwoPi, kTwoPi, 1.0, 1.0};
    for (int k = 0; k < np_; ++k) out[k] = host[ids[k]] * unit[ids[k]];
    return AP_OK;
}

// Window arguments of species i: leaving storage column col, injected
// particles (or none) required in window column in_col.
template <typename T> WindowArgs<T> window_args(ap_ctx *c, int i, int col, int in_col, const ap_inject *inject) {
    const RunShape &s = c->s;
    const ap_particles &p = c->buf.sp[i];
    WindowArgs<T> a{};
    a.cell = p.cell;
    a.id = p.id;
    for (int k = 0; k < 3; ++k) {
        a.off[k] = axis_active(s.dim, k) ? static_cast<T *>(p.off[k]) : nullptr;
        a.u[k] = static_cast<T *>(p.u[k]);
    }
    a.w = static_cast<T *>(p.w);
    a.proxy = s.has_proxy[i] ? static_cast<T *>(p.proxy) : nullptr;
    a.n = (int32_t)s.np[i];
    a.ncell = (uint32_t)s.ncell;
    a.nx = s.n[0];
    a.fnx = FastDiv((uint32_t)s.n[0]);
    a.col = col;
    a.freemap = c->wp<uint32_t>(c->L.wmap[i]);
    a.free_slot = c->wp<int32_t>(c->L.wslot[i]);
    a.miss = c->wp<unsigned long long>(c->L.wcnt) + 1 + 2 * kMaxSpecies + i;
    a.frank = c->wp<int32_t>(c->L.wfrank);
    a.words = (int32_t)((s.np[i] + 31) / 32);
    a.in_col = in_col;
    if (inject && inject[i].n > 0) {
        const ap_inject &in = inject[i];
        a.in_cell = in.cell;
        for (int k = 0; k < 3; ++k) {
            a.in_off[k] = axis_active(s.dim, k) ? static_cast<const T *>(in.off[k]) : nullptr;
            a.in_u[k] = static_cast<const T *>(in.u[k]);
        }
        a.in_w = static_cast<const T *>(in.w);
        a.n_inj = (int32_t)in.n;
    }
    return a;
}

// Free-id maps from the free slots passed at ap_init; ids checked for range.
template <typename T> ap_status window_init(ap_ctx *c) {
    const RunShape &s = c->s;
    unsigned long long *cnt = c->wp<unsigned long long>(c->L.wcnt);
    HIPCHK(launch_fill_zero<unsigned long long>(cnt, kWinCounters, c->stream), "ap_init");
    for (int i = 0; i < s.nsp; ++i) {
        WindowArgs<T> a = window_args<T>(c, i, 0, 0, nullptr);
        HIPCHK(launch_fill_zero<uint32_t>(a.freemap, (size_t)a.words, c->stream), "ap_init");
        a.count = cnt;
        a.count_free = cnt + 1 + i;
        HIPCHK(launch_window_init<T>(a, c->stream), "ap_init");
    }
    unsigned long long h[kWinCounters];
    HIPCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream), "ap_init");
    HIPCHK(hipStreamSynchronize(c->stream), "ap_init");
    HIPCHK(launch_fill_zero<unsigned long long>(cnt, kWinCounters, c->stream), "ap_init");
    if (h[0] != 0) return fail(AP_E_ARG, "particle ids must lie in [0, n) (moving window)");
    for (int i = 0; i < s.nsp; ++i) c->n_free[i] = (int64_t)h[1 + i];
    return AP_OK;
}

// One shift of the ring window: the storage column that leaves (the
// window's first column for dir = +1, its last for dir = -1) is cleared and
// becomes the entering column; its particles are freed and the injected ones
// take the smallest free ids.  One synchronisation, for the checks.
template <typename T> ap_status shift_window_impl(ap_ctx *c, int32_t dir, const ap_inject *inject) {
    const RunShape &s = c->s;
    const int nx = s.n[0];
    const int col = dir > 0 ? s.xo : (s.xo + nx - 1) % nx;
    const int in_col = dir > 0 ? nx - 1 : 0;
    unsigned long long *cnt = c->wp<unsigned long long>(c->L.wcnt);
    // validate everything before changing anything
    for (int i = 0; i < s.nsp; ++i) {
        const int64_t k = inject ? inject[i].n : 0;
        if (k < 0 || k > s.np[i]) return fail(AP_E_ARG, "species " + std::to_string(i) + ": bad injection count");
        if (k > 0) {
            const ap_inject &in = inject[i];
            bool okp = in.cell && in.u[0] && in.u[1] && in.u[2] && in.w;
            for (int a = 0; a < 3; ++a) okp = okp && (axis_active(s.dim, a) ? in.off[a] != nullptr : true);
            if (!okp) return fail(AP_E_ARG, "species " + std::to_string(i) + ": a required injection array is NULL");
        }
    }
    // injected particles checked; the leavers of the last shift read back;
    // where the injection exceeds the free slots known so far, this shift's
    // leavers counted ahead
    for (int i = 0; i < s.nsp; ++i) {
        WindowArgs<T> a = window_args<T>(c, i, col, in_col, inject);
        a.count = cnt;
        HIPCHK(launch_window_check_inject<T>(a, c->stream), "shift window");
        a.count = cnt + 1 + kMaxSpecies + i;
        if (inject && inject[i].n > c->n_free[i]) HIPCHK(launch_window_count_leavers<T>(a, c->stream), "shift window");
    }
    unsigned long long h[kWinCounters];
    HIPCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream), "shift window");
    HIPCHK(hipStreamSynchronize(c->stream), "shift window");
    HIPCHK(launch_fill_zero<unsigned long long>(cnt, kWinCounters, c->stream), "shift window");
    for (int i = 0; i < s.nsp; ++i) c->n_free[i] += (int64_t)h[1 + i];
    if (h[0] != 0)
        return fail(AP_E_ARG, "injected particles must sit in the entering column (window column " +
                                  std::to_string(in_col) + ") with offsets in [0, 1)");
    for (int i = 0; i < s.nsp; ++i) {
        const int64_t k = inject ? inject[i].n : 0;
        const int64_t avail = c->n_free[i] + (k > c->n_free[i] ? (int64_t)h[1 + kMaxSpecies + i] : 0);
        if (k > avail)
            return fail(AP_E_ARG, "species " + std::to_string(i) + ": " + std::to_string(k) +
                                      " injected particles but " + std::to_string(avail) + " free slots");
    }
    // apply: the column's fields, then per species leavers and injection
    T *grid = static_cast<T *>(c->buf.grid);
    T *F[6];
    for (int k = 0; k < 6; ++k) F[k] = grid + (size_t)k * (size_t)s.ncell;
    HIPCHK(launch_window_column<T>(F, col, nx, (size_t)s.ncell, c->stream), "shift window");
    // 2-D runs push in place between full sorts, moving a particle less than
    // a cell per step: a particle now in the leaving column sat, at the last
    // sort, within S = (steps since) cells of it, so its slot lies in the
    // range of a tile column meeting [col - S, col + S] -- unless it was
    // injected since, and then it is listed.  Otherwise (3-D, 1-D rows, a
    // pending re-sort, an overflowed list) every cell is read.
    LeaveTiles lt{};
    bool by_tiles = false;
    if (s.dim == 2 && c->sorted_once && !c->need_sort && !c->inj_overflow) {
        const int64_t S = c->step - c->sort_step;
        const int TX = s.tile[0], ntx = s.ntile[0];
        if (S >= 0 && 2 * S + 1 < nx) {
            const int lo = (int)(((col - S) % nx + nx) % nx), hi = (int)((col + S) % nx);
            const int tlo = lo / TX, thi = hi / TX;
            lt.tx0 = tlo;
            // tile columns from lo's to hi's; an interval that crosses the ring's
            // end and comes back into lo's tile column meets all of them
            lt.ncols = lo <= hi ? thi - tlo + 1 : (thi >= tlo ? ntx : ntx - tlo + thi + 1);
            lt.ntile_x = ntx;
            lt.ntile_z = s.ntile[2];
            by_tiles = lt.ncols < ntx;
        }
    }
    for (int i = 0; i < s.nsp; ++i) {
        if (s.np[i] == 0) continue;
        WindowArgs<T> a = window_args<T>(c, i, col, in_col, inject);
        a.count = cnt + 1 + i;   // leavers, read back at the next shift
        if (by_tiles) {
            lt.start = c->wp<int32_t>(c->L.start[i]);
            lt.list = c->wp<int32_t>(c->L.winj[i]);
            lt.list_n = (int32_t)c->inj_n[i];
            HIPCHK(launch_window_leave_tiles<T>(a, lt, c->stream), "shift window");
        } else {
            HIPCHK(launch_window_leave<T>(a, c->stream), "shift window");
        }
        if (a.n_inj == 0) continue;
        int32_t *pop = c->wp<int32_t>(c->L.wpop);
        int32_t *frank = c->wp<int32_t>(c->L.wfrank);
        HIPCHK(launch_window_popcount(a.freemap, a.words, pop, c->stream), "shift window");
        HIPCHK(launch_scan(pop, frank, a.words, c->wp<int32_t>(c->L.wpart), c->stream), "shift window");
        if (s.dim == 2 && !c->inj_overflow && c->inj_n[i] + a.n_inj <= c->L.winj_cap[i])
            a.inj_list = c->wp<int32_t>(c->L.winj[i]) + c->inj_n[i];
        HIPCHK(launch_window_fill<T>(a, c->stream), "shift window");
        if (a.inj_list) c->inj_n[i] += a.n_inj;
        else if (s.dim == 2) c->inj_overflow = true;
        HIPCHK(launch_window_clear(a.freemap, frank, a.words, a.n_inj, c->stream), "shift window");
        c->n_free[i] -= a.n_inj;
    }
    c->s.x_min[0] += dir * s.dx[0];
    c->s.xo = (s.xo + dir + nx) % nx;
    // 2-D and 3-D pushes take particles outside their tile; 1-D rows need
    // every particle in its row's range, and the 3-D re-sort ranks the last
    // push wrote no longer match the freed and filled slots
    if (s.dim != 2) c->need_sort = true;
    c->keys_valid = false;
    c->rec_n = 0;
    return AP_OK;
}

template <typename T> ap_status step_gridded(ap_ctx *c, uint32_t flags) {
    const RunShape &s = c->s;
    const WorkLayout &L = c->L;
    T *grid = static_cast<T *>(c->buf.grid);
    const size_t nc = (size_t)s.ncell;
    T *F[9];
    for (int k = 0; k < 9; ++k) F[k] = grid + (size_t)k * nc;
    const FastDiv fnx((uint32_t)s.n[0]);
    const FastDiv fnxy((uint32_t)(s.n[0] * s.n[1]));
    if (flags & AP_STEP_RECORD) {
        const int64_t k = c->step - c->rec_step0;
        const int64_t slot = record_slot(c, k);
        if (slot >= 0) {
            const ap_status st = save_ckpt<T>(c, ckpt_outer(c, slot));
            if (st != AP_OK) return st;
        }
    }
    // Re-sort.  1-D and 2-D runs (and recording or replaying steps) sort in
    // full every sort_every steps and push in place between sorts.  3-D runs
    // sort in full once; afterwards each push writes, per particle, its rank
    // in the tile of its new cell, and the next step builds from those ranks
    // the permutation its push reads through, writing the particles in tile
    // order into the other buffer (caller's arrays / workspace copy).
    const bool fuse = s.dim == 3 && !(flags & AP_STEP_RECORD) && !c->no_fuse;
    if (!fuse && c->state_alt) {
        const ap_status st = restore_primary<T>(c);
        if (st != AP_OK) return st;
    }
    const bool do_sort = !c->sorted_once || c->need_sort || (fuse ? !c->keys_valid : (c->step % s.sort_every) == 0);
    const bool from_perm = fuse && !do_sort;
    bool from_alt = false;
    if (do_sort) {
        if (c->state_alt) {
            const ap_status st = restore_primary<T>(c);
            if (st != AP_OK) return st;
        }
        Timer tm(c, 2);
        for (int i = 0; i < s.nsp; ++i) {
            // The first sort starts from the caller's order (typically cell
            // by cell) and interleaves it; later sorts start from an
            // interleaved order, which ranks within a tile preserve, so they
            // keep it (and write their slots contiguously).
            const double ppc = (double)s.np[i] / (double)s.ncell;
            int M = (int)std::lround(ppc);
            M = M < 1 ? 1 : (M > 64 ? 64 : M);
            int32_t *free_slot = (s.options & AP_GRID_MOVING_WINDOW) ? c->wp<int32_t>(L.wslot[i]) : nullptr;
            const ap_status st = tile_sort_to_alt<T>(c, i, live_block<T>(c, i), c->sorted_once ? 1 : M, free_slot);
            if (st != AP_OK) return st;
        }
        c->sorted_once = true;
        c->need_sort = false;
        c->sort_step = c->step;
        for (int i = 0; i < kMaxSpecies; ++i) c->inj_n[i] = 0;
        c->inj_overflow = false;
        from_alt = true;
    } else if (from_perm) {
        // the permutation from the ranks the last push wrote (into the buffer holding the state)
        Timer tm(c, 2);
        for (int i = 0; i < s.nsp; ++i) {
            int32_t *count = c->wp<int32_t>(L.count[i]);
            int32_t *start = c->wp<int32_t>(L.start[i]);
            const int32_t *stay = c->wp<int32_t>(L.stay[i]);
            HIPCHK(launch_resort_counts(stay, c->wp<int32_t>(L.mcount[i]), count, (int32_t)s.ntiles, c->stream),
                   "re-sort counts");
            HIPCHK(launch_scan(count, start, (int32_t)s.ntiles, c->wp<int32_t>(L.scan_part), c->stream), "tile scan");
            PermArgs pa{};
            pa.cell = c->state_alt ? c->wp<int32_t>(L.alt_cell[i]) : c->buf.sp[i].cell;
            pa.key = c->wp<int32_t>(L.key[i]);
            pa.start = start;
            pa.stay = stay;
            // mover ranks: the entering counts are no longer needed once summed
            pa.mrank = c->wp<int32_t>(L.mcount[i]);
            HIPCHK(launch_fill_zero<int32_t>(pa.mrank, (size_t)s.ntiles, c->stream), "re-sort counts");
            pa.perm = c->wp<int32_t>(L.perm[i]);
            pa.ncell = (uint32_t)s.ncell;
            pa.n = (int)s.np[i];
            pa.dim = s.dim;
            pa.fnx = fnx;
            pa.fnxy = fnxy;
            pa.ftx = FastDiv((uint32_t)s.tile[0]);
            pa.fty = FastDiv((uint32_t)s.tile[1]);
            pa.ftz = FastDiv((uint32_t)s.tile[2]);
            for (int k = 0; k < 3; ++k) pa.ntile[k] = s.ntile[k];
            HIPCHK(launch_resort_perm(pa, c->stream), "re-sort permutation");
        }
    }
    if (fuse) {
        // this push counts the particles entering each tile
        Timer tm(c, 2);
        for (int i = 0; i < s.nsp; ++i)
            HIPCHK(launch_fill_zero<int32_t>(c->wp<int32_t>(L.mcount[i]), (size_t)s.ntiles, c->stream), "re-sort counts");
    }
    // buffers the push reads and writes: after a full sort, the sorted
    // workspace copy -> caller's arrays; fused 3-D steps, the buffer holding
    // the state -> the other one; otherwise in place
    const bool in_alt = from_alt || (from_perm && c->state_alt);
    const bool out_alt = from_perm && !c->state_alt;
    PushArgs<T> a{};
    a.nsp = s.nsp;
    for (int i = 0; i < s.nsp; ++i) {
        const ap_particles &p = c->buf.sp[i];
        SpeciesIO<T> &io = a.sp[i];
        for (int k = 0; k < 3; ++k) {
            const bool act = axis_active(s.dim, k);
            T *pr_off = act ? static_cast<T *>(p.off[k]) : nullptr;
            T *al_off = act ? c->wp<T>(L.alt_off[i][k]) : nullptr;
            io.off_out[k] = out_alt ? al_off : pr_off;
            io.u_out[k] = out_alt ? c->wp<T>(L.alt_u[i][k]) : static_cast<T *>(p.u[k]);
            io.off_in[k] = in_alt ? al_off : pr_off;
            io.u_in[k] = in_alt ? c->wp<T>(L.alt_u[i][k]) : static_cast<T *>(p.u[k]);
        }
        io.cell_out = out_alt ? c->wp<int32_t>(L.alt_cell[i]) : p.cell;
        io.w_out = out_alt ? c->wp<T>(L.alt_w[i]) : static_cast<T *>(p.w);
        io.id_out = out_alt ? c->wp<int32_t>(L.alt_id[i]) : p.id;
        io.cell_in = in_alt ? c->wp<int32_t>(L.alt_cell[i]) : p.cell;
        io.w_in = in_alt ? c->wp<T>(L.alt_w[i]) : static_cast<T *>(p.w);
        io.id_in = in_alt ? c->wp<int32_t>(L.alt_id[i]) : p.id;
        io.copy_static = (from_alt || from_perm) ? 1 : 0;
        T *pr_proxy = s.has_proxy[i] ? static_cast<T *>(p.proxy) : nullptr;
        T *al_proxy = s.has_proxy[i] ? c->wp<T>(L.alt_proxy[i]) : nullptr;
        io.proxy_out = out_alt ? al_proxy : pr_proxy;
        io.proxy_in = in_alt ? al_proxy : pr_proxy;
        io.tile_start = c->wp<int32_t>(L.start[i]);
        io.perm = from_perm ? c->wp<int32_t>(L.perm[i]) : nullptr;
        io.key_out = fuse ? c->wp<int32_t>(L.key[i]) : nullptr;
        io.mcount = fuse ? c->wp<int32_t>(L.mcount[i]) : nullptr;
        io.stay = fuse ? c->wp<int32_t>(L.stay[i]) : nullptr;
        io.n = (int)s.np[i];
        io.q_over_m = s.q[i] / s.m[i];
        io.q = s.q[i];
    }
    a.xo = s.xo;
    for (int k = 0; k < 3; ++k) {
        a.E[k] = F[k];
        a.B[k] = F[3 + k];
        a.J[k] = F[6 + k];
        a.Jacc[k] = s.prec == AP_F32 ? c->wp<double>(L.jacc) + (size_t)k * nc : reinterpret_cast<double *>(F[6 + k]);
        a.n[k] = s.n[k];
        a.tile[k] = s.tile[k];
        a.ntile[k] = s.ntile[k];
        a.dx[k] = s.dx[k];
        a.x_min[k] = s.x_min[k];
        a.reg[k] = axis_active(s.dim, k) ? s.tile[k] + kHaloLo + kHaloHi : 1;
    }
    a.fnx = fnx;
    a.fnxy = fnxy;
    a.fntx = FastDiv((uint32_t)s.ntile[0]);
    a.fntxy = FastDiv((uint32_t)(s.ntile[0] * s.ntile[1]));
    a.splits = s.splits;
    a.n_logical = (int32_t)(s.ntiles * s.splits);
    a.xcd_chunk = s.dim == 3 && s.splits == 1 && s.ntile[0] >= 8 ? s.ntile[0] / 8 : 1;
    a.dt = s.dt;
    a.t = s.t0 + (double)c->step * s.dt;
    a.n_fast = c->counters() + 0;
    a.n_bad = c->counters() + 1;
    a.n_offtile = c->counters() + 4;
    a.q_slice = c->P.q_slice;
    a.pulse = c->P.type;
    a.W = plain_vars<T>(c->P, a.t);
    // grid-sampled pulse: the push gathers E2 + E1 and B2 + B1 from the
    // workspace and evaluates nothing per particle
    const bool on_grid = c->P.sampling == AP_SAMPLE_GRID && c->P.type != PT_NONE;
    if (on_grid) {
        Timer tm(c, 3);
        SampleArgs<T> sa{};
        T *S = c->wp<T>(L.esamp);
        for (int k = 0; k < 6; ++k) {
            sa.F[k] = F[k];
            sa.S[k] = S + (size_t)k * nc;
        }
        sa.xo = s.xo;
        for (int k = 0; k < 3; ++k) {
            sa.n[k] = s.n[k];
            sa.dx[k] = s.dx[k];
            sa.x_min[k] = s.x_min[k];
            a.E[k] = sa.S[k];
            a.B[k] = sa.S[3 + k];
        }
        sa.dim = s.dim;
        sa.fnx = fnx;
        sa.fnxy = fnxy;
        sa.q_slice = c->P.q_slice;
        sa.W = a.W;
        sa.fd_b = (c->P.current && c->P.fd) ? 1 : 0;
        sa.fd_delta = c->P.fd_delta;
        HIPCHK(launch_sample_pulse<T>(c->P.type, sa, c->stream), "sample pulse");
    }
    // launched through the x_min boundary: no analytic field anywhere
    const bool launch = c->P.sampling == AP_SAMPLE_BOUNDARY && c->P.type != PT_NONE;
    const int push_pulse = (on_grid || launch) ? (int)PT_NONE : c->P.type;

    {
        Timer tm(c, 3);
        HIPCHK(launch_fill_zero<double>(a.Jacc[0], 3 * nc, c->stream), "clear J");
    }
    double *rho0 = c->wp<double>(L.rho0), *rho1 = c->wp<double>(L.rho1);
    auto deposit_rho = [&](double *rho, bool use_in) -> ap_status {
        HIPCHK(launch_fill_zero<double>(rho, nc, c->stream), "rho");
        for (int i = 0; i < s.nsp; ++i) {
            RhoArgs<T> ra{};
            ra.cell = use_in ? a.sp[i].cell_in : a.sp[i].cell_out;
            for (int k = 0; k < 3; ++k) ra.off[k] = use_in ? a.sp[i].off_in[k] : a.sp[i].off_out[k];
            ra.w = use_in ? a.sp[i].w_in : a.sp[i].w_out;
            ra.n = (int)s.np[i];
            ra.q = s.q[i];
            for (int k = 0; k < 3; ++k) ra.nn[k] = s.n[k];
            ra.fnx = fnx;
            ra.fnxy = fnxy;
            ra.dim = s.dim;
            ra.rho = rho;
            HIPCHK(launch_rho<T>(ra, c->stream), "rho");
        }
        return AP_OK;
    };
    if (flags & AP_STEP_CONTINUITY) {
        Timer tm(c, 3);
        const ap_status st = deposit_rho(rho0, true);
        if (st != AP_OK) return st;
    }
    {
        Timer tm(c, 0);
        hipError_t e = s.dim == 1   ? launch_push_deposit_1d<T>(push_pulse, a, 256, c->stream)
                       : s.dim == 2 ? launch_push_deposit_2d<T>(push_pulse, a, 256, c->stream)
                                  : launch_push_deposit_3d<T>(push_pulse, a, 256, c->stream);
        if (e != hipSuccess) return hip_fail(e, "push/deposit");
        for (int i = 0; i < s.nsp; ++i) c->push_since_read += s.np[i];
        c->keys_valid = fuse;
        c->state_alt = out_alt;
    }
    if (s.prec == AP_F32) {
        // one rounding of the FP64 sum per node keeps continuity at FP32 round-off
        Timer tm(c, 3);
        HIPCHK(launch_round_current<T>(a.Jacc[0], F[6], 3 * nc, c->stream), "round J");
    }
    if (flags & AP_STEP_CONTINUITY) {
        Timer tm(c, 3);
        const ap_status st = deposit_rho(rho1, false);
        if (st != AP_OK) return st;
        T *J[3] = {F[6], F[7], F[8]};
        HIPCHK(launch_continuity<T>(s.dim, s.n, s.dx, s.dt, rho0, rho1, J, c->counters() + 2, c->counters() + 3,
                                    c->stream), "continuity");
    }
    if (c->P.current) {
        // Sec. IV: E2, B2 are driven by J - J1, J1 at t^{n+1/2}
        Timer tm(c, 3);
        CurrentArgs<T> ca{};
        ca.xo = s.xo;
        for (int k = 0; k < 3; ++k) {
            ca.J[k] = F[6 + k];
            ca.n[k] = s.n[k];
            ca.dx[k] = s.dx[k];
            ca.x_min[k] = s.x_min[k];
        }
        ca.dim = s.dim;
        ca.fnx = fnx;
        ca.fnxy = fnxy;
        ca.q_slice = c->P.q_slice;
        ca.W = plain_vars<T>(c->P, a.t + 0.5 * s.dt);
        ca.wp2z = c->P.wp2z;
        ca.fd = c->P.fd;
        HIPCHK(launch_analytic_current<T>(c->P.type, ca, c->stream), "analytic current");
    }
    {
        Timer tm(c, 1);
        YeeArgsBase yb;
        for (int k = 0; k < 3; ++k) { yb.n[k] = s.n[k]; yb.dx[k] = s.dx[k]; }
        yb.dt = s.dt;
        yb.open_x = (s.options & AP_GRID_OPEN_X) ? 1 : 0;
        yb.src = nullptr;
        if (launch && !(flags & AP_STEP_NO_YEE)) {
            BoundaryArgs<T> ba{};
            ba.S = c->wp<T>(L.bsrc);
            ba.rows = s.n[1] * s.n[2];
            ba.ny = s.n[1];
            for (int k = 0; k < 3; ++k) {
                ba.x_min[k] = s.x_min[k];
                ba.dx[k] = s.dx[k];
            }
            ba.q_slice = c->P.q_slice;
            ba.s0 = c->s0;
            ba.W = plain_vars<T>(c->P, a.t + 0.5 * s.dt);
            HIPCHK(launch_boundary_source<T>(c->P.type, ba, c->stream), "boundary source");
            yb.src = ba.S;
        }
        HIPCHK(launch_yee<T>(s.dim, F, yb, (flags & AP_STEP_NO_YEE) ? 1 : 0, c->stream), "yee");
    }
    return AP_OK;
}

// The particle state back from the workspace copy into the caller's arrays
// (fused 3-D re-sort); the re-sort keys stay valid (same slots).
template <typename T> ap_status restore_primary(ap_ctx *c) {
    if (!c->state_alt) return AP_OK;
    const RunShape &s = c->s;
    const WorkLayout &L = c->L;
    for (int i = 0; i < s.nsp; ++i) {
        const size_t N = (size_t)s.np[i];
        if (N == 0) continue;
        const ap_particles &p = c->buf.sp[i];
        HIPCHK(hipMemcpyAsync(p.cell, c->wp<int32_t>(L.alt_cell[i]), N * 4, hipMemcpyDeviceToDevice, c->stream),
               "restore state");
        HIPCHK(hipMemcpyAsync(p.id, c->wp<int32_t>(L.alt_id[i]), N * 4, hipMemcpyDeviceToDevice, c->stream),
               "restore state");
        for (int k = 0; k < 3; ++k) {
            if (axis_active(s.dim, k))
                HIPCHK(hipMemcpyAsync(p.off[k], c->wp<T>(L.alt_off[i][k]), N * sizeof(T), hipMemcpyDeviceToDevice,
                                      c->stream), "restore state");
            HIPCHK(hipMemcpyAsync(p.u[k], c->wp<T>(L.alt_u[i][k]), N * sizeof(T), hipMemcpyDeviceToDevice, c->stream),
                   "restore state");
        }
        HIPCHK(hipMemcpyAsync(p.w, c->wp<T>(L.alt_w[i]), N * sizeof(T), hipMemcpyDeviceToDevice, c->stream),
               "restore state");
        if (s.has_proxy[i])
            HIPCHK(hipMemcpyAsync(p.proxy, c->wp<T>(L.alt_proxy[i]), 2 * N * sizeof(T), hipMemcpyDeviceToDevice,
                                  c->stream), "restore state");
    }
    c->state_alt = false;
    return AP_OK;
}

}  // namespace
