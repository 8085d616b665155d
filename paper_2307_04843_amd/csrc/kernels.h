// Kernel argument structs and launcher declarations shared by the host
// runtime (apt_host.cpp) and the kernel translation units.
#pragma once

#include "common.h"
#include "pulse_dev.h"

namespace apt {

// Tile halo: a particle in tile cell range [X0, X0+TX) may drift kDrift cells
// out of it between re-sorts and still use the LDS copy.  The quadratic
// gather needs nodes [c-1, c+2] and the deposit [c-2, c+3] around cell c.
constexpr int kDrift = 2;
constexpr int kHaloLo = 2 + kDrift;
constexpr int kHaloHi = 3 + kDrift;

template <typename T> struct SpeciesIO {
    // source (read) arrays
    const int32_t *cell_in;
    const T *off_in[3];
    const T *u_in[3];
    const T *w_in;
    const int32_t *id_in;
    // destination (write) arrays
    int32_t *cell_out;
    T *off_out[3];
    T *u_out[3];
    T *w_out;
    int32_t *id_out;
    const T *proxy_in;           // emission proxy (sum, compensation) per particle, or null
    T *proxy_out;
    const int32_t *tile_start;   // [n_tiles + 1]
    int32_t copy_static;         // write w and id (source != destination)
    // fused re-sort (3-D): the particle of output slot j is read from input
    // slot perm[j] (perm null: j); key_out[j] (null: none) gets its rank in
    // the tile of its new cell when that is this block's tile, else -1;
    // mcount[t] counts the particles entering tile t (atomics) and stay[t]
    // those staying in it (written by tile t's block)
    const int32_t *perm;
    int32_t *key_out;
    int32_t *mcount;
    int32_t *stay;
    int32_t n;
    double q_over_m;
    double q;
};

template <typename T> struct PushArgs {
    SpeciesIO<T> sp[kMaxSpecies];
    int32_t nsp;
    const T *E[3];
    const T *B[3];
    T *J[3];
    double *Jacc[3];             // FP64 accumulator of this step's current (J itself in FP64 runs)
    int32_t n[3];                // cells per axis
    int32_t tile[3];             // tile shape
    int32_t ntile[3];            // tiles per axis
    FastDiv fnx, fnxy, fntx, fntxy;
    int32_t splits;              // workgroups per tile
    int32_t n_logical;           // n_tiles * splits
    int32_t xcd_chunk;           // 3-D: consecutive logical tiles per XCD run (block -> tile map)
    int32_t reg[3];              // LDS region extent per axis
    double dx[3];
    double x_min[3];             // lab position of the window's first node
    int32_t xo;                  // moving window: storage column of the window's first column
    double dt;
    double t;                    // time of the positions read (t^n)
    unsigned long long *n_fast;  // moves the kernel could not take (dropped), see push_move_ok
    unsigned long long *n_bad;   // skipped pushes of invalid particles (free slots not counted)
    unsigned long long *n_offtile;   // pushes that left the staged region (global-memory path)
    double q_slice;              // lab y sampled by an (x, z) grid
    int32_t pulse;               // PulseType
    PulseVar<T> W;               // pulse constants of this step
};

template <typename T> struct GridlessArgs {
    const int32_t *icell[3];     // source state
    const T *off[3];
    const T *u[3];
    int32_t *icell_out[3];       // destination state (may alias the source)
    T *off_out[3];
    T *u_out[3];
    T *proxy;                    // 2 per particle or null
    int32_t n;
    double q_over_m;
    double dx[3];                // virtual cell size
    double x_min[3];
    double dt;
    double t;
    unsigned long long *n_bad;
    PulseVar<T> W;
};

// Grid-sampled pulse: S[c] = F[c] + (E1, B1)[c] at component c's staggered node.
template <typename T> struct SampleArgs {
    const T *F[6];               // E2x E2y E2z B2x B2y B2z
    T *S[6];                     // sums, same layout
    int32_t n[3];
    int32_t dim;
    FastDiv fnx, fnxy;
    double dx[3];
    double x_min[3];
    int32_t xo;                  // moving window origin (storage column of window column 0)
    double q_slice;              // lab y of an (x, z) grid
    PulseVar<T> W;               // pulse constants of this step
    int32_t fd_b;                // B1 with the finite-duration correction of an analytic current
    double fd_delta;             // its factor 1 - v_phi/v_g
};
template <typename T> hipError_t launch_sample_pulse(int pulse, const SampleArgs<T> &a, hipStream_t s);

// Analytic current (Sec. IV): J[c] -= J1_c at component c's E node, t^{n+1/2}.
template <typename T> struct CurrentArgs {
    T *J[3];
    int32_t n[3];
    int32_t dim;
    FastDiv fnx, fnxy;
    double dx[3];
    double x_min[3];
    int32_t xo;                  // moving window origin
    double q_slice;
    PulseVar<T> W;               // pulse constants at t^{n+1/2}
    double wp2z;                 // omega_p^2 zeta / omega
    int32_t fd;                  // finite-duration correction kept
};
template <typename T> hipError_t launch_analytic_current(int pulse, const CurrentArgs<T> &a, hipStream_t s);

// Gridded runs, frozen-grid reading: the E2, B2 the push gathered at step n
// are a recorded external field; their position dependence enters dL/dx.
template <typename T> struct AdjointGrid {
    const int32_t *cell;         // linear cell of each particle (x fastest)
    const int32_t *id;           // particle id: index of its adjoint state
    const T *F[6];               // E2x E2y E2z B2x B2y B2z at the start of step n
    int32_t n[3];
    FastDiv fnx, fnxy;
    double q_slice;              // lab y of an (x, z) grid
};

template <typename T> struct AdjointArgs {
    const int32_t *icell[3];     // state x^n, u^{n-1/2} of the step being reversed (gridless)
    const T *off[3];
    const T *u[3];
    double *lam[6];              // dL/dx (lab, internal units), dL/du (in: step n+1, out: step n)
    const T *lam_proxy;          // dL/dproxy per particle or null
    double *partial;             // [blocks][5] gradient partials (a0, w0, focus, beta_f, chirp)
    int32_t slot[4];             // parameter id carried by tangent 3 + k (-1: unused)
    int32_t n;
    double q_over_m;
    double dx[3];
    double x_min[3];
    int32_t xo;                  // moving window origin (gridded runs)
    double dt;
    double t;
    PulseDev P;
    int32_t dim;                 // 0 (gridless), 1, 2 or 3 (grid: G is used, icell is not)
    AdjointGrid<T> G;
    // fully coupled reading of gridded runs (lJ[0] != null): the deposit and
    // the gather are differentiated as well
    const T *w;                  // particle weights, same order as off/u
    double q;                    // species charge
    const double *lJ[3];         // E adjoint after the first half of the reverse Yee step (E nodes)
    double *lEg[3], *lBg[3];     // grid adjoints of E2^n, B2^n: the gather's adjoint is added here
    double *gx0;                 // coupled 2-D/3-D: [6][n] per-particle values between the reverse passes
    // coupled 2-D/3-D, or null: [ntile + 1] slot ranges of the tiles; the
    // gather's adjoint then runs one block per tile, over the tile's box
    // widened by tile_margin cells (whole axes where that box would cover
    // the axis)
    const int32_t *tile_start;
    int32_t ntile, tile_dim[3], tile_n[3], tile_margin;
    int32_t scatter_cap;         // LDS entries of the gather's adjoint box (0: the default budget)
};
template <typename T> hipError_t launch_adjoint_step(int pulse, const AdjointArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_adjoint_step_coupled(int pulse, const AdjointArgs<T> &a, hipStream_t s);
// LDS entries (doubles) of the coupled gather's adjoint box in dim-D runs
int adjoint_scatter_lds_entries(int dim);

// Checks that id[0..n) is a permutation of 0..n-1: seen[] (n ints, zeroed by
// the caller) counts each id; *bad counts ids out of range or repeated.
hipError_t launch_check_ids(const int32_t *id, int n, int32_t *seen, unsigned long long *bad, hipStream_t s);
template <typename T> hipError_t launch_adjoint_init(double *const lam[6], const T *dl_du, int n, hipStream_t s);

struct YeeArgsBase {
    int32_t n[3];
    double dx[3];
    double dt;
    int32_t open_x;              // incoming/outgoing-wave x ends (App. B)
    const void *src;             // open x: [rows][2] boundary source S_y, S_z at t^{n+1/2}, or null
};

// Incoming-wave boundary source (App. B): per row, S0/E0 times the pulse's
// transverse E at (x_min, row) and the step's half time.
template <typename T> struct BoundaryArgs {
    T *S;                        // [rows][2], row = j + ny k
    int32_t rows;
    int32_t ny;                  // rows along y (3-D), else 1
    double x_min[3], dx[3];
    double q_slice;
    double s0;                   // S0 / E0
    PulseVar<T> W;               // pulse constants at t^{n+1/2}
};
template <typename T> hipError_t launch_boundary_source(int pulse, const BoundaryArgs<T> &a, hipStream_t s);
// Reverse split Yee step on FP64 adjoints (lE, lB: 3 x ncell each): from the
// adjoints of E^{n+1}, B^{n+1} to those of E^n, B^n, leaving in lJt the E
// adjoint after its first half (dL/dJ^{n+1/2} = -dt lJt).  Periodic grids.
hipError_t launch_yee_adjoint(int dim, double *lE, double *lB, double *lJt, const YeeArgsBase &a, hipStream_t s);

// launchers (hipStream_t passed through)
template <typename T>
hipError_t launch_push_deposit_1d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s);
template <typename T>
hipError_t launch_push_deposit_2d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s);
template <typename T>
hipError_t launch_push_deposit_3d(int pulse, const PushArgs<T> &a, int threads, hipStream_t s);
template <typename T>
hipError_t launch_gridless(int pulse, const GridlessArgs<T> &a, hipStream_t s);
// fd_delta != 0: B1 with the finite-duration correction of an analytic current.
template <typename T>
hipError_t launch_eval_pulse(int pulse, const PulseVar<T> &W, double fd_delta, int64_t n, const double *xyz, T *E,
                             T *B, hipStream_t s);
template <typename T>
hipError_t launch_yee(int dim, T *const F[9], const YeeArgsBase &g, int no_yee, hipStream_t s);
template <typename T>
hipError_t launch_fill_zero(T *p, size_t n, hipStream_t s);
// out[p] = pair[2p] - pair[2p+1] in FP64: the proxy of each particle from its compensated pair.
template <typename T> hipError_t launch_proxy_value(const T *pair, double *out, int n, hipStream_t s);
// J = (T) Jacc over n values: the step's current rounded once to the working type.
template <typename T> hipError_t launch_round_current(const double *jacc, T *J, size_t n, hipStream_t s);

struct SortArgs {
    const int32_t *cell;
    uint32_t ncell;              // cells outside [0, ncell) are binned to tile 0
    int32_t n;
    int32_t dim;
    FastDiv fnx, fnxy;           // decompose linear cell
    FastDiv ftx, fty, ftz;       // cell -> tile
    int32_t ntile[3];
    int32_t *count;              // [n_tiles]
    int32_t *rank;               // [n]
};
hipError_t launch_tile_count(const SortArgs &a, hipStream_t s);
// start[0..n_tiles] = exclusive scan of count (start[n_tiles] = total).
// part: scratch of 2 * scan_part_len(n_tiles) ints.
int32_t scan_part_len(int32_t n_tiles);
hipError_t launch_scan(const int32_t *count, int32_t *start, int32_t n_tiles, int32_t *part, hipStream_t s);

// Moving window (Sec. III.C).  The grid is a ring along x: window column l
// lives in storage column (l + xo) mod nx, so a shift moves the origin xo
// instead of the data.  A free particle slot holds cell kDeadCell and zero
// offsets, momentum and weight (its id is a free id).
constexpr int32_t kDeadCell = -1;

// Tile of a free or invalid slot p in the tile sort and the 3-D re-sort:
// blocks of 256 such slots are spread over the tiles, so that spare capacity
// does not pile up in one tile (the push skips them at the cost of a load).
AP_D inline int dead_tile(int p, int ntiles) { return (int)(((unsigned)p >> 8) % (unsigned)ntiles); }

// Window column of storage column i (origin xo, nx columns).
AP_D inline int win_col(int i, int xo, int nx) {
    const int l = i - xo;
    return l < 0 ? l + nx : l;
}

// A particle the push can advance has finite momentum and weight (a
// non-finite one would put NaN into the current); its cell and offsets are
// checked by each kernel.  Skipped particles are counted, free slots not.
template <typename T> AP_D bool finite_state(T ux, T uy, T uz, T w) {
    return __builtin_isfinite(ux) && __builtin_isfinite(uy) && __builtin_isfinite(uz) && __builtin_isfinite(w);
}
AP_D void count_skipped(unsigned long long *n_bad, int32_t cell) {
    if (cell != kDeadCell) atomicAdd(n_bad, 1ull);
}
// A move is taken when 1/gamma is positive (gamma did not overflow the
// working type) and the displacement is below one cell.  A particle is never
// faster than c and dt is below the Yee limit, so only a momentum whose gamma
// overflows (|u| above ~1e19 in FP32) can fail; its move is dropped and counted.
template <typename T> AP_D bool push_move_ok(T inv_gamma, T d) {
    return inv_gamma > T(0) && fabs(d) < T(1);
}
template <typename T> struct WindowArgs {
    int32_t *cell; const int32_t *id; T *off[3]; T *u[3]; T *w; T *proxy;   // one species, in place
    int32_t n;
    uint32_t ncell;
    int32_t nx;
    FastDiv fnx;
    int32_t col;                 // storage column leaving the window (it becomes the entering one)
    uint32_t *freemap;           // bit id set: the particle id is free (its slot holds no particle)
    const int32_t *frank;        // [words + 1]: exclusive scan of the popcounts of freemap's words
    int32_t words;               // ceil(n / 32)
    const int32_t *in_cell;      // injected particles (device, n_inj): window cells, entering column
    const T *in_off[3]; const T *in_u[3]; const T *in_w;
    int32_t n_inj;
    int32_t in_col;              // window column the injected particles must sit in
    unsigned long long *count;   // bad ids / bad injected particles / leavers
    unsigned long long *count_free;   // free slots (window_init)
    int32_t *free_slot;          // [n] by id: the slot a free id was last seen in (a hint, verified on use)
    unsigned long long *miss;    // injected particles whose hint was stale (window_fill)
    int32_t *inj_list;           // or null: slot of injected particle r written to inj_list[r] (window_fill)
};
// The leaving column's particles found through the tile ranges of the last
// full sort (2-D runs, particles in place since): tile columns tx0 ..
// tx0 + ncols - 1 (mod ntile_x), every tile row, plus the slots listed in
// list[0 .. list_n) (particles injected since that sort).  Each leaver is
// freed once (compare-and-swap of its cell); count[0] += leavers.
struct LeaveTiles {
    const int32_t *start;        // [n_tiles + 1] slot ranges of the last full sort
    int32_t tx0, ncols, ntile_x, ntile_z;
    const int32_t *list;
    int32_t list_n;
};
template <typename T> hipError_t launch_window_leave_tiles(const WindowArgs<T> &a, const LeaveTiles &lt, hipStream_t s);
// freemap from the free slots (bits of their ids, the map zeroed first);
// count[0] += ids out of range, count_free[0] += free slots.
template <typename T> hipError_t launch_window_init(const WindowArgs<T> &a, hipStream_t s);
// count[0] += injected particles outside the entering column or with offsets outside [0, 1).
template <typename T> hipError_t launch_window_check_inject(const WindowArgs<T> &a, hipStream_t s);
// count[0] += particles in the leaving column (no change).
template <typename T> hipError_t launch_window_count_leavers(const WindowArgs<T> &a, hipStream_t s);
// Particles in the leaving column: freed (state zeroed, id bit set, slot
// hint written); count[0] += leavers.
template <typename T> hipError_t launch_window_leave(const WindowArgs<T> &a, hipStream_t s);
// pop[w] = popcount(freemap[w]).
hipError_t launch_window_popcount(const uint32_t *freemap, int32_t words, int32_t *pop, hipStream_t s);
// The free ids ranked below n_inj take the injected particles in rank order
// (cells mapped to storage through col): first through the slot hints (a
// hint is used when its slot is free and holds that id, else *miss counts
// it), then, only if *miss > 0, by a pass over every slot for the rest.
template <typename T> hipError_t launch_window_fill(const WindowArgs<T> &a, hipStream_t s);
// Clears the bits of the n_inj smallest free ids (after launch_window_fill).
hipError_t launch_window_clear(uint32_t *freemap, const int32_t *frank, int32_t words, int32_t n_inj,
                               hipStream_t s);
// Zeroes storage column col of the six fields.
template <typename T> hipError_t launch_window_column(T *const F[6], int32_t col, int32_t nx, size_t ncell,
                                                      hipStream_t s);

template <typename T> struct ScatterArgs {
    const int32_t *cell_src; const T *off_src[3]; const T *u_src[3]; const T *w_src; const int32_t *id_src;
    int32_t *cell_dst; T *off_dst[3]; T *u_dst[3]; T *w_dst; int32_t *id_dst;
    const T *proxy_src; T *proxy_dst;   // 2 per particle, or null
    const int32_t *rank;
    const int32_t *start;
    uint32_t ncell;
    int32_t interleave;          // mean particles per cell: within-tile ragged transpose stride
    int32_t n, dim;
    FastDiv fnx, fnxy, ftx, fty, ftz;
    int32_t ntile[3];
    int32_t *free_slot;          // moving window: slot of each free id (a hint), or null
};
template <typename T> hipError_t launch_scatter(const ScatterArgs<T> &a, hipStream_t s);

// Fused re-sort: count[t] = stay[t] + mcount[t] (input of the tile scan).
hipError_t launch_resort_counts(const int32_t *stay, const int32_t *mcount, int32_t *count, int32_t n_tiles,
                                hipStream_t s);
// Fused re-sort: perm[start[t] + rank] = p for every particle p of the
// buffer the last push wrote (cell, key as written by it), with stayers
// first in each tile (their key is the rank) and the particles entering it
// after them (key -1; ranks handed out by atomics on mrank, zeroed).
struct PermArgs {
    const int32_t *cell;
    const int32_t *key;
    const int32_t *start;
    const int32_t *stay;
    int32_t *mrank;
    int32_t *perm;
    uint32_t ncell;
    int32_t n, dim;
    FastDiv fnx, fnxy, ftx, fty, ftz;
    int32_t ntile[3];
};
hipError_t launch_resort_perm(const PermArgs &a, hipStream_t s);

// diagnostics
constexpr int kDiagVals = 16;    // per-species partial-sum slots
template <typename T> struct DiagArgs {
    const T *u[3];
    const T *w;
    const T *proxy;
    const T *off[3];
    const int32_t *cell;         // gridded runs: linear cells (kDeadCell = free slot), else null
    uint32_t ncell;
    int32_t n;
    int32_t dim;
    double *partial;             // [blocks][kDiagVals]
    int32_t blocks;
};
template <typename T> hipError_t launch_diag_particles(const DiagArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_diag_fields(T *const F[6], size_t ncell, double *partial, int blocks, hipStream_t s);
hipError_t launch_sum_partials(const double *partial, int blocks, int nvals, double *out, hipStream_t s);

template <typename T> struct RhoArgs {
    const int32_t *cell; const T *off[3]; const T *w;
    int32_t n; double q;
    int32_t nn[3]; FastDiv fnx, fnxy; int32_t dim;
    double *rho;
};
template <typename T> hipError_t launch_rho(const RhoArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_continuity(int dim, const int32_t n[3], const double dx[3], double dt,
                             const double *rho0, const double *rho1, T *const J[3],
                             unsigned long long *res_max, unsigned long long *j_max,
                             hipStream_t s);

}  // namespace apt
