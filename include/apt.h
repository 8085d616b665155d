/*
 * apt.h -- C ABI of the MI355X analytic-pulse particle-in-cell hot path.
 *
 * The method (Weichman et al., "Analytic pulse technique for computational
 * electromagnetics", Sec. II, Eqs. (3)-(4) and Fig. 1): the electromagnetic
 * field is split as E = E1 + E2, B = B1 + B2.  (E1, B1) is a closed-form
 * vacuum solution -- the laser -- evaluated here at every particle; (E2, B2)
 * is the plasma response carried on a periodic Yee grid and advanced with the
 * physical current only.  One step = gather E2, B2 at the particles, add the
 * analytic E1, B1, relativistic Boris push, move, charge-conserving
 * (Esirkepov) deposition of J, Yee update of E2, B2.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Units at the API: "lambda units" -- lengths in laser wavelengths,
 *   times in lambda/c, fields in m c omega/|e| (the paper's a0), densities
 *   and weights in the critical density n_c, momenta u = gamma*beta.
 * - Memory: every device buffer is owned by the caller and borrowed by the
 *   context from ap_init until ap_destroy.  The library never allocates or
 *   frees device memory.  Host structs are read during the call only.
 * - Streams: all work is enqueued on the HIP stream given to ap_init (a
 *   hipStream_t passed as void*; NULL means the null stream).  ap_step and
 *   ap_set_pulse are asynchronous; ap_gather_diag, ap_backward and
 *   ap_timing_read synchronise that stream.
 * - Errors: every call returns an ap_status.  Arguments are validated
 *   before any state changes; on error nothing is modified and
 *   ap_last_error() returns a thread-local message.  HIP failures map to
 *   AP_E_DEVICE with the HIP error text.  No C++ exception crosses the ABI.
 * - One context must not be used from two threads at once.
 */
#ifndef APT_H
#define APT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ap_status;
#define AP_OK               0
#define AP_E_ARG           -1   /* invalid argument or undersized buffer       */
#define AP_E_STATE         -2   /* call out of order (e.g. step before pulse)  */
#define AP_E_DEVICE        -3   /* HIP runtime error                           */
#define AP_E_NOMEM         -4   /* host allocation failed                      */
#define AP_E_UNSUPPORTED   -5   /* valid but not implemented combination       */
#define AP_E_NUMERIC       -6   /* non-finite particle state or CFL violation  */

#define AP_MAX_SPECIES      4

/* Arithmetic type of particle and grid arrays. */
#define AP_F32              0
#define AP_F64              1

/* Analytic pulse families (Sec. II.A Eq. (15); Sec. III.A Eqs. (20)-(23);
 * Sec. III.C Eqs. (24)-(26)). */
#define AP_PULSE_NONE       0
#define AP_PULSE_PLANE      1   /* pulsed plane wave, Eqs. (15), (17)           */
#define AP_PULSE_GAUSS      2   /* paraxial Gaussian, Eq. (21), D = d_f          */
#define AP_PULSE_LG         3   /* Laguerre-Gaussian LG_p^l, d_f = 3             */
#define AP_PULSE_FF         4   /* Gaussian flying focus, Sec. III.C              */
#define AP_PULSE_GAUSS_NP   5   /* Gaussian with nonparaxial corrections          */

/* Numerical dispersion constants used for E1, B1 (Sec. II.A). */
#define AP_DISP_PAPER2      0   /* second-order forms, Eqs. (12)-(14)            */
#define AP_DISP_EXACT       1   /* exact Yee forms, Eqs. (10)-(11)               */
#define AP_DISP_VACUUM      2   /* v_phi = v_g = c, B0 = E0                      */
#define AP_DISP_PLASMA      3   /* exact Yee forms with the analytic current J1
                                   of a linear plasma response (Sec. IV)        */

/* ap_step flags */
#define AP_STEP_CONTINUITY  0x1u  /* track max |(rho1-rho0)/dt + div J| (FP64)  */
#define AP_STEP_NO_YEE      0x2u  /* keep E2, B2 frozen (J is still deposited)  */
#define AP_STEP_RECORD      0x4u  /* keep adjoint checkpoints (ap_backward)    */

/* ap_grid_desc options */
#define AP_GRID_PULSE_ON_GRID 0x1  /* allow AP_SAMPLE_GRID (reserves workspace)  */
#define AP_GRID_PROXY         0x2  /* gridded species may carry an emission
                                      proxy (reserves its re-sort workspace)  */
#define AP_GRID_MOVING_WINDOW 0x8  /* gridded runs: reserves the workspace of
                                      ap_shift_window (not with AP_GRID_OPEN_X) */
#define AP_GRID_OPEN_X        0x4  /* gridded runs: the x ends of every row
                                      are incoming/outgoing-wave boundaries for
                                      E2, B2 (App. B, first order, normal
                                      incidence; on 2-D and 3-D grids the
                                      boundary update omits the transverse
                                      derivatives of B_x).  E nodes 0 and n[0]-1 are the
                                      boundary nodes; the transverse B nodes at
                                      n[0]-1/2 lie outside and are held at 0;
                                      J is not applied at the boundary nodes.
                                      Particles stay periodic in x: keep plasma
                                      away from the ends.                      */

/* Temporal envelopes (Sec. II.A sin^2 form; Sec. II.B super-Gaussian runs). */
#define AP_ENV_SIN2         0   /* a0 sin^2(pi eta / tau) on [0, tau]           */
#define AP_ENV_SGAUSS       1   /* a0 exp(-((eta - tau/2)/tau_g)^(2g)) on [0, tau],
                                   tau_g from the intensity FWHM              */

/* Where E1, B1 are evaluated (Fig. 1). */
#define AP_SAMPLE_PARTICLES 0   /* at every particle (default)                  */
#define AP_SAMPLE_GRID      1   /* at the staggered Yee nodes, added to E2, B2
                                   before the gather (gridded runs with
                                   AP_GRID_PULSE_ON_GRID)                      */
#define AP_SAMPLE_BOUNDARY  2   /* nowhere: the traditional run of Fig. demo.
                                   A PLANE pulse (no analytic current) enters
                                   through the x_min boundary of an
                                   AP_GRID_OPEN_X run: the source is S0/E0 of
                                   App. B (exact form, vacuum Yee wavenumber
                                   along x) times the pulse's transverse E at
                                   (x_min, row) at t^{n+1/2}; the particles
                                   feel E2, B2 alone                          */

/* ap_gather_diag masks */
#define AP_DIAG_PARTICLES   0x1u  /* moments, energies, proxy, NaN count       */
#define AP_DIAG_FIELDS      0x2u  /* E2, B2 field energy                        */

typedef struct ap_ctx ap_ctx;    /* opaque */

/* Grid and run description.
 *   dim        0 = gridless test particles (3-D motion, no E2/B2/J),
 *              1 = rows of independent 1-D grids along x (1D-3V: three
 *              velocity components, motion, fields and current along x
 *              only; the reduced-dimensionality series of Sec. III.B),
 *              2 = (x, z) Cartesian grid, 3 = (x, y, z) grid.
 *   precision  AP_F32 or AP_F64: type of every real device array.
 *   n[3]       cells along x, y, z (n[1] ignored for dims 1, 2; unused for 0).
 *              dim 1: n[2] >= 1 rows; row k lies at lab z = x_min[2] +
 *              k*dx[2] (dx[2] >= 0) and at the pulse's y slice; particles
 *              keep their row (cell = k*n[0] + i, an x offset only).
 *              The grid is periodic: a field component has n nodes per axis.
 *   tile[3]    particle tile shape in cells (0 = default: 32 x 8 on (x, z)
 *              grids, 8 x 4 x 4 in 3-D, 32 cells on 1-D rows); the push
 *              kernel stages each tile's fields plus a halo in LDS.  3-D
 *              tiles must be 8x4x4, 8x8x4 or 8x8x8 (AP_E_ARG otherwise).
 *   dx[3]      cell size per axis (lambda).  For dim 0 it is the size of
 *              the virtual cells that hold positions as (cell, offset).
 *   x_min[3]   grid origin (lambda).  Node i of axis a is at
 *              x_min[a] + i*dx[a]; Yee components are staggered by half
 *              cells (Ex at i+1/2, Ey at j+1/2, Ez at k+1/2, B dual).
 *   t0         simulation time at step 0 (lambda/c).
 *   dt         time step (lambda/c); 0 selects c dt/dx = 0.95/sqrt(D)
 *              with the smallest dx (the rule stated after Eq. (14)).
 *   sort_every steps between tile re-sorts (0 = default: 8 in 1-D and 2-D,
 *              1 in 3-D).
 *   options    AP_GRID_* bits (0 = none).  AP_GRID_PULSE_ON_GRID reserves
 *              the workspace for the grid-sampled pulse (AP_SAMPLE_GRID):
 *              6 more reals per cell.
 */
typedef struct ap_grid_desc {
    int32_t dim;
    int32_t precision;
    int32_t n[3];
    int32_t tile[3];
    double  dx[3];
    double  x_min[3];
    double  t0;
    double  dt;
    int32_t sort_every;
    int32_t options;
} ap_grid_desc;

/* One particle species: charge in |e|, mass in m_e, count of macroparticles. */
typedef struct ap_species_desc {
    double  q;
    double  m;
    int64_t n;
} ap_species_desc;

/* Device arrays of one species, structure of arrays, each with n entries.
 * A particle's position is (cell, offset): on axis a it is
 *     x_min[a] + (i_a + off[a]) * dx[a],   0 <= off[a] < 1.
 *   cell      dim 2/3: linear cell index i + n[0]*(j + n[1]*k) (j = 0 in 2-D)
 *   icell[3]  dim 0: per-axis virtual cell index (may be negative)
 *   off[3]    real offsets; dim 2 uses off[0] (x) and off[2] (z)
 *   u[3]      real momenta gamma*beta (stored at half steps, u^{n-1/2})
 *   w         real weight: density contribution per cell, in n_c
 *   id        int32 particle id, carried through re-sorts
 *   proxy     optional (NULL): two reals per particle, interleaved
 *             (sum s, compensation c; the proxy is s - c), accumulating
 *             the emission proxy; gridded runs need AP_GRID_PROXY and
 *             re-sort it with the particle.
 * Unused pointers must be NULL. */
typedef struct ap_particles {
    int32_t *cell;
    int32_t *icell[3];
    void    *off[3];
    void    *u[3];
    void    *w;
    int32_t *id;
    void    *proxy;
} ap_particles;

/* Sizes the caller must allocate (bytes; 256-byte alignment suffices).
 *   grid_bytes  one block holding Ex,Ey,Ez,Bx,By,Bz,Jx,Jy,Jz, each
 *               n[0]*n[1]*n[2] reals, x fastest (0 for dim 0).
 *   work_bytes  library workspace: sort buffers, tile tables, reductions. */
typedef struct ap_layout {
    size_t grid_bytes;
    size_t work_bytes;
    size_t real_bytes;       /* 4 or 8 */
    int64_t n_cells;
    int64_t n_tiles;
    size_t ckpt_slot_bytes;  /* dim 0: bytes of one adjoint checkpoint slot */
} ap_layout;

typedef struct ap_buffers {
    void        *grid;       /* grid_bytes, zero-filled by ap_init          */
    void        *work;       /* work_bytes                                   */
    ap_particles sp[AP_MAX_SPECIES];
} ap_buffers;

/* Pulse parameters, lambda units (Sec. II.B lists the run-time set the
 * paper used: amplitude, frequency, duration, envelope delay and the phase
 * at a reference position).
 *   a0           peak field of the envelope (for LG: peak over the mode)
 *   tau          full zero-to-zero duration of the sin^2 field envelope
 *   t_ref,x_ref  the envelope peak passes x_ref at t_ref
 *   phi0         carrier phase at (t_ref, x_ref)
 *   chirp        fractional linear frequency sweep across tau
 *   x_f, w0      focal position and waist (Eqs. (21)-(23))
 *   y_c, z_c     transverse position of the beam axis
 *   q_slice      lab y sampled by an (x, z) grid
 *   d_f          focusing dimensionality D of Eq. (21): 2 or 3
 *   lg_l, lg_p   LG azimuthal and radial index
 *   pol          0: primary E along y; 1: primary E along z
 *   beta_f, x0_ff, t0_ff   flying focus: v_f/c, focus at x0_ff at t0_ff
 *   dispersion   AP_DISP_*; dx_prop, dt_prop: grid spacing along x and
 *                time step that fix v_phi, v_g, B0/E0 (0 = use the grid's)
 *   np_order     nonparaxial order (0 or 4) for AP_PULSE_GAUSS_NP
 *   envelope     AP_ENV_*; sg_order g >= 1 and fwhm (intensity full width at
 *                half maximum, lambda/c) for AP_ENV_SGAUSS, centred in the
 *                support [0, tau] (the reading of the paper's super-Gaussian)
 *   sampling     AP_SAMPLE_*
 *   wp2, zeta, no_fd   AP_DISP_PLASMA only (Sec. IV): the pulse propagates
 *                in a plasma whose linear response is the analytic current
 *                J1, dJ1/dt = wp2 zeta E1 (wp2 = omega_p^2/omega^2 of the
 *                density J1 stands for, e.g. n_e/n_c for electrons; zeta the
 *                factor of the plasma's discrete response, 0 meaning 1).
 *                v_phi, v_g and B0/E0 solve the Yee relation with that
 *                current; every step the grid's Yee update is driven by
 *                J - J1 (J1 at t^{n+1/2} on the E nodes).  B1 and J1 keep
 *                the lowest-order finite-duration corrections unless
 *                no_fd != 0.  Needs a gridded run, AP_SAMPLE_GRID and a
 *                pulse type other than AP_PULSE_GAUSS_NP. */
typedef struct ap_pulse_params {
    double  a0, tau, t_ref, x_ref, phi0, chirp;
    double  x_f, w0, y_c, z_c, q_slice;
    double  beta_f, x0_ff, t0_ff;
    double  dx_prop, dt_prop;
    int32_t d_f, lg_l, lg_p, pol, dispersion, np_order;
    int32_t envelope, sg_order, sampling, no_fd;
    double  fwhm;
    double  wp2, zeta;
} ap_pulse_params;

/* FP64 diagnostics: reductions of the current state (the quantities the
 * paper inspects: field energy, particle energy and moments, Sec. II.B and
 * the energy balance of Sec. IV), the continuity residual of the
 * charge-conserving deposition (Sec. II.B names second-order charge-
 * conserving deposition), and numeric flags.  Every per-species sum is over
 * valid particles only (free slots and invalid particles are left out).
 * The step counters (continuity_max, j_max, n_fast, n_offtile, n_skipped)
 * cover the steps since the previous ap_gather_diag (or ap_init): each call
 * resets them. */
typedef struct ap_diag {
    double  t;                          /* lambda/c                        */
    int64_t step;
    double  field_energy;               /* sum over cells of (E2^2 + B2^2)/2 times
                                           the cell volume dx dy dz (2-D: dx dz, per
                                           unit length along y; 1-D rows: dx, per
                                           unit transverse area, summed over rows);
                                           internal units: m c^2 n_c (c/omega)^D  */
    double  sum_w[AP_MAX_SPECIES];
    double  kinetic[AP_MAX_SPECIES];    /* m sum w (gamma - 1), in m_e c^2 n_c per cell */
    double  mean_u[AP_MAX_SPECIES][3];  /* weighted means sum w u / sum w  */
    double  mean_u2[AP_MAX_SPECIES][3]; /* sum w u_k^2 / sum w             */
    double  mean_gamma[AP_MAX_SPECIES];
    double  proxy_sum[AP_MAX_SPECIES];  /* sum of per-particle proxies (s - c) */
    double  continuity_max;             /* max over checked steps (AP_STEP_CONTINUITY)
                                           of max|(rho1-rho0)/dt + div J|      */
    double  j_max;                      /* max |J| over the same steps      */
    int64_t n_nonfinite;                /* AP_DIAG_PARTICLES: particles whose state
                                           is invalid now (non-finite momentum,
                                           weight or offset, cell off the grid,
                                           offset outside [0, 1)); free slots of a
                                           moving window are not counted */
    int64_t n_fast;                     /* pushes whose move was dropped: a particle
                                           never outruns c and dt is below the Yee
                                           limit, so this counts momenta whose gamma
                                           overflows the working type            */
    int64_t n_offtile;                  /* pushes whose stencil left the LDS-staged
                                           tile region (served from global memory
                                           instead; a measure of sort staleness) */
    int64_t n_skipped;                  /* pushes skipped because the particle was
                                           invalid (left unchanged)             */
} ap_diag;

/* Accumulated device time of each kernel family since the last reset. */
typedef struct ap_timing {
    double  ms_push;        /* fused gather+analytic+Boris+move+deposit      */
    double  ms_yee;         /* Yee update of E2, B2                          */
    double  ms_sort;        /* tile count + scan + scatter                   */
    double  ms_other;       /* J clear, diagnostics                          */
    int64_t n_push, n_yee, n_sort, n_other;
    int64_t pushes;         /* particle pushes covered by ms_push            */
} ap_timing;

/* Sizes of every caller-owned device buffer for this grid and species set:
 * the internal fields E2, B2 and the current J of the field split (Sec. II,
 * Eqs. (3)-(4)) and the particle workspace of the loop of Fig. 1.
 * AP_E_ARG for an invalid description (see ap_init). */
ap_status ap_query_layout(const ap_grid_desc *grid, const ap_species_desc *species,
                          int32_t n_species, ap_layout *out);

/* Bind caller-owned buffers and the stream; zero the grid block (E2 = B2 = 0:
 * the internal field starts empty, Sec. II, Eq. (4)).  Time step rule: the
 * one stated after Eq. (14).
 * The particle arrays must already hold the initial state (u at t0 - dt/2).
 * Validation: dim in {0,1,2,3}; n >= 4 cells per active axis; dx > 0;
 * dt > 0 and below the Yee limit 1/sqrt(sum 1/dx^2); 1 <= n_species <= 4;
 * m > 0; every required pointer non-NULL.  Writes *out on success only. */
ap_status ap_init(const ap_grid_desc *grid, const ap_species_desc *species,
                  int32_t n_species, const ap_buffers *buffers, void *hip_stream,
                  ap_ctx **out);

/* Select the analytic pulse (E1, B1): the closed-form vacuum solution of the
 * field split (Sec. II, Eq. (3)) with the run-time parameters of Sec. II.B
 * (amplitude, frequency, duration, envelope delay, phase at a reference
 * position) and the families of Eqs. (15), (21) and Sec. III.  Validates the parameters (tau > 0,
 * w0 > 0 for focused types, d_f in {2,3}, LG needs d_f = 3, beta_f != 1,
 * finite values) and precomputes its FP64 constants on the host.
 * AP_PULSE_NONE removes the laser. */
ap_status ap_set_pulse(ap_ctx *ctx, int32_t pulse_type, const ap_pulse_params *params);

/* Advance n_steps time steps (asynchronous): the loop of Fig. 1 with the
 * field split of Sec. II -- per step, gather E2, B2 at the particles, add
 * E1, B1 (Eq. (3), evaluated at each particle, or on the grid with
 * AP_SAMPLE_GRID), relativistic Boris push, move, charge-conserving
 * second-order deposition of J (Sec. II.B), and the Yee update of E2, B2
 * driven by J alone (Eqs. (4), (7)-(9)).  Requires ap_set_pulse first.
 * AP_E_ARG for unknown flags or a too small checkpoint buffer when recording. */
ap_status ap_step(ap_ctx *ctx, int64_t n_steps, uint32_t flags);

/* FP64 reductions of the current state into *out (host), synchronising
 * (the diagnostics of Sec. II.B and Sec. IV; the continuity residual of the
 * charge-conserving deposition).  what: AP_DIAG_* bits.  Returns AP_E_NUMERIC
 * (after filling *out) when n_nonfinite, n_fast or n_skipped is non-zero;
 * AP_E_ARG for a NULL argument or unknown bits. */
ap_status ap_gather_diag(ap_ctx *ctx, uint32_t what, ap_diag *out);

/* ap_gather_diag for callers that cannot allocate device memory (code under
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * reductions, results, counter resets and return codes, with the reduction
 * partials in a library-held static device array (66,176 bytes per GPU,
 * resolved by ap_init on the stream's device and held until the process
 * ends) instead of the context workspace.  Its scratch size does not depend
 * on the run, so no run is too large for it.  Calls no allocating routine.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (other host threads, other streams) race and must be serialised by the
 * caller.  AP_E_ARG for a NULL argument or unknown bits. */
ap_status ap_gather_diag_static(ap_ctx *ctx, uint32_t what, ap_diag *out);

/* Current simulation time (lambda/c) and step count. */
ap_status ap_get_time(const ap_ctx *ctx, double *t, int64_t *step);

/* Evaluate the current pulse's E1, B1 at n points, with the same device
 * function the push uses (test and diagnostic aid; Sec. II.A Fig. 2(a)
 * style field maps).  xyz: device, 3 arrays of n FP64 lab positions
 * (x, then y, then z; lambda units).  E, B: device, 3 arrays of n reals
 * each (context precision, component-major).  t in lambda/c.
 * Asynchronous on the context stream. */
ap_status ap_eval_pulse(ap_ctx *ctx, int64_t n, const double *xyz, double t, void *E, void *B);

/* Emission proxy of every particle of a species (the radiated-power proxy
 * the gradients of ap_backward observe: the Lienard power without its constant,
 * summed over the steps), read out as FP64 values s - c of each particle's
 * compensated pair, in the current slot order of the species' arrays (pair
 * them with the id array for a by-id view).  dst: device, n doubles, written
 * asynchronously on the context stream.  AP_E_ARG for a species without a
 * proxy, a species index out of range or a NULL dst. */
ap_status ap_read_proxy(ap_ctx *ctx, int32_t species, double *dst);

/* Adjoint checkpoint storage.  dev: caller-owned device buffer of `bytes`;
 * segment K: steps between stored states.  Recording n steps needs
 * ap_checkpoint_bytes(ctx, n, K) bytes (AP_E_ARG at the recording ap_step
 * call if the buffer is smaller).  Gridless runs: ceil(n/K) + K slots of
 * ap_layout.ckpt_slot_bytes (outer checkpoints plus the replay buffer of one
 * segment).  Gridded runs: the whole state (every species, E2, B2) every K
 * steps, a copy of the final state, K replay slots (E2, B2 and one
 * species), and the FP64 adjoint state of the largest species.  The buffer
 * must stay allocated and untouched until the last ap_backward call. */
ap_status ap_set_checkpoints(ap_ctx *ctx, void *dev, size_t bytes, int32_t segment);

/* Reading of the adjoint of gridded runs (ap_backward).
 *   AP_ADJ_FROZEN   (default) the E2, B2 each push gathered are a recorded
 *                   external field: one species is differentiated.
 *   AP_ADJ_COUPLED  the whole loop is differentiated: every species' push,
 *                   its charge-conserving current (positions before and
 *                   after the step, and the out-of-plane velocity), the Yee
 *                   update (transposed, periodic grids only) and the gather
 *                   of E2, B2; the parameters reach the observed species
 *                   also through the plasma's response.  Every species'
 *                   ids must be a permutation of 0..n-1.
 * Setting the mode drops the checkpoint buffer and any recording (the
 * layout depends on it): call before ap_set_checkpoints.  AP_E_ARG for an
 * unknown mode or a gridless run, AP_E_UNSUPPORTED with AP_GRID_OPEN_X. */
#define AP_ADJ_FROZEN   0
#define AP_ADJ_COUPLED  1
ap_status ap_set_adjoint_mode(ap_ctx *ctx, int32_t mode);

/* Checkpoint bytes for recording n_steps >= 1 steps with segment K >= 1
 * (written to *bytes, host). */
ap_status ap_checkpoint_bytes(const ap_ctx *ctx, int64_t n_steps, int32_t segment, size_t *bytes);

/* Binomial checkpointing (the schedule of Griewank's revolve, restated): a
 * fixed budget of `slots` whole states, whatever the number of recorded
 * steps, at the cost of re-advancing.  With the state of step l stored and s
 * slots free, C(s + t + 1, s + 1) steps are reversed when every step is
 * advanced at most t times beyond the recording sweep; the recording sweep
 * stores step 0 and the states of the recursion's first descent, and
 * ap_backward runs the recursion (each reverse step reads its state from a
 * slot: no replay buffer).  Gridless runs: slots + 1 slots of
 * ap_layout.ckpt_slot_bytes; gridded runs: the whole state (every species,
 * E2, B2) per slot, a copy of the final state and the FP64 adjoint state.
 * Gradients equal those of ap_set_checkpoints' segments: bit for bit in
 * gridless runs, up to the deposit's summation order in gridded ones.
 * ap_set_revolve selects it (replacing segments; AP_E_ARG if slots < 1 or the
 * buffer is smaller than ap_revolve_bytes); ap_set_checkpoints selects
 * segments again.  ap_revolve_plan (no context) gives, for n_steps and
 * slots, the repetitions t and the forward steps the reverse sweep takes
 * (the recording sweep excluded). */
ap_status ap_set_revolve(ap_ctx *ctx, void *dev, size_t bytes, int32_t slots);
ap_status ap_revolve_bytes(const ap_ctx *ctx, int32_t slots, size_t *bytes);
ap_status ap_revolve_plan(int64_t n_steps, int32_t slots, int64_t *repeats, int64_t *forward_steps);

/* Gradient of a particle observable with respect to pulse parameters (the
 * differentiated form of the push and of the analytic field of
 * Sec. II-III) over
 * the steps of the last ap_step call made with AP_STEP_RECORD (the state
 * must not have been advanced, nor the pulse changed, since).  The observable is
 *     L = sum_p dL_du[p] . u_p(final) + dL_dproxy[p] * proxy_p(final),
 * i.e. the caller passes the cotangents of the final momenta (device,
 * component-major, 3 arrays of n reals of the context precision) and,
 * optionally, of the emission proxies (device, n reals, or NULL).  The
 * reverse sweep replays each segment from its checkpoint and runs the
 * hand-written adjoint of the analytic field, Boris push, move and proxy.
 * param_ids (host): AP_PARAM_* values, each at most once; the focal position
 * is x_f (x0_ff for the flying focus).  Writes n_params FP64 derivatives to
 * dL_dparams (host) in lambda units.  Synchronises the stream.
 *
 * Gridded runs (dim 1, 2, 3) take the frozen-grid reading: the E2, B2 that
 * each push gathered are a recorded external field, so the gradient follows
 * the parameters through the particles' own analytic fields and through the
 * position dependence of the gather, not through the plasma's response on
 * the grid.  There dL_du and dL_dproxy are indexed by particle id (the
 * species' ids must be a permutation of 0..n-1, else AP_E_ARG), dL_dproxy
 * needs a species that carries a proxy (else AP_E_ARG), and the
 * pulse must be evaluated per particle (AP_SAMPLE_PARTICLES, else
 * AP_E_UNSUPPORTED).  The reverse sweep replays each segment with the full
 * loop (push, deposit, field update), then restores the final state; the
 * next step re-sorts.  A replayed step reproduces the recorded one up to the
 * summation order of the current deposit. */
#define AP_PARAM_A0      0
#define AP_PARAM_W0      1
#define AP_PARAM_XF      2
#define AP_PARAM_BETA_F  3
#define AP_PARAM_CHIRP   4
ap_status ap_backward(ap_ctx *ctx, int32_t species, const void *dL_du,
                      const void *dL_dproxy, const int32_t *param_ids,
                      int32_t n_params, double *dL_dparams);

/* Per-kernel device timing with HIP events on the context's stream. */
ap_status ap_timing_enable(ap_ctx *ctx, int32_t enable);
ap_status ap_timing_read(ap_ctx *ctx, ap_timing *out, int32_t reset);

/* Moving window (Sec. III.C: a window that follows the pulse, e.g. the
 * intensity peak of a flying focus, which moves at v_f in either direction).
 * Needs AP_GRID_MOVING_WINDOW.  The grid is a ring along x: window column l
 * (l = 0 at the window's x_min) is stored in column (l + origin) mod n[0] of
 * every field array and of the particles' cell indices, so a shift moves the
 * origin, not the data.  At ap_init origin = 0 (storage = window columns).
 *
 * ap_shift_window moves the window by one cell: dir = +1 along +x (x_min
 * grows by dx[0]; the window's first column leaves and a new last column
 * enters), dir = -1 along -x (x_min falls by dx[0]; the last column leaves,
 * a new first column enters).  Lab positions and the lab values of E2, B2
 * are kept; the entering column's E2, B2 are zero.  Particles in the leaving
 * column fall out of the window: their slots become free and their ids
 * free ids.  A free slot holds cell -1 and zero offsets, momentum, weight
 * (and proxy); the caller may pass such slots at ap_init as spare capacity.
 * Each species' ids must be a permutation of 0..n-1 (the range is checked
 * at ap_init: AP_E_ARG).
 * inject: NULL, or one ap_inject per species (n = 0 for none): device arrays
 * in the species layout of the new particles, cells given in window columns
 * (the entering column: n[0]-1 for dir = +1, 0 for dir = -1, any row) with
 * offsets in [0, 1) (else AP_E_ARG, nothing changed); momenta and weights
 * are the caller's (the injected plasma).  They take the smallest free ids,
 * in order, and the slots holding them; the proxy of an injected particle
 * starts at zero.  More injected particles than free slots: AP_E_ARG,
 * nothing changed.  Drops any adjoint recording; 1-D and 3-D runs re-sort at
 * the next step.  One synchronisation of the stream (the checks); the work
 * is a pass over the particles' cells and one over the free slots.  In 2-D
 * runs, once the particles have been sorted by ap_step and while no re-sort
 * is pending, the leaving particles are looked up instead in the slot
 * ranges of the tile columns they can have reached since that sort (a
 * particle moves less than a cell per step) and among the particles
 * injected since: this relies on the particle arrays being changed only by
 * ap_step and ap_shift_window between the two (a caller that edits cells
 * there calls ap_step first, or passes the particles anew to ap_init). */
typedef struct ap_inject {
    const int32_t *cell;
    const void    *off[3];      /* active axes; NULL on the others           */
    const void    *u[3];
    const void    *w;
    int64_t        n;
} ap_inject;
ap_status ap_shift_window(ap_ctx *ctx, int32_t dir, const ap_inject *inject);

/* The window's lab x_min (lambda) and its storage origin (the storage column
 * of window column 0); either output may be NULL. */
ap_status ap_get_window(const ap_ctx *ctx, double *x_min, int32_t *origin);

/* Shift schedule of a window moving at beta c (beta = v_f / c of a flying
 * focus, Sec. III.C, any sign): the window's x_min should be
 * x_ref + beta (t - t_ref) at the current time t (lambda, lambda/c).  With
 * d = (that position - x_min) / dx[0]: *dir = +1 if d >= 1/2, -1 if
 * d < -1/2 (shift once and ask again), else 0. */
ap_status ap_window_due(const ap_ctx *ctx, double beta, double x_ref, double t_ref, int32_t *dir);

/* Release the context (does not free caller buffers). NULL is accepted. */
ap_status ap_destroy(ap_ctx *ctx);

/* Message of the last non-OK status on this thread ("" if none).  The string
 * stays valid until the thread's next ap_* call. */
const char *ap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* APT_H */
