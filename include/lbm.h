/*
 * lbm.h -- C ABI of the MI355X (gfx950) thermal lattice Boltzmann library (D2Q37, D2Q17 or D2Q9
 * velocity stencil) with a perfectly matched layer (PML) and open outer boundaries, after
 * arXiv 2504.20169.
 *
 * One time step follows Sec. 2 (algorithm outline) and Secs. 3-4:
 *   pull streaming  f_i(x, n+1) = f*_i(x - e_i, n)                      (eq. lbe)
 *   outer boundary  zero-gradient copy from x_f (eq. zg-bc), or the characteristic
 *                   non-reflecting fill feq(U_tgt) + f^neq(x_f) (eqs. PNR,
 *                   thermal_LODI_macro_evo and the non-equilibrium extrapolation)
 *   moments         rho, u, T (eq. macro, e = (d/2) T)
 *   PML auxiliary   Q^{n+1} = Q^n + (fhat^n + fhat^{n+1})/2 (eq. PMLQ, trapezoid rule)
 *   collision       f* = f - (f - feq)/tau - sigma (e.grad Q + 2 fhat + sigma Q)
 *                   (BGK with eq. feq-4 on D2Q37, eq. feq-3 on D2Q17 or eq. feq-2 on D2Q9,
 *                   and eq. PMLCOLL;
 *                   sigma ramp eq. PML_ramp)
 *
 * Units: rho, u, T in thermal units (sound-speed unit c_s = 1, xi_i = r e_i with the stencil's
 * scale, r = 1.19698... for D2Q37, 1.64343... for D2Q17, sqrt 3 for D2Q9); lengths and times in lattice
 * units (one cell, one step).
 *
 * Grid: the bulk is nx x ny; every side carrying a PML of width W adds W layers, so the full
 * grid is Nx = nx + W*(#PML x-sides), Ny likewise.  The outermost 3 layers of an open side are
 * its boundary nodes (and, with a PML, also its PML levels W, W-1, W-2), for every stencil: the
 * paper's boundary depth is the displacement bound 3 under which its stencils are minimal.  Host field arrays are
 * row-major [Ny][Nx] float64; population arrays are [q][Ny][Nx] float64 (q = 37, 17 or 9) in the
 * order returned by lbm_velocities().
 *
 * Conventions: every call returns an lbm_status; no exception or abort crosses the ABI.
 * lbm_last_error() returns a thread-local message for the last failure.  Configuration order:
 * lbm_create -> lbm_set_pml / lbm_set_bc -> lbm_init_fields -> lbm_step...; setters after
 * lbm_init_fields return LBM_ERR_STATE.  A handle is used by one host thread at a time.  Work
 * is enqueued on the run's HIP stream; device faults surface at the next synchronising call
 * (lbm_moments, lbm_populations, lbm_error_norms, lbm_check, lbm_synchronize).  Host arrays
 * are caller-owned and copied; device memory is library-owned, obtained through the optional
 * allocator hook.
 */
#ifndef PAPER_2504_20169_LBM_H
#define PAPER_2504_20169_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_run *lbm_handle;
typedef struct lbm_group *lbm_group_handle;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = 1,         /* invalid argument (message says which) */
    LBM_ERR_STATE = 2,       /* call not allowed in the handle's current state */
    LBM_ERR_OOM = 3,         /* device allocation failed */
    LBM_ERR_DEVICE = 4,      /* a HIP call failed */
    LBM_ERR_UNSTABLE = 5,    /* lbm_check found a non-finite value, rho <= 0 or T <= 0 */
    LBM_ERR_UNSUPPORTED = 6
} lbm_status;

/* Population storage.  LBM_F64 stores f - fbar in float64 and computes in float64.
 * LBM_F32_DEV stores f - fbar in float32 and computes in float32.  LBM_F16_DEV stores
 * (f - fbar) * s in float16 with a per-run power-of-two scale s, computing in float32.  fbar
 * is the mean equilibrium feq(rho0, u0, T0) of eq. decomp-NJ (the rest weights w_i when the
 * mean state is rho0 = T0 = 1, u0 = 0).  The characteristic boundary and the error norms
 * always compute in float64. */
typedef enum { LBM_F64 = 0, LBM_F32_DEV = 1, LBM_F16_DEV = 2 } lbm_storage;

/* Side masks. */
enum { LBM_XMIN = 1, LBM_XMAX = 2, LBM_YMIN = 4, LBM_YMAX = 8, LBM_ALL = 15 };

/* Outer-edge treatment of a side.  PERIODIC must be set on both sides of an axis.  NRBC: the
 * perfectly non-reflecting LODI boundary (Sec. 4, eqs. PNR and thermal_LODI_macro_evo; the
 * paper's scheme B).  NRBC_A: the characteristic boundary with transverse and viscous terms and
 * relaxed incoming amplitudes (Sec. 4 eq. thermal_CBC_macro_evo, Sec. 5.2 eq. CBC-Relax; the
 * paper's CBC (A), which it applies at the outlet): on the nodes of a side that lie on no other
 * open side; corner nodes take the LODI target of each normal.  Stable on every side with D2Q17;
 * with D2Q37, whose sound speed exceeds one cell per step, only on outflow sides (on inflow or
 * tangential-flow sides its round-off grows). */
typedef enum { LBM_BC_PERIODIC = 0, LBM_BC_ZG = 1, LBM_BC_NRBC = 2, LBM_BC_NRBC_A = 3 } lbm_bc;

/* Optional device allocator: alloc returns device memory of at least `bytes` (256-byte
 * aligned) or NULL; free releases it.  Used for every device buffer of a run or group. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} lbm_allocator;

typedef struct {
    int32_t nx, ny;              /* bulk size, >= 1 */
    double tau;                  /* BGK relaxation time, > 0.5 (Sec. 2) */
    double rho0, ux0, uy0, T0;   /* mean state: fbar, PML target and deviation reference */
    int32_t storage;             /* lbm_storage */
    double f16_scale;            /* LBM_F16_DEV: scale s (power of two); 0 = chosen at init */
    const lbm_allocator *allocator; /* NULL = hipMalloc / hipFree */
    void *stream;                /* hipStream_t to enqueue on; NULL = a stream the run owns (only
                                    then can lbm_launch.overlap put the boundary/PML kernels on a
                                    side stream beside the bulk kernel) */
    int32_t layout;              /* population layout in HBM: 0 = the q population rows of each
                                    grid row adjacent (default), 1 = one plane per velocity */
    int32_t row_pad;             /* layout 0: extra elements after each population row (rows
                                    are first rounded up to 64 elements); 0 = automatic (64 for
                                    FP64 and FP32 storage, none for FP16: the fastest measured on
                                    large grids), -1 = none, 1..4096 = that many elements */
    int32_t lattice;             /* velocity stencil (Sec. 2, "Velocity stencils"): 0 or 37 =
                                    D2Q37 with eq. feq-4 (default), 17 = D2Q17 with eq. feq-3,
                                    9 = D2Q9 with eq. feq-2 */
} lbm_desc;

/* Launch configuration (set by lbm_set_launch or lbm_autotune).  bulk_tx in {64,128,256}
 * nodes along x, bulk_ty rows per block with bulk_tx*bulk_ty = 256; graph_steps: steps per
 * captured HIP graph in lbm_step (even, 0 disables graphs; steps are also launched eagerly in
 * batches of this many, 32 when 0, each closed by one bookkeeping launch); overlap: how the
 * boundary/PML work of a step meets the bulk kernel: 0 runs the kernels of a step in order on
 * the run's stream; 1 runs the boundary/PML chain on a side stream beside the bulk kernel (only
 * for a run that owns its stream; eager launches, no graphs); 2 launches phase A (characteristic
 * fill of the ring, PML Q update) and the bulk tiles as one grid, so they run beside the
 * streaming tiles (one stream, graphs and groups allowed); split places the phase-A blocks in
 * that grid: after split/8 of the bulk tiles (0..8, rounded down to a multiple of 8 blocks), or
 * -1 for the measured default (after all of the tiles when they outnumber the phase-A blocks
 * eightfold, as on large grids; else after half of them for D2Q37 in FP64, first otherwise).
 * Every schedule and placement gives the same bits.  Default {64, 4, 32, 2, -1}. */
typedef struct {
    int32_t bulk_tx, bulk_ty;
    int32_t graph_steps;
    int32_t overlap;
    int32_t split;
} lbm_launch;

/* Create a run (Sec. 2).  Validates the descriptor (LBM_ERR_ARG: tau <= 0.5, size < 1,
 * non-finite mean state, rho0 <= 0, T0 <= 0, unknown storage, layout or lattice).  No device memory is touched
 * until lbm_init_fields.  *out receives the handle (caller owns it until lbm_destroy). */
lbm_status lbm_create(const lbm_desc *desc, lbm_handle *out);

/* PML of width W on the sides in side_mask with ramp sigma(l) = sigma_max (l/W)^2 on ring
 * level l = 1..W (eq. PML_ramp; Chebyshev level at corners).  W = 0 removes it.  Errors:
 * LBM_ERR_ARG for W < 0, sigma_max < 0 or non-finite; LBM_ERR_STATE after init. */
lbm_status lbm_set_pml(lbm_handle h, unsigned side_mask, int32_t W, double sigma_max);

/* Outer-edge treatment for the sides in side_mask (Sec. 4).  Default: periodic on all
 * sides.  Errors: LBM_ERR_ARG for an unknown kind; LBM_ERR_STATE after init.  Consistency
 * (periodic on both sides of an axis, no PML on a periodic side, N >= 7 on an open axis) is
 * checked by lbm_init_fields. */
lbm_status lbm_set_bc(lbm_handle h, unsigned side_mask, lbm_bc kind);

/* Appendix (eq. NSF-CHAR-PML): make the characteristic boundary consistent with the PML by
 * adding, at NRBC boundary nodes inside a PML (sigma > 0), the velocity moments of the PML
 * collision term to the one-step target update: bit 0 term I (divergence of the auxiliary flux
 * moments, sum_i phi_i e_i . grad Q_i), bit 1 term II (2 (U - Ubar)), bit 2 term III
 * (sigma sum_i phi_i Q_i), phi = (1, xi, |xi|^2/2), entering as +sigma (I + II + III) in
 * conserved variables (the appendix's signs) and converted to (rho, u, T) at U^n.  Default 0: the plain LODI target of
 * Sec. 4.  Errors: LBM_ERR_ARG for bits outside 0..2; LBM_ERR_STATE after init. */
lbm_status lbm_set_nrbc_pml_terms(lbm_handle h, unsigned flags);

/* Debug flags of a run (lbm_set_debug).  LBM_DEBUG_POISON: a NaN canary.  Before the kernels of
 * every step, the buffers that the step writes in full -- the destination population buffer,
 * the new moment strips, and on characteristic sides the ring's fill and targets -- are filled
 * with NaN in their storage type, so a node or component that a step leaves unwritten and a
 * later kernel reads shows up as NaN in the moments (and in lbm_check).  A correct step gives
 * the same bits with and without it.  Costs one extra pass over those buffers per step; in a
 * group, the canary is on for every member while any member has it on.  Not part of the paper:
 * a test aid.  LBM_DEBUG_RANGES: every lbm_step call is enclosed in a roctx range named
 * "lbm_step <nsteps>" (lbm_group_step: "lbm_group_step <runs> <largest count>", while any member
 * has the flag), which rocprofv3 --marker-trace records, so a trace ties kernels to the calls
 * that launched them.  The range covers the host call that enqueues the steps; launches and
 * results are unchanged. */
enum { LBM_DEBUG_POISON = 1, LBM_DEBUG_RANGES = 2 };

/* Set the run's debug flags (0 clears them).  Allowed at any time; captured step graphs are
 * recaptured.  Errors: LBM_ERR_ARG for a NULL handle or an unknown flag. */
lbm_status lbm_set_debug(lbm_handle h, unsigned flags);

/* Full grid size for the current configuration: the bulk extended by W layers on each side
 * that carries a PML, Nx = nx + W (per PML x side), Ny likewise (Sec. 3: the computational
 * domain (L_x + 2W) x (L_y + 2W) when every side has a layer; Sec. 5 uses that layout).  Host
 * only.  Errors: LBM_ERR_ARG for NULL pointers. */
lbm_status lbm_grid(lbm_handle h, int32_t *Nx, int32_t *Ny);

/* Node counts of the run's kernel classes for the current configuration (host only): out[0]
 * interior nodes updated by the branch-free bulk kernel, out[1] frame nodes (boundary layers, PML
 * and moment strips) updated by the frame kernel, out[2] nodes carrying the PML auxiliary field Q
 * (Sec. 3: the layer plus the first bulk ring, eqs. PMLQ and FD-dx-center), out[3] boundary
 * nodes of characteristic sides (the outer 3 layers, Sec. 4) filled by phase A.  out holds 4
 * entries.  Errors: LBM_ERR_ARG for NULL pointers or an inconsistent configuration. */
lbm_status lbm_node_classes(lbm_handle h, int64_t out[4]);

/* Bytes of device memory the run needs at its peak (populations, PML Q, moment strips, ring
 * buffers, descriptor, and the transient staging of the input fields while lbm_init_fields runs),
 * for admission control. */
lbm_status lbm_footprint(lbm_handle h, size_t *bytes);

/* Allocate device state and set f*(x, 0) = feq(rho, u, T)(x), Q = 0 (Sec. 2 algorithm
 * outline; eq. PMLQ).  rho, ux, uy, T: host float64 [Ny][Nx], copied.  Errors: LBM_ERR_ARG
 * for NULL, non-finite, rho <= 0 or T <= 0 inputs or an inconsistent configuration;
 * LBM_ERR_OOM; LBM_ERR_STATE if already initialised; LBM_ERR_ARG if the allocator hook returns
 * two live buffers that overlap (nothing else is touched then).  Synchronises the stream. */
lbm_status lbm_init_fields(lbm_handle h, const double *rho, const double *ux,
                           const double *uy, const double *T);

/* Advance nsteps >= 0 time steps (Sec. 2 algorithm outline, each step: pull streaming, eq. lbe;
 * the outer boundary, eq. zg-bc or the characteristic fill of Sec. 4; the moments, eq. macro;
 * the PML auxiliary update, eq. PMLQ with the trapezoid rule; the collision, BGK with
 * eq. PMLCOLL), asynchronously on the run's stream.  Errors: LBM_ERR_ARG for nsteps < 0;
 * LBM_ERR_STATE before lbm_init_fields or while the run is in a group; LBM_ERR_DEVICE if a
 * launch fails (faults during the steps surface at the next synchronising call). */
lbm_status lbm_step(lbm_handle h, int64_t nsteps);

/* Stability checks inside lbm_step (failure detection, not part of the paper): with every > 0,
 * lbm_step advances in chunks of `every` steps and after each chunk scans the state as lbm_check
 * does (one synchronisation per chunk); at the first failure it stops and returns
 * LBM_ERR_UNSTABLE, the run then standing after that chunk (lbm_step_count says where).  0 (the
 * default) turns the checks off.  A multiple of lbm_launch.graph_steps keeps the graph replays.
 * Allowed at any time.  Errors: LBM_ERR_ARG for a NULL handle or every < 0. */
lbm_status lbm_set_check_interval(lbm_handle h, int64_t every);

/* Steps taken since init. */
lbm_status lbm_step_count(lbm_handle h, int64_t *steps);

#define LBM_DEVICE_PTRS 1u
/* Moments (rho, ux, uy, T) of the post-stream, post-boundary populations of the last step
 * (Sec. 2; eq. macro); after 0 steps those of f*(0).  Each output is [Ny][Nx] float64; NULL
 * skips it.  flags & LBM_DEVICE_PTRS: outputs are device pointers (stream-ordered), else host
 * pointers (the call synchronises). */
lbm_status lbm_moments(lbm_handle h, double *rho, double *ux, double *uy, double *T,
                       unsigned flags);

/* Post-collision populations f*(x, n) as float64 [q][Ny][Nx] host array (fbar + stored
 * deviation), in lbm_velocities() order.  Synchronises. */
lbm_status lbm_populations(lbm_handle h, double *f);

/* PML auxiliary field Q (eq. PMLQ) as float64 [q][Ny][Nx] host array, zero outside the Q
 * region.  Synchronises. */
lbm_status lbm_pml_q(lbm_handle h, double *Q);

/* The library's velocity order of a stencil (lattice 37 or 0: D2Q37, 17: D2Q17, 9: D2Q9; Sec. 2,
 * "Velocity stencils"): e[2*i], e[2*i+1] integer lattice vector of population i (e holds 2q
 * entries); w[i] its weight; *r the thermal scale (xi = r e).  Host only; any pointer may be
 * NULL.  LBM_ERR_ARG for another lattice. */
lbm_status lbm_velocities(int32_t lattice, int32_t *e, double *w, double *r);

/* Global relative L2 errors of Sec. 5 (Reference Simulation) over the bulk,
 * e_Z = sqrt(sum ((Z - Zref)/Zref)^2) for Z = rho, ux, T, accumulated in float64 in a fixed
 * order.  ref_*: host float64 [ny][nx] bulk arrays.  out[3] host.  Synchronises. */
lbm_status lbm_error_norms(lbm_handle h, const double *ref_rho, const double *ref_ux,
                           const double *ref_T, double out[3]);

/* lbm_error_norms for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): the same three norms with the same
 * bits, but every pointer is device memory and the call only enqueues kernels on the run's stream
 * (no allocation, no copy, no synchronisation; the caller synchronises before reading out).
 * ref_*: device float64 [ny][nx] bulk arrays; out: device float64[3].  The per-row partial sums
 * live in a library-owned device array of 16384 rows (384 KiB, one per device, held until the
 * process ends); the run's device must be current.  Calls that overlap on one device share that
 * array and race: order them on one stream.  Errors: LBM_ERR_ARG for NULL pointers or a bulk of
 * more than 16384 rows; LBM_ERR_STATE before lbm_init_fields; LBM_ERR_DEVICE if a launch fails. */
lbm_status lbm_error_norms_noalloc(lbm_handle h, const double *ref_rho, const double *ref_ux,
                                   const double *ref_T, double *out);

/* Scan the current state for non-finite values, rho <= 0 or T <= 0: LBM_OK or
 * LBM_ERR_UNSTABLE.  In the bounds-checked build, LBM_ERR_DEVICE first if a kernel of the run
 * met an index out of range since the run's descriptor was last uploaded.  Synchronises. */
lbm_status lbm_check(lbm_handle h);

/* How this library was built: 0 for the normal build, LBM_BUILD_BOUNDS for the bounds-checked
 * debug build (liblbm_mi355x_bounds.so, same ABI).  That build checks every element index of
 * the step kernels against its buffer (populations, Q, the moment strips, the ring's G and
 * targets) and the grid coordinates of the boundary nodes; an index out of range is counted on
 * the run and replaced by 0, so the kernel does not fault, and lbm_check reports it.  It gives
 * the same results as the normal build and runs slower.  Host only; never fails. */
#define LBM_BUILD_BOUNDS 1
int32_t lbm_build_flags(void);

/* Wait for the run's stream. */
lbm_status lbm_synchronize(lbm_handle h);

/* Tile shape; takes effect at the next lbm_step.  LBM_ERR_ARG for unsupported shapes. */
lbm_status lbm_set_launch(lbm_handle h, const lbm_launch *cfg);
lbm_status lbm_get_launch(lbm_handle h, lbm_launch *cfg);

/* Time every supported bulk tile shape in each schedule -- in order, on a side stream (for a
 * run that owns its stream), and fused with the phase-A blocks after 0, 2, 4, 6 or 8 eighths of
 * the tiles -- on a scratch copy of this run's geometry (the run's own state is untouched) and
 * keep the fastest; if cache_path is non-NULL the choice is read from / appended to that text
 * file, one line "Nx Ny storage lattice bulk_tx overlap split" per choice (a line without the
 * split reads as split -1).  *chosen may be NULL. */
lbm_status lbm_autotune(lbm_handle h, int32_t steps, const char *cache_path,
                        lbm_launch *chosen);

/* Per-kernel-class timing with HIP events (the wall time of the boundary/PML kernels vs the
 * bulk kernel; Sec. 5 "Computational Cost").  mode 1: every kernel class runs in order on the
 * run's stream and events time each class: ms[0] bulk kernel, ms[1] frame kernel (collision of
 * the boundary layers and the PML), ms[2] phase A (characteristic fill of the ring and PML
 * auxiliary update).  mode 2: the schedule lbm_launch.overlap selects, with events timing its step grid in
 * ms[0] (the grid of phase A and the bulk tiles in the fused schedule, else the bulk kernel) and
 * the frame kernel in ms[1].  mode 3: as mode 2 on every fourth step only (a sampled average that
 * leaves the other steps free of events).  The kernels' events are attached to their dispatch and
 * take the kernel's own start and end.  mode 0 turns timing off.  Any mode other than 0 makes
 * lbm_step launch eagerly (no graphs; the same kernel sequence); a mode outside 0..3 is
 * LBM_ERR_ARG.  lbm_profile_read synchronises and returns the summed milliseconds and launch
 * counts since the last reset. */
lbm_status lbm_profile(lbm_handle h, int enable);
lbm_status lbm_profile_read(lbm_handle h, double ms[3], int64_t launches[3], int reset);

/* Checkpoint: write / read the full state (populations, Q, moment strips, step count,
 * configuration) to a binary file with a header and checksum.  lbm_load needs a handle
 * created and configured identically and initialised (any fields); a file of another format
 * version (the layout of Q and the moment strips follows the library's frame numbering) or
 * another configuration is refused with LBM_ERR_ARG. */
lbm_status lbm_save(lbm_handle h, const char *path);
lbm_status lbm_load(lbm_handle h, const char *path);

void lbm_destroy(lbm_handle h);

const char *lbm_last_error(void);

/* ---- Batched runs: one launch per kernel class advances many independent runs ---------- */

/* A group advances its runs together on one stream; it does not own the runs.  Runs keep
 * their own state; a run may belong to one group at a time.  lbm_group_add requires an
 * initialised run of the group's storage and stencil (LBM_ERR_STATE, LBM_ERR_ARG otherwise) and
 * holds at most 4096 runs per group (LBM_ERR_ARG beyond); adding or removing a run synchronises
 * the group's stream and recaptures its step graphs at the next lbm_group_step. */
lbm_status lbm_group_create(void *stream, const lbm_allocator *allocator,
                            lbm_group_handle *out);
lbm_status lbm_group_add(lbm_group_handle g, lbm_handle h);
lbm_status lbm_group_remove(lbm_group_handle g, lbm_handle h);
/* Advance every member: run k by steps[k] steps (steps may be NULL: all by nsteps), in
 * member order as added; the group issues max(steps) batched steps and a run stops after its
 * own count.  Asynchronous. */
lbm_status lbm_group_step(lbm_group_handle g, const int64_t *steps, int64_t nsteps);
/* Launch configuration of the group's batched steps: bulk_tx/bulk_ty as for a run; with
 * graph_steps = G > 0, lbm_group_step replays a captured HIP graph of G batched steps (runs
 * past their own count skip every kernel, so one graph serves any mix of counts) and launches
 * the remainder eagerly; the graph is recaptured after the membership changes.  overlap 0 or 2
 * (a group runs on one stream).  Default {64, 4, 32, 2}.  LBM_ERR_ARG for unsupported values. */
lbm_status lbm_group_set_launch(lbm_group_handle g, const lbm_launch *cfg);
lbm_status lbm_group_get_launch(lbm_group_handle g, lbm_launch *cfg);
/* Time every bulk tile shape, in order and fused with the phase-A blocks after 0, 2, 4, 6 or 8
 * eighths of the tiles (18 configurations), on a scratch group that holds one scratch run (mean
 * state) per distinct member geometry (grid, PML, boundaries, storage, layout) and keep the
 * fastest for this group.  The members' state is untouched; the scratch memory is freed before return.
 * LBM_ERR_STATE for an empty group.  *chosen may be NULL. */
lbm_status lbm_group_autotune(lbm_group_handle g, int32_t steps, lbm_launch *chosen);
lbm_status lbm_group_size(lbm_group_handle g, int32_t *n);
/* lbm_check of every member with one synchronisation: flags[k] (host, caller-owned, one entry
 * per member in member order) receives 0 for a healthy state, 1 for a non-finite value, rho <= 0
 * or T <= 0, and, in the bounds-checked build only, 2 for a run whose kernels met an index out of
 * range.  Synchronises the group's stream.  Errors: LBM_ERR_ARG for NULL pointers. */
lbm_status lbm_group_check(lbm_group_handle g, int32_t *flags);
lbm_status lbm_group_synchronize(lbm_group_handle g);
void lbm_group_destroy(lbm_group_handle g);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2504_20169_LBM_H */
