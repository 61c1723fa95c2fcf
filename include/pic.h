/*
 * pic.h -- C ABI of the MI355X (gfx950) engine for the 1D electrostatic
 * particle-in-cell (PIC) cycle of S. Markidis and G. Lapenta, "Development and
 * performance analysis of a UPC Particle-in-Cell code" (PGAS10).
 *
 * Model (Sec. 2): one dimension, electrostatic, mobile electrons of charge-to-
 * mass ratio qm over an immobile uniform ion background rho0, periodic domain
 * [0, L) split into ng cells of width dx = L/ng with nodes at (g + 1/2) dx
 * (Appendix A), epsilon_0 = 1.  One step advances the state
 * (x^n, v^{n-1/2}, E^n) to (x^{n+1}, v^{n+1/2}, E^{n+1}):
 *   1. linear (two-node) gather of E^n at each particle (Sec. 2.3);
 *   2. leapfrog kick v^{n+1/2} = v^{n-1/2} + qm E_p^n dt (Sec. 2.1);
 *   3. drift x^{n+1} = x^n + v^{n+1/2} dt and periodic wrap (Sec. 2.1);
 *   4. linear charge deposit with the same two-node weights (Sec. 2.3),
 *      particle charge Q = sign(qm) rho0 L / np (Appendix A);
 *   5. periodic three-point Poisson solve and central-difference field
 *      (Sec. 2.2), solved exactly with zero-mean potential, or by the
 *      paper's fixed-iteration CG (PIC_SOLVE_CG_PAPER).
 *
 * Numerics.  Particle state and push in FP32 (PIC_FP32) or FP64 (PIC_FP64).
 * A particle is u = x/dx in [0, ng) and w = v dt/dx; the engine stores
 * s = u + 1/2 (the exact same number shifted, so that the cell index is
 * floor(s - 1) with ghost nodes at both ends of its tables).
 * The deposit is exact fixed point: with U = floor(u 2^32) (exact, from the
 * bits of u), j = floor((U - 2^31) / 2^32) and F = U - 2^31 - j 2^32, node
 * j mod ng receives 2^32 - F and node j+1 mod ng receives F as int64, so the
 * grid sum S_g is independent of summation order and sum_g S_g = np 2^32
 * exactly; rho_g = rho0 + (Q/dx) 2^-32 S_g.  Solve and diagnostics in FP64.
 *
 * Ownership.  Host arrays passed in are borrowed for the call and copied.
 * A caller-provided device buffer (dev_mem) is borrowed for the lifetime of
 * the run and must be at least pic_footprint() bytes, 256-byte aligned; with
 * dev_mem == NULL the library allocates (and later frees) its own.  Output
 * arrays are caller-allocated with explicit capacities.
 *
 * Errors.  Every call returns a pic_status; negative values are errors and
 * pic_last_error() then holds a thread-local message.  Nothing is thrown
 * across the ABI and nothing aborts.  Device faults of asynchronous work
 * surface at the next synchronising call as PIC_EDEVICE, after which the run
 * is sticky in PIC_ESTATE.  Calls on one handle must be serialised by the
 * caller; different handles may be used from different threads.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  All
 * device work of a run or batch is enqueued on its stream.
 */
#ifndef PIC1D_PIC_H
#define PIC1D_PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,   /* invalid argument or parameter                      */
    PIC_ENOMEM = -2,   /* device or host allocation failed / buffer too small */
    PIC_EDEVICE = -3,  /* HIP runtime or device error                         */
    PIC_ESTATE = -4,   /* handle in an error state, or call out of order      */
    PIC_EBUDGET = -5   /* batch: the run does not fit the HBM budget now      */
} pic_status;

typedef enum { PIC_FP32 = 0, PIC_FP64 = 1 } pic_precision;

/* Run parameters (Appendix A lists the paper's: L, ng, np, dt, qm, rho0).
 * Validation: ng in [2, PIC_MAX_NG]; 1 <= np < 2^31; L > 0; dt > 0;
 * qm != 0; rho0 > 0; all finite; precision PIC_FP32 or PIC_FP64;
 * solver PIC_SOLVE_EXACT or PIC_SOLVE_CG_PAPER; 0 <= cg_iters <= 100000;
 * sort_every >= PIC_SORT_AUTO. */
typedef struct pic_params {
    double  L;            /* periodic domain length                          */
    int32_t ng;           /* cells = grid nodes                              */
    int32_t precision;    /* pic_precision of the particle state and push    */
    int64_t np;           /* computational particles                         */
    double  dt;           /* time step                                       */
    double  qm;           /* charge-to-mass ratio (electrons: -1)            */
    double  rho0;         /* ion background density (paper: 1)              */
    int32_t sort_every;   /* cell sort every K > 0 steps; 0 never (no room
                             reserved); PIC_SORT_AUTO: K chosen at creation */
    int32_t tile;         /* particles per tile (multiple of 1024); 0 = default */
    int64_t history_cap;  /* per-step history rows kept on the device        */
    int32_t solver;       /* PIC_SOLVE_EXACT (default) or PIC_SOLVE_CG_PAPER   */
    int32_t cg_iters;     /* CG iterations for PIC_SOLVE_CG_PAPER; 0 = 150     */
} pic_params;

/* Field solvers of the periodic three-point system (Sec. 2.2).
 * PIC_SOLVE_EXACT: exact solution with zero-mean potential (prefix sum of
 *   the face field); equal to the converged CG.
 * PIC_SOLVE_CG_PAPER: the paper's matrix-free conjugate gradient (Sec. 2.2,
 *   Sec. 3.3): potential at node 0 held at zero, started from zero, a fixed
 *   number of iterations (the paper uses 150), then the central difference.
 *   It reproduces the paper's closing step including its non-convergence at
 *   large ng (150 iterations do not converge for ng above ~150). */
#define PIC_SOLVE_EXACT 0
#define PIC_SOLVE_CG_PAPER 1

#define PIC_MAX_NG 8192

/* Diagnostics of the current state (x^N, v^{N-1/2}, E^N) after N steps. */
typedef struct pic_diag {
    int64_t  step;             /* N                                            */
    double   time;             /* N dt                                         */
    double   kinetic;          /* (m/2) sum_p (v_p^{N-1/2})^2, m = Q/qm        */
    double   field;            /* W_E^N = (1/2) sum_g (E_g^N)^2 dx              */
    double   momentum;         /* m sum_p v_p^{N-1/2}                          */
    int64_t  charge_fixed_sum; /* sum_g S_g of the deposit of x^N (= np 2^32)  */
    double   net_charge;       /* sum_g rho_g dx (ions + particles)            */
    uint32_t flags;            /* PIC_FLAG_* seen since creation              */
    uint32_t pad_;
} pic_diag;

#define PIC_FLAG_NONFINITE 1u  /* a non-finite position was reset to 0       */
#define PIC_FLAG_MULTIWRAP 2u  /* a particle moved more than L in one step   */
#define PIC_FLAG_SORT      4u  /* internal: a cell sort lost track of a slot  */

/* One row per step n (0-based) of the per-step history:
 *   [0] KE^n  = (m/4) sum_p ((v^{n-1/2})^2 + (v^{n+1/2})^2)  (time-centred)
 *   [1] W_E^n = field energy of E^n, the field that step n gathers
 *   [2] P^{n+1/2} = m sum_p v^{n+1/2}
 *   [3] K^{n+1/2} = (m/2) sum_p (v^{n+1/2})^2                            */
#define PIC_HIST_COLS 4

typedef struct pic_run pic_run;
typedef struct pic_batch pic_batch;

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *pic_last_error(void);

/* Library version string. */
const char *pic_version(void);

/* Device bytes a run with these parameters needs (state, sort scratch, grids,
 * per-tile partials, history, descriptor).  EINVAL on invalid parameters. */
pic_status pic_footprint(const pic_params *params, size_t *bytes);

/* Create a run from host positions x0[np] in [0, L) and velocities
 * v_mhalf[np] (the velocity at t = -dt/2, the leapfrog half step of Sec. 2.1),
 * both FP64 and copied.  Requires max |v| dt < L (one wrap per step).
 * Deposits x0 and solves for E^0 on the device (enqueued on `stream`).
 * dev_mem/dev_bytes: see Ownership above.  On success *out owns the run. */
pic_status pic_create(const pic_params *params, const double *x0, const double *v_mhalf,
                      void *dev_mem, size_t dev_bytes, void *stream, pic_run **out);

/* Device-side loader: the initial particles are drawn on the GPU instead of
 * being uploaded.  Draw i of stream s is the SplitMix64 output (Steele, Lea
 * and Flood, OOPSLA 2014) for the counter base(seed, s) + (i + 1) gamma,
 * base(seed, s) = mix(seed * 0x100000001B3 + s * 0x9E37 + 1), gamma =
 * 0x9E3779B97F4A7C15; uniforms u = (draw >> 11) 2^-53; normals
 * n = sqrt(-2 log1p(-u)) cos(2 pi u') from draws i of streams vel_stream
 * and vel_stream + 1.  Particle i:
 *   x0 = L u_i (stream pos_stream), or the lattice x0 = (i + 1/2) L / np,
 *   x = x0 + amp sin(k x0) wrapped to [0, L),
 *   v^{-1/2} = s_i v0 + vth n_i with the beam sign s_i of `beams`,
 * a uniform or single-mode-displaced plasma with drifting beams and a
 * Maxwellian spread (the loads of Sec. 4 and the appendix).  The lattice is
 * the appendix's quiet start: with np a multiple of ng it puts np/ng
 * particles at the centres of equal sub-intervals of every cell.  Random
 * beam signs are the appendix's: +v0 when a uniform u''_i (stream
 * vel_stream + 2) is below 1/2.  A host can reproduce every value; device
 * sin/log1p/cos may differ from a host library's in the last bit. */
typedef struct pic_loader {
    uint64_t seed;
    int32_t  pos_stream;   /* stream of the position uniforms, 0..2^30     */
    int32_t  vel_stream;   /* first of the streams of the normals (then the
                              beam signs at vel_stream + 2), 0..2^30         */
    double   amp;          /* displacement amplitude (length)              */
    double   k;            /* its wavenumber                               */
    double   v0;           /* drift speed                                  */
    double   vth;          /* thermal spread, >= 0                         */
    int32_t  beams;        /* PIC_BEAMS_*: the beam sign s_i                */
    int32_t  lattice;      /* 1: lattice positions, 0: uniform random       */
} pic_loader;

enum {
    PIC_BEAMS_ONE = 0,        /* s_i = 1: one drifting (or resting) species     */
    PIC_BEAMS_ALTERNATE = 1,  /* s_i = +1 for even i, -1 for odd i              */
    PIC_BEAMS_RANDOM = 2      /* s_i = +1 if u''_i < 1/2, else -1               */
};

/* pic_create with the particles drawn on the device by `loader` (no host
 * arrays, no upload).  EINVAL if (|v0| + 8.58 vth) dt >= L: the normals are
 * bounded by sqrt(-2 ln 2^-53) < 8.58, so the single-wrap contract holds. */
pic_status pic_create_loaded(const pic_params *params, const pic_loader *loader, void *dev_mem,
                             size_t dev_bytes, void *stream, pic_run **out);

/* sort_every = PIC_SORT_AUTO (single runs only): at creation the engine
 * times the particle pass on the loaded state, the cell sort, and the pass
 * on the sorted state (HIP events, on a saved copy of the state that is put
 * back, so the run's results are as without the trial), and sorts every
 * K = ceil(2 t_sort / (t_unsorted - t_sorted)) steps if sorting makes the
 * pass faster, else never.  Room for the sort is reserved either way.
 * The storage order, and with it the rounding of the FP64 kinetic-energy
 * and momentum sums, then depends on the K chosen; particle values and the
 * deposit do not.  pic_sort_period reports K. */
#define PIC_SORT_AUTO (-1)

/* The run's cell-sort period after creation: K > 0, or 0 for never. */
pic_status pic_sort_period(pic_run *run, int32_t *k);

/* Enqueue `nsteps` >= 0 steps (asynchronous; returns before they run).
 * With sort_every = K > 0, the particles are reordered by cell (pic_sort)
 * before steps K+1, 2K+1, ... counted from creation. */
pic_status pic_step(pic_run *run, int64_t nsteps);

/* Enqueue a cell sort now (asynchronous): a stable reorder of the
 * particles by the cell of their left node, the locality step the engine
 * also runs every sort_every steps.  Positions, velocities and every later
 * result are unchanged as a multiset; only the storage order changes (and
 * with it the per-tile summation order of the kinetic-energy and momentum
 * diagnostics).  PIC_ESTATE if the run was created with sort_every = 0
 * (no room for the sort's alternate arrays). */
pic_status pic_sort(pic_run *run);

/* Same as pic_step but the steps are replayed from a captured HIP graph of
 * `graph_steps` launches (captured on first use, reused afterwards). */
pic_status pic_step_graph(pic_run *run, int64_t nsteps, int32_t graph_steps);

/* Enqueue `nsteps` >= 1 plain (ungraphed) steps with HIP events around each
 * of the step's two launches (particle pass, field solve), wait for them,
 * and report the mean duration of each launch in milliseconds.  For
 * measurement; the steps are real and advance the run. */
pic_status pic_step_profiled(pic_run *run, int64_t nsteps, double *ms_particle, double *ms_solve);

/* Achievable-bandwidth reference of the particle pass (measurement only, no
 * part of the method): swaps the contents of the device arrays a[n] and
 * b[n] of FP32 values, `reps` >= 1 times on `stream`, with the pass's memory
 * pattern (16-byte loads and stores, all CUs; cached = 0: non-temporal,
 * 1: ordinary cached accesses, the pass's two cache policies) and nothing
 * else, i.e. 16 bytes per element pair per swap, and reports the mean
 * duration of one swap in milliseconds (HIP events around the `reps`
 * back-to-back launches, after one warm-up launch; waits for them).
 * a and b are caller-owned device buffers, 16-byte aligned, n a multiple
 * of 4, cached 0 or 1 (else EINVAL); their contents end swapped if reps is
 * even (reps + 1 launches). */
pic_status pic_bandwidth_probe(void *a, void *b, int64_t n, int32_t reps, int32_t cached, void *stream,
                               double *ms);

/* Synchronise the run's stream and report diagnostics of the current state.
 * rho_out/E_out (FP64, ng_cap >= ng entries) may be NULL. */
pic_status pic_diagnostics(pic_run *run, pic_diag *diag, double *rho_out, double *E_out,
                           int32_t ng_cap);

/* Synchronise and copy the particles out in physical units
 * (x = u dx, v^{N-1/2} = w dx/dt) in their current storage order (the cell
 * sort permutes them).  cap >= np. */
pic_status pic_read_particles(pic_run *run, double *x, double *v, int64_t cap);

/* Synchronise and copy the raw engine state: u[np], w[np] in the run's
 * precision (float for PIC_FP32, double for PIC_FP64). cap >= np. */
pic_status pic_read_raw(pic_run *run, void *u, void *w, int64_t cap);

/* Synchronise and copy the fixed-point sums S[ng] of the current positions,
 * the FP64 node field E[ng] and the FP32 gather table Ehat[ng] =
 * float(E qm dt^2/dx).  Any pointer may be NULL; cap >= ng. */
pic_status pic_read_grid(pic_run *run, int64_t *S, double *E, float *Ehat, int32_t cap);

/* Phase-space density of the current particles: the (x, v) plane that the
 * two-stream figure of Sec. 4 plots point by point, binned on the device
 * into counts[iv * nx + ix] (nv rows of nx uint32 counts, caller-allocated).
 * From the stored state s = x/dx + 1/2, w = v dt/dx and c = dt/dx, in FP64:
 *   ix = min(floor((s - 1/2) nx / ng), nx - 1),
 *   y = (w - vmin c) * (nv / ((vmax - vmin) c)),  iv = floor(y) if 0 <= y < nv;
 * particles with y outside [0, nv) are counted in *outside (may be NULL).
 * Every particle is counted once: sum(counts) + outside = np.  Needs
 * 1 <= nx nv <= 16384 and finite vmin < vmax (else EINVAL).  Synchronises;
 * allocates 8 + 4 nx nv bytes of device memory for the call. */
pic_status pic_phase_space(pic_run *run, int32_t nx, int32_t nv, double vmin, double vmax, uint32_t *counts,
                           int64_t *outside);

/* pic_phase_space for callers that cannot allocate device memory (code that
 * must not call hipMalloc/hipFree, such as tight serving loops or harnesses
 * that forbid allocation): the same image, arguments and errors, binned in
 * a fixed device scratch of 8 + 4 * 16384 bytes that the library holds per
 * GPU for the life of the process; it allocates nothing.  nx nv above 16384
 * (the scratch's capacity) is EINVAL.  The scratch is shared by every call on
 * a GPU and cleared at the start of each call: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the
 * caller.  Synchronises, like pic_phase_space. */
pic_status pic_phase_space_noalloc(pic_run *run, int32_t nx, int32_t nv, double vmin, double vmax,
                                   uint32_t *counts, int64_t *outside);

/* Synchronise and copy history rows [first, first+count) (PIC_HIST_COLS
 * doubles each).  Rows beyond min(steps taken, history_cap) are EINVAL. */
pic_status pic_read_history(pic_run *run, int64_t first, int64_t count, double *rows);

/* Wait for the run's queued work, release what the library allocated. */
pic_status pic_destroy(pic_run *run);

/* ---------------------------------------------------------------------
 * Batched engine and continuous-batching service.
 *
 * A batch steps many independent runs of different (np, ng) with two
 * launches per step, replayed from a captured HIP graph: one persistent
 * particle pass over the chunks of every unfinished run, then one solve
 * launch with two workgroups (field, diagnostics) per unfinished run.  Runs
 * are admitted at any time against an HBM budget (bytes of the
 * batch's device arena), keep their state resident, stop at their own step
 * count and release their memory on pic_batch_release.  The result of a run
 * is the same alone and in any mix: its tiles, deposit and solve depend only
 * on its own (np, ng).
 * ------------------------------------------------------------------- */
typedef struct pic_batch_config {
    size_t  hbm_budget;    /* bytes of the device arena for run state        */
    void   *arena;         /* caller device buffer of hbm_budget bytes, or NULL */
    int32_t max_runs;      /* run-table capacity                              */
    int32_t ng_max;        /* largest ng admitted (sizes the LDS)             */
    int32_t graph_steps;   /* kernel launches captured per graph              */
    int32_t grid_blocks;   /* persistent workgroups; 0 = device default       */
} pic_batch_config;

pic_status pic_batch_create(const pic_batch_config *cfg, void *stream, pic_batch **out);

/* Admit a run that will take `nsteps` steps from host x0[np], v_mhalf[np]
 * (as pic_create; FP32 state only, ng <= ng_max, sort_every >= 0).  PIC_EBUDGET if its
 * footprint does not fit the arena or the run table is full now (nothing is
 * changed; retry after releases).  Asynchronous: the particles are converted
 * into pinned staging memory before the call returns (the caller's arrays
 * are free again), then upload, grid clearing and the initial deposit and
 * solve are enqueued on the batch stream; the host does not wait.  The run
 * joins the next pic_batch_step launch.  A failure after work was enqueued
 * puts the batch in the error state (PIC_EDEVICE, then PIC_ESTATE). */
pic_status pic_batch_admit(pic_batch *b, const pic_params *params, const double *x0,
                           const double *v_mhalf, int64_t nsteps, int64_t *run_id);

/* pic_batch_admit with the particles drawn on the device by `loader`. */
pic_status pic_batch_admit_loaded(pic_batch *b, const pic_params *params, const pic_loader *loader,
                                  int64_t nsteps, int64_t *run_id);

/* Advance every unfinished run by up to `nsteps` steps (asynchronous). */
pic_status pic_batch_step(pic_batch *b, int64_t nsteps);

/* pic_batch_step with HIP events around each launch (no graph), waiting
 * for completion and reporting the mean particle-pass and solve durations
 * in milliseconds over the launches issued. */
pic_status pic_batch_step_profiled(pic_batch *b, int64_t nsteps, double *ms_particle,
                                   double *ms_solve);

/* Report runs that reached their step count since the last poll
 * (non-blocking: only completed device work is reported). */
pic_status pic_batch_poll(pic_batch *b, int64_t *done_ids, int32_t cap, int32_t *n_done);

/* Borrow the pic_run view of a batch member, valid until its release; the
 * read/diagnostic calls above work on it (pic_step/pic_destroy do not). */
pic_status pic_batch_run(pic_batch *b, int64_t run_id, pic_run **view);

/* Diagnostics of batch member `run_id` (as pic_diagnostics, without the
 * grids): its step count N and the energies, momentum and charge of its state
 * after N steps (Sec. 2 model; the sums are defined at pic_diag).  Waits for
 * the work queued on the batch stream unless the member was already
 * reported complete by pic_batch_poll, in which case it reads without
 * waiting for the other members.  EINVAL for an unknown or released id. */
pic_status pic_batch_diagnostics(pic_batch *b, int64_t run_id, pic_diag *diag);

/* Retire a run: its table slot and arena space become free for later
 * admissions at once.  Asynchronous and safe while work is queued: reuse is
 * ordered after that work on the batch stream.  Its pic_run view and its
 * results are gone; read them (pic_diagnostics etc. on the view) before.
 * Releasing an unfinished run stops it. */
pic_status pic_batch_release(pic_batch *b, int64_t run_id);

/* Bytes of the arena in use / free, and runs admitted and not released. */
pic_status pic_batch_usage(pic_batch *b, size_t *used, size_t *free_bytes, int32_t *nruns);

pic_status pic_batch_destroy(pic_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* PIC1D_PIC_H */
