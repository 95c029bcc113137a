/*
 * weno_l2is.h -- C ABI of the MI355X (gfx950) library for the right-hand
 * side and SSP-RK3 update of the L2-norm regularized incremental-stencil WENO
 * scheme (Zhu & Hu, arXiv 1908.02464) for the compressible Euler equations on
 * uniform structured 1D/2D/3D grids.
 *
 * What is computed (paper references):
 *   semi-discretization  dU/dt = -(F_{j+1/2} - F_{j-1/2}) / dx      Eq.(19)
 *   per face: Roe average, eigensystem, characteristic projection,
 *     flux splitting, WENO reconstruction, back projection          Sec. 2.3
 *   candidate fluxes, smoothness indicators, reference tau5        Eq.(6),(11)
 *   L2-norm error terms and regularized weights                    Eq.(27),(28)
 *   discontinuity detector, regularization parameter               Eq.(30)-(32)
 *   hybrid switch to the optimal linear upwind flux                Eq.(33)-(35)
 *   third-order TVD Runge-Kutta with CFL 0.5                       Sec. 4
 * Multi-D grids are treated dimension by dimension (the paper states 1D).
 *
 * Data layout (every state array): FP64, structure of arrays
 * [nvar][nz][ny][nx], x fastest, interior cells only (no ghost layers),
 * nvar = 2 + dim, dim = 1 if ny == nz == 1, 2 if nz == 1 < ny, 3 if nz > 1
 * (nz > 1 requires ny > 1).  Variables: rho, rho*u_x, [rho*u_y, [rho*u_z]], E.
 *
 * Pointers named U, dUdt, U0 are DEVICE pointers on the current HIP device;
 * the caller owns them.  The library owns its scratch (stage buffers, the
 * device time-step word, status), allocated in *_create / *_admit and freed
 * in *_destroy / *_fetch.
 *
 * Errors: every int-returning call returns 0 on success, a negative
 * WL2_E_* code on invalid input or a HIP failure (nothing is enqueued then),
 * or WL2_S_NONPHYSICAL (> 0) from the calls that report device status.  No
 * call aborts or throws; weno_l2is_strerror names a code.
 */
#ifndef WENO_L2IS_H
#define WENO_L2IS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WL2_OK = 0,
  WL2_E_NULL = -1,        /* a required pointer is NULL                     */
  WL2_E_SHAPE = -2,       /* n < 1, nz > 1 with ny == 1, or 2^32 cells+     */
  WL2_E_PARAM = -3,       /* dx, gamma, cfl, thresholds or enums invalid    */
  WL2_E_BC = -4,          /* unpaired periodic side, reflective with n < 3,
                             inflow misplaced or its state not set          */
  WL2_E_HIP = -5,         /* a HIP runtime call failed                       */
  WL2_E_NOMEM = -6,       /* device allocation failed                        */
  WL2_E_BUDGET = -7,      /* batch: HBM budget or slot table exhausted;
                             rhs_noalloc: grid beyond its static scratch     */
  WL2_E_SLOT = -8,        /* batch: slot not in use / not finished           */
  WL2_S_NONPHYSICAL = 1   /* rho <= 0, p <= 0 or non-finite state detected   */
};

/* Boundary rule of a side, applied through three ghost cells (the paper
 * names the conditions of its tests only): PERIODIC wraps (both sides of a
 * direction); TRANSMISSIVE copies the boundary cell (outflow); REFLECTIVE
 * mirrors the interior with the normal momentum negated (Sec. 4.3, 4.7);
 * INFLOW gives the ghosts a prescribed state per x line, set with
 * weno_l2is_set_inflow (the left side of the jet of Sec. 4.7; allowed on the
 * x- side of a 1D or 2D grid held by a context only).  The state sides of
 * the double Mach reflection (Sec. 4.5), on the y sides of 2D grids (not in
 * the batch engine): STATE_WALL gives the ghosts under the cells centred
 * left of x = bgeom[0] the state bstate[0] and mirrors the interior (as
 * REFLECTIVE) elsewhere; STATE_FRONT gives a ghost centred at (x, y) the
 * state bstate[0] if x < bgeom[1] + bgeom[2] y + bgeom[3] t, else bstate[1]
 * (a straight front moving along x; t = the stage's time on the context's
 * clock: t, t + dt, t + dt/2 within a step of weno_l2is_advance, the
 * clock's t for a right-hand side; the stateless calls use t = 0).  Cell
 * centres lie at ((i + 1/2) dx, (j + 1/2) dx). */
enum { WL2_BC_PERIODIC = 0, WL2_BC_TRANSMISSIVE = 1, WL2_BC_REFLECTIVE = 2,
       WL2_BC_INFLOW = 3, WL2_BC_STATE_WALL = 4, WL2_BC_STATE_FRONT = 5 };

/* Flux-splitting speed alpha^s of Eq.(21): LLF = max over the six stencil
 * cells of |lambda^s(U_m)| (the hot path); LF = max over the whole grid per
 * direction, recomputed every stage; ROE = |lambda^s| of the Roe matrix. */
enum { WL2_SPLIT_LLF = 0, WL2_SPLIT_LF = 1, WL2_SPLIT_ROE = 2 };

/* Hybrid switch of Eq.(33)/(35): PER_FIELD = linear flux for field s iff
 * sigma^s < eps (default); PER_FACE = linear for all fields iff
 * max_s sigma^s < eps; WENO_ONLY = regularized WENO everywhere;
 * LINEAR_ONLY = optimal linear upwind scheme everywhere. */
enum { WL2_HYB_PER_FIELD = 0, WL2_HYB_PER_FACE = 1, WL2_HYB_WENO_ONLY = 2,
       WL2_HYB_LINEAR_ONLY = 3 };

/* Weights of the nonlinear reconstruction: L2IS = the regularized weights of
 * the present scheme, Eq.(28) (default); IS = the original WENO-IS weights,
 * Eq.(8); IS_B01 = WENO-IS with the 3-point indicator beta_01 of Eq.(15)
 * multiplying the ratios of the two 2-point stencils, Eq.(14) (the
 * "WENO-IS" scheme the paper compares against).  The two comparison forms
 * do not use lambda; with WL2_HYB_WENO_ONLY they are those schemes. */
enum { WL2_W_L2IS = 0, WL2_W_IS = 1, WL2_W_IS_B01 = 2 };

typedef struct weno_l2is_params {
  double cfl;       /* CFL number, 0.5 (Sec. 4)                               */
  double c_reg;     /* c in lambda = c * sigma^s, Eq.(32): 1                  */
  double eps_weno;  /* epsilon of the weights, Eq.(28): 1e-20                 */
  double thr_C;     /* C of the threshold eps = C (dx/L)^alpha, Eq.(35): 1    */
  int thr_alpha;    /* alpha of Eq.(35): 3                                    */
  int split;        /* WL2_SPLIT_*                                            */
  int hybrid;       /* WL2_HYB_*                                              */
  int bc[6];        /* x-, x+, y-, y+, z-, z+ : WL2_BC_*; periodic is paired  */
  double thr_L[3];  /* L of Eq.(35) per direction; default n_d * dx           */
  int weights;      /* WL2_W_*: weights of the WENO branch; default L2IS      */
  double bstate[2][5];  /* conserved states of STATE_WALL / STATE_FRONT ghosts
                           (first nvar values); default 0                   */
  double bgeom[4];  /* wall start x; front x0, dx/dy, dx/dt; default 0        */
} weno_l2is_params;

typedef struct weno_l2is_ctx weno_l2is_ctx;

/* Defaults above for an nx*ny*nz grid of spacing dx, transmissive sides. */
int weno_l2is_params_default(weno_l2is_params *p, int nx, int ny, int nz,
                             double dx);

/* Create a solver context for one grid.  hip_stream: hipStream_t (NULL =
 * the null stream); all of the context's work is enqueued there.  Allocates
 * the two RK stage buffers, one accumulator (per-direction path), the
 * correction list (8 bytes per cell), a 6.4 KB control block, for 2D
 * grids of 131072 cells or more the face-once correction buffers (68 bytes
 * per cell), and for 3D grids a face buffer (120 bytes per cell) where the
 * corrections compute each face once: with every face WENO (LLF
 * splitting), and with the hybrid switch (per field or per face), which
 * also lists the faces that need the WENO flux (12 bytes per cell).  About
 * 4.4 GB for a 256^3 grid with the hybrid switch (4.2 GB with every face
 * WENO, 2.2 GB with every face linear). */
int weno_l2is_create(int nx, int ny, int nz, double dx, double gamma,
                     const weno_l2is_params *p, void *hip_stream,
                     weno_l2is_ctx **out);

/* Right-hand side of Eq.(19): dUdt = -sum_d (F_{j+1/2} - F_{j-1/2})_d / dx,
 * for the state U (device).  Stateless form: enqueued on the null stream,
 * asynchronous; an internal context per shape and device is cached and
 * reused until weno_l2is_rhs_release.  U and dUdt must not overlap
 * (WL2_E_PARAM if they share a byte). */
int weno_l2is_rhs(const double *U, int nx, int ny, int nz, double dx,
                  double gamma, const weno_l2is_params *params, double *dUdt);

/* Release every context that weno_l2is_rhs keeps (one per grid shape and
 * device, about 2.2 GB for a 256^3 grid; they are otherwise held until the
 * process ends).  Waits for their work to finish, then frees their device
 * memory; a later weno_l2is_rhs builds its context again.  Must not run
 * while another thread is inside weno_l2is_rhs on a shape being released
 * (the cache itself is guarded by a lock).  Returns the number of contexts
 * released (>= 0), or WL2_E_HIP if a device could not be selected. */
int weno_l2is_rhs_release(void);

/* Bytes of the static device scratch of weno_l2is_rhs_noalloc (per GPU). */
#define WL2_NOALLOC_SCRATCH_BYTES (64u << 20)

/* weno_l2is_rhs without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid it).  The same dU/dt, bit for bit, enqueued on hip_stream
 * (hipStream_t; NULL = the null stream).  Its scratch (control block and
 * correction list: 8 bytes per cell plus 6.4 KB, and 8 bytes per column
 * tile and plane in 3D) lives in a static device array of
 * WL2_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, held until the
 * process ends; grids whose scratch does not fit (about 8.3M cells) are
 * refused with WL2_E_BUDGET before any device work.  Every call on a GPU
 * shares that GPU's array (the control block is cleared by a kernel at the
 * start of each call): calls that overlap on one GPU (different streams,
 * different threads) race, so the caller orders them.  No inflow or state
 * side (WL2_E_BC).  Other arguments and errors as weno_l2is_rhs.  (The
 * library allocates nothing here; the builds of some schemes keep spilled
 * registers in private memory, which the HIP runtime reserves for a queue
 * at the first launch of such a build on it, as for any kernel.) */
int weno_l2is_rhs_noalloc(const double *U, int nx, int ny, int nz, double dx,
                          double gamma, const weno_l2is_params *params,
                          double *dUdt, void *hip_stream);

/* The same on a context (its stream and scratch); the same overlap rule. */
int weno_l2is_rhs_ctx(weno_l2is_ctx *ctx, const double *U, double *dUdt);

/* One SSP-RK3 step of U in place (Shu-Osher form:
 *   U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U  = 1/3 U + 2/3 (U2 + dt L(U2))).
 * dt > 0: use it.  dt <= 0: the CFL step cfl*dx / max_cells sum_d(|u_d|+c)
 * is reduced on the device from U (no host round trip) and non-physical
 * cells set the status word.  Asynchronous on the context's stream. */
int weno_l2is_step(weno_l2is_ctx *ctx, double *U, double dt);

/* Advance U by n_steps CFL steps (dt from the device each step), stopping
 * exactly at t_end (> 0; the last step is clipped, later steps are no-ops).
 * Steps after a non-physical state was seen (status bit set) are no-ops too:
 * U keeps the last state the CFL reduction flagged.
 * The simulated time is kept on the device and read by weno_l2is_time.
 * The result equals n_steps calls of weno_l2is_step with the clock rule, bit
 * for bit; internally the CFL maximum of a step is folded out of the
 * previous step's last stage, and 1D grids of up to 1024 cells (not with
 * global Lax-Friedrichs splitting) run all steps in one single-workgroup
 * launch.  Asynchronous on the context's stream. */
int weno_l2is_advance(weno_l2is_ctx *ctx, double *U, int n_steps,
                      double t_end);

/* Ghost state of the inflow side (Sec. 4.7: the left boundary of the jet
 * prescribes the state (rho, u, v, p) of its ghosts, one state inside the
 * jet and another outside).  state: DEVICE pointer to the conserved state
 * [nvar][ny] (x fastest layout of one column: element v*ny + y is variable
 * v of the three ghost cells left of row y).  Checked (rho > 0, p > 0,
 * finite) and copied into the context before the call returns; the caller
 * keeps ownership.  A refused state (WL2_E_PARAM) changes nothing: the
 * context keeps the last accepted state and its time-step bound.  The
 * context must
 * have been created with bc[0] == WL2_BC_INFLOW (else WL2_E_BC); until this
 * call has been made, every call that evaluates the right-hand side
 * (rhs_ctx, step, advance, face_debug) returns WL2_E_BC.  The stateless
 * weno_l2is_rhs and the batch engine refuse WL2_BC_INFLOW (WL2_E_BC). */
int weno_l2is_set_inflow(weno_l2is_ctx *ctx, const double *state);

/* Reset the device clock of the context to t (for weno_l2is_advance). */
int weno_l2is_set_time(weno_l2is_ctx *ctx, double t);

/* CFL time step of U (device reduction; with an inflow side the speed of
 * its ghost states bounds it too).  If dt_host is not NULL the call
 * synchronizes the stream and stores it.  Returns WL2_S_NONPHYSICAL if a
 * non-physical cell was found (only known when dt_host != NULL). */
int weno_l2is_cfl_dt(weno_l2is_ctx *ctx, const double *U, double *dt_host);

/* Synchronize and read the dt used by the latest step, the device clock and
 * the number of clock steps taken since the context was created (steps of
 * weno_l2is_advance that advanced the clock).  Any pointer may be NULL. */
int weno_l2is_time(weno_l2is_ctx *ctx, double *t_host, double *last_dt_host,
                   unsigned *steps);

/* Per-face switch flags (1 = linear flux) and detector values sigma^s of
 * Eq.(30) along direction dir, computed by the same device code as the
 * sweeps (the fused kernels evaluate the detector in another operation
 * order, a few ulp apart, so a flag can differ only where sigma^s lies
 * within that of the threshold).  Layout [nvar][..] with n_dir + 1 faces
 * along dir (face f lies
 * between cells f-1 and f), the other extents unchanged, x fastest; both
 * are DEVICE pointers and may not overlap U or each other (WL2_E_PARAM).
 * Asynchronous. */
int weno_l2is_face_debug(weno_l2is_ctx *ctx, const double *U, int dir,
                         unsigned char *flags, double *sigma);

/* Synchronize and return the sticky status bits (bit 0: non-physical state
 * seen by a CFL reduction).  Returns WL2_S_NONPHYSICAL if any bit is set.
 * clear != 0 resets the bits. */
int weno_l2is_status(weno_l2is_ctx *ctx, unsigned *status_bits, int clear);

/* Kernel path and tuning of a context.  path: WL2_PATH_AUTO or
 * WL2_PATH_FUSED (the single-pass stage kernel of the grid's dimension: 3D
 * column tiles marching in z, or 1D/2D rows of 63 cells marching in y),
 * WL2_PATH_SWEEPS (one kernel per direction, partial sums through memory),
 * WL2_PATH_FUSED_CELLS (the fused stage kernel with the nonlinear
 * corrections computed per listed cell even where the default corrects
 * each flagged face once: 2D grids of 131072 cells or more, and 3D grids
 * with every face WENO or the hybrid switch).
 * zchunk: z planes (3D) or rows (2D, at most 62) per work item of the fused
 * kernels (0 = automatic).  waves_per_simd: register budget of the 3D fused
 * kernel, 1 or 2 (0 = default 2).  The sweeps agree with the fused kernels
 * to round-off; the chunk, the register budget and the correction mode
 * change no result bit. */
enum { WL2_PATH_AUTO = 0, WL2_PATH_SWEEPS = 1, WL2_PATH_FUSED = 2, WL2_PATH_FUSED_CELLS = 3 };
int weno_l2is_tune(weno_l2is_ctx *ctx, int path, int zchunk, int waves_per_simd);

/* Per-launch kernel timing with HIP events recorded on the context's stream
 * around every kernel the context enqueues.  enable != 0 starts (and clears)
 * collection; 0 stops it.  Costs two event records per launch. */
int weno_l2is_timing_enable(weno_l2is_ctx *ctx, int enable);

/* Synchronize and report the collected launches grouped by kernel: for
 * k < *n_kernels (at most cap), names + 64*k holds a NUL-terminated kernel
 * name, total_ms[k] the summed event time and launches[k] the count.  Any
 * of names/total_ms/launches may be NULL to skip it. */
int weno_l2is_timing_read(weno_l2is_ctx *ctx, int cap, char *names,
                          double *total_ms, long long *launches,
                          int *n_kernels);

/* Free the context and its scratch (synchronizes its stream first). */
void weno_l2is_destroy(weno_l2is_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched and served form: many independent 1D/2D runs of uneven sizes
 * advanced together.  Each step is one replay of a captured hipGraph whose
 * persistent kernels walk tables of work items over all admitted runs (an
 * item is 63 columns x a chunk of rows of one run: the unit of the
 * single-grid 1D/2D stage kernel); every run keeps its own CFL dt, clock
 * (stopping exactly at its t_end, or at a non-physical state) and status.  A
 * run's result is bit-identical to running it alone through
 * weno_l2is_advance (same device code, same operation order).
 * The engine allocates `hbm_budget_bytes` once at creation and sub-allocates
 * runs from it: admission fails with WL2_E_BUDGET when a run's footprint
 * (3 state arrays) does not fit or all `max_slots` slots are taken.  Beside
 * the budget it holds a correction list of budget/72 entries of 8 bytes (one
 * per admissible cell), the slot table and the work tables (which grow, with
 * a new graph, when the admitted runs need more items than ever before).
 * LF splitting (WL2_SPLIT_LF) and 3D grids are not supported in a batch
 * (WL2_E_PARAM / WL2_E_SHAPE).
 * All calls are asynchronous on the engine's stream unless noted.
 * ------------------------------------------------------------------------ */
typedef struct weno_l2is_batch weno_l2is_batch;

int weno_l2is_batch_create(size_t hbm_budget_bytes, int max_slots,
                           void *hip_stream, weno_l2is_batch **out);

/* Admit a run: copies U0 (host pointer if u0_on_host, else device pointer,
 * layout as everywhere) into engine memory, clock 0, target t_end > 0.
 * Returns its slot in *slot.  Footprint in bytes in *bytes (may be NULL). */
int weno_l2is_batch_admit(weno_l2is_batch *b, int nx, int ny, int nz,
                          double dx, double gamma, const weno_l2is_params *p,
                          const double *U0, int u0_on_host, double t_end,
                          int *slot, size_t *bytes);

/* Enqueue n_steps batched SSP-RK3 steps of all admitted runs, then a
 * snapshot of every run's clock and status for weno_l2is_batch_poll. */
int weno_l2is_batch_advance(weno_l2is_batch *b, int n_steps);

/* Non-blocking: if the latest snapshot has landed, store up to `cap` slots
 * that reached t_end (or stopped on a non-physical state) and were not
 * reported before; *n_done = number stored (0 if nothing new or the snapshot
 * is still in flight). */
int weno_l2is_batch_poll(weno_l2is_batch *b, int *done_slots, int cap,
                         int *n_done);

/* Synchronize, copy the run's state to U_out (host if out_on_host, else
 * device), report its time, status bits and number of steps taken (t_out,
 * status, steps may be NULL), and free the slot and its memory.  A run that
 * has not reached t_end is cancelled where it stands.  Returns WL2_E_SLOT
 * for a slot not in use. */
int weno_l2is_batch_fetch(weno_l2is_batch *b, int slot, double *U_out,
                          int out_on_host, double *t_out, unsigned *status,
                          unsigned *steps);

/* Launch shape of the batched stage kernels: `rows` rows per work item of a
 * 2D run (1..62; a work item is 63 columns of one run, one wavefront) and
 * `blocks` workgroups in the persistent grid (64..65536); 0 keeps the
 * current value.  Results do not depend on either (every face is computed by
 * the same arithmetic), only the speed does.  Returns WL2_E_PARAM for values
 * outside these ranges. */
int weno_l2is_batch_tune(weno_l2is_batch *b, int rows, int blocks);

/* Bytes of the budget in use and number of admitted runs. */
int weno_l2is_batch_usage(weno_l2is_batch *b, size_t *used_bytes,
                          int *active);

void weno_l2is_batch_destroy(weno_l2is_batch *b);

/* Static string for a return code. */
const char *weno_l2is_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
