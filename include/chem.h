/*
 * chem.h - C ABI of the batched FP64 Rosenbrock (ROS4) chemistry integrator for MI355X (gfx950).
 *
 * Every cell of a CFD domain (or sub-domain) is advanced independently over one
 * operator-splitting step at constant pressure.  The state of a cell is
 * Phi = {T, V, n_1 .. n_{K-1}} per unit mass, the last species being the bath
 * gas closed by the ideal-gas law (paper Sec. 2.1, eqs. (state_vec), (n_nsp)).
 * Each cell is integrated with a linearly implicit Rosenbrock method of the
 * paper's solver table (Table T:solvers) - the four-stage, fourth-order ROS4
 * by default, or ROS3, RODAS3, RODAS4 - in the transformed form of Sec. 2.3
 * (one LU of (I/(h gamma) - J) per step, analytical Jacobian J of eq. (jac)),
 * with adaptive steps from rtol/atol (Sec. 3.1).  One batched call integrates all
 * cells, and each cell's last internal step is returned for reuse as its next
 * initial step (Sec. 2.4.1, the batched chemistry model).
 *
 * Conventions
 *  - Units: SI.  T in K, P in Pa, dt and h in s, W in kg/kmol.
 *  - Layout: species arrays are structure-of-arrays, Y[k * ldY + cell], the
 *    cell index fastest; ldY >= n_cells.
 *  - Pointers to states, outputs and parameters are DEVICE pointers owned by
 *    the caller; the library never frees them.  Handles, workspaces and
 *    checkpoints are library-owned and released by the matching *_free call.
 *  - All calls are asynchronous on `stream` (0 = the null stream); none
 *    synchronises the host unless stated.
 *  - Return codes: 0 success; negative on API errors (see CHEM_E*).  A cell
 *    that fails to integrate does not fail the call: its outcome goes to
 *    status[cell] (CHEM_CELL_*) and it keeps its last accepted state.
 *  - A handle is immutable after load and may be used from several streams;
 *    calls on one stream are ordered, calls on different streams use
 *    separate workspaces.
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define CHEM_OK 0
#define CHEM_EINVAL (-1)       /* null pointer, n < 0, dt <= 0, rtol <= 0, ldY < n, bad option */
#define CHEM_EPARSE (-2)       /* mechanism file missing or malformed */
#define CHEM_EHIP (-3)         /* HIP runtime error */
#define CHEM_ENOMEM (-4)       /* device allocation failed */
#define CHEM_EUNSUPPORTED (-5) /* mechanism larger than the compiled limits, or a method the
                                  call does not support (the adjoint is ROS4 only) */
#define CHEM_ENONDET (-6)      /* checkpointed integration: a repeated pass took other
                                  steps than the first (a non-deterministic launch) */

/* ---- per-cell outcome (status[cell]) ----------------------------------- */
#define CHEM_CELL_OK 0
#define CHEM_CELL_MAX_STEPS 1  /* max_steps attempts reached before dt */
#define CHEM_CELL_H_MIN 2      /* step size fell below h_min */
#define CHEM_CELL_NONFINITE 3  /* ten consecutive non-finite steps */
#define CHEM_CELL_SINGULAR 4   /* ten consecutive zero pivots */

/* ---- scheduling modes (chem_opts.mode) ---------------------------------- */
#define CHEM_MODE_AUTO 0        /* autotuned choice (cached per mechanism/size) */
#define CHEM_MODE_PLAIN 1       /* one cell per thread, one launch of ceil(n/wg) groups */
#define CHEM_MODE_PERSISTENT 2  /* one cell per thread, resident grid, atomic work queue */
#define CHEM_MODE_TEAM 3        /* a team per cell: one wavefront (N <= 64) or a work-group of
                                   four (N <= 128); J and LU in LDS and registers */
#define CHEM_MODE_TEAM_PERSISTENT 4 /* a team per cell, resident grid, work queue.  Above
                                   N = 128 both team modes run one cell per thread, and so
                                   do they where the four-wavefront work-group's LDS (J plus
                                   four copies of the stage vectors) exceeds a CU's 160 KB:
                                   the six-stage CHEM_METHOD_RODAS4 above N = 124. */

/* ---- dispatch order (chem_opts.order) ---------------------------------- */
#define CHEM_ORDER_INDEX 0      /* cells are taken in index order */
#define CHEM_ORDER_HOT_FIRST 1  /* hottest cells first (T_in in 12 K buckets, descending): the
                                   step count grows steeply with temperature, so the longest
                                   cells start first and the tail of the launch is bounded by
                                   the longest cell rather than by its position in the batch;
                                   cells of similar cost also share a wavefront in the
                                   one-cell-per-thread modes.  Results do not depend on it. */

/* ---- integration method (chem_opts.method), Table T:solvers ------------ */
#define CHEM_METHOD_ROS4 0      /* 4 stages, order 4(3), Hairer-Wanner L-stable set (default) */
#define CHEM_METHOD_ROS3 1      /* 3 stages, order 3(2), Sandu et al. */
#define CHEM_METHOD_RODAS3 2    /* 4 stages, order 3(2), stiffly accurate, Sandu et al. */
#define CHEM_METHOD_RODAS4 3    /* 6 stages, order 4(3), stiffly accurate, Hairer-Wanner */
#define CHEM_METHOD_ROS34PW2 4  /* 4 stages, order 3(2), stiffly accurate W-method (Rang and
                                   Angermann 2005): keeps its order with a Jacobian kept over
                                   several steps (chem_opts.jac_every), the paper's future work */

/* ---- error estimate (chem_opts.estimator) ------------------------------ */
#define CHEM_EST_EMBEDDED 0     /* the method's own: difference of the two solutions */
#define CHEM_EST_FILTERED 1     /* the same, times (I - h gamma J)^-1 (one more solve per
                                   step): keeps the h^elo term, takes the estimate of a
                                   strongly damped mode to zero.  For ROS4 the embedded
                                   solution keeps 0.55 of such a mode, so the embedded
                                   estimate rejects steps that relax fast transients;
                                   the filtered one is less conservative at a given tol. */

typedef struct chem_mech_s* chem_mech_t; /* opaque, library-owned */
typedef struct chem_graph_s* chem_graph_t; /* opaque, library-owned captured split step */
typedef struct chem_ckpt_s* chem_ckpt_t; /* opaque, library-owned adjoint checkpoint */

/* Integration options.  Fill with chem_opts_default() and override. */
typedef struct {
  double rtol, atol;      /* ignored here: the chem_integrate arguments rule */
  double h_min;           /* smallest step before CHEM_CELL_H_MIN (1e-20 s) */
  double safety;          /* step-size safety factor (0.9) */
  double fac_min;         /* smallest step ratio (0.2) */
  double fac_max;         /* largest step ratio (6) */
  double T_cut;           /* cells with T_in < T_cut are copied, not integrated (0 = off) */
  int32_t max_steps;      /* attempted steps per cell before CHEM_CELL_MAX_STEPS (100000) */
  int32_t mode;           /* CHEM_MODE_* (CHEM_MODE_AUTO) */
  int32_t wg_size;        /* work-group size in threads (0 = library choice) */
  int32_t waves_per_cu;   /* persistent modes: resident waves per CU (0 = occupancy limit) */
  int32_t order;          /* dispatch order of the cells: CHEM_ORDER_* (CHEM_ORDER_HOT_FIRST) */
  int32_t method;         /* CHEM_METHOD_* (CHEM_METHOD_ROS4) */
  int32_t estimator;      /* CHEM_EST_* (CHEM_EST_EMBEDDED) */
  int32_t team_waves;     /* team modes: wavefronts per cell, 0 = library choice: 1 for
                             N <= 64, 4 for 64 < N <= 128 (the only sizes each is built for:
                             another value is CHEM_EUNSUPPORTED; not 0, 1 or 4: CHEM_EINVAL) */
  int32_t jac_every;      /* J is evaluated at every jac_every-th accepted state of a cell and
                             kept in between (1: every step; only a W-method keeps its order
                             with a kept J).  > 1 is CHEM_EUNSUPPORTED with four wavefronts per
                             cell on a plain grid or without allocation, and for checkpoints */
  unsigned long long* stats; /* nullable DEVICE pointer to 4 counters that the call adds to:
                                attempted steps, accepted steps, rejected steps, Jacobian
                                evaluations (all cells) */
} chem_opts;

/* Defaults listed above. */
void chem_opts_default(chem_opts* o);

/* Parse the text mechanism at `path` (format in the library's generator
 * documentation: species with NASA-7 coefficients, reversible reactions of
 * elementary, third-body, Lindemann and Troe type) and upload its tables to
 * `device`.  *out receives the handle.  Errors: CHEM_EPARSE, CHEM_EUNSUPPORTED
 * (more than 255 species or 4095 reactions), CHEM_EHIP, CHEM_ENOMEM. */
int chem_mech_load(const char* path, int device, chem_mech_t* out);

/* Species, reaction and element counts of a loaded mechanism. */
int chem_mech_info(chem_mech_t m, int32_t* n_species, int32_t* n_reactions, int32_t* n_elements);

/* Release the handle, its device tables and every cached workspace
 * (synchronises the device). */
void chem_mech_free(chem_mech_t m);

/* Integrate n_cells cells over [0, dt] (one split step): the batched
 * chemistry integration of Sec. 2.4.1 - every cell advanced independently at
 * constant pressure (Sec. 2.1), from (T, P, Y) converted to the state of
 * eq. (state_vec) through eq. (conc_form1) and back, by the Rosenbrock method
 * of Sec. 2.3 with the analytical Jacobian of eq. (jac) and adaptive steps
 * from rtol/atol (Sec. 3.1).
 *   T_in[n], P[n], Y_in[K][ldY]  initial temperature, pressure, mass fractions
 *   T_out[n], Y_out[K][ldY]      results; may alias T_in / Y_in
 *   dt        split-step length (> 0); rtol (> 0), atol (>= 0) the tolerances
 *   h_io[n]   nullable; in: first step per cell (<= 0 means dt), out: the
 *             controller's next step after the last accepted one (the step
 *             reused by the next split step, Sec. 2.4.1)
 *   n_steps[n], status[n]  nullable int32 outputs: accepted steps, outcome
 *   lnA[Nr]   nullable; replaces every reaction's ln A (falloff reactions
 *             move their low-pressure A by the same factor), for
 *             differentiation with respect to ln A
 *   opts      nullable (defaults)
 *   ckpt_out  nullable; non-null records every accepted step (state and h;
 *             the adjoint recomputes the stage vectors) for
 *             chem_integrate_adjoint; *ckpt_out receives a new checkpoint
 *             that the caller frees.  One pass records into an arena sized
 *             from the handle's previous checkpointed call (records per cell,
 *             at most a quarter of the free device memory); if it fills up,
 *             the call runs once more with the exact size from that pass's
 *             step counts (same resolved options, from copies of the inputs).
 *             Synchronises the stream
 * All pointers are device pointers owned by the caller.  The library uses a
 * per-(handle, stream) workspace that it allocates on first use and grows.
 * Errors: CHEM_EINVAL (null pointer, n < 0, dt <= 0, rtol <= 0, atol < 0,
 * ldY < n, an option out of range), CHEM_EHIP, CHEM_ENOMEM, CHEM_ENONDET.
 * Asynchronous on `stream` unless ckpt_out is given. */
int chem_integrate(chem_mech_t m, int64_t n_cells, const double* T_in, const double* P,
                   const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                   double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                   const double* lnA, const chem_opts* opts, chem_ckpt_t* ckpt_out,
                   hipStream_t stream);

/* chem_integrate without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments and results as chem_integrate (no
 * checkpoint), with the team launches only (one or four wavefronts per cell,
 * N <= 128), mode CHEM_MODE_AUTO, CHEM_MODE_TEAM or CHEM_MODE_TEAM_PERSISTENT
 * (AUTO and an autotuned one-cell-per-thread choice run the persistent team
 * launch; an explicit one-cell-per-thread mode, and a team launch whose LDS
 * exceeds a CU's - CHEM_METHOD_RODAS4 above N = 124 - are
 * CHEM_EUNSUPPORTED).  With
 * four wavefronts per cell (64 < N <= 128) a rejected step evaluates the
 * Jacobian again instead of reloading a saved copy (the same values, so the
 * results equal chem_integrate's).
 * Scratch: a fixed array in the library's device image, one per device, held
 * until the process ends - the work-queue counter, the dispatch-order bins and
 * the cell order, 4 MiB + 2.3 KiB: at most 1,048,576 cells per call
 * (CHEM_EINVAL above).  Every call on a device shares that device's array, so
 * calls that overlap on one device (on different streams, or from several
 * threads) race and must be serialised by the caller; the counter and bins
 * are cleared by kernels at the start of each call (no memset).
 * Errors: CHEM_EINVAL, CHEM_EUNSUPPORTED, CHEM_EHIP.  Asynchronous on `stream`. */
int chem_integrate_noalloc(chem_mech_t m, int64_t n_cells, const double* T_in, const double* P,
                           const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                           double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                           const double* lnA, const chem_opts* opts, hipStream_t stream);

/* Discrete adjoint of the checkpointed integration: reverse sweep over every
 * cell's accepted steps with the step sizes frozen, through the stages of the
 * transformed Rosenbrock step of Sec. 2.3 (ROS4), the state conversion of
 * eq. (conc_form1) and the source terms of eq. (dphidt).  (The paper does not
 * differentiate the integration; this is the discrete adjoint of the method
 * it uses.)
 *   gT[n], gY[K][ldY]   dL/dT_final, dL/dY_final (device)
 *   g_lnA               [Nr] dL/d ln A summed over cells (per_cell = 0) or
 *                       [Nr][n] per cell (per_cell = 1), overwritten
 *   gT0[n], gY0[K][ldY] nullable: dL/dT_in, dL/dY_in
 * One wavefront per cell: needs N <= 64 and the per-cell LDS (one N x (N+1)
 * matrix, the vectors in doubles and in dual numbers, and Nr accumulators)
 * within the device's LDS per work-group (160 KiB on MI355X), and a
 * checkpoint taken with ROS4, else CHEM_EUNSUPPORTED.  The sum over cells is taken in a fixed order.
 * Errors: CHEM_EINVAL, CHEM_EHIP, CHEM_ENOMEM, CHEM_EUNSUPPORTED.
 * Synchronises the stream when per_cell = 0 (it frees the per-cell scratch). */
int chem_integrate_adjoint(chem_mech_t m, chem_ckpt_t ckpt, const double* gT, const double* gY,
                           int64_t ldY, double* g_lnA, int32_t per_cell, double* gT0,
                           double* gY0, hipStream_t stream);

/* Release a checkpoint (synchronises its stream). */
void chem_ckpt_free(chem_ckpt_t c);

/* Number of records in a checkpoint: for each cell, one per accepted step
 * plus one for the final state; -1 for a null handle. */
int64_t chem_ckpt_records(chem_ckpt_t c);

/* Copy a checkpoint to host memory (synchronises): off[n+1] record offsets of
 * the cells (host), records[chem_ckpt_records][N+1] = (Phi_n, h_n) of each
 * accepted step then (Phi_final, 0) per cell (host).  Either may be null.
 * For inspection and tests. */
int chem_ckpt_export(chem_ckpt_t c, int64_t* off, double* records);

/* Autotuner.  Times the launch configurations (one wavefront per cell,
 * plain or persistent with 1..4 resident waves per CU, or a work-group of four
 * wavefronts per cell for 64 < N <= 128; and, for mechanisms with N <= 16 or
 * N > 128, one cell per thread with 64- or 256-thread groups) on a strided
 * sample of the given batch - sixteen cells per resident wavefront of the
 * device (16,384 on MI355X), at least 4,096 - two runs each,
 * and keeps the fastest for this mechanism and the batch-size bucket
 * floor(log2(n_cells)).  CHEM_MODE_AUTO then uses it.  The choice is kept
 * with the handle and, when the environment variable CHEM_AUTOTUNE_CACHE
 * names a file, appended there and read back by later handles of the same
 * mechanism shape.  *chosen (nullable) receives the winning options; ms
 * (nullable, 8 entries) the best time of each candidate in the order tried
 * (unused entries -1).  Synchronises `stream`. */
int chem_autotune(chem_mech_t m, int64_t n_cells, const double* T_in, const double* P,
                  const double* Y_in, int64_t ldY, double dt, double rtol, double atol,
                  chem_opts* chosen, double* ms, hipStream_t stream);

/* Capture one split step - chem_integrate with exactly these arguments, no
 * checkpoint - into a HIP graph (the work-queue reset is a kernel node, so
 * the graph holds no memset node).  The pointers are baked in: a replay reads
 * and writes the same buffers, so the caller refreshes the inputs (and h_io,
 * which a step overwrites) between replays.  Replays of one graph must not
 * overlap; the graph uses its own workspace.  Errors as chem_integrate. */
int chem_graph_create(chem_mech_t m, int64_t n_cells, const double* T_in, const double* P,
                      const double* Y_in, int64_t ldY, double* T_out, double* Y_out, double dt,
                      double rtol, double atol, double* h_io, int32_t* n_steps, int32_t* status,
                      const double* lnA, const chem_opts* opts, chem_graph_t* out);

/* Replay a captured split step on `stream` (asynchronous). */
int chem_graph_launch(chem_graph_t g, hipStream_t stream);

/* Release a captured split step (synchronises the device). */
void chem_graph_free(chem_graph_t g);

/* Evaluate the source terms f(Phi) (eq. (dphidt)) and, if J is non-null, the
 * dense Jacobian (eq. (jac)) for n cells.  phi[N][ld], f[N][ld],
 * J[N*N][ld] (row-major element (i, j) at J[(i*N + j)*ld + cell]), P[n].
 * lnA nullable as in chem_integrate.  For testing the pieces of a step. */
int chem_eval(chem_mech_t m, int64_t n, const double* phi, int64_t ld, const double* P,
              const double* lnA, double* f, double* J, hipStream_t stream);

/* The factorisation every attempted step makes of its stage matrix
 * (Sec. 2.3: each stage solves a system in M = I/(h gamma) - J), alone: LU
 * with partial pivoting of M = d I - A for n matrices of order N, by the
 * integrator's own routines, for testing that piece and timing it.
 *   A       [N*N][ld] device, read only: element (i, j) of matrix c at
 *           A[(i*N + j)*ld + c] (the layout of chem_eval's J); ld >= n
 *   d       the diagonal shift (1 / (h gamma) in a step)
 *   F       [N*N][ld] device, out: row k holds row k of L left of the diagonal
 *           (unit diagonal implied) and row k of U from the diagonal on, in
 *           pivot order: row k of L U is row perm[k] of M
 *   perm    [N][ld] int32 device, out: the row of M pivoted at step k
 *   status  [n] int32 device, out: 0, 1 (zero pivot) or 2 (non-finite pivot
 *           column), the first failure in column order; F and perm of a
 *           matrix that failed are unspecified
 *   launch  0: the team launches' factorisation (one wavefront per matrix
 *           for N <= 64, a work-group of four for 64 < N <= 128; the pivot is
 *           the largest |M_ik| over the rows not yet used, ties to the lowest
 *           row of M); 1: the one-cell-per-thread launches' (explicit row
 *           swaps, ties to the lowest current position, N <= 256)
 * Errors: CHEM_EINVAL (n < 0, N < 1, ld < n, launch not 0 or 1, a null
 * pointer with n > 0), CHEM_EUNSUPPORTED (N above the launch's limit),
 * CHEM_EHIP.  Runs on the current device, asynchronous on `stream`. */
int chem_lu(int64_t n, int32_t N, const double* A, int64_t ld, double d, double* F, int32_t* perm,
            int32_t* status, int32_t launch, hipStream_t stream);

/* Human-readable text of a return code. */
const char* chem_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* CHEM_H */
