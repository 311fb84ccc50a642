/*
 * acch — energy-stable Allen–Cahn/Cahn–Hilliard time stepping on one MI355X (gfx950).
 *
 * Each accepted time step solves the nonlinear system of scheme (2.20)
 * (Section 2: (U^{n+1} - U^n)/dt_n = -A~ G~^S with the truncated-series discrete
 * variational derivative G~^S of Lemma 2.2 / eq. D2-1) by the Newton–Krylov–Schwarz
 * method of Section 3.1 (inexact Newton + line search, right-preconditioned restarted
 * GMRES, restricted additive Schwarz with subdomain ILU(0)), with the adaptive time
 * step control of Section 3.2 (eq. sencondt, sqrt(2) retries, eta doubling).
 *
 * Conventions for every entry point below
 *  - Return value: ACCH_OK (0) or one of the ACCH_E* codes; no exceptions cross this
 *    boundary.  acch_strerror() names a code; acch_last_error() returns a message
 *    for the last failure on the calling thread.
 *  - "host" pointers point to CPU memory, "device" pointers to GPU memory of the
 *    device that was current at acch_create.  The library never allocates device
 *    memory: every device buffer is carved out of the caller's workspace
 *    (acch_params.workspace), which must stay alive until acch_destroy.
 *  - Fields are FP64 arrays of nx*ny (2D) cells, x fastest; a "state vector" is
 *    2*ncell doubles: the u field followed by the v field.
 *  - Work is enqueued on acch_params.stream (a hipStream_t, NULL = default stream);
 *    calls that return host values synchronise that stream.
 *  - A context is not thread safe; distinct contexts may be used concurrently.
 */
#ifndef ACCH_H
#define ACCH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ACCH_OK = 0,
  ACCH_EINVAL = 1,     /* invalid argument or parameter, workspace too small      */
  ACCH_EDOMAIN = 2,    /* a state outside the admissible set u+-v in (0,1)         */
  ACCH_EDIVERGED = 3,  /* Newton–Krylov–Schwarz failed at dt_min (or the fixed dt) */
  ACCH_EDEVICE = 4,    /* a HIP runtime error                                      */
  ACCH_EUNSUPPORTED = 5/* a configuration the library does not implement            */
};

enum { ACCH_BC_PERIODIC = 0, ACCH_BC_NEUMANN = 1 };
/* On/off switches of acch_params (ilu_reuse, mass_projection, log_energy): 0, the
 * value of a zero-filled struct, selects the documented default, which is on. */
enum { ACCH_OFF = -1, ACCH_SWITCH_DEFAULT = 0, ACCH_ON = 1 };
/* Schwarz variant (Section 3.1): left-restricted (restricted extension, the paper's
 * choice), right-restricted (restricted restriction) or classical (eq. invM). */
enum { ACCH_RAS_LEFT = 0, ACCH_RAS_RIGHT = 1, ACCH_AS_CLASSICAL = 2 };
/* Subdomain solver for inv(A_k) (Section 3.1: sparse LU or incomplete LU; the four
 * solvers of Table 2): ILU(0) on the Jacobian stencil (default), ILU(k) on the
 * level-of-fill pattern with k = acch_params.fill_level, the exact LU, or ILU(k) whose
 * level-0 pattern is the "box" pattern (every coupling of two cells at most 2 apart
 * along each axis, u and v both ways: the structure a structured-grid sparse-matrix
 * library allocates for this stencil; k = fill_level, 0 allowed, 0 is ILU(0) on it).
 * The paper does not state its ILU pattern.  All but ILU(0) on the stencil are 2D and
 * single-instance.  ILU(k), box ILU(k) with k >= 1 and LU need padded subdomain boxes
 * (owned width + 2 overlap) of at most 55 cells in x (54 with the box pattern): they
 * store the band of A_k in the natural order (half bandwidth 4 box widths, plus 5 with
 * the box pattern) and factor it without pivoting.  Box ILU(0) has kernels of its own
 * (compact records, wavefront sweeps) and takes padded boxes up to 144 x 160 cells. */
enum { ACCH_SUB_ILU0 = 0, ACCH_SUB_ILUK = 1, ACCH_SUB_LU = 2, ACCH_SUB_ILUK_BOX = 3 };
/* Precision of the subdomain ILU(0) factors and triangular solves; the residual,
 * Jacobian products, Arnoldi process, Newton update and diagnostics stay FP64. */
enum { ACCH_PREC_FP64 = 0, ACCH_PREC_MIXED = 1 };
/* Time level of the mobility c(u,v) inside A~ (Section 2 writes c^n but builds the
 * scheme by the trapezoidal rule at the half step): midpoint state (default),
 * average of the two end values, or the explicit level-n value. */
enum { ACCH_MOB_MIDPOINT = 0, ACCH_MOB_AVERAGE = 1, ACCH_MOB_EXPLICIT = 2 };

typedef struct {
  int dim;              /* 2 or 3 (3D: left-restricted Schwarz, single instances)    */
  int n[3];             /* cells per direction (x, y, z)                              */
  double L[3];          /* domain lengths; 0 means 1.0                                */
  int bc;               /* ACCH_BC_*                                                  */
  double alpha, beta, theta, gamma, rho;  /* Section 1 coefficients, all > 0         */
  int S;                /* series order of Lemma 2.2; 0 means 10 (Section 4)          */
  int adaptive;         /* 1: eq. sencondt control; 0: fixed dt_fixed                 */
  double dt_fixed, dt_min, dt_max, eta0;
  double newton_rtol, newton_atol;        /* eps_r, eps_a of Section 3.1; 0 -> 1e-8, 1e-13 */
  int newton_max_it;                      /* 0 -> 50                                  */
  double gmres_rtol, gmres_atol;          /* xi_r, xi_a; 0 -> 1e-8, 1e-14             */
  int gmres_restart;                      /* 0 -> 30 (maximum 30)                     */
  int gmres_max_restarts;                 /* 0 -> 10                                  */
  int ras_type;                           /* ACCH_RAS_LEFT / _RIGHT / ACCH_AS_CLASSICAL */
  int sub[3];                             /* subdomains per direction                 */
  int overlap;                            /* delta, cell layers                       */
  int ilu_reuse;                          /* ACCH_ON (default): factor once per step
                                             attempt; ACCH_OFF: at every Newton iteration */
  int precision;                          /* ACCH_PREC_*                              */
  int mobility_mode;                      /* ACCH_MOB_*                               */
  int xd_norm;                            /* 0: plain 2-norm of X^n - X^{n-1};
                                             1: cell-volume weighted                 */
  int mass_projection;                    /* ACCH_ON (default): remove the mean of the u
                                             part of each Newton direction; ACCH_OFF */
  int log_energy;                         /* ACCH_ON (default): energy and mass per step;
                                             ACCH_OFF: NaN in the step records        */
  double ilu_shift;                       /* sigma >= 0: the subdomain ILU(0) factors
                                             A_k + sigma diag(A_k); 0 is plain ILU(0)
                                             (also ILU(k); the exact LU ignores it)    */
  int subsolver;                          /* ACCH_SUB_* (0: ILU(0))                      */
  int fill_level;                         /* k of ACCH_SUB_ILUK (1..8) and of
                                             ACCH_SUB_ILUK_BOX (0..8)                  */
  void *workspace;                        /* device buffer, >= acch_workspace_bytes    */
  size_t workspace_bytes;
  void *stream;                           /* hipStream_t                              */
} acch_params;

typedef struct {
  double t, dt, eta, energy, mass, fnorm;
  int newton_its;       /* Newton iterations of all attempts of this step          */
  int gmres_its;        /* GMRES iterations of all attempts of this step           */
  int retries;          /* diverged attempts before acceptance                       */
  int status;           /* ACCH_OK                                                   */
} acch_step_info;

typedef struct acch_ctx acch_ctx;

/* Fill unset fields with the documented defaults (paper values of Section 4 where
 * it states them).  Host pointer; never fails on a valid pointer. */
void acch_params_default(acch_params *p);

/* Device bytes the workspace must hold for parameters p (host pointer). */
int acch_workspace_bytes(const acch_params *p, size_t *bytes);

/* Create a solver for the initial fields u0, v0 (host arrays, copied).  Validates the
 * parameters and the admissible set (ACCH_EDOMAIN), carves the workspace, builds the
 * subdomain maps of Section 3.1.  *out receives a context owned by the library. */
int acch_create(const acch_params *p, const double *u0, const double *v0, acch_ctx **out);

/* Advance nsteps accepted time steps.  info (host, may be NULL) receives one record
 * per accepted step; *accepted (may be NULL) the number accepted.  On ACCH_EDIVERGED
 * the state stays at the last accepted step. */
int acch_step(acch_ctx *c, int nsteps, acch_step_info *info, int *accepted);

/* Discrete energy E~ (eqs. relations, freeenergy, exact Phi) and mass sum(u) h^d of
 * the current state, as host doubles. */
int acch_energy(acch_ctx *c, double *energy, double *mass);

int acch_destroy(acch_ctx *c);

/* Copy the current state out to / in from host arrays of ncell doubles each.
 * set_fields checks admissibility (ACCH_EDOMAIN) and resets the step history
 * (the next adaptive step predicts as a first step) but keeps t and eta. */
int acch_get_fields(acch_ctx *c, double *u, double *v);
int acch_set_fields(acch_ctx *c, const double *u, const double *v);

/* Controller state: time, last accepted dt, eta. */
int acch_get_time(acch_ctx *c, double *t, double *dt_prev, double *eta);

/* ---- operator level entry points (one stage of the per-step solve each) ----
 * All vectors are device state vectors (2*ncell doubles) unless stated. */

/* F(X; Xn, dt) of scheme (2.20) into F.  *fnorm2 (host, may be NULL) = ||F||^2;
 * *inadmissible (host, may be NULL) = number of cells of X outside the admissible set. */
int acch_residual(acch_ctx *c, const double *X, const double *Xn, double dt, double *F,
                  double *fnorm2, int *inadmissible);

/* Analytic Jacobian dF/dX at (X; Xn, dt) (Section 3.1, J_m) into the context's
 * matrix storage: slot arrays J[slot][cell], 24 slots in 2D:
 *   u-row/u-col offsets (dx,dy): 0:(0,0) 1:(-1,0) 2:(1,0) 3:(0,-1) 4:(0,1) 5:(-2,0)
 *     6:(2,0) 7:(0,-2) 8:(0,2) 9:(-1,-1) 10:(1,-1) 11:(-1,1) 12:(1,1)
 *   u-row/v-col: 13:(0,0) 14:(-1,0) 15:(1,0) 16:(0,-1) 17:(0,1)
 *   v-row/v-col: 18:(0,0) 19:(-1,0) 20:(1,0) 21:(0,-1) 22:(0,1)
 *   v-row/u-col: 23:(0,0)
 * In 3D, 40 slots per cell (offsets (dx,dy,dz)):
 *   u-row/u-col 0:(0,0,0) 1..6: (-1,0,0) (1,0,0) (0,-1,0) (0,1,0) (0,0,-1) (0,0,1)
 *     7..12: (-2,0,0) (2,0,0) (0,-2,0) (0,2,0) (0,0,-2) (0,0,2)
 *     13..24: (-1,-1,0) (1,-1,0) (-1,1,0) (1,1,0) (-1,0,-1) (1,0,-1) (-1,0,1) (1,0,1)
 *             (0,-1,-1) (0,1,-1) (0,-1,1) (0,1,1)
 *   u-row/v-col 25..31, v-row/v-col 32..38: the cell then its 6 faces in the order above
 *   v-row/u-col 39: the cell
 * Entries whose neighbour lies outside a Neumann domain are zero. */
int acch_jacobian(acch_ctx *c, const double *X, const double *Xn, double dt);

/* y = J x with the context's Jacobian. */
int acch_apply_jacobian(acch_ctx *c, const double *x, double *y);

/* Extract the subdomain matrices A_k = R_k J R_k^T and factor them with the
 * subdomain solver of acch_params.subsolver: ILU(0) or ILU(k) of A_k + ilu_shift *
 * diag(A_k), or the exact LU of A_k. */
int acch_factor(acch_ctx *c);

/* z = M^{-1} r, the Schwarz preconditioner with the current factors. */
int acch_precondition(acch_ctx *c, const double *r, double *z);

/* Solve J S = -F by right-preconditioned restarted (flexible) GMRES from S = 0 with
 * the context's Jacobian and factors; *iterations and *resid (host, may be NULL)
 * receive the total iterations and the final residual estimate. */
int acch_gmres(acch_ctx *c, const double *F, double *S, int *iterations, double *resid);

/* One Newton solve of scheme (2.20) at the given dt from the current state, without
 * the dt controller; on success the state advances (t += dt).  info may be NULL. */
int acch_solve_step(acch_ctx *c, double dt, acch_step_info *info);

/* Copy an internal buffer to a device buffer `out` of at least *bytes bytes
 * (call with out = NULL to query *bytes):
 *   ACCH_EXPORT_JACOBIAN: J[slot][cell] FP64 (layout above);
 *   ACCH_EXPORT_FACTORS:  ILU(0) factors as FP64 [sub][slot][by][bx] over each
 *     subdomain box (box-lexicographic, x fastest), 24 slots in 2D:
 *     L of the u-row (unit diagonal): 0:u(-1,0) 1:u(-2,0) 2:u(1,-1) 3:u(0,-1)
 *       4:u(-1,-1) 5:u(0,-2) 6:v(-1,0) 7:v(0,-1);  L of the v-row: 8:v(-1,0)
 *       9:v(0,-1) 10:u(0,0);
 *     U of the u-row: 11: 1/diag, 12:u(1,0) 13:u(2,0) 14:u(-1,1) 15:u(0,1)
 *       16:u(1,1) 17:u(0,2) 18:v(0,0) 19:v(1,0) 20:v(0,1);
 *     U of the v-row: 21: 1/diag, 22:v(1,0) 23:v(0,1).
 *   ACCH_EXPORT_BOXES: int32 [sub][4] = box origin x, y (unwrapped) and box
 *     width, height (all boxes padded to the same width/height).
 *   ACCH_EXPORT_BAND: the ILU(k) / exact-LU factors as FP64 [sub][R][d], R over the
 *     2 bw bh unknowns of the padded box (cell (i, j) of the box: R = 2 (j bw + i) for
 *     u, + 1 for v), d = 0 .. 2 kl for column R + d - kl (kl = 4 bw, or 4 bw + 5 for
 *     ACCH_SUB_ILUK_BOX); L below the diagonal
 *     (unit diagonal implied), U on and above it, with 1/u_RR stored on the diagonal.
 *     Box cells outside the grid are identity rows. */
enum { ACCH_EXPORT_JACOBIAN = 0, ACCH_EXPORT_FACTORS = 1, ACCH_EXPORT_BOXES = 2, ACCH_EXPORT_BAND = 3 };
int acch_export(acch_ctx *c, int which, void *out, size_t *bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): acch_residual without a
 * context or workspace.  p describes the grid and the coefficients (dim 2; of the
 * device fields only p->stream is used, NULL = default stream); X, Xn and F are
 * device state vectors of 2*nx*ny doubles owned by the caller.  F receives F(X; Xn, dt),
 * *fnorm2 and *inadmissible (host, may be NULL) as for acch_residual.  The norm's block
 * partials and result live in a static 1 MiB device array of the library (one per
 * GPU, held until the process ends), so grids of more than 65504 tiles of 32 x 8
 * cells (about 16.7 M cells) are rejected with ACCH_EINVAL before any device work.
 * Calls that overlap on one GPU race on that array.  Synchronises p->stream. */
int acch_residual_noalloc(const acch_params *p, const double *X, const double *Xn, double dt, double *F,
                          double *fnorm2, int *inadmissible);

/* Number of cells and of subdomains, the padded box size, and the kernel-launch
 * statistics of the last acch_step call (launches, host synchronisations). */
int acch_info(acch_ctx *c, long *ncell, int *nsub, int *box_w, int *box_h);

/* Kernel classes of the per-step solve, for acch_kernel_stats. */
enum {
  ACCH_KERNEL_RESIDUAL = 0, ACCH_KERNEL_JACOBIAN = 1, ACCH_KERNEL_FACTOR = 2, ACCH_KERNEL_RAS = 3,
  ACCH_KERNEL_SPMV_DOTS = 4, ACCH_KERNEL_ORTH = 5, ACCH_KERNEL_GMRES_START = 6, ACCH_KERNEL_GMRES_UPDATE = 7,
  ACCH_KERNEL_ENERGY = 8, ACCH_KERNEL_SPMV = 9, ACCH_KERNEL_OTHER = 10, ACCH_KERNEL_KINDS = 11
};

/* Enable (1) or disable (0) per-kernel timing: HIP events recorded on the context's
 * stream around every launch, accumulated per kernel class.  2: sampled timing of the
 * Schwarz preconditioner only (events around one ACCH_KERNEL_RAS launch in 16, none
 * elsewhere), for timing a run without the events' own cost on every launch.  Resets
 * the totals and the launch / synchronisation counters.  Synchronises the stream. */
int acch_timing(acch_ctx *c, int enable);

/* Accumulated device time (ms, host double) and launch count of one kernel class
 * since the last acch_timing call. */
int acch_kernel_stats(acch_ctx *c, int kind, double *total_ms, long *count);

/* Tuning options (process-wide): ACCH_OPT_RAS_PREFETCH = wavefronts of factors the
 * 2D triangular-solve kernel loads ahead of their use (3, 4, 5 or 6; default 5);
 * ACCH_OPT_RAS3D_WINDOW = 1 (default) lets the 3D preconditioner keep the recent
 * levels of a box in LDS when the box allows it, 0 forces the variant that keeps
 * the whole box in device memory (same arithmetic).  c may be NULL. */
enum { ACCH_OPT_RAS_PREFETCH = 0, ACCH_OPT_RAS3D_WINDOW = 1 };
int acch_set_option(acch_ctx *c, int option, long value);

/* Kernel launches and host synchronisations since the last acch_timing call. */
int acch_counters(acch_ctx *c, long *launches, long *syncs);

/* ---- Discrete adjoint of the time-step map ----------------------------------
 * A step solves F(X1; X0, dt) = 0 (scheme (2.20), Section 3.1).  With the step sizes
 * held fixed, reverse differentiation of a loss L through the steps needs, per step,
 *   J^T lambda = dL/dX1 (J = dF/dX1, the Newton Jacobian at the converged X1),
 *   dL/dX0 = -(dF/dX0)^T lambda,   dL/dp -= lambda . dF/dp,
 * for p = (alpha, beta, theta, gamma).  Vectors are device arrays of 2*ncell
 * doubles (u then v), owned by the caller.  These calls reuse the context's
 * Jacobian, factor and Krylov storage (its state, time and step history are left
 * alone); the next acch_step refactors as usual. */

/* y = J^T x with the context's Jacobian. */
int acch_apply_jacobian_transpose(acch_ctx *c, const double *x, double *y);

/* z = M^{-T} r: the exact transpose of the Schwarz preconditioner with the current
 * factors, sum_k (R_k^delta)^T (L_k U_k)^{-T} R_k^0 r (left-restricted; the other
 * variants likewise).  Needs overlap <= the smallest subdomain width and an ILU(0)
 * subdomain solver, on the stencil or the box pattern (ACCH_EUNSUPPORTED otherwise). */
int acch_precondition_transpose(acch_ctx *c, const double *r, double *z);

/* Gradient of the discrete energy E~ (eqs. relations, freeenergy) at the device
 * state X (NULL: the context's current state): g receives dE~/dX, dparams (host,
 * 4 doubles) receives dE~/d(alpha, beta, theta, gamma). */
int acch_energy_gradient(acch_ctx *c, const double *X, double *g, double *dparams);

/* One step back: assemble J at (X1; X0, dt), factor, solve J^T lambda = g by GMRES
 * preconditioned with M^{-T} (the context's tolerances and restart limits; no mass
 * projection), then g_prev = -(dF/dX0)^T lambda and dparams[k] -= lambda . dF/dp_k
 * (host, 4 doubles, accumulated).  g_prev may be g.  gmres_its / resid (host, may
 * be NULL) receive the GMRES iterations and final residual estimate.  Returns
 * ACCH_EDIVERGED if GMRES does not converge. */
int acch_adjoint_step(acch_ctx *c, const double *X1, const double *X0, double dt, const double *g, double *g_prev,
                      double *dparams, int *gmres_its, double *resid);

/* ---- Batches of independent instances ----------------------------------------
 * count instances, each described by its own acch_params (grid, boundary,
 * parameters, subdomains), advanced together at the common fixed dt of instance 0
 * (adaptive must be 0; overlap, precision, dt_fixed and the subdomain solver must
 * agree; the left-restricted variant with ILU(0) on the stencil pattern or on the box
 * pattern, ACCH_SUB_ILUK_BOX with fill_level 0, else ACCH_EUNSUPPORTED).  Every kernel of
 * a Newton-Krylov-Schwarz stage runs once for all instances: all subdomain
 * factorisations and triangular solves of all instances in one launch each; Newton
 * iterations, line searches and GMRES cycles run in lockstep with per-instance
 * masks, so every instance follows the operation sequence of its own
 * single-instance run.  The Arnoldi steps of a GMRES cycle are recorded once into
 * HIP graphs and replayed (ACCH_BATCH_OPT_GRAPH, default on, recorded at the first
 * step or when the option is switched on; the stream of instance 0 must then be a
 * created stream, not the null stream).  Instance 0 also
 * supplies the tolerances, restart limits, ilu_shift, mass projection, workspace
 * (acch_batch_workspace_bytes) and stream. */
typedef struct acch_batch acch_batch;
enum { ACCH_BATCH_OPT_GRAPH = 0 };

int acch_batch_workspace_bytes(const acch_params *inst, int count, size_t *bytes);

/* u0[i], v0[i]: host arrays of instance i's ncell doubles (x fastest), copied. */
int acch_batch_create(const acch_params *inst, int count, const double *const *u0, const double *const *v0,
                      acch_batch **out);

/* nsteps fixed-dt steps of every instance; newton_its / gmres_its (host arrays of
 * count ints, may be NULL) are incremented per instance.  If any instance fails
 * the call returns ACCH_EDIVERGED and no instance advances in that step. */
int acch_batch_step(acch_batch *b, int nsteps, int *newton_its, int *gmres_its);

/* Discrete energy and mass of every instance (host arrays of count doubles). */
int acch_batch_energy(acch_batch *b, double *energy, double *mass);

/* Copy instance i's state to host arrays of its ncell doubles each. */
int acch_batch_get_fields(acch_batch *b, int i, double *u, double *v);

/* z = M^{-1} r for every instance at once (one launch over all subdomains) with the
 * factors of the last step's first Newton iteration; r, z are batched device
 * vectors (instance i's u then v at element offset xoff[i], see acch_batch_info).
 * Asynchronous on the batch stream. */
int acch_batch_precondition(acch_batch *b, const double *r, double *z);

/* Total cells, subdomains, padded box size and the element offset of each instance
 * in batched vectors (xoff: host array of count longs, may be NULL). */
int acch_batch_info(acch_batch *b, long *ncell, int *nsub, int *box_w, int *box_h, long *xoff);

int acch_batch_set_option(acch_batch *b, int option, long value);

/* Kernel launches, graph launches and host synchronisations so far. */
int acch_batch_counters(acch_batch *b, long *launches, long *graph_launches, long *syncs);

int acch_batch_destroy(acch_batch *b);

const char *acch_strerror(int code);
const char *acch_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ACCH_H */
