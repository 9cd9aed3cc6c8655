/*
 * eclqr.h -- C ABI of the MI355X (gfx950) solver for linear
 * equality-constrained LQR problems.
 *
 * Problem (paper: Section II, eq. (problem)), with the mixed rows and the
 * state-only rows of a stage merged into one block:
 *
 *   min  sum_{i<N} 1/2 x_i'Q_i x_i + x_i'M_i u_i + 1/2 u_i'R_i u_i + q_i'x_i + r_i'u_i
 *        + 1/2 x_N'Q_N x_N + q_N'x_N
 *   s.t. x_0 = x0,
 *        x_{i+1} = A_i x_i + B_i u_i + c_i               (i < N)
 *        E_i x_i + F_i u_i + g_i = 0   (k_i rows)         (i < N)
 *        E_N x_N + g_N = 0             (k_N rows, terminal)
 *
 * Dimensions may vary by stage (x_i in R^{n_i}, u_i in R^{m_i}); rows may be
 * dependent or absent.  The solve follows Algorithm 1: the feasible-domain
 * suffix scan over affine endpoint relations (Sections III-IV), the
 * stage-parallel elimination (Section V), an associative-scan Riccati solve of
 * the reduced LQR (Section VI), primal recovery (eq. (recovery-maps)) and the
 * multipliers of Section VII (by default the minimum-norm solution of the
 * stationarity equations; optionally the factor-reusing route).
 *
 * Conventions
 * - All floating-point data are FP64.  Integers are int32 unless stated.
 * - Matrices are row-major and dense.  Each field is one flat array: the
 *   blocks of all stages of instance 0 in stage order, then instance 1, ...
 *   The per-stage element offsets come from eclqr_plan_layout().
 * - Q, q, E, g have N+1 blocks per instance (the last is the terminal block:
 *   Q_N, q_N, E_N, g_N); R, r, M, A, B, c, F have N blocks; x0 has one.
 * - Outputs: x has the layout of q (N+1 blocks), u the layout of r, lam the
 *   layout of q (lam_0 .. lam_N, lam_{i+1} multiplies the dynamics of stage i
 *   and lam_0 = -alpha, alpha the multiplier of x_0 = x0), mu the layout of g
 *   (mu_i multiplies the rows of stage i, mu_N the terminal rows).  The
 *   Lagrangian sign is f + nu'c(w) (Section VII).
 * - Pointers named "device" must be device memory of the current HIP device;
 *   "host" pointers are host memory.  The caller owns every buffer it passes.
 * - `stream` is a hipStream_t (NULL = the default stream).  Solve and backward
 *   only enqueue work; nothing synchronises except where stated.
 * - Synchronous errors are returned as eclqr_status; a text description of
 *   the last error of the calling thread is given by eclqr_last_error().
 *   Numerical outcomes are written per instance to the device array status[]
 *   (bit set, 0 = OK).  Outputs of an instance whose status is not OK are NaN.
 */
#ifndef ECLQR_H
#define ECLQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ECLQR_ABI_VERSION 3

/* synchronous return codes */
typedef enum {
  ECLQR_SUCCESS = 0,
  ECLQR_INVALID_ARGUMENT = 1,   /* bad dims, NULL pointer, misaligned buffer */
  ECLQR_WORKSPACE_TOO_SMALL = 2,
  ECLQR_HIP_ERROR = 3,          /* a HIP runtime call failed */
  ECLQR_UNSUPPORTED = 4,        /* dims beyond what the kernels handle */
  ECLQR_NO_DEVICE = 5
} eclqr_status;

/* per-instance outcome bits written to status[b] (device int32) */
#define ECLQR_OK 0
#define ECLQR_INFEASIBLE_SUFFIX 1   /* some suffix relation reads 0 = gamma (Algorithm 1) */
#define ECLQR_INFEASIBLE_INITIAL 2  /* x0 outside X_0 (eq. (initial-feasibility)) */
#define ECLQR_RANK_INCONSISTENT 4   /* nonzero residual after Lemma 2 (rank decisions) */
#define ECLQR_NOT_CONVEX 8          /* the costs are not positive definite on the feasible set: the scan
                                       route's reduced input Hessians are not, and the sequential
                                       fallback (which solves every instance whose minimiser is unique)
                                       found no unique minimiser either; ECLQR_NO_MINIMIZER when it shows
                                       that none exists, neither bit added when it cannot decide (a
                                       singular stage Hessian whose null space meets the state feedback) */
#define ECLQR_INVALID_INPUT 16      /* NaN or Inf in the data */
#define ECLQR_CAPACITY 32           /* a relation outgrew its on-chip tile */
#define ECLQR_DUAL_FAILED 64        /* the multiplier (stationarity) solve failed; its own
                                       outcome bits are repeated in bits 8..15 */
#define ECLQR_TIMEOUT (1 << 16)      /* a bounded wait of a persistent scan kernel expired (2 s of wall
                                       clock): the outputs are not valid */
#define ECLQR_NO_MINIMIZER (1 << 17)  /* with ECLQR_NOT_CONVEX: the problem has no minimiser (the cost falls
                                        without bound on the feasible set; Section II, the paragraph after
                                        eq. (convexity)) */
#define ECLQR_NOT_UNIQUE (1 << 18)    /* informational, outputs valid: the costs are not positive definite on the
                                        feasible set; a minimiser exists but is not unique and the one
                                        returned has no component along the flat input directions.  Test
                                        (status & ~ECLQR_NOT_UNIQUE) == 0 for usable outputs */
#define ECLQR_NOT_DIFFERENTIABLE 128 /* eclqr_backward only: the instance's constraint rows are
                                       dependent (LICQ fails: a redundant row, or rows that together
                                       with x_0 = x0 restrict x_0), so its multipliers are not unique
                                       (Section VII, the remark after the multiplier proposition) and
                                       the solution is not differentiable in the data; its gradients
                                       are NaN */

/* fields of the problem layout */
enum {
  ECLQR_F_Q = 0, ECLQR_F_q, ECLQR_F_R, ECLQR_F_r, ECLQR_F_M, ECLQR_F_A, ECLQR_F_B,
  ECLQR_F_c, ECLQR_F_E, ECLQR_F_F, ECLQR_F_g, ECLQR_F_x0, ECLQR_NUM_FIELDS
};

typedef struct eclqr_plan eclqr_plan;

/* Problem dimensions (host arrays, copied by eclqr_plan_create).
 *   horizon[b] = N_b >= 1                     (batch entries)
 *   nx: sum_b (N_b+1) state dims, instance-major (n_0 may be 0)
 *   nu: sum_b N_b input dims
 *   nc: sum_b (N_b+1) row counts, the last of each instance = terminal rows */
typedef struct {
  int32_t batch;
  const int32_t* horizon;
  const int32_t* nx;
  const int32_t* nu;
  const int32_t* nc;
} eclqr_dims;

/* Options (Section VIII numerical policy).  Fill with eclqr_default_options. */
typedef struct {
  double rank_tol;        /* pivot counts toward rank if > rank_tol*max(1,|largest pivot|); 1e-10 */
  double cons_tol;        /* 0 = gamma accepted if |gamma| <= cons_tol*max(1,|offsets|); 1e-8 */
  double dual_cons_tol;   /* same test inside the multiplier solve; 1e-6 */
  double refine_tol;      /* an instance stops refining once ||correction|| <= refine_tol*||(x,u)||; 1e-8 */
  double accept_tol;      /* an instance whose KKT backward error (see eclqr_plan_backward_error) after the
                           * first solve is <= accept_tol takes no refinement step; 1e-10 (0: always refine).
                           * Measured on every workload, the first pass's relative error against the exact
                           * solution is at most about 0.7 times this backward error */
  int32_t multipliers;    /* 0: primal only; 1: lam and mu as the minimum-norm solution of the stationarity
                           * equations of Section VII (computed as the tuning field multiplier_route selects:
                           * by default the theta LQR over the normal coordinates of the feasible domains,
                           * else the reversed-time problem); 2: factor-reusing route (Section VIII, subsection
                           * "Reference implementation"): one representative from the primal pass's domains
                           * and scans -- equal to route 1 where the multipliers are unique (LICQ), otherwise a
                           * valid multiplier vector that need not have minimum norm; 3: the contraction-expansion
                           * route of Section VII: the dual base relations (eq. (dual-base-system)) composed by a
                           * balanced up-sweep, the minimum-norm lambda_0 of the root relation, the tree expanded
                           * from the root with each shared costate the minimum-norm solution of its two operand
                           * relations (eq. (middle-dual-map) with rho_j = 0), then the minimum-norm mu_i of each
                           * stage's stationarity rows; computed at the refined primal point (the refinement
                           * itself uses route 1).  Equal to route 1 under LICQ, otherwise another valid
                           * representative. 1 */
  int32_t refine;         /* most steps of iterative refinement per instance (0..4); 2 (no instance of the
                           * benchmark workloads takes more; every step is one vector-only pass whose
                           * launches run even when no instance refines).  A refined instance whose final
                           * KKT backward error exceeds dual_cons_tol reports ECLQR_DUAL_FAILED */
  int32_t use_graph;      /* 1: capture the launch sequence of eclqr_solve once per set of pointers and
                           * replay it as a hipGraph; 0 */
  int32_t scan_schedule;  /* parenthesization of the associative scans (Proposition 1 allows any): 1 balanced
                           * up/down sweep (about 2 L tasks in 2 log2 L levels per instance of L = N + 1
                           * leaves); 2 recursive doubling (about L log2 L tasks in log2 L levels); 0 (default)
                           * hybrid: the fewest balanced up-sweep levels after which the batch has at most 2048
                           * interval nodes (512 when a state dim exceeds 16), doubling over those nodes, then
                           * the balanced down-sweep (pure doubling for up to 2048 leaves) */
  int32_t reversed_time;  /* with multipliers = 1: 1 also lays out the reversed-time stationarity problem in the
                           * workspace, so the tuning field multiplier_route can select it; 0 (default) only when
                           * the theta route is unavailable (a stage with k_i + n_{i+1} > 64) */
  int32_t domain_shortcut; /* 1 (default): an instance with no terminal rows whose every F_i has full row rank
                           * (Section VI: every domain is the whole space) skips the relation scan; 0: every
                           * instance runs it.  Both give the same solution */
  int32_t reserved[2];
} eclqr_options;

/* Device pointers to the problem data (layout from eclqr_plan_layout).  M may
 * be NULL (zero cross terms). */
typedef struct {
  const double *Q, *q, *R, *r, *M, *A, *B, *c, *E, *F, *g, *x0;
} eclqr_problem;

/* Device output buffers.  lam and mu may be NULL when multipliers = 0.
 * info (may be NULL) receives, per instance, the stage of its failure: the
 * largest stage index at which a kernel of the problem's own pass (the
 * relation scan, the state parameterization, the stage elimination, the
 * feedback gains) set an outcome bit.  Algorithm 1 runs from the terminal
 * stage backwards, so this is the first failing stage in its order: for
 * ECLQR_INFEASIBLE_SUFFIX the largest i whose suffix set is empty, 0 for
 * ECLQR_INFEASIBLE_INITIAL.  -1 when the problem's pass flagged nothing
 * (status OK, or only the multiplier solve failed). */
typedef struct {
  double *x, *u, *lam, *mu;
  int32_t* status;   /* [batch] */
  int32_t* info;     /* [batch] or NULL */
} eclqr_solution;

/* Device buffers for the backward pass: dL/dx, dL/du (layouts of q, r) and,
 * optionally (NULL = zero), dL/dlam (layout of q) and dL/dmu (layout of g). */
typedef struct {
  const double *dx, *du, *dlam, *dmu;
} eclqr_cotangent;

/* Device gradient buffers, same layouts as the problem fields (M may be
 * NULL).  status (may be NULL) receives per instance the forward outcome
 * bits, ECLQR_NOT_DIFFERENTIABLE, and ECLQR_DUAL_FAILED (with the adjoint
 * solve's bits in 8..15) when the adjoint solve failed; the gradients of an
 * instance with any bit set are NaN. */
typedef struct {
  double *Q, *q, *R, *r, *M, *A, *B, *c, *E, *F, *g, *x0;
  int32_t* status;   /* [batch] or NULL */
} eclqr_grads;

int eclqr_abi_version(void);
void eclqr_default_options(eclqr_options* opt);
const char* eclqr_status_string(int32_t status);
const char* eclqr_last_error(void);

/* Builds the host-side plan: layout, workspace map and the associative-scan
 * schedules (balanced up-sweep / down-sweep, Section IV "Suffix scan").  Does
 * not touch the GPU.  Errors: INVALID_ARGUMENT for N_b < 1, negative dims,
 * UNSUPPORTED for a dimension above 64.  *out is NULL on error. */
eclqr_status eclqr_plan_create(eclqr_plan** out, const eclqr_dims* dims, const eclqr_options* opt);
void eclqr_plan_destroy(eclqr_plan* plan);

/* Per-stage element offsets of one field.  *offsets points to plan-owned host
 * memory valid until eclqr_plan_destroy; *count entries (stages or instances
 * for x0); *total = elements of the flat array. */
eclqr_status eclqr_plan_layout(const eclqr_plan* plan, int32_t field, const int64_t** offsets,
                               int64_t* count, int64_t* total);

/* Bytes of device workspace one solve (and one backward) needs; the caller
 * allocates it with 256-byte alignment. */
eclqr_status eclqr_plan_workspace_size(const eclqr_plan* plan, size_t* bytes);

/* Forward solve (Algorithm 1 + Section VII).  Enqueued on `stream`; the first
 * call with a given workspace uploads the plan's tables into it (one H2D copy).
 * The workspace keeps the factorizations of this solve: refinement steps and
 * eclqr_backward replay them on new vectors, so keep it between the two. */
eclqr_status eclqr_solve(eclqr_plan* plan, const eclqr_problem* prob, eclqr_solution* sol, void* ws,
                         size_t ws_bytes, void* stream);

/* eclqr_solve for callers that cannot allocate device memory (code under
 * stream capture, serving loops that forbid allocation): the same solve, with
 * the workspace in a static device array of the library (64 MiB, one per GPU,
 * held until the process ends) instead of a caller buffer.  The caller still
 * passes the problem and the solution buffers.  Calls no allocating routine:
 * no hipMalloc/hipFree, no stream, event or graph creation (launches are
 * eager on `stream`; the plan's overlapped second stream is used only if an
 * earlier eclqr_solve of the plan created it).  Errors:
 * ECLQR_WORKSPACE_TOO_SMALL when eclqr_plan_workspace_size exceeds 64 MiB,
 * the other errors of eclqr_solve.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (the solve initialises what it
 * reads): calls that overlap on one GPU (two host threads, or unsynchronised
 * streams) race and give undefined results.  eclqr_backward cannot follow a
 * call of this entry point. */
eclqr_status eclqr_solve_noalloc(eclqr_plan* plan, const eclqr_problem* prob, eclqr_solution* sol, void* stream);

/* Gradients of a loss L(x, u, lam, mu) with respect to every problem field
 * (implicit differentiation of the KKT system; the adjoint is the same
 * constrained LQR with linear costs dL/dx, dL/du and the offsets
 * c_i <- dL/dlam_{i+1}, g_i <- dL/dmu_i, x0 <- dL/dlam_0).  Requires the
 * forward solve's outputs (x, u, lam, mu) and its workspace: the last solve
 * made in ws must be the one of this problem and solution (same pointers),
 * with the plan's current multiplier route, else ECLQR_INVALID_ARGUMENT.  The
 * adjoint replays the factorizations that solve left there (no factorization
 * is recomputed).  Gradients exist where the multipliers are unique (LICQ);
 * instances where the rank decisions of the forward pass show dependent rows
 * get ECLQR_NOT_DIFFERENTIABLE and NaN gradients. */
eclqr_status eclqr_backward(eclqr_plan* plan, const eclqr_problem* prob, const eclqr_solution* sol,
                            const eclqr_cotangent* ct, eclqr_grads* grads, void* ws, size_t ws_bytes,
                            void* stream);

/* KKT residual of Section IX per instance: out[4*b + j], j = 0 initial,
 * 1 dynamics, 2 equalities (rows normalised by max(1, |coefficients|, |offset|)),
 * 3 stationarity; infinity norms.  out is device memory [4*batch]. */
eclqr_status eclqr_kkt_residual(eclqr_plan* plan, const eclqr_problem* prob, const eclqr_solution* sol,
                                double* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Interior-point driver for bound-constrained problems.  Section I motivates
 * the method by interior-point and SQP solvers, which solve a sequence of
 * equality-constrained LQR problems of fixed structure whose cost weights
 * change; this driver is that use, on the GPU: the problem above plus bounds
 *   lo <= u_i <= hi (i < N),   lo <= x_i <= hi (1 <= i <= N),
 * solved by Mehrotra's predictor-corrector primal-dual method (SIAM J. Optim.
 * 2(4), 1992).  With bound multipliers z_lo, z_hi >= 0, distances
 * d_lo = v - lo, d_hi = hi - v and complementarity targets t_lo, t_hi, each
 * linear system of the method is the equality-constrained LQR problem with
 *   Q_i + diag(z_lo/d_lo + z_hi/d_hi),  R_i likewise,
 *   q_i = grad_x f - t_lo/d_lo + t_hi/d_hi,  r_i likewise,
 *   c_i = A_i x_i + B_i u_i + c_i - x_{i+1},  g_i = E_i x_i + F_i u_i + g_i,
 *   x0 = x0 - x_0
 * at the current iterate (M, A, B, E, F unchanged); its solution is the step
 * and its multipliers the new equality multipliers.  Per iteration and
 * instance, with mu the mean complementarity product: the predictor (targets
 * 0) is a full solve; sigma = min(1, (mu_aff/mu)^3) from the complementarity
 * after its largest feasible step; the corrector (targets sigma mu minus the
 * predictor's second-order term) has the same matrices and replays the
 * predictor's factorizations; the step is the largest <= 1 that keeps the
 * iterate strictly inside the bounds and z positive (fraction tau to the
 * boundary).  An instance stops once its mu is below mu_stop.  The start
 * point is the equality-constrained solution moved inside the bounds.
 * --------------------------------------------------------------------------- */

/* Device bound arrays (NULL = no bound on that side; an infinite entry is an
 * absent bound).  u_lo, u_hi: layout of r; x_lo, x_hi: layout of q (the block
 * of x_0 is ignored: x_0 = x0 is fixed).  Where both sides are finite lo < hi
 * is required (a fixed variable belongs in the equality rows); an instance
 * with lo >= hi or a NaN bound gets ECLQR_INVALID_INPUT. */
typedef struct {
  const double *u_lo, *u_hi, *x_lo, *x_hi;
} eclqr_bounds;

/* Method parameters (eclqr_ipm_default_params: 30, 1e-8, 0.995, 100, 0.25, 1, 2). */
typedef struct {
  int32_t iterations; /* predictor-corrector iterations at most (every instance is solved in each; >= 0) */
  double mu_stop;     /* an instance stops once its mean complementarity is below this (the Newton
                       * matrices' diagonal grows like z^2 / mu: much below 1e-8 their factorizations lose
                       * the accuracy the refinement needs) */
  double tau;         /* fraction to the boundary, in (0, 1) */
  double mu0;         /* initial z = mu0 / (distance to the bound), > 0 */
  double interior;    /* start point: at least this fraction of a two-sided gap (one-sided: of
                       * max(1, |bound|)) inside each finite bound, in (0, 0.5) */
  int32_t corrector_replay; /* 1: the corrector replays the predictor's factorizations (its matrices are
                             * the same); 0: the corrector is a full solve */
  int32_t newton_refine;    /* refinement steps of each Newton solve (0..4; the plan's refine applies to the
                             * start solve only).  Fewer steps are faster, but near the solution the Newton
                             * matrices are ill-conditioned and the multipliers of an unrefined pass leave
                             * stationarity residuals of about 1e-5 on the test instances; 2 */
} eclqr_ipm_params;

/* Device outputs: the last iterate of each instance. */
typedef struct {
  double *x, *u, *lam, *mu;   /* layouts of q, r, q, g (lam, mu: equality multipliers, as eclqr_solution) */
  double *z_ulo, *z_uhi;      /* bound multipliers of the inputs, layout of r */
  double *z_xlo, *z_xhi;      /* bound multipliers of the states, layout of q (zero on the block of x_0) */
  double* comp;               /* [batch] mean complementarity at the returned iterate, or NULL */
  int32_t* steps;             /* [batch] iterations the instance took, or NULL */
  int32_t* status;            /* [batch]: the start solve's outcome bits, ECLQR_INVALID_INPUT for bad bounds,
                               * or the bits of the first predictor or corrector solve that failed (the
                               * instance stops there and keeps its last iterate).  A Newton solve whose
                               * refinement stops above dual_cons_tol is not a failure: its inexact step is
                               * taken */
} eclqr_ipm_solution;

void eclqr_ipm_default_params(eclqr_ipm_params* prm);

/* Bytes of device workspace eclqr_ipm_solve needs (the plan's solve
 * workspace plus the Newton problem's data, the predictor's and corrector's
 * solutions and the driver's per-instance state); 256-byte aligned by the
 * caller. */
eclqr_status eclqr_ipm_workspace_size(const eclqr_plan* plan, size_t* bytes);

/* Runs the start solve and up to prm->iterations predictor-corrector
 * iterations, all enqueued on `stream` (no synchronisation; every iteration
 * solves the whole batch, the stopped instances' results unused).  The
 * Newton problems live at fixed addresses in ws, so with use_graph one
 * iteration is captured once (per set of pointers and parameters) and
 * replayed.  Requires a plan with multipliers 1, 2 or 3 (the Newton
 * multipliers are the equality multipliers' update; with 3 the corrector's
 * multipliers come from the minimum-norm route, equal where they are
 * unique).  Errors: INVALID_ARGUMENT for NULL pointers, a plan without
 * multipliers or bad parameters, WORKSPACE_TOO_SMALL, and the errors of
 * eclqr_solve.  After this call ws holds Newton factorizations, not a solve
 * of prob: eclqr_backward cannot follow it. */
eclqr_status eclqr_ipm_solve(eclqr_plan* plan, const eclqr_problem* prob, const eclqr_bounds* bounds,
                             const eclqr_ipm_params* prm, eclqr_ipm_solution* sol, void* ws, size_t ws_bytes,
                             void* stream);

/* Kernel classes timed by the optional profiler. */
enum {
  ECLQR_K_VALIDATE = 0, ECLQR_K_BASE_RELATION, ECLQR_K_REL_COMPOSE, ECLQR_K_DOMAIN, ECLQR_K_ELIMINATE,
  ECLQR_K_RIC_COMBINE, ECLQR_K_GAINS, ECLQR_K_FWD_COMBINE, ECLQR_K_RECOVER, ECLQR_K_MULTIPLIER_IO,
  ECLQR_K_REFINE_IO, ECLQR_K_OTHER,
  ECLQR_K_REPLAY, /* every kernel of a vector-only pass (recovery included) */
  ECLQR_K_MULT_FAST, /* the factor-reusing multiplier route (multipliers = 2) */
  ECLQR_K_MULT_THETA, /* local systems, initial state and read-out of the theta-LQR minimum-norm route */
  ECLQR_K_MULT_CX,    /* the contraction-expansion multiplier route (multipliers = 3) */
  ECLQR_K_IPM,        /* the interior-point driver's own kernels (Newton data, step, complementarity) */
  ECLQR_NUM_KERNEL_CLASSES
};

/* Profiler: when on, every later solve/backward records a HIP event pair
 * around each launch of every kernel class on the launch stream.
 * eclqr_plan_profile synchronises the recorded events and returns, per class,
 * the summed milliseconds and the number of launches (arrays of
 * ECLQR_NUM_KERNEL_CLASSES, host memory), then clears them if reset != 0. */
eclqr_status eclqr_plan_set_profiling(eclqr_plan* plan, int32_t on);

/* Launch configuration of a plan. */
typedef struct {
  int32_t use_graph;      /* replay the solve as a captured hipGraph */
  int32_t level_buckets;  /* relation-scan levels with >= 2048 tasks launch in LDS-size buckets */
  int32_t pool_in_lds;    /* value-function combines: 0 work pool in global scratch, 1 pool in LDS, 2 operands,
                             result and pool in LDS, 3 (default) the operands read more than once staged in LDS
                             with a compact pool, the result written once to global memory (the same bits in
                             every mode); a mode whose LDS does not fit falls back to the next lower one */
  int32_t grid_divisor;   /* grid of the stage-parallel kernels = its maximum / grid_divisor (1..64) */
  double ms_per_solve;    /* time of the configuration chosen by eclqr_plan_autotune (0 if never tuned) */
  int32_t register_compose; /* relation compositions that fit (<= 64 stacked rows, <= 128 columns) keep the
                             * stacked system in registers instead of LDS */
  int32_t stage_lds;      /* stage eliminations and feedback gains keep their working arrays in LDS when these
                             need at most 20 KiB (eliminations) or 32 KiB (gains) per workgroup (1, default), only
                             the feedback gains do (2), or neither (0: global scratch) */
  int32_t overlap_dual;   /* with the minimum-norm multipliers, 1: the multiplier route's problem is factored
                           * (matrix data only) on a second stream while the primal pass runs, and its vector-only
                           * replay at the primal solution gives the multipliers; 0: one stream, full pass after
                           * the primal pass.  Route 0 forks at the start of the solve (the reversed-time problem
                           * needs no primal data), route 1 once the primal pass has the domains.  Default 0 on
                           * plans whose default route is 1 (it pays only on large batches), else 1 */
  int32_t multiplier_route; /* how the minimum-norm multipliers (multipliers = 1) are computed: 1 (default where
                           * the stage input capacity k_i + n_{i+1} <= 64): from the primal pass's domains and
                           * scans, as an unconstrained LQR over the normal coordinates theta_i of the domains
                           * (minimum-norm local systems, value-function scan, gains, forward scan); 0: the
                           * reversed-time stationarity problem solved by the full engine.  Both give the
                           * minimum-norm multipliers; they differ in rounding.  Route 0 needs a plan made with
                           * the option reversed_time = 1 (else the field stays 1).  eclqr_backward needs the
                           * workspace of a solve made with the same route. */
  int32_t split_combine;  /* value-function combines of a level whose tasks all fit the device at once run on two
                           * wavefronts (J, eta, A, b on one, the C update on the other; same bits) (1, default) or
                           * one (0) */
  int32_t fused_scans;    /* 1: the vector-only replays (refinement steps, the multipliers at the refined point, the
                           * adjoint) run each scan as one persistent launch over all its levels: the grid is
                           * bounded by the co-resident workgroups the runtime reports, tasks are taken in level
                           * order from a counter and wait, boundedly (2 s, then ECLQR_TIMEOUT), for the levels
                           * before theirs.  0 (default): one launch per level.  Experimental: on the device the
                           * persistent form did not complete its waits (see the design notes); the autotuner does
                           * not select it */
  int32_t refine_gate;    /* 1: eclqr_solve reads back, after the first pass, how many instances still need a
                           * refinement step (their backward error above accept_tol) and enqueues the refinement
                           * steps only if some does; the calling thread then waits for that first pass.  A
                           * solve enqueued on a stream under capture, eclqr_solve_noalloc and the interior-point
                           * driver never wait (they run as with 0).  0 (default): every step is enqueued and its
                           * launches return at once for instances that are done; eclqr_solve never waits.  Same
                           * results either way */
} eclqr_tuning;

/* Time the caller's problem under alternative launch configurations
 * (coordinate search over the fields of eclqr_tuning, 1 warm-up + 3 timed
 * solves each, an alternative kept only if 2% faster) and keep the fastest in
 * the plan.  Synchronous: enqueues solves on `stream` and waits for them.  The
 * solution buffers hold the last solve's result on return. */
eclqr_status eclqr_plan_autotune(eclqr_plan* plan, const eclqr_problem* prob, eclqr_solution* sol, void* ws,
                                 size_t ws_bytes, void* stream, eclqr_tuning* out);
eclqr_status eclqr_plan_get_tuning(const eclqr_plan* plan, eclqr_tuning* out);
eclqr_status eclqr_plan_set_tuning(eclqr_plan* plan, const eclqr_tuning* t);

/* Turn the captured-graph path of eclqr_solve on or off (the use_graph
 * option).  With it on, the first solve with a given set of pointers (problem,
 * solution, workspace) captures its launch sequence into a hipGraph on the
 * stream and launches it; later solves with the same pointers launch the graph
 * (new values in the same buffers are picked up).  Different pointers
 * re-capture.  Profiling bypasses the graph. */
eclqr_status eclqr_plan_set_graph(eclqr_plan* plan, int32_t on);
eclqr_status eclqr_plan_profile(eclqr_plan* plan, double* ms, int64_t* launches, int32_t reset);
const char* eclqr_kernel_class_name(int32_t k);

/* Reduced dimensions n-bar_i, m-bar_i (Section V) computed by the last solve
 * in workspace ws, copied to host arrays of length sum_b (N_b + 1) (m-bar of a
 * terminal stage is 0).  which = 0: the problem; 1: the reversed-time
 * stationarity problem of the multipliers; 2: the theta LQR of the
 * minimum-norm route (normal dims r_i, free dims of the local systems; plans
 * without it return ECLQR_INVALID_ARGUMENT).  Synchronises the device. */
eclqr_status eclqr_plan_reduced_dims(const eclqr_plan* plan, const void* ws, int32_t which, int32_t* nbar,
                                     int32_t* mbar);

/* Refinement steps each instance took in the last solve in ws (host array of
 * batch entries).  Synchronises the device. */
eclqr_status eclqr_plan_refine_steps(const eclqr_plan* plan, const void* ws, int32_t* steps);

/* KKT backward error of each instance at the point returned by the last
 * eclqr_solve (or eclqr_backward, for the adjoint) in ws: the max over rows
 * of |residual| / sum |terms| (componentwise), except on rows where that sum
 * is below 1000 * (terms) * eps times the row's normwise scale
 * ||coefficients||_1 * max|unknowns| + |offset|, which take the normwise scale
 * as denominator (Arioli, Demmel and Duff's two-category backward error; a
 * row whose data and solution are of rounding size would otherwise count as
 * inaccurate).  Host array of batch entries; 0 when refine = 0.
 * Synchronises. */
eclqr_status eclqr_plan_backward_error(const eclqr_plan* plan, const void* ws, double* omega);

/* Row counts of every slot of the feasible-domain scan after the last solve
 * in ws (rows of the affine relation each slot holds); *nslots receives the
 * slot count, rows (host, may be NULL) nslots entries.  Synchronises. */
eclqr_status eclqr_plan_scan_rows(const eclqr_plan* plan, const void* ws, int32_t which, int32_t* rows,
                                  int32_t* nslots);

/* Form of the value-function combine that produced every scan slot in the
 * last solve in ws (reduced LQR scan, Section VI): 0 none (a leaf, or an
 * instance that was skipped), 1 Cholesky-factored, 2 LU (the middle value
 * function was not numerically positive definite).  forms (host, may be NULL)
 * receives *nslots entries.  Synchronises. */
eclqr_status eclqr_plan_combine_forms(const eclqr_plan* plan, const void* ws, int32_t which, int32_t* forms,
                                      int32_t* nslots);

/* Device bytes of one engine's parts in the workspace (which: 0 the problem,
 * 1 the reversed-time problem, 2 the theta LQR; ECLQR_INVALID_ARGUMENT when
 * the plan has no such engine): out[0] stage arenas (the stage kernels'
 * results and kept factors), out[1] relation-scan factor logs, out[2]
 * value-function-scan factor logs, out[3] scan slot arenas.  A vector-only
 * pass reads out[0] + out[1] + out[2]. */
eclqr_status eclqr_plan_footprint(const eclqr_plan* plan, int32_t which, int64_t* out);

/* Interval of every scan slot: instance, first leaf, one past the last leaf
 * (leaf N_b is the terminal; a slot whose end is N_b + 1 is unary).  Host
 * arrays of *nslots entries (may be NULL to query *nslots only). */
eclqr_status eclqr_plan_slot_info(const eclqr_plan* plan, int32_t which, int32_t* inst, int32_t* first,
                                  int32_t* last, int32_t* nslots);

/* Introspection of the scan schedule (tests): number of levels and, for
 * level l (0..levels-1, up-sweep then down-sweep), the task triples
 * (left slot, right slot, output slot) in plan-owned host memory. */
eclqr_status eclqr_plan_schedule(const eclqr_plan* plan, int32_t dual, int32_t* levels, int32_t level,
                                 const int32_t** tasks, int32_t* ntasks);

#ifdef __cplusplus
}
#endif

#endif /* ECLQR_H */
