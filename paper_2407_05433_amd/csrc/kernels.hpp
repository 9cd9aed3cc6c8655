// Launch interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace eclqr {

// Device view of one engine's tables inside the bound workspace.
struct DevEngine {
  const StageInfo* st;
  const int64_t* slot_off;    // [SCAN_COUNT * nslots]
  const int32_t* slot_sa;     // [2 * nslots] global stage of the left endpoint (REL/RIC, FWD)
  const int32_t* slot_sb;     // [2 * nslots] global stage of the right endpoint, -1 = unary
  const int32_t* slot_cap;    // REL row capacity
  int32_t* slot_rows;         // REL rows written by the kernels
  const int32_t* tasks;       // (left, right, out) triples
  const int32_t* ric_perm;    // launch order of the value-function combines (absolute task indices), null = identity
  int32_t* nbar;              // reduced state dim per stage
  int32_t* mbar;              // reduced input dim per stage
  double* arena;              // stage arenas
  double* scan[SCAN_COUNT];   // slot arenas
  double* theta;              // fast multiplier route: theta maps, laid out like the forward scan
  double* resid;              // [4 * S]
  const int64_t* rel_log_off; // per slot, -1 = none
  const int64_t* ric_log_off;
  double* rel_log;            // factor logs of the relation scan
  double* ric_log;            // factor logs of the value-function scan
  const int32_t* vac;         // per-instance whole-space domains (relation scan skipped), null = none
  const int32_t* gate;        // per-instance refinement state, null = every instance runs
  const int32_t* live;        // instances still refining; 0 makes the kernels of a refinement step return at once
  int32_t* info;              // per instance: largest stage at which the pass flagged a failure (-1 none), null = not kept
  double* gw;                 // per-workgroup global tiles for stacked relation systems beyond LDS, null = none
  int64_t gw_stride;          // doubles per tile
  int32_t gw_blocks;          // tiles (workgroups of a launch that uses them)
  double* scratch;            // per-workgroup global scratch
  int64_t scratch_per_block;  // doubles
  int64_t S;
  int32_t B;
  int32_t nslots;
  const int32_t* stage_perm;  // stages in the plan's size order (stage-kernel launch ranges), null = stage order
  int32_t nblocks;            // grid size of the stage-parallel kernels (grid-stride)
  int32_t task_grid;          // grid cap of the kernels without per-workgroup global scratch: large (one workgroup
                              // per task, so the dispatcher balances tasks of unequal cost) or nblocks
  int32_t pool_lds;           // value-function combine LDS mode (0 global pool, 1 LDS pool, 2 all in LDS,
                              // 3 staged operands and compact pool in LDS)
  int32_t reg_compose;        // 1: relation compositions that fit run register-resident
  int32_t elim_lds;           // working arrays in LDS when they fit: 1 stage eliminations and feedback gains,
                              // 2 feedback gains only, 0 neither
  int32_t split_combine;      // 1: value-function combines of a level that fits the device run on two wavefronts
};

// Pointers to one problem's data (caller layout of the engine).
struct Inputs {
  const double* f[IN_COUNT];  // Q q R r M A B c E F g (M may be null)
  const double* x0;
};

struct Tols {
  double rank;
  double cons;
  int check_lemma2;
};

void launch_validate(const DevEngine& e, const Inputs& in, int32_t* status, hipStream_t s);
void relations_set_max_lds(int bytes);
void eliminate_set_max_lds(int bytes);
void lqr_set_max_lds(int bytes);
void lqr_set_device(int lds_per_cu, int num_cu);
void replay_set_max_lds(int bytes);
// Grid of a grid-stride launch of `fn` (workgroups of `block` lanes, `lds`
// bytes of dynamic LDS): `want`, capped at the workgroups the current device
// runs at once for that kernel (a grid a little above that capacity runs its
// surplus as a second round of the whole per-workgroup loop on an almost idle
// device).  Cached per device, kernel and LDS size.
int fit_grid(const void* fn, int block, size_t lds, int64_t want);
// Grid of `ntasks` independent tasks for a kernel that needs no per-workgroup
// global scratch (e.task_grid caps it).
inline int task_grid(const DevEngine& e, int64_t ntasks) {
  const int64_t g = ntasks < e.task_grid ? ntasks : e.task_grid;
  return (int)(g < 1 ? 1 : g);
}
size_t rel_lds_bytes(int maxp, int ldw);
size_t domain_lds_bytes(int maxn);
size_t elim_lds_bytes(int maxm, int maxq);
size_t ric_lds_bytes(int maxd);
size_t gains_lds_bytes(int maxm);
// per-instance test of the domain shortcut (vac preset to 1; failing instances get 0)
void launch_vacuous(const DevEngine& e, const Inputs& in, Tols t, int32_t* vac, int maxk, int maxm, hipStream_t s);
// a stacked relation system of maxp x ldw fits LDS or a global tile of the plan
bool rel_fits(const DevEngine& e, int maxp, int ldw);
void launch_base_relation(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxp, int ldw,
                          int64_t first, int64_t count, hipStream_t s);
// maxkc: most coefficient columns (n_a + n_c) of a result in the launch
void launch_rel_compose(const DevEngine& e, int64_t first_task, int64_t ntasks, Tols t, int32_t* status, int maxp,
                        int ldw, int maxkc, hipStream_t s);
// stage kernels: the stages at positions [first, first + count) of the plan's size order
void launch_domain(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxn, int64_t first,
                   int64_t count, hipStream_t s);
void launch_eliminate(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxm, int maxq, int maxn,
                      int maxk, int64_t first, int64_t count, hipStream_t s);
void launch_ric_combine(const DevEngine& e, int64_t first_task, int64_t ntasks, int32_t* status, int maxd,
                        hipStream_t s);
// the same combines, one lane per task where every reduced dim is <= 4 (the
// rest by the wavefront: inline, or with defer_count non-null (zero on entry)
// through defer_list (ntasks entries) and a second launch, one per
// wavefront); for engines whose reduced dims are mostly tiny
void launch_ric_combine_lane(const DevEngine& e, int64_t first, int64_t ntasks, int32_t* defer_count,
                             int32_t* defer_list, hipStream_t s);
void launch_gains(const DevEngine& e, int32_t* status, int maxm, int maxn, int64_t first, int64_t count,
                  hipStream_t s);
void launch_fwd_combine(const DevEngine& e, int64_t first_task, int64_t ntasks, hipStream_t s);
void launch_recover(const DevEngine& e, double* x, double* u, hipStream_t s);

// Levels of one scan for the persistent scan kernels: the nonempty levels in
// order, each a contiguous range of the task list.
constexpr int kMaxScanLevels = 64;
struct ScanLevels {
  int32_t n;
  int64_t begin[kMaxScanLevels];
  int64_t count[kMaxScanLevels];
};
// control block of one persistent scan: [next task, done count per level]
constexpr int kScanCtrlInts = 1 + kMaxScanLevels;
void replay_set_device(int num_cu, int wall_clock_khz);
// One launch for every level of a scan's vector-only replay: workgroups take
// tasks in level order from a counter in ctrl (zero on entry) and wait,
// boundedly, until the levels before a task's level are complete.  kind:
// SCAN_REL, SCAN_RIC or SCAN_FWD.  An expired wait sets *abort and the
// kernel's workgroups return.
void launch_scan_vec(const DevEngine& e, int kind, const ScanLevels& lv, int32_t* ctrl, int32_t* abort,
                     hipStream_t s);
// status[b] |= bit for every instance when *abort is set
void launch_apply_abort(int32_t* status, const int32_t* abort, int32_t bit, int32_t B, hipStream_t s);

// Interior-point driver (bounds on u_i and on x_i, i >= 1): bound arrays
// (null = no bound on that side), bound multipliers and the Newton
// problem's own fields (layouts of the problem's fields).
struct IpmBounds {
  const double *u_lo, *u_hi, *x_lo, *x_hi;
};
struct IpmDuals {
  double *ul, *uh, *xl, *xh;
};
struct IpmNewton {
  double *Q, *q, *R, *r, *c, *g, *x0;
};
// status[b] = nstatus[b], act[b] = (status == 0), steps[b] = 0
void launch_ipm_start(const int32_t* nstatus, int32_t* status, int32_t* act, int32_t* steps, int32_t B,
                      hipStream_t s);
// iterate moved inside the bounds, z = mu0 / distance; bad bounds flag the instance
void launch_ipm_init(const DevEngine& p, const IpmBounds& bd, double* x, double* u, const IpmDuals& z, double mu0,
                     double interior, int32_t* status, int32_t* act, hipStream_t s);
// mean complementarity per instance (part: 2 S doubles); instances below mu_stop stop
void launch_ipm_mu(const DevEngine& p, const int64_t* sbase, const IpmBounds& bd, const double* x, const double* u,
                   const IpmDuals& z, double* part, double mu_stop, double* mu, int32_t* act, hipStream_t s);
// Newton data at the iterate: predictor (ax null: zero targets, every field)
// or corrector (targets from the predictor step ax, au and smu; with
// vectors_only only q and r are written)
void launch_ipm_newton(const DevEngine& p, const Inputs& in, const IpmBounds& bd, const double* x, const double* u,
                       const IpmDuals& z, const double* ax, const double* au, const double* smu, int vectors_only,
                       const IpmNewton& nw, hipStream_t s);
// predictor step length (alpha), complementarity after it and smu = sigma mu
void launch_ipm_centering(const DevEngine& p, const int64_t* sbase, const IpmBounds& bd, const double* x,
                          const double* u, const IpmDuals& z, const double* ax, const double* au,
                          unsigned long long* alpha, double* part, double* mu, double* smu, const int32_t* act,
                          hipStream_t s);
// Newton outcome, corrector step length and update of the active instances
void launch_ipm_step(const DevEngine& p, const IpmBounds& bd, double* x, double* u, double* lam, double* mu_eq,
                     const IpmDuals& z, const double* dx, const double* du, const double* lam_new,
                     const double* mu_new, const double* ax, const double* au, const double* smu,
                     const int32_t* nstatus, const int32_t* cstatus, int32_t* status, double tau,
                     unsigned long long* alpha, int32_t* act, int32_t* steps, hipStream_t s);

// Sequential fallback for instances the scan rejects as not convex: doubles
// of work arrays per workgroup; the solve (classification, x, u, the value
// functions and z of the scans' suffix slots) of every eligible instance;
// their gates held out of refinement.
void launch_dp_fallback(const DevEngine& e, const Inputs& in, const int64_t* sbase, double* x, double* u,
                        int32_t* status, int32_t* info, int32_t* dpflag, double* scratch, int64_t stride,
                        int32_t blocks, int maxn, int maxm, hipStream_t s);
void launch_dp_hold(const int32_t* dpflag, int32_t* gate, int32_t B, hipStream_t s);
// out[b] |= bit where flag[b] != 0
void launch_flag_where(const int32_t* flag, int32_t* out, int32_t bit, int32_t B, hipStream_t s);

// vector-only replays of the kernels above (factors logged by the full pass)
void launch_base_relation_vec(const DevEngine& e, const Inputs& in, int64_t logmax, hipStream_t s);
void launch_rel_compose_vec(const DevEngine& e, int64_t first, int64_t ntasks, int64_t logmax, hipStream_t s);
void launch_domain_vec(const DevEngine& e, const Inputs& in, hipStream_t s);
void launch_eliminate_vec(const DevEngine& e, const Inputs& in, hipStream_t s);
void launch_ric_combine_vec(const DevEngine& e, int64_t first, int64_t ntasks, int maxd, hipStream_t s);
void launch_gains_vec(const DevEngine& e, hipStream_t s);
void launch_fwd_combine_vec(const DevEngine& e, int64_t first, int64_t ntasks, hipStream_t s);

// reversed-time stationarity problem and refinement helpers
struct DualPtrs {
  double* f[IN_COUNT];     // data of the reversed-time problem (its own layout)
  const int64_t* pbase;    // first primal stage of each instance
  const int64_t* dbase;    // first reversed-time stage of each instance
};
struct CorrPtrs {
  double *q, *r, *c, *g, *x0;
};
struct GradPtrs {
  double* f[IN_COUNT];
  double* x0;
};

void launch_dual_matrices(const DevEngine& p, const Inputs& in, const DevEngine& d, const DualPtrs& dp,
                          hipStream_t s);
void launch_dual_vectors(const DevEngine& p, const Inputs& in, const double* x, const double* u, const DevEngine& d,
                         const DualPtrs& dp, hipStream_t s);
void launch_dual_extract(const DevEngine& p, const DevEngine& d, const double* dx, const double* du, double* lam,
                         double* mu, const DualPtrs& dp, hipStream_t s);
void launch_correction(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                       const double* mu, const CorrPtrs& cp, hipStream_t s);
// refinement control: an instance in state kGateDone is skipped by every kernel
constexpr int32_t kGateActive = 0;  // still refining: its reversed-time outcome is not reported
constexpr int32_t kGateFinal = 1;   // this step's update is its last: report the reversed-time outcome
constexpr int32_t kGateDone = 2;    // converged in an earlier step
void launch_refine_update(const DevEngine& p, double* x, double* u, const double* dx, const double* du,
                          double* norms, hipStream_t s);
void launch_refine_decide(const DevEngine& p, const int64_t* sbase, const double* norms, double tol, int last,
                          int32_t* gate, int32_t* steps, hipStream_t s);
void launch_gate_advance(int32_t* gate, int32_t* live, int32_t B, hipStream_t s);
// per-instance componentwise backward error (as the bit pattern of a
// non-negative double, max-accumulated: clear to 0 first)
// max-accumulates the backward error per instance into omega (wmax: B
// entries of scratch for the scale of the unknowns)
// clear = false: the scales of the instances measured were cleared by
// launch_gate_refined (the others keep theirs)
void launch_backward_error(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                           const double* mu, unsigned long long* wmax, unsigned long long* omega, hipStream_t s,
                           bool clear = true);
void launch_gate_refined(const int32_t* steps, int32_t* gate, unsigned long long* wmax, unsigned long long* omega,
                         int32_t B, hipStream_t s);
void launch_accept(const unsigned long long* omega, const int32_t* dstatus, double tol, int32_t* gate, int32_t B,
                   hipStream_t s);
void launch_fill_u64(unsigned long long* y, unsigned long long v, int64_t n, hipStream_t s);
// status |= bit (+ the other outcome in bits 8..15) where other & mask
void launch_merge_dual_bits(int32_t* status, const int32_t* other, int32_t bit, int32_t mask, int32_t B,
                            hipStream_t s);
// status |= bit where an instance took refinement steps and its final backward error exceeds tol
void launch_flag_unconverged(const unsigned long long* omega, const int32_t* steps, double tol, int32_t* status,
                             int32_t bit, int32_t B, hipStream_t s);
void launch_fill(double* y, double v, int64_t n, hipStream_t s);
void launch_fill_i32(int32_t* y, int32_t v, int64_t n, hipStream_t s);
// merges only instances whose gate equals `want` (all instances if gate is null)
void launch_merge_status(int32_t* status, const int32_t* other, int32_t bit, int32_t B, const int32_t* gate,
                         int32_t want, hipStream_t s);
void launch_finalize(const DevEngine& p, const int32_t* status, double* x, double* u, double* lam, double* mu,
                     hipStream_t s);
void launch_kkt_residual(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                         const double* mu, const int64_t* sbase, double* out, hipStream_t s);
// factor-reusing multipliers (reuse the primal pass's scans; run right after it)
void fast_set_max_lds(int bytes);
size_t mult_local_lds_bytes(int maxrow, int ldw);
// false (nothing launched) when the tile exceeds the device's LDS
bool launch_mult_local(const DevEngine& e, const Inputs& in, const double* x, const double* u, Tols t,
                       int32_t* status, int maxrow, int ldw, hipStream_t s);
void launch_theta_combine(const DevEngine& e, int64_t first, int64_t ntasks, hipStream_t s);
void launch_mult_final(const DevEngine& e, double* lam, double* mu, int accumulate, hipStream_t s);
// minimum-norm multipliers through the theta LQR (p: the primal engine, th:
// the theta engine over the same schedule)
void theta_set_max_lds(int bytes);
size_t theta_local_lds_bytes(int maxq, int ldw, int maxr);
// mode 0: full pass; 1: vector pass reusing the local factors of the last
// full or matrix pass (new vectors, same matrices; with status, the vector
// column's consistency is checked); 2: matrix pass (every vector zero; reads
// neither x, u nor the primal's value-function and forward scans)
bool launch_theta_local(const DevEngine& p, const DevEngine& th, const Inputs& in, const double* x, const double* u,
                        Tols t, int32_t* status, int maxq, int ldw, int maxr, int mode, int64_t first,
                        int64_t count, hipStream_t s);
void launch_theta_init(const DevEngine& th, hipStream_t s);
void launch_theta_final(const DevEngine& p, const DevEngine& th, double* lam, double* mu, int accumulate,
                        hipStream_t s);
// gradients of every field from the solution and the adjoint solution; the
// gradients of an instance whose gstatus is nonzero are NaN
// contraction-expansion multipliers (c: the engine of the dual relations, p:
// the problem's engine)
void cx_set_max_lds(int bytes);
bool cx_fits(int base_p, int base_ld, int exp_n, int exp_p, int leaf_k, int leaf_r);
void launch_cx_base(const DevEngine& c, const DevEngine& p, const int64_t* psbase, const Inputs& in, const double* x,
                    const double* u, Tols t, int32_t* status, int maxp, int ldw, hipStream_t s);
void launch_cx_root(const DevEngine& c, const DevEngine& p, const int64_t* csbase, const int64_t* psbase, double* lam,
                    Tols t, int maxn, int maxp, hipStream_t s);
void launch_cx_expand(const DevEngine& c, const DevEngine& p, const int64_t* psbase, int64_t first, int64_t ntasks,
                      double* lam, Tols t, int32_t* status, int maxn, int maxp, hipStream_t s);
void launch_cx_leaf(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                    double* mu, Tols t, int32_t* status, int maxk, int maxr, hipStream_t s);
void launch_grad_assemble(const DevEngine& p, const double* x, const double* u, const double* lam, const double* mu,
                          const double* ax, const double* au, const double* al, const double* am, const GradPtrs& g,
                          const int32_t* gstatus, hipStream_t s);
// gstatus[b] = fstatus[b], plus ECLQR_NOT_DIFFERENTIABLE where the forward
// pass's rank decisions show dependent constraint rows: the feasible set has
// dimension sum_i m-bar_i, so the rows have full rank exactly when
// sum_{i<N} (m_i - m-bar_i) = sum_{i<=N} k_i
void launch_licq(const DevEngine& p, const int64_t* sbase, const int32_t* fstatus, int32_t* gstatus, hipStream_t s);
// adjoint offsets from dL/dlam: c_i <- dlam_{i+1} (layout of c), x0 <- dlam_0
void launch_adjoint_offsets(const DevEngine& p, const double* dlam, double* c, double* x0, hipStream_t s);

}  // namespace eclqr
