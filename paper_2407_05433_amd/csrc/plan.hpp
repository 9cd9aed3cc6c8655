// Host-side plan: caller layout, workspace map and the associative-scan
// schedule for one problem structure (the primal problem, or the reversed-time
// stationarity problem that yields the multipliers).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <array>
#include <vector>

#include "common.hpp"
#include "eclqr.h"

namespace eclqr {

struct Engine {
  int32_t B = 0;
  std::vector<int32_t> N;        // horizon per instance
  std::vector<int64_t> sbase;    // first global stage of each instance
  int64_t S = 0;                 // stages, sum_b (N_b + 1)
  std::vector<StageInfo> st;

  // caller layout
  std::vector<int64_t> off[ECLQR_NUM_FIELDS];
  int64_t total[ECLQR_NUM_FIELDS] = {0};

  // scans: slot tables shared by the three scans (same ids, different sizes)
  int32_t nslots = 0;
  std::vector<int32_t> slot_inst, slot_s, slot_e;
  std::vector<int32_t> slot_na[SCAN_COUNT], slot_nb[SCAN_COUNT];
  std::vector<int32_t> slot_cap;  // REL row capacity
  std::vector<int64_t> slot_off[SCAN_COUNT];
  int64_t scan_arena[SCAN_COUNT] = {0, 0, 0};

  // levels: 0..D-1 up-sweep (level l combines nodes of level l), D..2D-1
  // down-sweep (from the top down).  Tasks are (left, right, out) slot triples.
  int32_t D = 0;
  std::vector<int32_t> tasks;
  std::vector<int64_t> lvl_begin, lvl_count;
  std::vector<int32_t> lvl_rows;    // REL: max (cap_left + cap_right) over the level
  std::vector<int32_t> lvl_dim;     // max endpoint dim over the level's operands
  std::vector<int32_t> lvl_ldw;     // REL: max (n_a + n_b + n_c + 1) over the level
  // launch buckets of each level: task ranges with their own LDS sizing
  std::vector<int64_t> bkt_begin, bkt_count;
  std::vector<int32_t> bkt_rows, bkt_ldw, bkt_dim, bkt_kc;
  std::vector<int32_t> bkt_fit;     // every task of the bucket fits the register-resident composition
  std::vector<int32_t> lvl_kc;      // REL: max (n_a + n_c) over the level
  std::vector<int32_t> lvl_bkt_first, lvl_bkt_n;
  // value-function combine buckets: the tasks of each level reordered by their
  // endpoint dims (ric_perm: absolute task indices, in launch order) and cut
  // into ranges with their own LDS sizing (rbk_dim)
  std::vector<int32_t> ric_perm;
  std::vector<int64_t> rbk_begin, rbk_count;
  std::vector<int32_t> rbk_dim;
  std::vector<int32_t> lvl_rbk_first, lvl_rbk_n;
  // stage buckets: the stages ordered by size (stage_perm: absolute stage
  // indices, in launch order; empty = stage order, one bucket) and cut into
  // ranges whose stage kernels size their LDS to the range's largest stage
  struct StageBucket {
    int64_t begin = 0, count = 0;
    int32_t maxn = 1, maxm = 1, maxk = 0, base_maxp = 1, base_ldw = 1, elim_maxq = 1;
  };
  std::vector<int32_t> stage_perm;
  std::vector<StageBucket> sbk;

  // factor logs replayed by the vector-only pass, per output slot
  std::vector<int64_t> rel_log_off, ric_log_off;
  int64_t rel_log_total = 0, ric_log_total = 0;
  std::vector<int64_t> lvl_rel_log;  // largest relation log (doubles) of each level's outputs
  int64_t base_rel_log = 0;          // largest relation log of the leaves

  int64_t arena_total = 0;  // stage arena doubles
  int32_t maxn = 0, maxm = 0, maxk = 0;
  int32_t base_maxp = 0, base_ldw = 0, elim_maxq = 0;
  int32_t fast_rows = 0, fast_ldw = 0;  // LDS tile of the factor-reusing multiplier kernel
  bool need_rel = true;            // false: no relation-scan arenas or logs (an engine that only runs the LQR scans)
  bool shortcut = false;           // some instance may have whole-space domains (no terminal rows, k_i <= m_i)
  int64_t gw_stride = 0;           // doubles per global tile for stacked relation systems beyond LDS (0: none)
  int32_t gw_blocks = 0;           // tiles
  int32_t bal_levels_ = 1 << 30;   // balanced levels before recursive doubling (0: pure doubling)
  int32_t nblocks = 0;             // grid of the stage-parallel kernels
  int64_t scratch_per_block = 0;   // doubles

  // workspace map (byte offsets from the engine's base)
  size_t o_stage = 0, o_slot_off = 0, o_slot_na = 0, o_slot_nb = 0, o_slot_cap = 0, o_slot_rows = 0,
         o_tasks = 0, o_nbar = 0, o_mbar = 0, o_arena = 0, o_scan[SCAN_COUNT] = {0, 0, 0}, o_resid = 0,
         o_sbase = 0, o_scratch = 0, o_rel_log_off = 0, o_ric_log_off = 0, o_rel_log = 0, o_ric_log = 0,
         o_theta = 0, o_vac = 0, o_gw = 0, o_ric_perm = 0, o_stage_perm = 0;
  size_t bytes = 0;

  std::string build(const eclqr_dims* d);
};

struct Plan {
  eclqr_options opt;
  Engine primal, dual;
  // Minimum-norm multipliers from the primal pass's domains and scans: the
  // LQR over the normal coordinates theta_i of the domains (same schedule as
  // the primal; stage input capacity k_i + n_{i+1}).  theta_ok is false when
  // that capacity exceeds the kernels' limit; the reversed-time problem is
  // used then.
  Engine theta;
  bool theta_ok = false;
  // The contraction-expansion multiplier route (multipliers = 3): the dual
  // base relations over (lambda_i, lambda_{i+1}) composed by a balanced
  // up-sweep, then expanded from the root.  Its engine has the problem's
  // state dims, input dims k_i (the eliminated mu_i), and one more stage of
  // dimension zero so that the terminal relation has a right endpoint.
  Engine cx;
  bool cx_ok = false;
  size_t o_cx_eng = 0;
  int32_t cx_base_p = 1, cx_base_ld = 1;  // LDS tile of the dual base relations
  int32_t cx_exp_p = 1, cx_exp_n = 1;     // stacked operand rows and middle dim of an expansion step
  int32_t cx_leaf_q = 1, cx_leaf_r = 1;   // leaf systems: mu dims x stationarity rows
  bool has_dual = false;      // the reversed-time engine is in the workspace
  size_t o_theta_eng = 0;
  size_t o_defer = 0;         // per level: count of deferred combines (2 D ints), then one task list
  int32_t th_q = 1, th_ldw = 1, th_r = 1;  // LDS tile of the local minimum-norm systems
  std::vector<std::array<int32_t, 3>> th_bk;  // the same over each stage bucket of the problem (q, ldw, r)
  // the vector-only pass factors only terminal stages: its tile's (q, r) are
  // theirs (at least 16 each, so the tile's front also holds any stage's
  // q <= 64 multiplier values), its ldw the bucket's
  int32_t th_vq = 16, th_vr = 16;
  std::vector<std::array<int32_t, 2>> th_vbk;
  int32_t mult_route = 1;     // 1: theta LQR (when theta_ok), 0: reversed-time problem
  // What each workspace holds: the factorizations of the last solve made in
  // it (multiplier route, problem and solution pointers).  eclqr_backward
  // replays them only for that solve.
  struct WsRecord {
    const void* ws;
    int32_t route;
    uint64_t generation;
    std::vector<const void*> ptrs;  // problem fields, then x, u, lam, mu
  };
  std::vector<WsRecord> ws_records;
  uint64_t generation = 0;
  uint64_t uid = 0;           // unique per plan of the process (owner of a shared scratch buffer)
  // workspace regions (bytes from the workspace base)
  size_t o_primal = 0, o_dual = 0;
  size_t o_dprob[ECLQR_NUM_FIELDS] = {0};  // reversed-time stationarity problem data
  size_t o_dx = 0, o_du = 0, o_dstatus = 0;
  size_t o_corr[ECLQR_NUM_FIELDS] = {0};   // correction / adjoint problem vectors (q r c g x0)
  size_t o_cx = 0, o_cu = 0, o_clam = 0, o_cmu = 0, o_zero = 0;
  size_t o_flag = 0;   // per-instance status of the adjoint solve
  size_t o_gate = 0;   // per-instance refinement state (kGate*)
  size_t o_rnorm = 0;  // per-stage squared norms of correction and iterate
  size_t o_rsteps = 0; // per-instance count of refinement steps taken
  size_t o_live = 0;   // instances still refining (one int)
  size_t o_omega = 0;  // per-instance backward error after the first solve (double bits)
  size_t o_wmax = 0;   // per-instance scale of the unknowns of the backward error (double bits)
  size_t o_dp = 0;     // work arrays of the sequential fallback (dp_blocks x dp_stride doubles)
  size_t o_dpflag = 0; // per instance: solved by the sequential fallback
  int64_t dp_stride = 0;
  int32_t dp_blocks = 1;
  size_t o_info = 0;   // per-instance failing stage of the last solve (when the caller passes no info buffer)
  size_t o_adjc = 0, o_adjx0 = 0;  // adjoint offsets from dL/dlam (layouts of c and x0)
  size_t o_gstat = 0;  // per-instance outcome of the last backward (when the caller passes no status buffer)
  size_t o_ctrl = 0;   // control blocks of the persistent scans: 3 engines x 3 scans x kScanCtrlInts int32
  size_t o_abort = 0;  // set by a persistent scan whose bounded wait expired (one int32)
  size_t bytes = 0;
  void* bound_ws = nullptr;
  int bound_device = -1;
  // captured launch sequence of eclqr_solve (use_graph): valid for the
  // pointers it was captured with
  // tuning (eclqr_plan_autotune / eclqr_plan_set_tuning)
  int32_t level_buckets = 1;  // relation levels launch in LDS-size buckets
  int32_t stage_lds = 1;      // stage kernels' working arrays in LDS when small (20 KiB eliminations, 32 KiB gains)
  int32_t pool_lds = 3;       // value-function combine LDS mode (0 global pool, 1 LDS pool, 2 all in LDS,
                              // 3 staged operands and compact pool in LDS)
  int32_t grid_divisor = 1;   // grid of the stage-parallel kernels = nblocks / divisor
  int32_t reg_compose = 1;    // register-resident relation compositions where they fit
  int32_t overlap_dual = 1;   // factor the multiplier route's problem on a second stream beside the primal pass
                              // (plan default: 0 with the theta route, 1 without)
  int32_t split_combine = 1;  // two wavefronts per value-function combine on levels that fit the device
  int32_t fused_scans = 0;    // vector-only replays run each scan as one persistent launch (else one per level)
  int32_t refine_gate = 0;    // the host reads the count of instances still refining and skips unneeded steps
  double tuned_ms = 0.0;
  void* graph_exec = nullptr;
  // with refine_gate: graph_exec holds the first pass up to the accept test,
  // graph_ref the refinement steps, graph_tail the rest of the solve
  void* graph_ref = nullptr;
  void* graph_tail = nullptr;
  int32_t* gate_host = nullptr;    // pinned host word the count of instances still refining is read into
  void* capture_stream = nullptr;  // plan-owned stream the sequence is captured on
  void* aux_stream = nullptr;      // plan-owned stream of the overlapped reversed-time factorization
  void* ev_fork = nullptr;         // fork / join events between the two streams
  void* ev_join = nullptr;
  std::vector<const void*> graph_key;
  void* ipm_graph_exec = nullptr;          // one interior-point iteration, captured (eclqr_ipm_solve)
  std::vector<const void*> ipm_graph_key;
  ~Plan();
  // profiler: recorded (class, start, stop) event triples
  bool profiling = false;
  bool inexact_newton = false;  // set while the interior-point driver enqueues its Newton solves: an
                                // instance whose refinement stops above dual_cons_tol keeps its (inexact)
                                // step instead of reporting ECLQR_DUAL_FAILED
  std::vector<std::pair<int, std::pair<void*, void*>>> events;
  std::vector<void*> event_pool;
  size_t pool_next = 0;
};

std::string build_plan(Plan& p, const eclqr_dims* d, const eclqr_options* opt);
void release_graph(Plan& p);

}  // namespace eclqr

struct eclqr_plan {
  eclqr::Plan p;
};
