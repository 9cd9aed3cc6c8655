// Host-side checks of the plan builder (plan.cpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizer.py.
// Plans for random and edge-case dimension sets under every multiplier option;
// each must build (or be refused, for invalid dimensions) without a memory or
// undefined-behaviour error, and satisfy the invariants of its workspace map,
// scan schedule and launch orders.  No device code runs.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "plan.hpp"
#include "scratch.hpp"

using namespace eclqr;

// The solve entry points own the plan's device objects; the plans built here
// hold none.
Plan::~Plan() {}

static int g_fail = 0, g_cases = 0;
#define CHECK(c, ...)                                \
  do {                                               \
    if (!(c)) {                                      \
      std::fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);            \
      std::fprintf(stderr, "\n");                   \
      ++g_fail;                                      \
    }                                                \
  } while (0)

struct Dims {
  std::vector<int32_t> hor, nx, nu, nc;
  eclqr_dims view() const {
    return eclqr_dims{(int32_t)hor.size(), hor.data(), nx.data(), nu.data(), nc.data()};
  }
};

// Options with the defaults the public header documents.
static eclqr_options defaults() {
  eclqr_options o;
  std::memset(&o, 0, sizeof(o));
  o.rank_tol = 1e-10;
  o.cons_tol = 1e-8;
  o.dual_cons_tol = 1e-6;
  o.refine_tol = 1e-8;
  o.accept_tol = 1e-10;
  o.multipliers = 1;
  o.refine = 2;
  o.domain_shortcut = 1;
  return o;
}

static uint64_t g_rng = 0x9E3779B97F4A7C15ull;
static int rnd(int lo, int hi) {  // uniform in [lo, hi]
  g_rng ^= g_rng << 13;
  g_rng ^= g_rng >> 7;
  g_rng ^= g_rng << 17;
  return lo + (int)(g_rng % (uint64_t)(hi - lo + 1));
}

static Dims random_dims(int B, int Nmax, int nmax, int mmax, bool terminal_rows) {
  Dims d;
  for (int b = 0; b < B; ++b) {
    const int N = rnd(1, Nmax), n = rnd(1, nmax), m = rnd(1, mmax);
    d.hor.push_back(N);
    for (int i = 0; i <= N; ++i) {
      d.nx.push_back(n);
      if (i < N) {
        d.nu.push_back(m);
        d.nc.push_back(rnd(0, m));
      } else {
        d.nc.push_back(terminal_rows ? rnd(0, n - 1) : 0);
      }
    }
  }
  return d;
}

static void check_offsets(const std::vector<size_t>& offs, size_t bytes, const char* what) {
  for (size_t o : offs) {
    CHECK(o % 256 == 0, "%s: offset %zu not 256-aligned", what, o);
    CHECK(o <= bytes, "%s: offset %zu beyond %zu bytes", what, o, bytes);
  }
}

static void check_engine(const Engine& E, const char* what) {
  // stage order: a permutation of the stages, tiled by the stage buckets
  if (!E.stage_perm.empty()) {
    CHECK((int64_t)E.stage_perm.size() == E.S, "%s: stage order of %zu entries for %lld stages", what,
          E.stage_perm.size(), (long long)E.S);
    std::vector<char> seen((size_t)E.S, 0);
    for (int32_t s : E.stage_perm) {
      CHECK(s >= 0 && s < E.S, "%s: stage %d out of range", what, s);
      if (s >= 0 && s < E.S) {
        CHECK(!seen[s], "%s: stage %d twice in the stage order", what, s);
        seen[s] = 1;
      }
    }
  }
  int64_t t = 0;
  for (const auto& b : E.sbk) {
    CHECK(b.begin == t, "%s: stage bucket starts at %lld, expected %lld", what, (long long)b.begin, (long long)t);
    t += b.count;
    CHECK(b.maxn >= 1 && b.maxm >= 1 && b.base_maxp >= 1 && b.base_ldw >= 1, "%s: bucket sizes below 1", what);
  }
  CHECK(t == E.S, "%s: stage buckets cover %lld of %lld stages", what, (long long)t, (long long)E.S);
  // tasks: slot triples; every level's combine order is a permutation of it
  CHECK(E.tasks.size() % 3 == 0, "%s: task list not in triples", what);
  const int64_t ntask = (int64_t)E.tasks.size() / 3;
  for (int64_t i = 0; i < ntask; ++i)
    for (int k = 0; k < 3; ++k) {
      const int32_t v = E.tasks[3 * i + k];
      CHECK(v >= 0 && v < E.nslots, "%s: task %lld slot %d out of range", what, (long long)i, v);
    }
  CHECK((int64_t)E.ric_perm.size() == ntask, "%s: combine order of %zu for %lld tasks", what, E.ric_perm.size(),
        (long long)ntask);
  for (size_t l = 0; l < E.lvl_begin.size(); ++l) {
    const int64_t b0 = E.lvl_begin[l], nt = E.lvl_count[l];
    CHECK(b0 >= 0 && b0 + nt <= ntask, "%s: level %zu out of the task list", what, l);
    std::vector<char> seen((size_t)nt, 0);
    for (int64_t i = 0; i < nt && b0 + i < (int64_t)E.ric_perm.size(); ++i) {
      const int64_t v = (int64_t)E.ric_perm[b0 + i] - b0;
      CHECK(v >= 0 && v < nt, "%s: level %zu combine order leaves the level", what, l);
      if (v >= 0 && v < nt) {
        CHECK(!seen[v], "%s: level %zu task twice in the combine order", what, l);
        seen[v] = 1;
      }
    }
  }
  check_offsets({E.o_stage, E.o_slot_off, E.o_slot_na, E.o_slot_nb, E.o_slot_cap, E.o_slot_rows, E.o_tasks,
                 E.o_nbar, E.o_mbar, E.o_arena, E.o_scan[0], E.o_scan[1], E.o_scan[2], E.o_resid, E.o_sbase,
                 E.o_scratch, E.o_rel_log_off, E.o_ric_log_off, E.o_rel_log, E.o_ric_log, E.o_vac, E.o_gw,
                 E.o_ric_perm, E.o_stage_perm},
                E.bytes, what);
  CHECK(E.scratch_per_block >= ric_pool(1), "%s: scratch below one combine pool", what);
}

static void run(const Dims& d, bool valid, const char* what) {
  for (int mult = 0; mult <= 3; ++mult)
    for (int rev = 0; rev <= 1; ++rev)
      for (int sched = 0; sched <= 2; ++sched) {
        if (rev && mult != 1) continue;
        eclqr_options o = defaults();
        o.multipliers = mult;
        o.reversed_time = rev;
        o.scan_schedule = sched;
        Plan p;
        const eclqr_dims v = d.view();
        const std::string err = build_plan(p, &v, &o);
        ++g_cases;
        if (!valid) {
          CHECK(!err.empty(), "%s: invalid dimensions accepted", what);
          continue;
        }
        CHECK(err.empty(), "%s (multipliers %d, reversed %d, schedule %d): %s", what, mult, rev, sched, err.c_str());
        if (!err.empty()) continue;
        check_engine(p.primal, what);
        if (p.primal.S >= 4096)
          CHECK(!p.primal.stage_perm.empty() && p.primal.sbk.size() > 1, "%s: no stage buckets at %lld stages", what,
                (long long)p.primal.S);
        if (p.theta_ok) check_engine(p.theta, what);
        if (p.has_dual) check_engine(p.dual, what);
        CHECK(p.th_bk.empty() || p.th_bk.size() == p.primal.sbk.size(), "%s: theta tiles per stage bucket", what);
        CHECK(p.bytes >= p.primal.bytes, "%s: workspace smaller than the problem's engine", what);
        check_offsets({p.o_primal, p.o_dual, p.o_gate, p.o_omega, p.o_wmax, p.o_dp, p.o_dpflag}, p.bytes, what);
      }
}

int main() {
  // edge cases
  run(Dims{{1}, {1, 1}, {1}, {0, 0}}, true, "one stage");
  run(Dims{{3}, {0, 2, 2, 2}, {1, 1, 1}, {0, 1, 0, 1}}, true, "empty initial state");
  run(Dims{{2}, {64, 64, 64}, {64, 64}, {0, 0, 0}}, true, "largest dims");
  run(Dims{{2}, {12, 12, 12}, {6, 6}, {6, 3, 11}}, true, "full-rank rows");
  run(Dims{{0}, {3}, {}, {0}}, false, "empty horizon");
  run(Dims{{1}, {65, 3}, {2}, {0, 0}}, false, "state dim above 64");
  run(Dims{{1}, {3, 3}, {65}, {0, 0}}, false, "input dim above 64");
  // single long instance, random batches, and a batch wide enough for the
  // stage and combine buckets
  run(random_dims(1, 1024, 12, 6, true), true, "single long instance");
  for (int r = 0; r < 6; ++r) run(random_dims(rnd(1, 24), 40, 16, 8, r % 2 == 0), true, "random batch");
  run(random_dims(120, 80, 24, 12, true), true, "wide batch");
  std::printf("plan_check: %d plans, %d failures\n", g_cases, g_fail);
  return g_fail ? 1 : 0;
}
