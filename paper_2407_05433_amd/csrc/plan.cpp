// Host-side plan construction (no GPU calls).
//
// The feasible-domain scan, the Riccati scan and the forward pass are all
// inclusive suffix scans over L = N + 1 leaves per instance whose last leaf
// is unary (the terminal relation, the terminal cost, or the initial state of
// the reversed forward scan).  One balanced schedule (Section IV, "Suffix
// scan": an up-sweep composing interval aggregates, a down-sweep handing each
// interval the aggregate to its right) serves all three; only the slot sizes
// differ.  Tasks of every instance at the same level form one launch.
//
// Recursive doubling is the depth-optimal alternative: at level l every node
// j with j + 2^l < K combines its interval with the one 2^l nodes to its
// right; after ceil(log2 K) levels node j covers [start_j, L).  It has no
// down-sweep and about K log2 K tasks instead of 2K, so it wins while a
// level's tasks fit on the device at once and loses on wide levels.  The
// schedule built here is the hybrid: b balanced up-sweep levels (K = the
// nodes left), doubling over those K nodes, then the b balanced down-sweep
// levels.  b = 0 is pure doubling, b >= depth the plain balanced sweep.
#include "plan.hpp"
#include "kernels.hpp"
#include "scratch.hpp"

#include <algorithm>
#include <array>
#include <cstdio>

namespace eclqr {

namespace {

struct Node {
  int32_t s, e, slot;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

std::string Engine::build(const eclqr_dims* d) {
  B = d->batch;
  if (B < 1) return "batch must be >= 1";
  N.assign(d->horizon, d->horizon + B);
  sbase.resize(B);
  S = 0;
  for (int b = 0; b < B; ++b) {
    if (N[b] < 1) return "every horizon must be >= 1";
    sbase[b] = S;
    S += N[b] + 1;
  }
  // per-stage dims
  st.assign(S, StageInfo{});
  int64_t ui = 0;
  maxn = maxm = maxk = 0;
  for (int b = 0; b < B; ++b) {
    for (int i = 0; i <= N[b]; ++i) {
      int64_t s = sbase[b] + i;
      StageInfo& x = st[s];
      x.n = d->nx[s];
      x.k = d->nc[s];
      x.inst = b;
      x.i = i;
      x.N = N[b];
      x.terminal = (i == N[b]);
      if (i < N[b]) {
        x.np = d->nx[s + 1];
        x.m = d->nu[ui++];
      } else {
        x.np = 0;
        x.m = 0;
      }
      if (x.n < 0 || x.m < 0 || x.k < 0) return "negative dimension";
      if (x.n > kMaxDim || x.m > kMaxDim || x.k > kMaxDim)
        return "dimension above " + std::to_string(kMaxDim);
      maxn = std::max(maxn, x.n);
      maxm = std::max(maxm, x.m);
      maxk = std::max(maxk, x.k);
    }
  }
  // caller layout: blocks in stage order
  for (int f = 0; f < ECLQR_NUM_FIELDS; ++f) {
    off[f].assign(f == ECLQR_F_x0 ? B : S, -1);
    total[f] = 0;
  }
  for (int64_t s = 0; s < S; ++s) {
    StageInfo& x = st[s];
    const int64_t n = x.n, np = x.np, m = x.m, k = x.k;
    const int64_t sz[ECLQR_NUM_FIELDS - 1] = {n * n, n, m * m, m, n * m, np * n, np * m, np, k * n, k * m, k};
    for (int f = 0; f < ECLQR_NUM_FIELDS - 1; ++f) {
      bool present = !(x.terminal && (f == ECLQR_F_R || f == ECLQR_F_r || f == ECLQR_F_M || f == ECLQR_F_A ||
                                      f == ECLQR_F_B || f == ECLQR_F_c || f == ECLQR_F_F));
      off[f][s] = total[f];
      x.in[f] = total[f];
      if (present) total[f] += sz[f];
    }
    if (x.i == 0) {
      off[ECLQR_F_x0][x.inst] = total[ECLQR_F_x0];
      x.x0 = total[ECLQR_F_x0];
      total[ECLQR_F_x0] += n;
    }
  }
  // stage arenas
  arena_total = 0;
  for (int64_t s = 0; s < S; ++s) {
    st[s].ws = arena_total;
    arena_total += arena_layout(st[s].n, st[s].np, st[s].m, st[s].k).size;
  }

  // ---- scan schedule -------------------------------------------------------
  nslots = 0;
  slot_inst.clear(); slot_s.clear(); slot_e.clear(); slot_cap.clear();
  std::vector<std::vector<int32_t>> up_lv, dn_lv;  // tasks per level (flattened triples)
  D = 0;
  auto new_slot = [&](int b, int s, int e, int cap) {
    slot_inst.push_back(b);
    slot_s.push_back(s);
    slot_e.push_back(e);
    slot_cap.push_back(cap);
    return nslots++;
  };
  // balanced levels before the doubling phase (every instance the same, so
  // levels stay aligned across the batch): all of them for the balanced
  // schedule, none for pure doubling
  const int bal_levels = bal_levels_;
  std::vector<int32_t> top_suffix;
  for (int b = 0; b < B; ++b) {
    const int L = N[b] + 1;
    const int64_t s0 = sbase[b];
    auto ndim = [&](int i) { return st[s0 + i].n; };
    auto rel_dims = [&](int s, int e, int& na, int& nb) {
      na = ndim(s);
      nb = (e == L) ? 0 : ndim(e);
    };
    std::vector<std::vector<Node>> lv(1);
    for (int j = 0; j < L; ++j) {
      const StageInfo& x = st[s0 + j];
      int cap = (j < N[b]) ? std::min(x.np + x.k, x.n + x.np) : std::min(x.k, x.n);
      lv[0].push_back({j, j + 1, new_slot(b, j, j + 1, cap)});
    }
    int lev = 0;
    while (lv[lev].size() > 1 && lev < bal_levels) {
      const auto& cur = lv[lev];
      std::vector<Node> nxt;
      if ((int)up_lv.size() <= lev) up_lv.emplace_back();
      for (size_t j = 0; j < cur.size(); j += 2) {
        if (j + 1 < cur.size()) {
          const Node& a = cur[j];
          const Node& c = cur[j + 1];
          int na, nb;
          rel_dims(a.s, c.e, na, nb);
          int cap = std::min(slot_cap[a.slot] + slot_cap[c.slot], na + nb);
          int slot = new_slot(b, a.s, c.e, cap);
          up_lv[lev].insert(up_lv[lev].end(), {a.slot, c.slot, slot});
          nxt.push_back({a.s, c.e, slot});
        } else {
          nxt.push_back(cur[j]);
        }
      }
      lv.push_back(nxt);
      ++lev;
    }
    // recursive doubling over the nodes of the top balanced level: node j
    // covers [top[j].s, end_j); after ceil(log2 K) levels every node reaches L
    {
      const std::vector<Node>& top = lv[lev];
      const int K = (int)top.size();
      std::vector<int32_t> cur(K), cend(K);
      for (int j = 0; j < K; ++j) {
        cur[j] = top[j].slot;
        cend[j] = j + 1;  // end as a node index (K = the terminal end L)
      }
      int dl = lev;
      for (int span = 1; span < K; span *= 2, ++dl) {
        if ((int)up_lv.size() <= dl) up_lv.emplace_back();
        std::vector<int32_t> nxt(cur), nend(cend);
        for (int j = 0; j + span < K; ++j) {
          const int mid = cend[j], e = cend[mid];
          const int ee = (e == K) ? L : top[e].s;
          int na, nb;
          rel_dims(top[j].s, ee, na, nb);
          const int cap = std::min(slot_cap[cur[j]] + slot_cap[cur[mid]], na + nb);
          const int slot = new_slot(b, top[j].s, ee, cap);
          up_lv[dl].insert(up_lv[dl].end(), {cur[j], cur[mid], slot});
          nxt[j] = slot;
          nend[j] = e;
        }
        cur.swap(nxt);
        cend.swap(nend);
      }
      D = std::max(D, dl);
      top_suffix.assign(L + 1, -1);
      for (int j = 0; j < K; ++j) {
        if (cend[j] != K) return "internal error: doubling left a node short of the end";
        top_suffix[top[j].s] = cur[j];
      }
    }
    const int Db = lev;
    // down-sweep over the balanced levels: suffix slot of every leaf
    std::vector<int32_t> suf(top_suffix);
    for (int l = Db; l >= 1; --l) {
      const auto& par = lv[l];
      const auto& ch = lv[l - 1];
      // children of par[p] are ch[2p], ch[2p+1]
      for (size_t p = 0; p < par.size(); ++p) {
        if (2 * p + 1 >= ch.size()) continue;  // pass-through
        const Node& v = par[p];
        const Node& bn = ch[2 * p + 1];
        if (v.e == L) {
          suf[bn.s] = bn.slot;
        } else {
          int na = ndim(bn.s);
          int cap = std::min(slot_cap[bn.slot] + slot_cap[suf[v.e]], na);
          int slot = new_slot(b, bn.s, L, cap);
          // down level index counts from the top of this instance's tree: all
          // instances share the bottom level (l = 1) as the last launch.
          int di = l - 1;
          if ((int)dn_lv.size() <= di) dn_lv.resize(di + 1);
          dn_lv[di].insert(dn_lv[di].end(), {bn.slot, suf[v.e], slot});
          suf[bn.s] = slot;
        }
      }
    }
    for (int j = 0; j < L; ++j) {
      if (suf[j] < 0) return "internal error: leaf without suffix";
    }
    for (int j = 0; j < L; ++j) {
      StageInfo& x = st[s0 + j];
      x.elem[SCAN_REL] = x.elem[SCAN_RIC] = lv[0][j].slot;
      x.suf[SCAN_REL] = x.suf[SCAN_RIC] = suf[j];
      // forward scan: leaf j is the closed-loop map of stage N-1-j, leaf N the
      // initial state; the suffix of leaf j is z_{N-j}
      x.elem[SCAN_FWD] = (j < N[b]) ? lv[0][N[b] - 1 - j].slot : -1;
      x.suf[SCAN_FWD] = suf[N[b] - j];
    }
  }
  // levels: up 0..D-1, down D..2D-1 (down level index D-1-di so the top runs first)
  tasks.clear();
  lvl_begin.assign(2 * D, 0);
  lvl_count.assign(2 * D, 0);
  for (int l = 0; l < D; ++l) {
    lvl_begin[l] = tasks.size() / 3;
    if (l < (int)up_lv.size()) tasks.insert(tasks.end(), up_lv[l].begin(), up_lv[l].end());
    lvl_count[l] = tasks.size() / 3 - lvl_begin[l];
  }
  for (int l = 0; l < D; ++l) {
    int di = D - 1 - l;  // top first
    lvl_begin[D + l] = tasks.size() / 3;
    if (di < (int)dn_lv.size()) tasks.insert(tasks.end(), dn_lv[di].begin(), dn_lv[di].end());
    lvl_count[D + l] = tasks.size() / 3 - lvl_begin[D + l];
  }
  // slot dims and sizes per scan
  for (int k = 0; k < SCAN_COUNT; ++k) {
    slot_na[k].assign(nslots, 0);
    slot_nb[k].assign(nslots, 0);
    slot_off[k].assign(nslots, 0);
    scan_arena[k] = 0;
  }
  for (int32_t q = 0; q < nslots; ++q) {
    const int b = slot_inst[q], s = slot_s[q], e = slot_e[q];
    const int L = N[b] + 1;
    const int64_t s0 = sbase[b];
    const int na = st[s0 + s].n, nb = (e == L) ? 0 : st[s0 + e].n;
    slot_na[SCAN_REL][q] = slot_na[SCAN_RIC][q] = na;
    slot_nb[SCAN_REL][q] = slot_nb[SCAN_RIC][q] = nb;
    // forward scan reflects the leaf index: output z_{N-s}, input z_{N-e}
    const int fa = st[s0 + (N[b] - s)].n, fb = (e == L) ? 0 : st[s0 + (N[b] - e)].n;
    slot_na[SCAN_FWD][q] = fa;
    slot_nb[SCAN_FWD][q] = fb;
    slot_off[SCAN_REL][q] = scan_arena[SCAN_REL];
    if (need_rel) scan_arena[SCAN_REL] += rel_slot_size(slot_cap[q], na, nb);
    slot_off[SCAN_RIC][q] = scan_arena[SCAN_RIC];
    scan_arena[SCAN_RIC] += ric_layout(na, nb).size;
    slot_off[SCAN_FWD][q] = scan_arena[SCAN_FWD];
    scan_arena[SCAN_FWD] += fwd_slot_size(fa, fb);
  }
  // factor logs: leaves of the relation scan (base relations) and every task output
  rel_log_off.assign(nslots, -1);
  ric_log_off.assign(nslots, -1);
  rel_log_total = ric_log_total = 0;
  base_rel_log = 0;
  lvl_rel_log.assign(2 * D, 0);
  for (int32_t q = 0; q < nslots; ++q) {
    const int b = slot_inst[q], s = slot_s[q], e = slot_e[q];
    if (e != s + 1 || !need_rel) continue;
    const StageInfo& x = st[sbase[b] + s];
    const int P = x.terminal ? x.k : x.np + x.k;
    const int R = x.terminal ? 0 : std::min(x.m, P);
    rel_log_off[q] = rel_log_total;
    rel_log_total += rel_log_layout(P, R, slot_cap[q]).size;
    base_rel_log = std::max(base_rel_log, rel_log_layout(P, R, slot_cap[q]).size);
  }
  for (size_t t = 0; t < tasks.size() / 3; ++t) {
    const int a = tasks[3 * t], c = tasks[3 * t + 1], o = tasks[3 * t + 2];
    const int b = slot_inst[a];
    const int nmid = st[sbase[b] + slot_e[a]].n;
    const int P = slot_cap[a] + slot_cap[c];
    if (need_rel) {
      rel_log_off[o] = rel_log_total;
      rel_log_total += rel_log_layout(P, std::min(nmid, P), slot_cap[o]).size;
      for (int l = 0; l < 2 * D; ++l)
        if ((int64_t)t >= lvl_begin[l] && (int64_t)t < lvl_begin[l] + lvl_count[l])
          lvl_rel_log[l] = std::max(lvl_rel_log[l], rel_log_layout(P, std::min(nmid, P), slot_cap[o]).size);
    }
    ric_log_off[o] = ric_log_total;
    ric_log_total += ric_log_size(nmid);
  }
  // Launch buckets of the relation composition: the tasks of a wide level
  // (>= 2048 tasks) sorted by the LDS their composition needs and split where
  // that need doubles (buckets of fewer than 512 tasks join the next larger
  // one), so small tasks of a batch are not launched with the LDS of its
  // largest one.
  lvl_rows.assign(2 * D, 0);
  lvl_dim.assign(2 * D, 0);
  lvl_ldw.assign(2 * D, 1);
  lvl_kc.assign(2 * D, 0);
  bkt_kc.clear();
  bkt_fit.clear();
  bkt_begin.clear();
  bkt_count.clear();
  bkt_rows.clear();
  bkt_ldw.clear();
  bkt_dim.clear();
  lvl_bkt_first.assign(2 * D, 0);
  lvl_bkt_n.assign(2 * D, 0);
  auto task_ldw = [&](int a, int c) { return slot_na[SCAN_REL][a] + slot_nb[SCAN_REL][a] + slot_nb[SCAN_REL][c] + 1; };
  auto task_need = [&](int a, int c) { return (int64_t)(slot_cap[a] + slot_cap[c]) * task_ldw(a, c); };
  auto task_dim = [&](int a, int c) {
    return std::max({slot_na[SCAN_REL][a], slot_nb[SCAN_REL][a], slot_nb[SCAN_REL][c], slot_na[SCAN_FWD][a],
                     slot_nb[SCAN_FWD][a], slot_nb[SCAN_FWD][c]});
  };
  auto lg2 = [](int64_t v) {
    int k = 0;
    while ((int64_t(1) << (k + 1)) <= v) ++k;
    return k;
  };
  for (int l = 0; l < 2 * D; ++l) {
    const int64_t b0 = lvl_begin[l], nt = lvl_count[l];
    std::vector<std::array<int32_t, 3>> tv((size_t)nt);
    for (int64_t t = 0; t < nt; ++t) tv[t] = {tasks[3 * (b0 + t)], tasks[3 * (b0 + t) + 1], tasks[3 * (b0 + t) + 2]};
    // tasks that fit the register-resident composition first, each part by size
    auto fits = [&](int a, int c) {
      return slot_cap[a] + slot_cap[c] <= 64 && task_ldw(a, c) <= 128 &&
             slot_na[SCAN_REL][a] + slot_nb[SCAN_REL][c] <= 64;
    };
    std::stable_sort(tv.begin(), tv.end(), [&](const std::array<int32_t, 3>& x, const std::array<int32_t, 3>& y) {
      const bool fx = fits(x[0], x[1]), fy = fits(y[0], y[1]);
      if (fx != fy) return fx;
      return task_need(x[0], x[1]) < task_need(y[0], y[1]);
    });
    for (int64_t t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k) tasks[3 * (b0 + t) + k] = tv[t][k];
    lvl_bkt_first[l] = (int32_t)bkt_begin.size();
    int64_t t = 0;
    while (t < nt) {
      int64_t u = t + 1;
      const int cls = lg2(std::max<int64_t>(1, task_need(tv[t][0], tv[t][1])));
      const bool fit = fits(tv[t][0], tv[t][1]);
      // end of this fit class
      int64_t end = t + 1;
      while (end < nt && fits(tv[end][0], tv[end][1]) == fit) ++end;
      if (nt >= 2048) {
        while (u < end && lg2(std::max<int64_t>(1, task_need(tv[u][0], tv[u][1]))) == cls) ++u;
        while (u < end && u - t < 512) ++u;
        if (end - u < 512) u = end;
      } else {
        u = end;
      }
      int rows = 0, ldw = 1, dim = 0, kc = 0;
      for (int64_t v = t; v < u; ++v) {
        rows = std::max(rows, slot_cap[tv[v][0]] + slot_cap[tv[v][1]]);
        ldw = std::max(ldw, task_ldw(tv[v][0], tv[v][1]));
        dim = std::max(dim, task_dim(tv[v][0], tv[v][1]));
        kc = std::max(kc, slot_na[SCAN_REL][tv[v][0]] + slot_nb[SCAN_REL][tv[v][1]]);
      }
      bkt_begin.push_back(b0 + t);
      bkt_count.push_back(u - t);
      bkt_rows.push_back(rows);
      bkt_ldw.push_back(ldw);
      bkt_dim.push_back(dim);
      bkt_kc.push_back(kc);
      bkt_fit.push_back(fit ? 1 : 0);
      lvl_kc[l] = std::max(lvl_kc[l], kc);
      lvl_rows[l] = std::max(lvl_rows[l], rows);
      lvl_ldw[l] = std::max(lvl_ldw[l], ldw);
      lvl_dim[l] = std::max(lvl_dim[l], dim);
      t = u;
    }
    lvl_bkt_n[l] = (int32_t)bkt_begin.size() - lvl_bkt_first[l];
  }
  // Value-function combine buckets.  Its LDS grows with the square of the
  // largest endpoint dim of a launch, and LDS bounds how many workgroups a
  // compute unit holds; a wide level (>= 2048 tasks) is launched in ranges of
  // one dim class each (<= 8, 12, 16, 24, 32, 48, 64; ranges of fewer than
  // 512 tasks join the next class) over its tasks ordered by that dim.
  ric_perm.resize(tasks.size() / 3);
  rbk_begin.clear();
  rbk_count.clear();
  rbk_dim.clear();
  lvl_rbk_first.assign(2 * D, 0);
  lvl_rbk_n.assign(2 * D, 0);
  auto dim_class = [](int d) {
    const int bounds[] = {8, 12, 16, 24, 32, 48, 64};
    for (int b : bounds)
      if (d <= b) return b;
    return d;
  };
  for (int l = 0; l < 2 * D; ++l) {
    const int64_t b0 = lvl_begin[l], nt = lvl_count[l];
    std::vector<std::pair<int32_t, int32_t>> dv((size_t)nt);  // (dim, absolute task)
    for (int64_t t = 0; t < nt; ++t)
      dv[t] = {task_dim(tasks[3 * (b0 + t)], tasks[3 * (b0 + t) + 1]), (int32_t)(b0 + t)};
    if (nt >= 2048) std::stable_sort(dv.begin(), dv.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (int64_t t = 0; t < nt; ++t) ric_perm[b0 + t] = dv[t].second;
    lvl_rbk_first[l] = (int32_t)rbk_begin.size();
    int64_t t = 0;
    while (t < nt) {
      int64_t u = nt;
      if (nt >= 2048) {
        u = t + 1;
        while (u < nt && dim_class(dv[u].first) == dim_class(dv[t].first)) ++u;
        while (u < nt && u - t < 512) ++u;
        if (nt - u < 512) u = nt;
      }
      int dim = 0;
      for (int64_t v = t; v < u; ++v) dim = std::max(dim, dv[v].first);
      rbk_begin.push_back(b0 + t);
      rbk_count.push_back(u - t);
      rbk_dim.push_back(dim);
      t = u;
    }
    lvl_rbk_n[l] = (int32_t)rbk_begin.size() - lvl_rbk_first[l];
  }
  // per-stage kernel sizes
  base_maxp = 1;
  base_ldw = 1;
  elim_maxq = 1;
  fast_rows = 1;
  fast_ldw = 1;
  scratch_per_block = 64;
  for (int64_t s = 0; s < S; ++s) {
    const StageInfo& x = st[s];
    if (x.terminal) {
      base_maxp = std::max(base_maxp, x.k);
      base_ldw = std::max(base_ldw, x.n + 1);
    } else {
      base_maxp = std::max(base_maxp, x.np + x.k);
      base_ldw = std::max(base_ldw, x.m + x.n + x.np + 1);
      elim_maxq = std::max(elim_maxq, x.k + x.np);
    }
    // factor-reusing multipliers: (x, u) rows; mu, theta', H' and constant columns
    fast_rows = std::max(fast_rows, x.n + (x.terminal ? 0 : x.m));
    fast_ldw = std::max(fast_ldw, (x.k + x.np + x.n + 1) | 1);
    if (need_rel) scratch_per_block = std::max(scratch_per_block, elim_scratch(x.n, x.np, x.m, x.k));
    scratch_per_block = std::max(scratch_per_block, gains_scratch(x.n, x.np, x.m));
  }
  scratch_per_block = std::max(scratch_per_block, ric_pool(maxn));
  scratch_per_block = rup4(scratch_per_block);
  // Stage buckets.  The LDS of the stage kernels grows with the stacked
  // system of the stage's base relation ((n' + k) x (m + n + n' + 1)), and LDS
  // bounds how many workgroups a compute unit holds; with at least 4096
  // stages they are launched in ranges of one size class each (tile area
  // <= 128, 256, 512, 1024, 2048, 4096 doubles, or more; ranges of fewer than
  // 1024 stages join the next class) over the stages ordered by that area.
  stage_perm.clear();
  sbk.clear();
  {
    auto area = [&](int64_t s) -> int64_t {
      const StageInfo& x = st[s];
      return x.terminal ? (int64_t)x.k * (x.n + 1) : (int64_t)(x.np + x.k) * (x.m + x.n + x.np + 1);
    };
    auto size_class = [](int64_t a) -> int64_t {
      for (int64_t b = 128; b <= 4096; b *= 2)
        if (a <= b) return b;
      return 1 << 30;
    };
    std::vector<std::pair<int64_t, int32_t>> sv((size_t)S);
    for (int64_t s = 0; s < S; ++s) sv[s] = {area(s), (int32_t)s};
    const bool split = S >= 4096;
    if (split) {
      std::stable_sort(sv.begin(), sv.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      stage_perm.resize((size_t)S);
      for (int64_t s = 0; s < S; ++s) stage_perm[s] = sv[s].second;
    }
    int64_t t = 0;
    while (t < S) {
      int64_t u = S;
      if (split) {
        u = t + 1;
        while (u < S && size_class(sv[u].first) == size_class(sv[t].first)) ++u;
        while (u < S && u - t < 1024) ++u;
        if (S - u < 1024) u = S;
      }
      StageBucket b;
      b.begin = t;
      b.count = u - t;
      for (int64_t v = t; v < u; ++v) {
        const StageInfo& x = st[sv[v].second];
        b.maxn = std::max(b.maxn, std::max(x.n, x.np));  // a stage kernel also sizes its successor's state
        b.maxm = std::max(b.maxm, x.m);
        b.maxk = std::max(b.maxk, x.k);
        if (x.terminal) {
          b.base_maxp = std::max(b.base_maxp, x.k);
          b.base_ldw = std::max(b.base_ldw, x.n + 1);
        } else {
          b.base_maxp = std::max(b.base_maxp, x.np + x.k);
          b.base_ldw = std::max(b.base_ldw, x.m + x.n + x.np + 1);
          b.elim_maxq = std::max(b.elim_maxq, x.k + x.np);
        }
      }
      sbk.push_back(b);
      t = u;
    }
    if (S == 0) sbk.push_back(StageBucket{});
  }
  nblocks = (int32_t)std::min<int64_t>(std::max<int64_t>(S, 1), 8192);

  // global tiles for stacked relation systems: base relations that may
  // outgrow LDS (48 KiB and more: the device's LDS also holds the small work
  // arrays), and compositions whose LDS tile would exceed kRelComposeLds
  // (there a tile in global memory per workgroup, at many workgroups per
  // compute unit, is faster than LDS at a few), one tile per workgroup of
  // the widest launch (at most the stage-parallel grid)
  gw_stride = 0;
  gw_blocks = 0;
  if (need_rel) {
    const int64_t btile = (int64_t)base_maxp * (base_ldw | 1);
    int64_t ctile = 0, widest = S;
    for (size_t l = 0; l < lvl_rows.size(); ++l) {
      ctile = std::max(ctile, (int64_t)lvl_rows[l] * (lvl_ldw[l] | 1));
      widest = std::max(widest, lvl_count[l]);
    }
    const bool big_base = (int64_t)sizeof(double) * btile > 48 * 1024;
    const bool big_compose = (int64_t)sizeof(double) * ctile > kRelComposeLds;
    if (big_base || big_compose) {
      gw_stride = rup4(std::max(btile, ctile));
      gw_blocks = (int32_t)std::min<int64_t>(big_compose ? 8192 : 256, std::max<int64_t>(1, widest));
    }
  }

  // ---- workspace map -------------------------------------------------------
  size_t o = 0;
  o_stage = o; o = align256(o + sizeof(StageInfo) * S);
  o_slot_off = o; o = align256(o + sizeof(int64_t) * nslots * SCAN_COUNT);
  o_slot_na = o; o = align256(o + sizeof(int32_t) * nslots * SCAN_COUNT);
  o_slot_nb = o; o = align256(o + sizeof(int32_t) * nslots * SCAN_COUNT);
  o_slot_cap = o; o = align256(o + sizeof(int32_t) * nslots);
  o_slot_rows = o; o = align256(o + sizeof(int32_t) * nslots);
  o_tasks = o; o = align256(o + sizeof(int32_t) * tasks.size() + 16);
  o_ric_perm = o; o = align256(o + sizeof(int32_t) * ric_perm.size() + 16);
  o_stage_perm = o; o = align256(o + sizeof(int32_t) * stage_perm.size() + 16);
  o_nbar = o; o = align256(o + sizeof(int32_t) * S);
  o_mbar = o; o = align256(o + sizeof(int32_t) * S);
  o_resid = o; o = align256(o + sizeof(double) * 4 * S);
  o_sbase = o; o = align256(o + sizeof(int64_t) * B);
  o_vac = o; o = align256(o + sizeof(int32_t) * B);
  o_gw = o; o = align256(o + sizeof(double) * (size_t)gw_stride * gw_blocks);
  o_scratch = o; o = align256(o + sizeof(double) * scratch_per_block * nblocks);
  o_arena = o; o = align256(o + sizeof(double) * arena_total);
  o_rel_log_off = o; o = align256(o + sizeof(int64_t) * std::max<int32_t>(1, nslots));
  o_ric_log_off = o; o = align256(o + sizeof(int64_t) * std::max<int32_t>(1, nslots));
  o_rel_log = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, rel_log_total));
  o_ric_log = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, ric_log_total));
  for (int k = 0; k < SCAN_COUNT; ++k) {
    o_scan[k] = o;
    o = align256(o + sizeof(double) * scan_arena[k]);
  }
  // affine maps of the fast multiplier route, laid out like the forward scan
  o_theta = o;
  o = align256(o + sizeof(double) * std::max<int64_t>(1, scan_arena[SCAN_FWD]));
  bytes = o;
  return "";
}

std::string build_plan(Plan& p, const eclqr_dims* d, const eclqr_options* opt) {
  p.opt = *opt;
  if (opt->scan_schedule < 0 || opt->scan_schedule > 2) return "scan_schedule must be 0, 1 or 2";
  {
    // automatic: the smallest number of balanced levels after which the
    // batch has at most as many interval nodes as the device runs combines at
    // once (one wavefront each): 2048 up to state dim 16; 512 above, where a
    // combine's LDS tile leaves room for one workgroup per CU
    int64_t leaves = 0;
    for (int b = 0; b < d->batch; ++b) leaves += (d->horizon[b] >= 1) ? (int64_t)d->horizon[b] + 1 : 0;
    int maxn = 0;
    for (int64_t s = 0; s < leaves; ++s) maxn = std::max(maxn, d->nx[s]);
    const int64_t cap_nodes = maxn <= 16 ? 2048 : 512;
    int bl = 0;
    for (;; ++bl) {
      int64_t nodes = 0;
      for (int b = 0; b < d->batch; ++b)
        if (d->horizon[b] >= 1) nodes += (((int64_t)d->horizon[b] + 1) + (int64_t(1) << bl) - 1) >> bl;
      if (nodes <= cap_nodes || bl >= 30) break;
    }
    const int lv = opt->scan_schedule == 1 ? (1 << 30) : (opt->scan_schedule == 2 ? 0 : bl);
    p.primal.bal_levels_ = p.dual.bal_levels_ = p.theta.bal_levels_ = lv;
  }
  std::string err = p.primal.build(d);
  if (!err.empty()) return err;
  // domain shortcut (Section VI): possible for an instance with no terminal
  // rows and k_i <= m_i at every stage; the device tests the ranks
  if (opt->domain_shortcut) {
    Engine& E = p.primal;
    for (int b = 0; b < E.B && !E.shortcut; ++b) {
      bool ok = true;
      for (int64_t s = E.sbase[b]; s <= E.sbase[b] + E.N[b] && ok; ++s)
        ok = E.st[s].terminal ? E.st[s].k == 0 : E.st[s].k <= E.st[s].m;
      E.shortcut = ok;
    }
  }
  const Engine& P = p.primal;
  // theta engine: the primal's stages with input capacity k_i + n_{i+1}
  {
    std::vector<int32_t> tu;
    bool ok = true;
    for (int64_t s = 0; s < P.S; ++s) {
      const StageInfo& x = P.st[s];
      if (x.terminal) continue;
      tu.push_back(x.k + x.np);
      if (x.k + x.np > kMaxDim) ok = false;
    }
    if (ok) {
      std::vector<int32_t> hor(P.N.begin(), P.N.end()), nx(P.S), nc(P.S);
      for (int64_t s = 0; s < P.S; ++s) {
        nx[s] = P.st[s].n;
        nc[s] = P.st[s].k;
      }
      eclqr_dims td{P.B, hor.data(), nx.data(), tu.data(), nc.data()};
      p.theta.need_rel = false;
      ok = p.theta.build(&td).empty();
    }
    p.theta_ok = ok;
    p.mult_route = ok ? 1 : 0;
    // the theta factorization beside the primal pass pays only on large
    // batches (the autotuner tries it); the reversed-time one pays everywhere
    p.overlap_dual = ok ? 0 : 1;
    p.th_q = p.th_ldw = p.th_r = 1;
    p.th_bk.assign(P.sbk.size(), {1, 1, 1});
    p.th_vq = p.th_vr = 16;
    p.th_vbk.assign(P.sbk.size(), {16, 16});
    for (size_t b = 0; b < P.sbk.size(); ++b)
      for (int64_t t = P.sbk[b].begin; t < P.sbk[b].begin + P.sbk[b].count; ++t) {
        const StageInfo& x = P.st[P.stage_perm.empty() ? t : P.stage_perm[t]];
        const int q = x.terminal ? x.k : x.k + x.np, R = x.terminal ? x.n : x.n + x.m;
        auto& tb = p.th_bk[b];
        tb[0] = std::max(tb[0], q);
        tb[1] = std::max(tb[1], R | 1);
        tb[2] = std::max(tb[2], x.n);
        p.th_q = std::max(p.th_q, q);
        p.th_ldw = std::max(p.th_ldw, R | 1);
        p.th_r = std::max(p.th_r, x.n);
        if (x.terminal) {
          auto& vb = p.th_vbk[b];
          vb[0] = std::max(vb[0], q);
          vb[1] = std::max(vb[1], x.n);
          p.th_vq = std::max(p.th_vq, q);
          p.th_vr = std::max(p.th_vr, x.n);
        }
      }
    // the local systems are factored in one LDS tile per stage: where that
    // tile exceeds the device's LDS the reversed-time route is laid out
    // instead (decided here, so a plan never switches routes at solve time)
    if (p.theta_ok && theta_local_lds(p.th_q, p.th_ldw, p.th_r) > kDeviceLdsBytes) {
      p.theta_ok = false;
      p.mult_route = 0;
      p.overlap_dual = 1;
    }
  }

  // the reversed-time engine: needed when the minimum-norm multipliers have
  // no theta engine, or when the caller asks for both routes
  p.has_dual = (opt->multipliers == 1 || opt->multipliers == 3) && (!p.theta_ok || opt->reversed_time != 0);
  if (!p.has_dual) p.mult_route = 1;
  // Reversed-time stationarity problem (Section VII): stage 0 has an empty
  // state and input mu_N; stage j = 1..N is primal stage i = N - j with state
  // lambda_{i+1}, input mu_i and m_i mixed rows; the terminal state is lambda_0.
  std::vector<int32_t> hor(P.B), nx, nu, nc;
  for (int b = 0; b < P.B; ++b) {
    const int Nb = P.N[b];
    const int64_t s0 = P.sbase[b];
    hor[b] = Nb + 1;
    nx.push_back(0);
    for (int j = 1; j <= Nb + 1; ++j) nx.push_back(P.st[s0 + Nb - j + 1].n);
    nu.push_back(P.st[s0 + Nb].k);
    for (int j = 1; j <= Nb; ++j) nu.push_back(P.st[s0 + Nb - j].k);
    nc.push_back(0);
    for (int j = 1; j <= Nb; ++j) nc.push_back(P.st[s0 + Nb - j].m);
    nc.push_back(0);
  }
  eclqr_dims dd{P.B, hor.data(), nx.data(), nu.data(), nc.data()};
  if (p.has_dual) {
    err = p.dual.build(&dd);
    if (!err.empty()) return "dual: " + err;
  }

  // contraction-expansion route: engine over (lambda_i) with inputs mu_i
  p.cx_ok = false;
  if (opt->multipliers == 3) {
    std::vector<int32_t> chor(P.B), cnx, cnu, cnc;
    bool ok = true;
    for (int b = 0; b < P.B; ++b) {
      const int Nb = P.N[b];
      const int64_t s0 = P.sbase[b];
      chor[b] = Nb + 1;
      for (int i = 0; i <= Nb; ++i) {
        const StageInfo& x = P.st[s0 + i];
        cnx.push_back(x.n);
        cnu.push_back(x.k);
        // stacked stationarity rows n_i + m_i, held as n_{i+1} + c_i rows
        const int rows = x.n + (x.terminal ? 0 : x.m);
        const int np = x.terminal ? 0 : x.np;
        cnc.push_back(std::max(0, rows - np));
        p.cx_base_p = std::max(p.cx_base_p, rows);
        p.cx_base_ld = std::max(p.cx_base_ld, (x.k + x.n + np + 1) | 1);
        p.cx_leaf_q = std::max(p.cx_leaf_q, x.k);
        p.cx_leaf_r = std::max(p.cx_leaf_r, rows);
        if (std::max(0, rows - np) > kMaxDim) ok = false;
      }
      cnx.push_back(0);
      cnc.push_back(0);
    }
    if (ok) {
      eclqr_dims cd{P.B, chor.data(), cnx.data(), cnu.data(), cnc.data()};
      p.cx.bal_levels_ = 1 << 30;
      ok = p.cx.build(&cd).empty();
    }
    if (ok) {
      const Engine& C = p.cx;
      for (int l = 0; l < C.D; ++l)
        for (int64_t t = C.lvl_begin[l]; t < C.lvl_begin[l] + C.lvl_count[l]; ++t) {
          const int a = C.tasks[3 * t], c = C.tasks[3 * t + 1];
          const int b = C.slot_inst[a];
          p.cx_exp_p = std::max(p.cx_exp_p, C.slot_cap[a] + C.slot_cap[c]);
          p.cx_exp_n = std::max(p.cx_exp_n, C.st[C.sbase[b] + C.slot_e[a]].n);
        }
    }
    p.cx_ok = ok;
  }

  size_t o = 0;
  p.o_primal = o; o = align256(o + p.primal.bytes);
  p.o_dual = o; o = align256(o + p.dual.bytes);
  if (p.theta_ok) {
    p.o_theta_eng = o;
    o = align256(o + p.theta.bytes);
    int64_t widest = 1;
    for (int64_t c : p.theta.lvl_count) widest = std::max(widest, c);
    p.o_defer = o;
    o = align256(o + sizeof(int32_t) * (2 * (int64_t)p.theta.D + 4 + widest));
  }
  if (p.cx_ok) {
    p.o_cx_eng = o;
    o = align256(o + p.cx.bytes);
  }
  for (int f = 0; f < ECLQR_NUM_FIELDS; ++f) {
    p.o_dprob[f] = o;
    o = align256(o + sizeof(double) * std::max<int64_t>(1, p.dual.total[f]));
  }
  p.o_dx = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, p.dual.total[ECLQR_F_q]));
  p.o_du = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, p.dual.total[ECLQR_F_r]));
  p.o_dstatus = o; o = align256(o + sizeof(int32_t) * P.B);
  for (int f : {ECLQR_F_q, ECLQR_F_r, ECLQR_F_c, ECLQR_F_g, ECLQR_F_x0}) {
    p.o_corr[f] = o;
    o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[f]));
  }
  p.o_cx = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_q]));
  p.o_cu = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_r]));
  p.o_clam = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_q]));
  p.o_cmu = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_g]));
  p.o_flag = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_gate = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_rnorm = o; o = align256(o + sizeof(double) * 2 * std::max<int64_t>(1, P.S));
  p.o_rsteps = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_live = o; o = align256(o + sizeof(int32_t));
  p.o_omega = o; o = align256(o + sizeof(double) * std::max<int32_t>(1, P.B));
  p.o_wmax = o; o = align256(o + sizeof(double) * std::max<int32_t>(1, P.B));
  p.dp_stride = (int64_t)dp_stride(std::max(1, P.maxn), std::max(1, P.maxm));
  p.dp_blocks = std::max<int32_t>(1, std::min<int32_t>(P.B, 64));
  p.o_dp = o; o = align256(o + sizeof(double) * (size_t)p.dp_stride * p.dp_blocks);
  p.o_dpflag = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_info = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_gstat = o; o = align256(o + sizeof(int32_t) * std::max<int32_t>(1, P.B));
  p.o_adjc = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_c]));
  p.o_adjx0 = o; o = align256(o + sizeof(double) * std::max<int64_t>(1, P.total[ECLQR_F_x0]));
  p.o_ctrl = o; o = align256(o + sizeof(int32_t) * 9 * kScanCtrlInts);
  p.o_abort = o; o = align256(o + sizeof(int32_t));
  {
    int64_t nz = std::max<int64_t>(1, std::max(P.total[ECLQR_F_c], std::max(P.total[ECLQR_F_g], P.total[ECLQR_F_x0])));
    // the overlapped reversed-time factorization reads zero vectors
    for (int f : {ECLQR_F_q, ECLQR_F_r, ECLQR_F_c, ECLQR_F_g, ECLQR_F_x0}) nz = std::max(nz, p.dual.total[f]);
    p.o_zero = o; o = align256(o + sizeof(double) * nz);
  }
  p.bytes = o;
  return "";
}

}  // namespace eclqr
