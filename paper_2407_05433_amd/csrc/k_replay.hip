// Vector-only passes.  Every kernel of the method (Algorithm 1) produces
// matrices that depend only on Q, R, M, A, B, E, F and vectors that also
// depend on q, r, c, g, x0.  The refinement correction, the multipliers at a
// refined point and the adjoint of the gradient change only the vectors, so
// they replay the factorizations logged by the full pass:
//   relations    -- row scales, Householder reflectors and Gram-Schmidt steps
//                   applied to the new offset column (Lemma 1, eq.
//                   (composition-matrix));
//   domains      -- t = -H' h, z_0 = T'(x0 - t) (eqs. (state-param),
//                   (reduced-initial));
//   elimination  -- y from the QR of Gamma', c-bar, q-bar, r-bar and the
//                   element vectors from the Cholesky factor of R-bar;
//   value scan   -- b, eta of every combine from its logged factors;
//   gains / forward scan / recovery -- vector parts only.
// One wavefront per stage or task; vectors of at most 64 (states, inputs) or
// 256 (stacked relation rows) entries live in LDS.
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "scratch.hpp"

namespace eclqr {

namespace {

constexpr int kMaxRows = 4 * kMaxDim;  // stacked rows of a composition (two relations of <= 2n rows)

// Header of a relation log, clamped to the log's capacity: rows p, eliminated
// columns rho, kept rows rr.
struct RelHdr {
  int p, rho, rr;
};
__device__ inline RelHdr rel_header(const double* lg, int P, int R, int C) {
  int p = (int)lg[0], rho = (int)lg[1], rr = (int)lg[2];
  p = (p < 0) ? 0 : ((p > P) ? P : p);
  rho = (rho < 0) ? 0 : ((rho > R) ? R : rho);
  rho = (rho > p) ? p : rho;
  rr = (rr < 0) ? 0 : ((rr > C) ? C : rr);
  rr = (rr > p - rho) ? p - rho : rr;
  return RelHdr{p, rho, rr};
}

// dst[r * stride + k] = src[r * stride + k] for r < nr, k < len: eight
// ranges' loads in flight per lane.
__device__ inline void stage_ranges(double* dst, const double* src, int64_t stride, int nr, int len) {
  for (int r0 = 0; r0 < nr; r0 += 8)
    for (int k = ECLQR_TID; k < len; k += ECLQR_NT) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = (r0 + t < nr) ? src[(int64_t)(r0 + t) * stride + k] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (r0 + t < nr) dst[(int64_t)(r0 + t) * stride + k] = v[t];
    }
}

// Copy what a replay of the log reads into LDS at the log's own offsets:
// header, row scales, tau and reflectors of the rho eliminated columns (rows
// < p) and the rr Gram-Schmidt records (entries < 2 + C + p).
__device__ inline void stage_rel_log(double* dst, const double* lg, const RelLog& L, int P, int C, const RelHdr& h,
                                     bool scaled) {
  stage_ranges(dst, lg, 0, 1, 4);
  if (scaled) stage_ranges(dst + L.scale, lg + L.scale, 0, 1, h.p);
  stage_ranges(dst + L.tau, lg + L.tau, 0, 1, h.rho);
  stage_ranges(dst + L.V, lg + L.V, P, h.rho, h.p);
  stage_ranges(dst + L.gs, lg + L.gs, L.step, h.rr, 2 + C + h.p);
}

// Replay a relation log on the offset column o (LDS, p entries).  Returns the
// rows eliminated (rho) and kept (rr); the new offsets are o[rho .. rho+rr).
// o lives in LDS and the log is read only, so LDS-only barriers order every
// exchange.
// The logged Householder reflectors applied to the offsets o (LDS, p rows):
// step j takes w = (o_j + v_j'o_{j+1:}) tau_j, o_j -= w, o_{j+1:} -= w v_j.
// With at most one row per lane the next step's reflector entry and tau are
// loaded while this step runs (a log left in global memory then costs one
// round trip per step less); same rows per lane and order, so the same bits.
__device__ inline void apply_reflectors(double* o, const double* lg, const RelLog& L, int P, int p, int rho) {
  const int lane = ECLQR_TID;
  if (p <= ECLQR_NT) {
    double vn = 0.0, tn = 0.0;
    if (rho > 0) {
      vn = (1 + lane < p) ? lg[L.V + 1 + lane] : 0.0;
      tn = lg[L.tau];
    }
    for (int j = 0; j < rho; ++j) {
      const int row = j + 1 + lane;
      const double vj = vn, tj = tn;
      if (j + 1 < rho) {
        const int rn = row + 1;
        vn = (rn < p) ? lg[L.V + (int64_t)(j + 1) * P + rn] : 0.0;
        tn = lg[L.tau + j + 1];
      }
      double part = 0.0;
      if (row < p) part = fma(vj, o[row], part);
      const double w = (o[j] + wave_sum(part)) * tj;
      lds_sync();
      if (lane == 0) o[j] -= w;
      if (row < p) o[row] = fma(-w, vj, o[row]);
      lds_sync();
    }
    return;
  }
  for (int j = 0; j < rho; ++j) {
    const double* v = lg + L.V + (int64_t)j * P;
    double part = 0.0;
    for (int row = j + 1 + lane; row < p; row += ECLQR_NT) part = fma(v[row], o[row], part);
    const double w = (o[j] + wave_sum(part)) * lg[L.tau + j];
    lds_sync();
    if (lane == 0) o[j] -= w;
    for (int row = j + 1 + lane; row < p; row += ECLQR_NT) o[row] = fma(-w, v[row], o[row]);
    lds_sync();
  }
}

__device__ inline void rel_replay(double* o, const double* lg, const RelLog& L, int P, int R, int C, bool scaled,
                                  int* rho_out, int* rr_out) {
  const RelHdr h = rel_header(lg, P, R, C);
  const int p = h.p, rho = h.rho, rr = h.rr;
  if (scaled) {
    for (int r = ECLQR_TID; r < p; r += ECLQR_NT) o[r] *= lg[L.scale + r];
    lds_sync();
  }
  apply_reflectors(o, lg, L, P, p, rho);
  for (int sel = 0; sel < rr; ++sel) {
    const double* rec = lg + L.gs + (int64_t)sel * L.step;
    const int base = rho + sel;
    int best = (int)rec[0];
    best = (best < base || best >= p) ? base : best;
    if (best != base) {
      if (ECLQR_TID == 0) {
        const double a = o[base];
        o[base] = o[best];
        o[best] = a;
      }
      lds_sync();
    }
    double part = 0.0;
    for (int l = ECLQR_TID; l < sel; l += ECLQR_NT) part = fma(rec[2 + l], o[rho + l], part);
    const double nbv = (o[base] - wave_sum(part)) * rec[1];
    lds_sync();
    if (ECLQR_TID == 0) o[base] = nbv;
    for (int row = base + 1 + ECLQR_TID; row < p; row += ECLQR_NT) o[row] = fma(-rec[2 + C + row], nbv, o[row]);
    lds_sync();
  }
  *rho_out = rho;
  *rr_out = rr;
}

// Replay of the register-resident factorization's log: the reflectors as
// above, then the phase-2 records with the remaining rows' offsets held one
// per lane (q <= 64) and the chosen rows' offsets in selection order.
__device__ inline void rel_replay_reg(double* o, const double* lg, const RelLog& L, int P, int R, int C, int* rho_out,
                                      int* rr_out) {
  const int lane = ECLQR_TID;
  const RelHdr h = rel_header(lg, P, R, C);
  const int p = h.p, rho = h.rho;
  int q = p - rho;
  q = (q > 64) ? 64 : q;
  int rr = h.rr;
  rr = (rr > q) ? q : rr;
  rr = (rr > 64) ? 64 : rr;
  apply_reflectors(o, lg, L, P, p, rho);
  double v = (lane < q) ? o[rho + lane] : 0.0;
  bool chosen = lane >= q;
  double qoff = 0.0;
  // each record (pivot, 1 / norm, coefficients on the chosen rows, on the
  // remaining rows) is loaded one step ahead
  auto load = [&](int sel, double& r0, double& r1, double& ra, double& rb) {
    const double* rec = lg + L.gs + (int64_t)sel * L.step;
    r0 = rec[0];
    r1 = rec[1];
    ra = (lane < sel) ? rec[2 + lane] : 0.0;
    rb = (lane < q) ? rec[2 + C + lane] : 0.0;
  };
  double n0 = 0.0, n1 = 0.0, na = 0.0, nb = 0.0;
  if (rr > 0) load(0, n0, n1, na, nb);
  for (int sel = 0; sel < rr; ++sel) {
    const double r0 = n0, r1 = n1, ra = na, rb = nb;
    if (sel + 1 < rr) load(sel + 1, n0, n1, na, nb);
    int piv = (int)r0;
    piv = (piv < 0 || piv >= q) ? 0 : piv;
    const double vp = wave_bcast(v, piv);
    const double part = (lane < sel) ? ra * qoff : 0.0;
    const double nv = (vp - wave_sum(part)) * r1;
    if (lane == sel) qoff = nv;
    if (lane == piv) chosen = true;
    if (!chosen) v = fma(-rb, nv, v);
  }
  lds_sync();
  if (lane < rr) o[rho + lane] = qoff;
  lds_sync();
  *rho_out = rho;
  *rr_out = rr;
}

}  // namespace

// ---------------------------------------------------------------------------
// Logs of at most logcap doubles are staged in LDS before the replay.
__global__ void __launch_bounds__(kBlock) k_base_relation_vec(DevEngine e, Inputs in, int64_t logcap) {
  if (none_live(e)) return;
  __shared__ double o[kMaxRows];
  extern __shared__ double lgs[];
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const int slot = st.elem[SCAN_REL];
    const int cap = e.slot_cap[slot];
    const double* g = in.f[IN_g] + st.in[IN_g];
    const int P = st.terminal ? k : np + k;
    const int R = st.terminal ? 0 : ((m < P) ? m : P);
    const RelLog L = rel_log_layout(P, R, cap);
    const double* lg = e.rel_log + e.rel_log_off[slot];
    if (L.size <= logcap) {
      stage_rel_log(lgs, lg, L, P, cap, rel_header(lg, P, R, cap), true);
      lg = lgs;
    }
    if (st.terminal) {
      for (int r = ECLQR_TID; r < k; r += ECLQR_NT) o[r] = g[r];
    } else {
      const double* cv = in.f[IN_c] + st.in[IN_c];
      for (int r = ECLQR_TID; r < P; r += ECLQR_NT) o[r] = (r < np) ? cv[r] : g[r - np];
    }
    lds_sync();
    int rho = 0, rr = 0;
    rel_replay(o, lg, L, P, R, cap, true, &rho, &rr);
    const int lo = st.terminal ? n + 1 : n + np + 1;
    double* out = slot_ptr(e, SCAN_REL, slot);
    for (int r = ECLQR_TID; r < rr; r += ECLQR_NT) out[r * lo + lo - 1] = o[rho + r];
    lds_sync();
  }
}

// Vector replay of the composition task `task` (absolute index into the task
// list).  o: LDS offsets of kMaxRows; lgs: LDS for a staged log (logcap
// doubles, 0 = read in place).
__device__ inline void rel_compose_vec_task(const DevEngine& e, int64_t task, int64_t logcap, double* o, double* lgs) {
  const int a = e.tasks[3 * task];
  const int bsl = e.tasks[3 * task + 1];
  const int oo = e.tasks[3 * task + 2];
  const int sa = slot_a(e, 0, a), sb = slot_b(e, 0, a), sc = slot_b(e, 0, bsl);
  if (gated(e, e.st[sa].inst)) return;
  const int na = e.st[sa].n, nb = e.st[sb].n, nc = (sc >= 0) ? e.st[sc].n : 0;
  const int ra = e.slot_rows[a], rb = e.slot_rows[bsl];
  const int P = e.slot_cap[a] + e.slot_cap[bsl];
  if (ra + rb > P || P > kMaxRows) return;
  const int cap = e.slot_cap[oo];
  const RelLog L = rel_log_layout(P, (nb < P) ? nb : P, cap);
  const double* lg = e.rel_log + e.rel_log_off[oo];
  const double* Ls = slot_ptr(e, SCAN_REL, a);
  const double* Rs = slot_ptr(e, SCAN_REL, bsl);
  const int lda = na + nb + 1, ldb = nb + nc + 1;
  if (lg[3] == 1.0) {
    // composition of two full-rank relations: offsets -(a*, c*)
    if (ra != na + nb || rb != nb + nc) return;
    const int lo = na + nc + 1;
    double* out = slot_ptr(e, SCAN_REL, oo);
    for (int r = ECLQR_TID; r < na + nc; r += ECLQR_NT) {
      const double x = (r < na) ? -lane_dot(Ls + r, lda, Ls + lda - 1, lda, ra)
                                : -lane_dot(Rs + nb + (r - na), ldb, Rs + ldb - 1, ldb, rb);
      out[r * lo + lo - 1] = -x;
    }
    wg_sync();
    return;
  }
  const bool regfmt = lg[3] == 2.0;
  const int R = (nb < P) ? nb : P;
  if (L.size <= logcap) {
    stage_rel_log(lgs, lg, L, P, cap, rel_header(lg, P, R, cap), false);
    lg = lgs;
  }
  for (int r = ECLQR_TID; r < ra + rb; r += ECLQR_NT)
    o[r] = (r < ra) ? Ls[r * lda + na + nb] : Rs[(r - ra) * ldb + nb + nc];
  lds_sync();
  int rho = 0, rr = 0;
  if (regfmt) rel_replay_reg(o, lg, L, P, R, cap, &rho, &rr);
  else rel_replay(o, lg, L, P, R, cap, false, &rho, &rr);
  if (rr > e.slot_rows[oo]) rr = e.slot_rows[oo];
  const int lo = na + nc + 1;
  double* out = slot_ptr(e, SCAN_REL, oo);
  for (int r = ECLQR_TID; r < rr; r += ECLQR_NT) out[r * lo + lo - 1] = o[rho + r];
  lds_sync();
}

__global__ void __launch_bounds__(kBlock) k_rel_compose_vec(DevEngine e, int64_t first, int64_t ntasks, int64_t logcap) {
  if (none_live(e)) return;
  __shared__ double o[kMaxRows];
  extern __shared__ double lgs[];
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) rel_compose_vec_task(e, first + ti, logcap, o, lgs);
}

// t = -H' h; on stage 0, z_0 = T'(x0 - t).
__global__ void __launch_bounds__(kBlock) k_domain_vec(DevEngine e, Inputs in) {
  if (none_live(e)) return;
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n;
    const int suf = st.suf[SCAN_REL];
    const int r = e.slot_rows[suf];
    const double* H = slot_ptr(e, SCAN_REL, suf);
    const Arena ar = arena_layout(st.n, st.np, st.m, st.k);
    double* base = e.arena + st.ws;
    double* tv = base + ar.t;
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double v = 0.0;
      v = lane_chain<false>(v, H + i, (n + 1), H + n, (n + 1), r);
      tv[i] = -v;
    }
    wg_sync();
    if (st.i == 0) {
      const int nb = e.nbar[s];
      const double* T = base + ar.T;
      const double* x0 = in.x0 + st.x0;
      double* z0 = slot_ptr(e, SCAN_FWD, st.suf[SCAN_FWD]);
      for (int j = ECLQR_TID; j < nb; j += ECLQR_NT) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) v = fma(T[i * nb + j], x0[i] - tv[i], v);
        z0[j] = v;
      }
      wg_sync();
    }
  }
}

// Vector part of the stage elimination and of the value-function element.
__global__ void __launch_bounds__(kBlock) k_eliminate_vec(DevEngine e, Inputs in) {
  if (none_live(e)) return;
  __shared__ double tvs[kMaxDim], gam[2 * kMaxDim], yv[kMaxDim], atc[kMaxDim], cvv[kMaxDim], wv[kMaxDim],
      qt[kMaxDim], rz[kMaxDim], sv[kMaxDim];
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const Arena ar = arena_layout(n, np, m, k);
    double* base = e.arena + st.ws;
    const int nb = e.nbar[s];
    const double* T = base + ar.T;
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* qv = in.f[IN_q] + st.in[IN_q];
    double* ric = slot_ptr(e, SCAN_RIC, st.elem[SCAN_RIC]);
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) tvs[i] = base[ar.t + i];
    wg_sync();
    // Q t + q
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double a = qv[i];
      a = lane_chain<false>(a, Q + i * n, 1, tvs, 1, n);
      qt[i] = a;
    }
    wg_sync();
    if (st.terminal) {
      const RicLayout rl = ric_layout(n, 0);
      double* qb = base + ar.qb;
      for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
        double a = 0.0;
        a = lane_chain<false>(a, T + i, nb, qt, 1, n);
        qb[i] = a;
        ric[rl.eta + i] = -a;
      }
      wg_sync();
      continue;
    }
    const StageInfo& st1 = e.st[s + 1];
    const Arena ar1 = arena_layout(st1.n, st1.np, st1.m, st1.k);
    const double* T1 = e.arena + st1.ws + ar1.T;
    const double* t1 = e.arena + st1.ws + ar1.t;
    const int nb1 = e.nbar[s + 1];
    const int suf1 = st1.suf[SCAN_REL];
    const int r1 = e.slot_rows[suf1];
    const double* H1 = slot_ptr(e, SCAN_REL, suf1);
    const int ldh = np + 1;
    const double* A = in.f[IN_A] + st.in[IN_A];
    const double* B = in.f[IN_B] + st.in[IN_B];
    const double* cv = in.f[IN_c] + st.in[IN_c];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* g = in.f[IN_g] + st.in[IN_g];
    const double* R = in.f[IN_R] + st.in[IN_R];
    const double* Mm = in.f[IN_M] ? in.f[IN_M] + st.in[IN_M] : nullptr;
    const double* rv = in.f[IN_r] + st.in[IN_r];
    const int q = k + r1;
    const int mb = e.mbar[s];
    const int rho = m - mb;
    // gamma = rows-scaled [E t + g; H'(A t + c) + h']
    for (int i = ECLQR_TID; i < np; i += ECLQR_NT) {
      double a = cv[i];
      a = lane_chain<false>(a, A + i * n, 1, tvs, 1, n);
      atc[i] = a;
    }
    wg_sync();
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) {
      double a;
      if (j < k) {
        a = g[j];
        a = lane_chain<false>(a, E + j * n, 1, tvs, 1, n);
      } else {
        const int jj = j - k;
        a = H1[jj * ldh + np];
        a = lane_chain<false>(a, H1 + jj * ldh, 1, atc, 1, np);
      }
      gam[j] = a * base[ar.rsc + j];
    }
    wg_sync();
    // y = -Q1 R11^{-T} (P' gamma)_{1:rho}
    double xv = 0.0;
    if (ECLQR_TID < rho) {
      int pj = (int)base[ar.prm + ECLQR_TID];
      pj = (pj < 0 || pj >= q) ? 0 : pj;
      xv = gam[pj];
    }
    xv = lane_trsv_upper_t(base + ar.R11, rho, xv, rho);
    if (ECLQR_TID < rho) sv[ECLQR_TID] = xv;
    wg_sync();
    double* y = base + ar.y;
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double a = 0.0;
      a = lane_chain<false>(a, base + ar.Q1 + i * rho, 1, sv, 1, rho);
      y[i] = -a;
      yv[i] = -a;
    }
    wg_sync();
    // c-bar = T1'(A t + B y + c - t1)
    for (int i = ECLQR_TID; i < np; i += ECLQR_NT) {
      double a = atc[i] - t1[i];
      a = lane_chain<false>(a, B + i * m, 1, yv, 1, m);
      cvv[i] = a;
    }
    // rz = r + M' t ; w = rz + R y
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double a = rv[i];
      if (Mm)
        a = lane_chain<false>(a, Mm + i, m, tvs, 1, n);
      rz[i] = a;
      double b = a;
      b = lane_chain<false>(b, R + i * m, 1, yv, 1, m);
      wv[i] = b;
    }
    // (Q t + q) + M y, reused for q-bar
    if (Mm) {
      wg_sync();
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
        double a = qt[i];
        a = lane_chain<false>(a, Mm + i * m, 1, yv, 1, m);
        qt[i] = a;
      }
    }
    wg_sync();
    double* cb = base + ar.cb;
    double* qb = base + ar.qb;
    double* rb = base + ar.rb;
    const double* Y = base + ar.Y;
    const double* Z = base + ar.Z;
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double a = 0.0;
      a = lane_chain<false>(a, T1 + i, nb1, cvv, 1, np);
      cb[i] = a;
    }
    for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
      double a = 0.0;
      a = lane_chain<false>(a, T + i, nb, qt, 1, n);
      a = lane_chain<false>(a, Y + i, nb, wv, 1, m);
      qb[i] = a;
    }
    double rbl = 0.0;
    if (ECLQR_TID < mb) {
      rbl = lane_chain<false>(rbl, Z + ECLQR_TID, mb, wv, 1, m);
      rb[ECLQR_TID] = rbl;
    }
    // element: s = R-bar^{-1} r-bar, b_e = c-bar - B-bar s, eta_e = -(q-bar - M-bar s)
    double sl = lane_trsv_lower(base + ar.Lc, mb, rbl, mb);
    sl = lane_trsv_lower_t(base + ar.Lc, mb, sl, mb);
    if (ECLQR_TID < mb) sv[ECLQR_TID] = sl;
    wg_sync();
    const RicLayout rl = ric_layout(n, np);
    const double* Bb = base + ar.Bb;
    const double* Mb = base + ar.Mb;
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double a = cb[i];
      a = lane_chain<true>(a, Bb + i * mb, 1, sv, 1, mb);
      ric[rl.b + i] = a;
    }
    for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
      double a = qb[i];
      a = lane_chain<true>(a, Mb + i * mb, 1, sv, 1, mb);
      ric[rl.eta + i] = -a;
    }
    wg_sync();
  }
}

// b, eta of the value-function combine `task` from its logged factors.
// rs (maxd): [log: 4 + 2 maxd^2 + maxd | A1: maxd^2 | A2: maxd^2] in LDS; the
// factored form reads its factors and both A blocks from there (maxd = 0:
// read in place).  v1, v2, v3, piv: LDS vectors of kMaxDim.
__device__ inline void ric_combine_vec_task(const DevEngine& e, int64_t task, int maxd, double* v1, double* v2,
                                            double* v3, int* piv, double* rs) {
  const int a = e.tasks[3 * task];
  const int bsl = e.tasks[3 * task + 1];
  const int o = e.tasks[3 * task + 2];
  const int sa = slot_a(e, 0, a), sm = slot_b(e, 0, a), se = slot_b(e, 0, bsl);
  if (gated(e, e.st[sa].inst)) return;
  const int ds = e.nbar[sa], dm = e.nbar[sm], de = (se >= 0) ? e.nbar[se] : 0;
  const int ns = e.st[sa].n, nm = e.st[sm].n, ne = (se >= 0) ? e.st[se].n : 0;
  const RicLayout l1 = ric_layout(ns, nm), l2 = ric_layout(nm, ne), lo = ric_layout(ns, ne);
  const double* E1 = slot_ptr(e, SCAN_RIC, a);
  const double* E2 = slot_ptr(e, SCAN_RIC, bsl);
  double* Eo = slot_ptr(e, SCAN_RIC, o);
  const double *A1 = E1 + l1.A, *b1 = E1 + l1.b, *C1 = E1 + l1.C, *et1 = E1 + l1.eta;
  const double *A2 = E2 + l2.A, *b2 = E2 + l2.b, *et2 = E2 + l2.eta, *J2 = E2 + l2.J;
  const double* rlog = e.ric_log + e.ric_log_off[o];
  const bool binary = se >= 0;
  const bool factored = (dm > 0) && (rlog[0] == 1.0);
  if (factored && dm <= maxd && ds <= maxd && de <= maxd) {
    const int64_t lsz = 4 + 2 * (int64_t)maxd * maxd + maxd;
    double* A1s = rs + lsz;
    double* A2s = A1s + (int64_t)maxd * maxd;
    stage_ranges(rs, rlog, 0, 1, 4 + 2 * dm * dm);
    stage_ranges(A1s, A1, 0, 1, dm * ds);
    if (binary) stage_ranges(A2s, A2, 0, 1, de * dm);
    lds_sync();
    rlog = rs;
    A1 = A1s;
    A2 = A2s;
  }
  if (factored) {
    const double* Lj = rlog + 4;
    const double* Rg = rlog + 4 + (int64_t)dm * dm;
    // xi = L^{-1} eta2 ; d = G^{-1}(xi - L'b1) ; eta = eta1 + A1' L d ; b = A2 L^{-T}(xi - d) + b2
    // (with the log in global memory each solve preloads its operand rows)
    double xi = (ECLQR_TID < dm) ? et2[ECLQR_TID] : 0.0;
    xi = lane_trsv_lower_any(Lj, dm, xi, dm);
    double tvv = xi;
    if (ECLQR_TID < dm) tvv = lane_chain<true>(tvv, Lj + ECLQR_TID * dm + ECLQR_TID, dm, b1 + ECLQR_TID, 1, dm - ECLQR_TID);
    tvv = lane_trsv_lower_any(Rg, dm, tvv, dm);
    tvv = lane_trsv_lower_t_any(Rg, dm, tvv, dm);
    if (ECLQR_TID < dm) v1[ECLQR_TID] = tvv;
    lds_sync();
    if (ECLQR_TID < dm) v2[ECLQR_TID] = lane_chain<false>(0.0, Lj + ECLQR_TID * dm, 1, v1, 1, ECLQR_TID + 1);
    lds_sync();
    for (int i = ECLQR_TID; i < ds; i += ECLQR_NT) {
      double v = et1[i];
      v = lane_chain<false>(v, A1 + i, ds, v2, 1, dm);
      Eo[lo.eta + i] = v;
    }
    if (binary) {
      double yl = lane_trsv_lower_t_any(Lj, dm, xi - tvv, dm);
      if (ECLQR_TID < dm) v3[ECLQR_TID] = yl;
      lds_sync();
      for (int i = ECLQR_TID; i < de; i += ECLQR_NT) {
        double v = b2[i];
        v = lane_chain<false>(v, A2 + i * dm, 1, v3, 1, dm);
        Eo[lo.b + i] = v;
      }
    }
    lds_sync();
    return;
  }
  // LU form: eta = A1' Minv'(eta2 - J2 b1) + eta1 ; b = A2 Minv (b1 + C1 eta2) + b2
  const double* LU = rlog + 4;
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) {
    piv[i] = (int)rlog[4 + 2 * (int64_t)dm * dm + i];
    double v = et2[i];
    v = lane_chain<true>(v, J2 + i * dm, 1, b1, 1, dm);
    v1[i] = v;
    double w = b1[i];
    w = lane_chain<false>(w, C1 + i * dm, 1, et2, 1, dm);
    v3[i] = w;
  }
  lds_sync();
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) piv[i] = (piv[i] < i || piv[i] >= dm) ? i : piv[i];
  lds_sync();
  wg_lu_solve_t(LU, dm, dm, piv, v1, 1, 1);
  for (int i = ECLQR_TID; i < ds; i += ECLQR_NT) {
    double v = et1[i];
    v = lane_chain<false>(v, A1 + i, ds, v1, 1, dm);
    Eo[lo.eta + i] = v;
  }
  if (binary) {
    wg_lu_solve(LU, dm, dm, piv, v3, 1, 1);
    for (int i = ECLQR_TID; i < de; i += ECLQR_NT) {
      double v = b2[i];
      v = lane_chain<false>(v, A2 + i * dm, 1, v3, 1, dm);
      Eo[lo.b + i] = v;
    }
  }
  lds_sync();
}

__global__ void __launch_bounds__(kBlock) k_ric_combine_vec(DevEngine e, int64_t first, int64_t ntasks, int maxd) {
  if (none_live(e)) return;
  __shared__ double v1[kMaxDim], v2[kMaxDim], v3[kMaxDim];
  __shared__ int piv[kMaxDim];
  extern __shared__ double rs[];
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) ric_combine_vec_task(e, first + ti, maxd, v1, v2, v3, piv, rs);
}

// k = -H_uu^{-1} h_u from the logged Cholesky factor; forward leaf vector.
__global__ void __launch_bounds__(kBlock) k_gains_vec(DevEngine e) {
  if (none_live(e)) return;
  __shared__ double pc[kMaxDim], kv[kMaxDim];
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (st.terminal || gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m;
    const Arena ar = arena_layout(n, np, m, st.k);
    double* base = e.arena + st.ws;
    const int nb1 = e.nbar[s + 1], mb = e.mbar[s];
    const StageInfo& st1 = e.st[s + 1];
    const RicLayout l1 = ric_layout(st1.n, 0);
    const double* P1 = slot_ptr(e, SCAN_RIC, st1.suf[SCAN_RIC]) + l1.J;
    const double* et1 = slot_ptr(e, SCAN_RIC, st1.suf[SCAN_RIC]) + l1.eta;
    const double *Bb = base + ar.Bb, *cb = base + ar.cb, *rb = base + ar.rb;
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double v = -et1[i];
      v = lane_chain<false>(v, P1 + i * nb1, 1, cb, 1, nb1);
      pc[i] = v;
    }
    lds_sync();
    double hu = 0.0;
    if (ECLQR_TID < mb) {
      hu = rb[ECLQR_TID];
      hu = lane_chain<false>(hu, Bb + ECLQR_TID, mb, pc, 1, nb1);
    }
    hu = lane_trsv_lower(base + ar.Hc, mb, hu, mb);
    hu = lane_trsv_lower_t(base + ar.Hc, mb, hu, mb);
    if (ECLQR_TID < mb) {
      kv[ECLQR_TID] = -hu;
      base[ar.kk + ECLQR_TID] = -hu;
    }
    lds_sync();
    double* fs = slot_ptr(e, SCAN_FWD, st.elem[SCAN_FWD]) + (int64_t)np * n;
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double v = cb[i];
      v = lane_chain<false>(v, Bb + i * mb, 1, kv, 1, mb);
      fs[i] = v;
    }
    lds_sync();
  }
}

// f = F1 f2 + f1 of the forward-map composition `task` (F = F1 F2 is unchanged).
__device__ inline void fwd_combine_vec_task(const DevEngine& e, int64_t task) {
  const int a = e.tasks[3 * task];
  const int bsl = e.tasks[3 * task + 1];
  const int o = e.tasks[3 * task + 2];
  const int so = slot_a(e, 1, a), smid = slot_b(e, 1, a), sin_ = slot_b(e, 1, bsl);
  if (gated(e, e.st[so].inst)) return;
  const int dout = e.nbar[so], dmid = e.nbar[smid];
  const int nout = e.st[so].n, nmid = e.st[smid].n, nin = (sin_ >= 0) ? e.st[sin_].n : 0;
  const double* F1 = slot_ptr(e, SCAN_FWD, a);
  const double* f1 = F1 + (int64_t)nout * nmid;
  const double* F2 = slot_ptr(e, SCAN_FWD, bsl);
  const double* f2 = F2 + (int64_t)nmid * nin;
  double* Fo = slot_ptr(e, SCAN_FWD, o);
  double* fo = Fo + (int64_t)nout * nin;
  for (int i = ECLQR_TID; i < dout; i += ECLQR_NT) {
    double v = f1[i];
    v = lane_chain<false>(v, F1 + i * dmid, 1, f2, 1, dmid);
    fo[i] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_fwd_combine_vec(DevEngine e, int64_t first, int64_t ntasks) {
  if (none_live(e)) return;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) fwd_combine_vec_task(e, first + ti);
}

// ---------------------------------------------------------------------------
// Persistent scan kernels.  Tasks are taken in level order from a counter, so
// every task a workgroup waits for was taken earlier by a running workgroup
// whose own dependencies were taken earlier still: the waits end without any
// co-residency assumption.  A finished task publishes its slot with an
// agent-scope release (fence, then the level's done counter); a waiting
// workgroup reads the counters with agent-scope acquire loads.

// Waits until done >= target.  false when the wall clock passed the bound
// (the workgroup then sets *abort) or another workgroup aborted.
__device__ inline bool wait_count(const int32_t* done, int32_t target, int32_t* abort, int64_t ticks) {
  const int64_t t0 = wall_clock64();
  while (__hip_atomic_load(done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > ticks) {
      atomicOr(abort, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  return true;
}

template <int kKind>
__global__ void __launch_bounds__(kBlock) k_scan_vec(DevEngine e, ScanLevels lv, int32_t* ctrl, int32_t* abort,
                                                     int64_t ticks) {
  if (none_live(e)) return;
  __shared__ double o[kKind == SCAN_REL ? kMaxRows : 1];
  __shared__ double v1[kMaxDim], v2[kMaxDim], v3[kMaxDim];
  __shared__ int piv[kMaxDim];
  const int64_t first = lv.begin[0];
  const int64_t total = lv.begin[lv.n - 1] + lv.count[lv.n - 1] - first;
  for (;;) {
    int t = 0;
    if (threadIdx.x == 0) t = atomicAdd(ctrl, 1);
    t = wave_bcast_i(t, 0);
    if (t >= total) return;
    const int64_t task = first + t;
    int l = 0;
    while (l + 1 < lv.n && task >= lv.begin[l + 1]) ++l;
    for (int j = 0; j < l; ++j)
      if (!wait_count(ctrl + 1 + j, (int32_t)lv.count[j], abort, ticks)) return;
    if constexpr (kKind == SCAN_REL) rel_compose_vec_task(e, task, 0, o, nullptr);
    else if constexpr (kKind == SCAN_RIC) ric_combine_vec_task(e, task, 0, v1, v2, v3, piv, nullptr);
    else fwd_combine_vec_task(e, task);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(ctrl + 1 + l, 1);
  }
}

__global__ void k_apply_abort(int32_t* status, const int32_t* abort, int32_t bit, int32_t B) {
  if (*abort == 0) return;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) status[b] |= bit;
}

// ---------------------------------------------------------------------------
static unsigned grid_of(const DevEngine& e, int64_t ntasks) {
  return (unsigned)((ntasks < e.nblocks) ? ntasks : e.nblocks);
}

// Largest dynamic LDS (bytes) of each replay kernel: the device limit less the
// kernel's static LDS (the attribute cannot exceed that difference).
static int g_dyn_base = 65536 - 4096, g_dyn_compose = 65536 - 4096, g_dyn_ric = 65536 - 4096;
static int set_dyn_limit(const void* fn, int device_bytes) {
  hipFuncAttributes a{};
  int stat = 4096;
  if (hipFuncGetAttributes(&a, fn) == hipSuccess) stat = (int)a.sharedSizeBytes;
  const int dyn = device_bytes - stat;
  if (dyn > 0 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) == hipSuccess) return dyn;
  (void)hipGetLastError();
  return 65536 - stat > 0 ? 65536 - stat : 0;
}
void replay_set_max_lds(int bytes) {
  g_dyn_base = set_dyn_limit(reinterpret_cast<const void*>(k_base_relation_vec), bytes);
  g_dyn_compose = set_dyn_limit(reinterpret_cast<const void*>(k_rel_compose_vec), bytes);
  g_dyn_ric = set_dyn_limit(reinterpret_cast<const void*>(k_ric_combine_vec), bytes);
}
// Staging a log pays off for latency-bound launches (at most kStageTasks
// tasks: a few per compute unit) and up to 24 KiB per workgroup; on wider
// launches, or beyond that size, the lost occupancy costs more than the
// faster accesses save, so logs are read in place.
constexpr int64_t kStageCapBytes = 24 * 1024;
constexpr int64_t kStageTasks = 1024;
// doubles of dynamic LDS for a staged relation log
static int64_t rel_logcap(int64_t want, int dyn_bytes) {
  int64_t room = (int64_t)dyn_bytes / (int64_t)sizeof(double);
  if (room > kStageCapBytes / (int64_t)sizeof(double)) room = kStageCapBytes / (int64_t)sizeof(double);
  return want < room ? want : (room > 0 ? room : 0);
}
void launch_base_relation_vec(const DevEngine& e, const Inputs& in, int64_t logmax, hipStream_t s) {
  const int64_t cap = (e.S <= kStageTasks) ? rel_logcap(logmax, g_dyn_base) : 0;
  hipLaunchKernelGGL(k_base_relation_vec, dim3(e.nblocks), dim3(kBlock), sizeof(double) * cap, s, e, in, cap);
}
void launch_rel_compose_vec(const DevEngine& e, int64_t first, int64_t ntasks, int64_t logmax, hipStream_t s) {
  const int64_t cap = (ntasks <= kStageTasks) ? rel_logcap(logmax, g_dyn_compose) : 0;
  if (ntasks > 0)
    hipLaunchKernelGGL(k_rel_compose_vec, dim3(grid_of(e, ntasks)), dim3(kBlock), sizeof(double) * cap, s, e, first,
                       ntasks, cap);
}
void launch_domain_vec(const DevEngine& e, const Inputs& in, hipStream_t s) {
  hipLaunchKernelGGL(k_domain_vec, dim3(e.nblocks), dim3(kBlock), 0, s, e, in);
}
void launch_eliminate_vec(const DevEngine& e, const Inputs& in, hipStream_t s) {
  hipLaunchKernelGGL(k_eliminate_vec, dim3(e.nblocks), dim3(kBlock), 0, s, e, in);
}
void launch_ric_combine_vec(const DevEngine& e, int64_t first, int64_t ntasks, int maxd, hipStream_t s) {
  // staged factors need (4 + 2 d^2 + d) + 2 d^2 doubles; larger levels read them in place
  int d = (ntasks <= kStageTasks) ? maxd : 0;
  while (d > 0 && ((int64_t)sizeof(double) * (4 + 4 * (int64_t)d * d + d) > (int64_t)g_dyn_ric ||
                   (int64_t)sizeof(double) * (4 + 4 * (int64_t)d * d + d) > kStageCapBytes))
    --d;
  const size_t lds = d > 0 ? sizeof(double) * (4 + 4 * (size_t)d * d + d) : 0;
  if (ntasks > 0)
    hipLaunchKernelGGL(k_ric_combine_vec, dim3(grid_of(e, ntasks)), dim3(kBlock), lds, s, e, first, ntasks, d);
}
void launch_gains_vec(const DevEngine& e, hipStream_t s) {
  hipLaunchKernelGGL(k_gains_vec, dim3(e.nblocks), dim3(kBlock), 0, s, e);
}
void launch_fwd_combine_vec(const DevEngine& e, int64_t first, int64_t ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_fwd_combine_vec, dim3(grid_of(e, ntasks)), dim3(kBlock), 0, s, e, first, ntasks);
}

// Co-resident workgroups of each persistent scan kernel (occupancy times
// compute units) and the wall-clock bound of a wait (2 s).
static int g_scan_grid[SCAN_COUNT] = {1024, 1024, 1024};
static int64_t g_wait_ticks = 200000000;
template <int K>
static int resident(int num_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_scan_vec<K>), kBlock, 0) !=
          hipSuccess ||
      per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  return per_cu * num_cu;
}
void replay_set_device(int num_cu, int wall_clock_khz) {
  if (num_cu > 0) {
    g_scan_grid[SCAN_REL] = resident<SCAN_REL>(num_cu);
    g_scan_grid[SCAN_RIC] = resident<SCAN_RIC>(num_cu);
    g_scan_grid[SCAN_FWD] = resident<SCAN_FWD>(num_cu);
  }
  if (wall_clock_khz > 0) g_wait_ticks = (int64_t)wall_clock_khz * 2000;
}
void launch_scan_vec(const DevEngine& e, int kind, const ScanLevels& lv, int32_t* ctrl, int32_t* abort,
                     hipStream_t s) {
  if (lv.n <= 0) return;
  const int64_t total = lv.begin[lv.n - 1] + lv.count[lv.n - 1] - lv.begin[0];
  if (total <= 0) return;
  const unsigned grid = (unsigned)(total < g_scan_grid[kind] ? total : g_scan_grid[kind]);
  if (kind == SCAN_REL)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_vec<SCAN_REL>), dim3(grid), dim3(kBlock), 0, s, e, lv, ctrl, abort,
                       g_wait_ticks);
  else if (kind == SCAN_RIC)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_vec<SCAN_RIC>), dim3(grid), dim3(kBlock), 0, s, e, lv, ctrl, abort,
                       g_wait_ticks);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scan_vec<SCAN_FWD>), dim3(grid), dim3(kBlock), 0, s, e, lv, ctrl, abort,
                       g_wait_ticks);
}
void launch_apply_abort(int32_t* status, const int32_t* abort, int32_t bit, int32_t B, hipStream_t s) {
  const int grid = (B + 255) / 256;
  hipLaunchKernelGGL(k_apply_abort, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, status, abort, bit, B);
}

}  // namespace eclqr
