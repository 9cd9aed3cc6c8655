// Feasible-domain scan (paper Sections III-IV): input validation, base
// relations, relation composition, and the state parameterisation that turns
// each suffix relation into x_i = T_i z_i + t_i.
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "relreg.hpp"
#include "scratch.hpp"

namespace eclqr {

// ---------------------------------------------------------------------------
// NaN / Inf in any input block of a stage -> ECLQR_INVALID_INPUT.
__global__ void __launch_bounds__(kBlock) k_validate(DevEngine e, Inputs in, int32_t* status) {
  __shared__ int bad;
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo& st = e.st[s];
    if (gated(e, st.inst)) continue;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int64_t n = st.n, np = st.np, m = st.m, k = st.k;
    const int64_t sz[IN_COUNT] = {n * n, n, m * m, m, n * m, np * n, np * m, np, k * n, k * m, k};
    int mine = 0;
    for (int f = 0; f < IN_COUNT; ++f) {
      if (f == IN_M && in.f[IN_M] == nullptr) continue;
      const double* p = in.f[f] + st.in[f];
      for (int64_t j = threadIdx.x; j < sz[f]; j += blockDim.x)
        if (!isfinite(p[j])) mine = 1;
    }
    if (st.i == 0)
      for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
        if (!isfinite(in.x0[st.x0 + j])) mine = 1;
    if (mine) bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && bad) flag_at(e, status, st.inst, ECLQR_INVALID_INPUT, st.i);
    __syncthreads();
  }
}

// Divide each row of W (columns [0, ncoef) coefficients, column ncoef the
// offset) by the 2-norm of its coefficients (Section VIII item 1); returns
// max(1, max |offset|) of the scaled rows.
__device__ inline double scale_rows(double* W, int ld, int p, int ncoef, double* sh, double* scales) {
  for (int r = ECLQR_TID; r < p; r += ECLQR_NT) {
    double s = 0.0;
    s = lane_chain<false>(s, W + r * ld, 1, W + r * ld, 1, ncoef);
    const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 1.0;
    if (s > 0.0)
      for (int j = 0; j <= ncoef; ++j) W[r * ld + j] *= inv;
    scales[r] = inv;
  }
  wg_sync();
  double mx = 1.0;
  for (int r = ECLQR_TID; r < p; r += ECLQR_NT) mx = fmax(mx, fabs(W[r * ld + ncoef]));
  (void)sh;
  return wave_max(mx);
}

// The domain shortcut of Section VI.  X_i = R^{n_i} for every stage of an
// instance when it has no terminal rows and every F_i has full row rank: by
// induction from the terminal stage, if X_{i+1} is the whole space, stage i's
// rows E_i x + F_i u + g_i = 0 can be met by some u_i for every x_i, so the
// suffix relation of stage i has no rows.  Such an instance skips the
// relation scan (every relation of it is left empty: the suffixes, the only
// relations read after the scan, are exactly empty) and its domains are the
// whole spaces.  vac[b] starts at 1; a stage that fails the test stores 0.
// The test is stricter than the scan's rank decisions (pivots of the rows of
// F_i, each scaled by the norm of its whole row [F_i E_i g_i], above
// sqrt(rank_tol)), so an instance it accepts has no borderline row.
// LDS: W (maxk x (maxm | 1)) | tau | qr scratch | perm
__global__ void __launch_bounds__(kBlock) k_vacuous(DevEngine e, Inputs in, Tols t, int32_t* vac, int maxk,
                                                    int maxm) {
  extern __shared__ double lds[];
  const int ld = maxm | 1;
  double* W = lds;
  double* tau = W + (int64_t)maxk * ld;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + kMaxDim + 8);
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    const int n = st.n, m = st.terminal ? 0 : st.m, k = st.k;
    if (k == 0) continue;
    if (st.terminal || k > m) {
      if (ECLQR_TID == 0) vac[st.inst] = 0;
      continue;
    }
    if (vac[st.inst] == 0) continue;  // another stage already failed the test
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* F = in.f[IN_F] + st.in[IN_F];
    const double* g = in.f[IN_g] + st.in[IN_g];
    bool zero_row = false;  // a row with F = 0 (a state-only row) fails without a factorization
    for (int r = ECLQR_TID; r < k; r += ECLQR_NT) {
      double sf = 0.0, ss = g[r] * g[r];
      for (int j = 0; j < m; ++j) sf = fma(F[r * m + j], F[r * m + j], sf);
      for (int j = 0; j < n; ++j) ss = fma(E[r * n + j], E[r * n + j], ss);
      ss += sf;
      zero_row = zero_row || !(sf > 0.0);
      tau[r] = (ss > 0.0) ? 1.0 / sqrt(ss) : 0.0;
    }
    if (__ballot(zero_row) != 0) {
      if (ECLQR_TID == 0) vac[st.inst] = 0;
      lds_sync();
      continue;
    }
    lds_sync();
    for (int idx = ECLQR_TID; idx < k * m; idx += ECLQR_NT) {
      const int r = idx / m, j = idx - (idx / m) * m;
      W[r * ld + j] = F[idx] * tau[r];
    }
    lds_sync();
    const int rho = wg_qr_colpiv(W, ld, k, m, 0, m, sqrt(t.rank), tau, QRScratch{qd, perm});
    if (rho < k && ECLQR_TID == 0) vac[st.inst] = 0;
    lds_sync();
  }
}


// ---------------------------------------------------------------------------
// Base relation of stage i (eq. (base-system), (base-relation)):
//   [B; F] u + [[A, -I], [E, 0]] (x_i, x_{i+1}) + [c; g] = 0,
// u projected out with Lemma 1 by a column-pivoted Householder QR of the
// input columns; the remaining equations are replaced by an orthonormal row
// basis.  The terminal relation (eq. (terminal-relation)) is E_N x_N + g_N = 0.
// LDS: W (maxp x ldw) | tau (64) | qr scratch (64+8) | perm (64 ints) | rb scratch
// kGW: the stacked system in the workgroup's tile of global memory (e.gw)
// instead of LDS, for systems that outgrow the device's LDS; the small work
// arrays stay in LDS.
template <bool kGW>
__global__ void __launch_bounds__(kBlock) k_base_relation(DevEngine e, Inputs in, Tols t, int32_t* status, int maxp,
                                                          int ldw, int64_t first, int64_t count) {
  extern __shared__ double lds[];
  double* W = kGW ? e.gw + (int64_t)blockIdx.x * e.gw_stride : lds;
  double* tau = kGW ? lds : W + (int64_t)maxp * (ldw | 1);
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + kMaxDim + 8);
  double* rbs = (double*)(perm + kMaxDim);
  double* sh = rbs + 2 * maxp + 8 + 64;
  for (int64_t ti = blockIdx.x; ti < count; ti += gridDim.x) {
    const int64_t s = stage_at(e, first, ti);
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const int slot = st.elem[SCAN_REL];
    double* out = slot_ptr(e, SCAN_REL, slot);
    if (e.vac && e.vac[st.inst]) {  // whole-space domains: every relation of the instance is empty
      if (ECLQR_TID == 0) {
        double* glog = e.rel_log + e.rel_log_off[slot];
        glog[0] = glog[1] = glog[2] = glog[3] = 0.0;
        e.slot_rows[slot] = 0;
      }
      continue;
    }
    if (st.terminal) {
      const int p = k, ld = n + 1;
      const double* E = in.f[IN_E] + st.in[IN_E];
      const double* g = in.f[IN_g] + st.in[IN_g];
      for (int idx = ECLQR_TID; idx < p * ld; idx += ECLQR_NT) {
        const int r = idx / ld, j = idx % ld;
        W[r * ld + j] = (j < n) ? E[r * n + j] : g[r];
      }
      wg_sync();
      const int cap = e.slot_cap[slot];
      const RelLog lg = rel_log_layout(p, 0, cap);
      double* glog = e.rel_log + e.rel_log_off[slot];
      const double omax = scale_rows(W, ld, p, n, sh, glog + lg.scale);
      int b = 0;
      const int rr = wg_row_basis(W, ld, 0, p, 0, n, t.rank, t.cons * omax, &b, rbs, glog + lg.gs, lg.step, cap);
      for (int idx = ECLQR_TID; idx < rr * ld; idx += ECLQR_NT) out[idx] = W[idx];
      if (ECLQR_TID == 0) {
        glog[0] = p;
        glog[1] = 0;
        glog[2] = rr;
        glog[3] = 0;
        e.slot_rows[slot] = rr;
        if (b) flag_at(e, status, st.inst, ECLQR_INFEASIBLE_SUFFIX, st.i);
      }
      wg_sync();
      continue;
    }
    const int p = np + k;
    const int c = m + n + np + 1;
    const int ld = c | 1;  // odd: rows read one per lane hit distinct LDS banks
    const double* A = in.f[IN_A] + st.in[IN_A];
    const double* B = in.f[IN_B] + st.in[IN_B];
    const double* cv = in.f[IN_c] + st.in[IN_c];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* F = in.f[IN_F] + st.in[IN_F];
    const double* g = in.f[IN_g] + st.in[IN_g];
    for (int idx = ECLQR_TID; idx < p * c; idx += ECLQR_NT) {
      const int r = idx / c, j = idx % c;
      double v;
      if (r < np) {
        if (j < m) v = B[r * m + j];
        else if (j < m + n) v = A[r * n + (j - m)];
        else if (j < m + n + np) v = (j - m - n == r) ? -1.0 : 0.0;
        else v = cv[r];
      } else {
        const int q = r - np;
        if (j < m) v = F[q * m + j];
        else if (j < m + n) v = E[q * n + (j - m)];
        else if (j < m + n + np) v = 0.0;
        else v = g[q];
      }
      W[r * ld + j] = v;
    }
    wg_sync();
    const int cap = e.slot_cap[slot];
    const RelLog lg = rel_log_layout(p, (m < p) ? m : p, cap);
    double* glog = e.rel_log + e.rel_log_off[slot];
    const double omax = scale_rows(W, ld, p, c - 1, sh, glog + lg.scale);
    const int rho = wg_qr_colpiv(W, ld, p, c, 0, m, t.rank, tau, QRScratch{qd, perm});
    wg_log_reflectors(W, ld, p, 0, rho, tau, glog + lg.V, p, glog + lg.tau);
    int b = 0;
    const int rr =
        wg_row_basis(W, ld, rho, p, m, n + np, t.rank, t.cons * omax, &b, rbs, glog + lg.gs, lg.step, cap);
    const int lo = n + np + 1;
    for (int idx = ECLQR_TID; idx < rr * lo; idx += ECLQR_NT) {
      const int r = idx / lo, j = idx % lo;
      out[r * lo + j] = W[(rho + r) * ld + m + j];
    }
    if (ECLQR_TID == 0) {
      glog[0] = p;
      glog[1] = rho;
      glog[2] = rr;
      glog[3] = 0;
      e.slot_rows[slot] = rr;
      if (b) flag_at(e, status, st.inst, ECLQR_INFEASIBLE_SUFFIX, st.i);
    }
    wg_sync();
  }
}

// Composition of two full-rank relations (rows = endpoint dims, orthonormal
// coefficient rows, so the coefficient matrix is orthogonal): the endpoint
// values are -H' h.  Writes the point relation over (a, c) to out and sets
// *bad when the shared endpoint disagrees beyond cons * max(1, |values|).
// xs: LDS scratch of na + 2 nb + nc doubles.
__device__ inline void point_compose(const double* L, int lda, int ra, const double* Rr, int ldb, int rb, int na, int nb,
                                     int nc, double* xs, double cons, double* out, int* bad) {
  const int ldl = lda + 1, ldr = ldb + 1;
  double* xl = xs;            // (a*, b*) from the left relation
  double* xr = xs + lda;      // (b*, c*) from the right relation
  for (int i = ECLQR_TID; i < lda; i += ECLQR_NT) xl[i] = -lane_dot(L + i, ldl, L + lda, ldl, ra);
  for (int i = ECLQR_TID; i < ldb; i += ECLQR_NT) xr[i] = -lane_dot(Rr + i, ldr, Rr + ldb, ldr, rb);
  wg_sync();
  double dif = 0.0, sc = 1.0;
  for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
    dif = fmax(dif, fabs(xl[na + i] - xr[i]));
    sc = fmax(sc, fmax(fabs(xl[na + i]), fabs(xr[i])));
  }
  dif = wave_max(dif);
  sc = wave_max(sc);
  *bad = (dif > cons * sc) ? 1 : 0;
  const int lo = na + nc + 1;
  for (int idx = ECLQR_TID; idx < (na + nc) * lo; idx += ECLQR_NT) {
    const int r = idx / lo, j = idx - (idx / lo) * lo;
    double v;
    if (j < na + nc) v = (j == r) ? 1.0 : 0.0;
    else v = (r < na) ? -xl[r] : -xr[nb + (r - na)];
    out[idx] = v;
  }
  wg_sync();
}

// ---------------------------------------------------------------------------
// Composition R_ab o R_bc (eq. (composition-matrix)): stack
//   [R_ab | L_ab | 0    | l_ab]
//   [L_bc | 0    | R_bc | l_bc]
// over the columns (b | a | c | 1), eliminate b with Lemma 1 (pivoted
// Householder on the b columns) and keep an orthonormal row basis of the rest.
// A unary right operand (n_c = 0) gives a unary result.
template <bool kGW>
__global__ void __launch_bounds__(kBlock) k_rel_compose(DevEngine e, int64_t first, int64_t ntasks, Tols t,
                                                        int32_t* status, int maxp, int ldw) {
  extern __shared__ double lds[];
  double* W = kGW ? e.gw + (int64_t)blockIdx.x * e.gw_stride : lds;
  double* tau = kGW ? lds : W + (int64_t)maxp * (ldw | 1);
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + kMaxDim + 8);
  double* rbs = (double*)(perm + kMaxDim);
  double* sh = rbs + 2 * maxp + 8 + 64;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * (first + ti)];
    const int bsl = e.tasks[3 * (first + ti) + 1];
    const int o = e.tasks[3 * (first + ti) + 2];
    const int sa = slot_a(e, 0, a), sb = slot_b(e, 0, a), sc = slot_b(e, 0, bsl);
    if (gated(e, e.st[sa].inst)) continue;
    const int na = e.st[sa].n, nb = e.st[sb].n, nc = (sc >= 0) ? e.st[sc].n : 0;
    const int inst = e.st[sa].inst;
    int bad_full = 0;
    const int ra = e.slot_rows[a], rb = e.slot_rows[bsl];
    const int p = ra + rb;
    const int P = e.slot_cap[a] + e.slot_cap[bsl];
    const int cap = e.slot_cap[o];
    const RelLog lg = rel_log_layout(P, (nb < P) ? nb : P, cap);
    double* glog = e.rel_log + e.rel_log_off[o];
    if (p == 0) {  // no rows on either side: no rows in the composition
      if (ECLQR_TID == 0) {
        glog[0] = glog[1] = glog[2] = glog[3] = 0.0;
        e.slot_rows[o] = 0;
      }
      continue;
    }
    if (p > maxp || p > 2 * kMaxDim * 2) {
      if (ECLQR_TID == 0) {
        glog[0] = 0;
        glog[1] = 0;
        glog[2] = 0;
        glog[3] = 0;
        e.slot_rows[o] = 0;
        flag_at(e, status, inst, ECLQR_CAPACITY, e.st[sa].i);
      }
      wg_sync();
      continue;
    }
    const double* L = slot_ptr(e, SCAN_REL, a);
    const double* Rr = slot_ptr(e, SCAN_REL, bsl);
    if (ra == na + nb && rb == nb + nc && na + nc <= e.slot_cap[o]) {
      // Both relations have full rank: each pins its endpoints to one point,
      // (a*, b*) = -H_L' h_L and (b*, c*) = -H_R' h_R (orthonormal rows), the
      // two b* must agree, and the composition is the point relation
      // [I 0; 0 I](a, c) - (a*, c*) = 0.
      point_compose(L, na + nb, ra, Rr, nb + nc, rb, na, nb, nc, W, t.cons, slot_ptr(e, SCAN_REL, o), &bad_full);
      if (ECLQR_TID == 0) {
        glog[0] = 0;
        glog[1] = 0;
        glog[2] = na + nc;
        glog[3] = 1;
        e.slot_rows[o] = na + nc;
        if (bad_full) flag_at(e, status, inst, ECLQR_INFEASIBLE_SUFFIX, e.st[sa].i);
      }
      wg_sync();
      continue;
    }
    const int c = nb + na + nc + 1;
    const int ld = c | 1;  // odd: rows read one per lane hit distinct LDS banks
    const int lda = na + nb + 1, ldb = nb + nc + 1;
    for (int idx = ECLQR_TID; idx < p * c; idx += ECLQR_NT) {
      const int r = idx / c, j = idx % c;
      double v;
      if (r < ra) {
        if (j < nb) v = L[r * lda + na + j];
        else if (j < nb + na) v = L[r * lda + (j - nb)];
        else if (j < nb + na + nc) v = 0.0;
        else v = L[r * lda + na + nb];
      } else {
        const int q = r - ra;
        if (j < nb) v = Rr[q * ldb + j];
        else if (j < nb + na) v = 0.0;
        else if (j < nb + na + nc) v = Rr[q * ldb + nb + (j - nb - na)];
        else v = Rr[q * ldb + nb + nc];
      }
      W[r * ld + j] = v;
    }
    wg_sync();
    double mx = 1.0;
    for (int r = ECLQR_TID; r < p; r += ECLQR_NT) mx = fmax(mx, fabs(W[r * ld + c - 1]));
    const double omax = wave_max(mx);
    const int rho = wg_qr_colpiv(W, ld, p, c, 0, nb, t.rank, tau, QRScratch{qd, perm});
    wg_log_reflectors(W, ld, p, 0, rho, tau, glog + lg.V, P, glog + lg.tau);
    int bad = 0;
    const int rr =
        wg_row_basis(W, ld, rho, p, nb, na + nc, t.rank, t.cons * omax, &bad, rbs, glog + lg.gs, lg.step, cap);
    double* out = slot_ptr(e, SCAN_REL, o);
    const int lo = na + nc + 1;
    if (ECLQR_TID == 0) {
      glog[0] = p;
      glog[1] = rho;
      glog[2] = (rr > cap) ? 0 : rr;
      glog[3] = 0;
    }
    if (rr > cap) {
      if (ECLQR_TID == 0) {
        e.slot_rows[o] = 0;
        flag_at(e, status, inst, ECLQR_CAPACITY, e.st[sa].i);
      }
      wg_sync();
      continue;
    }
    for (int idx = ECLQR_TID; idx < rr * lo; idx += ECLQR_NT) {
      const int r = idx / lo, j = idx % lo;
      out[r * lo + j] = W[(rho + r) * ld + nb + j];
    }
    if (ECLQR_TID == 0) {
      e.slot_rows[o] = rr;
      if (bad) flag_at(e, status, inst, ECLQR_INFEASIBLE_SUFFIX, e.st[sa].i);
    }
    wg_sync();
  }
}


// ---------------------------------------------------------------------------
// The composition of k_rel_compose with the stacked system in registers
// (tasks with at most PR stacked rows, 64 NC columns and KC coefficient
// columns after the elimination).  Logs in the phase-2 replay format.
template <int PR, int NC, int KC>
__global__ void __launch_bounds__(kBlock) k_rel_compose_reg(DevEngine e, int64_t first, int64_t ntasks, Tols t,
                                                            int32_t* status) {
  constexpr int QROWS = (PR > KC) ? PR : KC;
  __shared__ double Qb[QROWS * (KC + 1)];
  __shared__ double vbuf[PR];
  __shared__ double vs[PR];
  __shared__ double pb[KC + 1];
  __shared__ double dots[KC];
  const int lane = ECLQR_TID;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * (first + ti)];
    const int bsl = e.tasks[3 * (first + ti) + 1];
    const int o = e.tasks[3 * (first + ti) + 2];
    const int sa = slot_a(e, 0, a), sb = slot_b(e, 0, a), sc = slot_b(e, 0, bsl);
    if (gated(e, e.st[sa].inst)) continue;
    const int na = e.st[sa].n, nb = e.st[sb].n, nc = (sc >= 0) ? e.st[sc].n : 0;
    const int inst = e.st[sa].inst;
    const int ra = e.slot_rows[a], rb = e.slot_rows[bsl];
    const int p = ra + rb;
    const int P = e.slot_cap[a] + e.slot_cap[bsl];
    const int cap = e.slot_cap[o];
    const RelLog lg = rel_log_layout(P, (nb < P) ? nb : P, cap);
    double* glog = e.rel_log + e.rel_log_off[o];
    const double* L = slot_ptr(e, SCAN_REL, a);
    const double* Rr = slot_ptr(e, SCAN_REL, bsl);
    double* out = slot_ptr(e, SCAN_REL, o);
    const int c = nb + na + nc + 1, kc = na + nc;
    if (p == 0) {  // no rows on either side: no rows in the composition
      if (lane == 0) {
        glog[0] = glog[1] = glog[2] = glog[3] = 0.0;
        e.slot_rows[o] = 0;
      }
      continue;
    }
    if (ra == na + nb && rb == nb + nc && kc <= cap) {
      int bad_full = 0;
      point_compose(L, na + nb, ra, Rr, nb + nc, rb, na, nb, nc, Qb, t.cons, out, &bad_full);
      if (lane == 0) {
        glog[0] = 0;
        glog[1] = 0;
        glog[2] = kc;
        glog[3] = 1;
        e.slot_rows[o] = kc;
        if (bad_full) flag_at(e, status, inst, ECLQR_INFEASIBLE_SUFFIX, e.st[sa].i);
      }
      lds_sync();
      continue;
    }
    if (p > PR || c > 64 * NC || kc > KC || cap > KC) {
      if (lane == 0) {
        glog[0] = 0;
        glog[1] = 0;
        glog[2] = 0;
        glog[3] = 0;
        e.slot_rows[o] = 0;
        flag_at(e, status, inst, ECLQR_CAPACITY, e.st[sa].i);
      }
      lds_sync();
      continue;
    }
    // stacked system over the columns (b | a | c | 1), one column per lane
    const int lda = na + nb + 1, ldb = nb + nc + 1;
    double col[NC][PR];
    double om = 0.0;
#pragma unroll
    for (int tt = 0; tt < NC; ++tt) {
      const int j = lane + 64 * tt;
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        double v = 0.0;
        if (r < p && j < c) {
          if (r < ra) {
            if (j < nb) v = L[r * lda + na + j];
            else if (j < nb + na) v = L[r * lda + (j - nb)];
            else if (j < nb + na + nc) v = 0.0;
            else v = L[r * lda + na + nb];
          } else {
            const int q = r - ra;
            if (j < nb) v = Rr[q * ldb + j];
            else if (j < nb + na) v = 0.0;
            else if (j < nb + na + nc) v = Rr[q * ldb + nb + (j - nb - na)];
            else v = Rr[q * ldb + nb + nc];
          }
        }
        col[tt][r] = v;
        if (j == c - 1) om = fmax(om, fabs(v));
      }
    }
    const double omax = fmax(1.0, wave_max(om));
    const int R = (nb < P) ? nb : P;
    const int rho = rr_phase1<PR, NC>(col, p, c, nb, t.rank, vbuf, vs, glog + lg.V, P, glog + lg.tau, R);
    // rows rho.. of the (a | c | 1) columns, one row per lane
    const int q = p - rho;
#pragma unroll
    for (int tt = 0; tt < NC; ++tt) {
      const int j = lane + 64 * tt;
      if (j >= nb && j < c) {
        const int k = (j == c - 1) ? KC : j - nb;
#pragma unroll
        for (int r = 0; r < PR; ++r)
          if (r >= rho && r < p) Qb[(r - rho) * (KC + 1) + k] = col[tt][r];
      }
    }
    for (int idx = lane; idx < q * (KC + 1); idx += 64) {
      const int k = idx % (KC + 1);
      if (k >= kc && k < KC) Qb[idx] = 0.0;
    }
    lds_sync();
    double row[KC];
    double off = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) row[k] = (lane < q) ? Qb[lane * (KC + 1) + k] : 0.0;
    if (lane < q) off = Qb[lane * (KC + 1) + KC];
    lds_sync();
    int bad = 0, over = 0;
    const int rr = rr_phase2<KC>(row, off, q, kc, t.rank, t.cons * omax, Qb, pb, dots, cap, glog + lg.gs, lg.step, &bad,
                                 &over);
    const int lo = kc + 1;
    if (!over)
      for (int idx = lane; idx < rr * lo; idx += 64) {
        const int r = idx / lo, j = idx - (idx / lo) * lo;
        out[idx] = Qb[r * (KC + 1) + ((j < kc) ? j : KC)];
      }
    if (lane == 0) {
      glog[0] = p;
      glog[1] = rho;
      glog[2] = over ? 0 : rr;
      glog[3] = 2;
      e.slot_rows[o] = over ? 0 : rr;
      if (over) flag_at(e, status, inst, ECLQR_CAPACITY, e.st[sa].i);
      else if (bad) flag_at(e, status, inst, ECLQR_INFEASIBLE_SUFFIX, e.st[sa].i);
    }
    lds_sync();
  }
}

// ---------------------------------------------------------------------------
// State parameterisation (eqs. (state-param), (left-inverse)): T_i is an
// orthonormal basis of null(H_i) (trailing columns of the Householder Q of
// H_i^T), t_i = -H_i^T h_i (minimum norm, H_i has orthonormal rows), S_i =
// T_i^T.  On stage 0 also eq. (initial-feasibility) and z_0 (eq.
// (reduced-initial)), written as the constant leaf of the forward scan.
// LDS: Ht (maxn x maxn) | X (maxn x maxn) | tau | qr scratch | perm
__global__ void __launch_bounds__(kBlock) k_domain(DevEngine e, Inputs in, Tols t, int32_t* status, int maxn,
                                                   int64_t first, int64_t count) {
  extern __shared__ double lds[];
  double* Ht = lds;
  double* X = Ht + maxn * maxn;
  double* tau = X + maxn * maxn;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + kMaxDim + 8);
  double* sh = (double*)(perm + kMaxDim);
  for (int64_t ti = blockIdx.x; ti < count; ti += gridDim.x) {
    const int64_t s = stage_at(e, first, ti);
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n;
    const int suf = st.suf[SCAN_REL];
    const int r = e.slot_rows[suf];
    const double* H = slot_ptr(e, SCAN_REL, suf);  // r x (n + 1)
    const int nb = n - r;
    const Arena ar = arena_layout(st.n, st.np, st.m, st.k);
    double* base = e.arena + st.ws;
    double* T = base + ar.T;
    double* tv = base + ar.t;
    // Ht = H^T (n x r)
    for (int idx = ECLQR_TID; idx < n * r; idx += ECLQR_NT) {
      const int i = idx / r, j = idx % r;
      Ht[i * r + j] = H[j * (n + 1) + i];
    }
    for (int idx = ECLQR_TID; idx < n * nb; idx += ECLQR_NT) {
      const int i = idx / nb, j = idx % nb;
      X[i * nb + j] = (i == r + j) ? 1.0 : 0.0;
    }
    wg_sync();
    wg_qr_colpiv(Ht, r, n, r, 0, r, 0.0, tau, QRScratch{qd, perm});
    wg_apply_q(Ht, r, n, 0, r, tau, X, nb, nb);
    for (int idx = ECLQR_TID; idx < n * nb; idx += ECLQR_NT) T[idx] = X[idx];
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double v = 0.0;
      v = lane_chain<false>(v, H + i, (n + 1), H + n, (n + 1), r);
      tv[i] = -v;
    }
    if (ECLQR_TID == 0) e.nbar[s] = nb;
    wg_sync();
    if (st.i == 0) {
      const double* x0 = in.x0 + st.x0;
      if (ECLQR_TID == 0) {
        double sc = 1.0, res = 0.0;
        for (int i = 0; i < n; ++i) sc = fmax(sc, fabs(x0[i]));
        for (int j = 0; j < r; ++j) {
          double v = H[j * (n + 1) + n];
          sc = fmax(sc, fabs(v));
          v = lane_chain<false>(v, H + j * (n + 1), 1, x0, 1, n);
          res = fmax(res, fabs(v));
        }
        if (res > t.cons * sc) flag_at(e, status, st.inst, ECLQR_INFEASIBLE_INITIAL, 0);
      }
      double* z0 = slot_ptr(e, SCAN_FWD, st.suf[SCAN_FWD]);
      for (int j = ECLQR_TID; j < nb; j += ECLQR_NT) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) v = fma(X[i * nb + j], x0[i] - tv[i], v);
        z0[j] = v;
      }
      wg_sync();
    }
    (void)sh;
  }
}

// ---------------------------------------------------------------------------
static int g_rel_max_lds = 65536;
void relations_set_max_lds(int bytes) {
  g_rel_max_lds = bytes;
  for (const void* f : {reinterpret_cast<const void*>(k_base_relation<false>),
                        reinterpret_cast<const void*>(k_base_relation<true>),
                        reinterpret_cast<const void*>(k_rel_compose<false>),
                        reinterpret_cast<const void*>(k_rel_compose<true>)})
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_domain), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

size_t rel_lds_bytes(int maxp, int ldw) {
  return sizeof(double) * ((size_t)maxp * (ldw | 1) + kMaxDim + kMaxDim + 8 + 2 * maxp + 8 + 64 + 16) +
         sizeof(int) * kMaxDim + 64;
}

size_t domain_lds_bytes(int maxn) {
  return sizeof(double) * (2 * (size_t)maxn * maxn + kMaxDim + kMaxDim + 8 + 16) + sizeof(int) * kMaxDim + 64;
}

void launch_validate(const DevEngine& e, const Inputs& in, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(e.nblocks), dim3(kBlock), 0, s, e, in, status);
}

void launch_vacuous(const DevEngine& e, const Inputs& in, Tols t, int32_t* vac, int maxk, int maxm, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)maxk * (maxm | 1) + 2 * kMaxDim + 8) + sizeof(int) * kMaxDim;
  hipLaunchKernelGGL(k_vacuous, dim3(e.nblocks), dim3(kBlock), lds, s, e, in, t, vac, maxk, maxm);
}

// The stacked system of maxp x ldw doubles goes to a global tile when it
// does not fit the device's LDS and the plan laid tiles out.
static bool rel_global(const DevEngine& e, int maxp, int ldw) {
  return rel_lds_bytes(maxp, ldw) > (size_t)g_rel_max_lds && e.gw && (int64_t)maxp * (ldw | 1) <= e.gw_stride;
}
static size_t rel_tile_bytes(int maxp, int ldw) { return sizeof(double) * (size_t)maxp * (ldw | 1); }
// compositions: the global tile already above kRelComposeLds
static bool rel_global_compose(const DevEngine& e, int maxp, int ldw) {
  return (rel_lds_bytes(maxp, ldw) > (size_t)kRelComposeLds && e.gw && (int64_t)maxp * (ldw | 1) <= e.gw_stride) ||
         rel_global(e, maxp, ldw);
}

void launch_base_relation(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxp, int ldw,
                          int64_t first, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  if (rel_global(e, maxp, ldw)) {
    int grid = e.nblocks < e.gw_blocks ? e.nblocks : e.gw_blocks;
    grid = (int)(count < grid ? count : grid);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_base_relation<true>), dim3(grid), dim3(kBlock),
                       rel_lds_bytes(maxp, ldw) - rel_tile_bytes(maxp, ldw), s, e, in, t, status, maxp, ldw, first,
                       count);
    return;
  }
  const size_t lds = rel_lds_bytes(maxp, ldw);
  const int grid = task_grid(e, count);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_base_relation<false>), dim3(grid), dim3(kBlock), lds, s, e, in, t, status, maxp,
                     ldw, first, count);
}

bool rel_fits(const DevEngine& e, int maxp, int ldw) {
  return rel_lds_bytes(maxp, ldw) <= (size_t)g_rel_max_lds || rel_global(e, maxp, ldw);
}

void launch_rel_compose(const DevEngine& e, int64_t first, int64_t ntasks, Tols t, int32_t* status, int maxp, int ldw,
                        int maxkc, hipStream_t s) {
  if (ntasks <= 0) return;
  const int grid = (int)(ntasks < e.nblocks ? ntasks : e.nblocks);  // the global-tile variant
  const int tg = task_grid(e, ntasks);
  // register-resident variant when every task of the launch fits it
  if (e.reg_compose && maxp <= 64 && ldw <= 128 && maxkc <= 64) {
    const bool r32 = maxp <= 32, r48 = maxp <= 48, c1 = ldw <= 64, k32 = maxkc <= 32;
#define ECLQR_REG(PRV, NCV, KCV) \
  hipLaunchKernelGGL((k_rel_compose_reg<PRV, NCV, KCV>), dim3(tg), dim3(kBlock), 0, s, e, first, ntasks, t, status)
    if (r32 && c1 && k32) ECLQR_REG(32, 1, 32);
    else if (r32 && c1) ECLQR_REG(32, 1, 64);
    else if (r32 && k32) ECLQR_REG(32, 2, 32);
    else if (r32) ECLQR_REG(32, 2, 64);
    else if (r48 && c1 && k32) ECLQR_REG(48, 1, 32);
    else if (r48 && k32) ECLQR_REG(48, 2, 32);
    else if (c1 && k32) ECLQR_REG(64, 1, 32);
    else if (c1) ECLQR_REG(64, 1, 64);
    else if (k32) ECLQR_REG(64, 2, 32);
    else ECLQR_REG(64, 2, 64);
#undef ECLQR_REG
    return;
  }
  if (rel_global_compose(e, maxp, ldw)) {
    const int g2 = grid < e.gw_blocks ? grid : e.gw_blocks;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rel_compose<true>), dim3(g2), dim3(kBlock),
                       rel_lds_bytes(maxp, ldw) - rel_tile_bytes(maxp, ldw), s, e, first, ntasks, t, status, maxp, ldw);
    return;
  }
  const size_t lds = rel_lds_bytes(maxp, ldw);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rel_compose<false>), dim3(tg), dim3(kBlock), lds, s, e, first, ntasks, t, status,
                     maxp, ldw);
}

void launch_domain(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxn, int64_t first,
                   int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const size_t lds = domain_lds_bytes(maxn);
  const int grid = task_grid(e, count);
  hipLaunchKernelGGL(k_domain, dim3(grid), dim3(kBlock), lds, s, e, in, t, status, maxn, first, count);
}

}  // namespace eclqr
