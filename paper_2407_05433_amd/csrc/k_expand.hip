// Multipliers by the contraction-expansion route of Section VII.
//
// The stationarity equations of stage i (eq. (stage-stationarity)), with the
// mixed and state-only rows merged,
//   [E_i'; F_i'] mu_i + [[-I, A_i'], [0, B_i']] (lambda_i, lambda_{i+1}) + [g^x_i; g^u_i] = 0,
// and the terminal equations g^x_N - lambda_N + E_N' mu_N = 0 are affine
// relations once mu is projected out (eq. (dual-base-system), Lemma 1).  They
// are composed by a balanced up-sweep over the stages (plus one empty leaf
// after the terminal one, so that every leaf is binary) down to a relation
// on lambda_0, whose minimum-norm point is taken; then the tree is expanded
// from the root: at every composition node with both outer costates known,
// the shared costate is the minimum-norm solution of the two operand
// relations (eq. (middle-dual-map) with the free coordinates rho_j = 0).
// Finally each stage's mu_i is the minimum-norm solution of its own
// stationarity rows (the leaf solves).
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "kernels.hpp"

namespace eclqr {

namespace {

// Minimum-norm solution of the consistent system M y = b (M: R x q), given
// W = M' (q x R, row-major, leading dimension ld) and b (R entries, LDS):
// Householder QR of W with column pivoting (rank: pivots above
// thr * max(1, first pivot)), z = R11^{-T} (P' b)_{1:rho}, y = Q [z; 0].  W
// is overwritten; y (q entries) and xz (R entries) are LDS.  Returns rho.
__device__ inline int wg_minnorm(double* W, int ld, int q, int R, const double* b, double thr, double* tau,
                                 QRScratch sc, double* y, double* xz) {
  const int rho = wg_qr_colpiv(W, ld, q, R, 0, R, thr, tau, sc);
  for (int j = ECLQR_TID; j < rho; j += ECLQR_NT) xz[j] = b[sc.perm[j]];
  wg_sync();
  wg_trsm_upper_t(W, ld, 0, xz, 1, rho, 1);
  for (int j = ECLQR_TID; j < q; j += ECLQR_NT) y[j] = (j < rho) ? xz[j] : 0.0;
  wg_sync();
  wg_apply_q(W, ld, q, 0, rho, tau, y, 1, 1);
  return rho;
}

// Objective gradients of primal stage ps at the solution (eq.
// (objective-gradients)): gx (n), gu (m; none at the terminal stage).
__device__ inline void objective_gradients(const StageInfo& st, const Inputs& in, const double* x, const double* u,
                                           double* gx, double* gu) {
  const int n = st.n, m = st.terminal ? 0 : st.m;
  const double* Q = in.f[IN_Q] + st.in[IN_Q];
  const double* xs = x + st.in[IN_q];
  const double* us = st.terminal ? nullptr : u + st.in[IN_r];
  const double* Mm = (in.f[IN_M] && !st.terminal) ? in.f[IN_M] + st.in[IN_M] : nullptr;
  for (int a = ECLQR_TID; a < n; a += ECLQR_NT) {
    double v = lane_chain<false>(in.f[IN_q][st.in[IN_q] + a], Q + a * n, 1, xs, 1, n);
    if (Mm) v = lane_chain<false>(v, Mm + a * m, 1, us, 1, m);
    gx[a] = v;
  }
  if (!st.terminal) {
    const double* R = in.f[IN_R] + st.in[IN_R];
    for (int c = ECLQR_TID; c < m; c += ECLQR_NT) {
      double v = lane_chain<false>(in.f[IN_r][st.in[IN_r] + c], R + c * m, 1, us, 1, m);
      if (Mm) v = lane_chain<false>(v, Mm + c, m, xs, 1, n);
      gu[c] = v;
    }
  }
  wg_sync();
}

// The primal stage of a stage of the contraction engine (-1 for its extra
// empty stage).
__device__ inline int64_t primal_stage(const DevEngine& c, const int64_t* psbase, int64_t cs) {
  const StageInfo& x = c.st[cs];
  return (x.i <= x.N - 1) ? psbase[x.inst] + x.i : -1;
}

}  // namespace

// Dual base relations (eq. (dual-base-system)): one wavefront per stage of
// the contraction engine.  The stacked system [mu | lambda_i | lambda_{i+1} | 1]
// has n_i + m_i rows (n_N at the terminal stage); rows are scaled by their
// coefficient norms, mu is eliminated by a column-pivoted Householder QR and
// the remaining rows are replaced by an orthonormal row basis over the two
// costates.  An inconsistent remainder (0 = gamma) flags the instance.
// LDS: W (maxp x ldw) | tau | qr scratch | perm | gradients | row-basis scratch
__global__ void __launch_bounds__(kBlock) k_cx_base(DevEngine c, DevEngine p, const int64_t* psbase, Inputs in,
                                                    const double* x, const double* u, Tols t, int32_t* status,
                                                    int maxp, int ldw) {
  extern __shared__ double lds[];
  double* W = lds;
  double* tau = W + (int64_t)maxp * ldw;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + kMaxDim + 8);
  double* gx = (double*)(perm + kMaxDim);
  double* gu = gx + kMaxDim;
  double* rbs = gu + kMaxDim;
  for (int64_t cs = blockIdx.x; cs < c.S; cs += gridDim.x) {
    const StageInfo& cst = c.st[cs];
    const int slot = cst.elem[SCAN_REL];
    const int64_t ps = primal_stage(c, psbase, cs);
    if (ps < 0) {  // the extra empty stage: no rows
      if (ECLQR_TID == 0) c.slot_rows[slot] = 0;
      continue;
    }
    const StageInfo st = p.st[ps];
    const bool term = st.terminal;
    const int n = st.n, np = term ? 0 : st.np, m = term ? 0 : st.m, k = st.k;
    const int rows = n + m, cols = k + n + np + 1, ld = cols | 1;
    objective_gradients(st, in, x, u, gx, gu);
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* F = term ? nullptr : in.f[IN_F] + st.in[IN_F];
    const double* A = term ? nullptr : in.f[IN_A] + st.in[IN_A];
    const double* B = term ? nullptr : in.f[IN_B] + st.in[IN_B];
    for (int idx = ECLQR_TID; idx < rows * cols; idx += ECLQR_NT) {
      const int r = idx / cols, j = idx - (idx / cols) * cols;
      double v;
      if (r < n) {
        if (j < k) v = E[j * n + r];
        else if (j < k + n) v = (j - k == r) ? -1.0 : 0.0;
        else if (j < k + n + np) v = A[(j - k - n) * n + r];
        else v = gx[r];
      } else {
        const int a = r - n;
        if (j < k) v = F[j * m + a];
        else if (j < k + n) v = 0.0;
        else if (j < k + n + np) v = B[(j - k - n) * m + a];
        else v = gu[a];
      }
      W[r * ld + j] = v;
    }
    wg_sync();
    // scale every row by the norm of its coefficients (Section VIII item 1)
    for (int r = ECLQR_TID; r < rows; r += ECLQR_NT) {
      double s2 = 0.0;
      for (int j = 0; j < cols - 1; ++j) s2 = fma(W[r * ld + j], W[r * ld + j], s2);
      if (s2 > 0.0) {
        const double inv = 1.0 / sqrt(s2);
        for (int j = 0; j < cols; ++j) W[r * ld + j] *= inv;
      }
    }
    wg_sync();
    double om = 1.0;
    for (int r = ECLQR_TID; r < rows; r += ECLQR_NT) om = fmax(om, fabs(W[r * ld + cols - 1]));
    om = wave_max(om);
    const int rho = (k > 0) ? wg_qr_colpiv(W, ld, rows, cols, 0, k, t.rank, tau, QRScratch{qd, perm}) : 0;
    int bad = 0;
    const int rr = wg_row_basis(W, ld, rho, rows, k, n + np, t.rank, t.cons * om, &bad, rbs);
    const int cap = c.slot_cap[slot];
    const int lo = n + np + 1;
    double* out = slot_ptr(c, SCAN_REL, slot);
    const int keep = rr < cap ? rr : cap;
    for (int idx = ECLQR_TID; idx < keep * lo; idx += ECLQR_NT) {
      const int r = idx / lo, j = idx - (idx / lo) * lo;
      out[idx] = W[(rho + r) * ld + k + j];
    }
    if (ECLQR_TID == 0) {
      c.slot_rows[slot] = keep;
      double* glog = c.rel_log + c.rel_log_off[slot];
      glog[0] = rows;
      glog[1] = rho;
      glog[2] = keep;
      glog[3] = 0;
      if (bad || rr > cap) flag(status, cst.inst, ECLQR_RANK_INCONSISTENT);
    }
    wg_sync();
  }
}

// Root of each instance's tree: the relation on lambda_0 left by the
// up-sweep; lambda_0 is its minimum-norm point.
// LDS: W (maxn x ldp) | b (maxp) | y (maxn) | xz (maxp) | tau | qr scratch (maxp + 8) | perm (maxp)
__global__ void __launch_bounds__(kBlock) k_cx_root(DevEngine c, DevEngine p, const int64_t* csbase,
                                                    const int64_t* psbase, double* lam, Tols t, int maxn, int maxp) {
  extern __shared__ double lds[];
  const int ldp = maxp | 1;
  double* W = lds;
  double* bv = W + (int64_t)maxn * ldp;
  double* y = bv + maxp;
  double* xz = y + maxn;
  double* tau = xz + maxp;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + maxp + 8);
  for (int b = blockIdx.x; b < c.B; b += gridDim.x) {
    const StageInfo& c0 = c.st[csbase[b]];
    const int root = c0.suf[SCAN_REL];
    const int n = c0.n, r = c.slot_rows[root];
    const double* H = slot_ptr(c, SCAN_REL, root);  // r x (n + 1)
    double* l0 = lam + p.st[psbase[b]].in[IN_q];
    if (n == 0) continue;
    for (int idx = ECLQR_TID; idx < n * r; idx += ECLQR_NT) {
      const int i = idx / r, j = idx - (idx / r) * r;
      W[i * ldp + j] = H[j * (n + 1) + i];
    }
    for (int j = ECLQR_TID; j < r; j += ECLQR_NT) bv[j] = -H[j * (n + 1) + n];
    wg_sync();
    wg_minnorm(W, ldp, n, r, bv, t.rank, tau, QRScratch{qd, perm}, y, xz);
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) l0[i] = y[i];
    wg_sync();
  }
}

// Expansion of one up-sweep level (eq. (middle-dual-map), rho_j = 0): task
// (a, c) -> o composes [s, mid) and [mid, e); with lambda_s and lambda_e
// known, lambda_mid is the minimum-norm solution of the operand rows
//   L_a(:, mid) lambda_mid = -(L_a(:, s) lambda_s + l_a),
//   L_c(:, mid) lambda_mid = -(L_c(:, e) lambda_e + l_c).
// A residual above cons times the rows' magnitudes flags the instance.
// LDS as k_cx_root.
__global__ void __launch_bounds__(kBlock) k_cx_expand(DevEngine c, DevEngine p, const int64_t* psbase, int64_t first,
                                                      int64_t ntasks, double* lam, Tols t, int32_t* status, int maxn,
                                                      int maxp) {
  extern __shared__ double lds[];
  const int ldp = maxp | 1;
  double* W = lds;
  double* bv = W + (int64_t)maxn * ldp;
  double* y = bv + maxp;
  double* xz = y + maxn;
  double* tau = xz + maxp;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + maxp + 8);
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = c.tasks[3 * (first + ti)];
    const int cc = c.tasks[3 * (first + ti) + 1];
    const int gs = slot_a(c, 0, a), gm = slot_b(c, 0, a), ge = slot_b(c, 0, cc);
    const int ns = c.st[gs].n, nm = c.st[gm].n, ne = (ge >= 0) ? c.st[ge].n : 0;
    if (nm == 0) continue;
    const int ra = c.slot_rows[a], rb = c.slot_rows[cc];
    const int P = ra + rb;
    const double* La = slot_ptr(c, SCAN_REL, a);   // ra x (ns + nm + 1)
    const double* Lc = slot_ptr(c, SCAN_REL, cc);  // rb x (nm + ne + 1)
    const int lda = ns + nm + 1, ldc = nm + ne + 1;
    const int64_t pms = primal_stage(c, psbase, gm);
    const double* ls = (ns > 0) ? lam + p.st[primal_stage(c, psbase, gs)].in[IN_q] : nullptr;
    const double* le = (ne > 0) ? lam + p.st[primal_stage(c, psbase, ge)].in[IN_q] : nullptr;
    for (int idx = ECLQR_TID; idx < nm * P; idx += ECLQR_NT) {
      const int i = idx / P, j = idx - (idx / P) * P;
      W[i * ldp + j] = (j < ra) ? La[j * lda + ns + i] : Lc[(j - ra) * ldc + i];
    }
    for (int j = ECLQR_TID; j < P; j += ECLQR_NT) {
      double v;
      if (j < ra) v = lane_chain<false>(La[j * lda + ns + nm], La + j * lda, 1, ls, 1, ns);
      else v = lane_chain<false>(Lc[(j - ra) * ldc + nm + ne], Lc + (j - ra) * ldc + nm, 1, le, 1, ne);
      bv[j] = -v;
    }
    wg_sync();
    wg_minnorm(W, ldp, nm, P, bv, t.rank, tau, QRScratch{qd, perm}, y, xz);
    // residual of every operand row at lambda_mid
    bool bad = false;
    for (int j = ECLQR_TID; j < P; j += ECLQR_NT) {
      const double* row = (j < ra) ? La + j * lda + ns : Lc + (j - ra) * ldc;
      double e = -bv[j], mag = fabs(bv[j]);
      for (int i = 0; i < nm; ++i) {
        const double tl = row[i] * y[i];
        e += tl;
        mag += fabs(tl);
      }
      if (!(fabs(e) <= t.cons * fmax(1.0, mag))) bad = true;
    }
    if (bad) flag(status, c.st[gs].inst, ECLQR_RANK_INCONSISTENT);
    double* lm = lam + p.st[pms].in[IN_q];
    for (int i = ECLQR_TID; i < nm; i += ECLQR_NT) lm[i] = y[i];
    wg_sync();
  }
}

// Leaf solves: mu_i, the minimum-norm solution of stage i's stationarity rows
// at the expanded costates,
//   [E_i'; F_i'] mu_i = -[g^x_i - lambda_i + A_i' lambda_{i+1}; g^u_i + B_i' lambda_{i+1}],
//   E_N' mu_N = lambda_N - g^x_N at the terminal stage.
// LDS: W (maxk x ldr) | b (maxr) | y (maxk) | xz (maxr) | tau | qr scratch (maxr + 8) | perm (maxr) | gx | gu
__global__ void __launch_bounds__(kBlock) k_cx_leaf(DevEngine p, Inputs in, const double* x, const double* u,
                                                   const double* lam, double* mu, Tols t, int32_t* status, int maxk,
                                                   int maxr) {
  extern __shared__ double lds[];
  const int ldr = maxr | 1;
  double* W = lds;
  double* bv = W + (int64_t)maxk * ldr;
  double* y = bv + maxr;
  double* xz = y + maxk;
  double* tau = xz + maxr;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + maxr + 8);
  double* gx = (double*)(perm + ((maxr + 1) & ~1));
  double* gu = gx + kMaxDim;
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    const bool term = st.terminal;
    const int n = st.n, np = term ? 0 : st.np, m = term ? 0 : st.m, k = st.k;
    if (k == 0) continue;
    const int R = n + m;
    objective_gradients(st, in, x, u, gx, gu);
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* F = term ? nullptr : in.f[IN_F] + st.in[IN_F];
    const double* A = term ? nullptr : in.f[IN_A] + st.in[IN_A];
    const double* B = term ? nullptr : in.f[IN_B] + st.in[IN_B];
    const double* li = lam + st.in[IN_q];
    const double* l1 = term ? nullptr : lam + p.st[s + 1].in[IN_q];
    for (int idx = ECLQR_TID; idx < k * R; idx += ECLQR_NT) {
      const int q = idx / R, r = idx - (idx / R) * R;
      W[q * ldr + r] = (r < n) ? E[q * n + r] : F[q * m + (r - n)];
    }
    for (int r = ECLQR_TID; r < R; r += ECLQR_NT) {
      double v;
      if (r < n) {
        v = gx[r] - li[r];
        if (!term) v = lane_chain<false>(v, A + r, n, l1, 1, np);
      } else {
        v = lane_chain<false>(gu[r - n], B + (r - n), m, l1, 1, np);
      }
      bv[r] = -v;
    }
    wg_sync();
    wg_minnorm(W, ldr, k, R, bv, t.rank, tau, QRScratch{qd, perm}, y, xz);
    bool bad = false;
    for (int r = ECLQR_TID; r < R; r += ECLQR_NT) {
      const double* G = (r < n) ? E + r : F + (r - n);
      const int ldg = (r < n) ? n : m;
      double e = -bv[r], mag = fabs(bv[r]);
      for (int q = 0; q < k; ++q) {
        const double tl = G[q * ldg] * y[q];
        e += tl;
        mag += fabs(tl);
      }
      if (!(fabs(e) <= t.cons * fmax(1.0, mag))) bad = true;
    }
    if (bad) flag(status, st.inst, ECLQR_RANK_INCONSISTENT);
    double* ms = mu + st.in[IN_g];
    for (int q = ECLQR_TID; q < k; q += ECLQR_NT) ms[q] = y[q];
    wg_sync();
  }
}

// ---------------------------------------------------------------------------
size_t cx_base_lds_bytes(int maxp, int ldw) {
  return sizeof(double) * ((size_t)maxp * ldw + kMaxDim + kMaxDim + 8 + 2 * kMaxDim + 2 * (size_t)maxp + 8 + 64) +
         sizeof(int) * kMaxDim + 64;
}
size_t cx_solve_lds_bytes(int maxn, int maxp) {
  return sizeof(double) * ((size_t)maxn * (maxp | 1) + 2 * (size_t)maxp + maxn + kMaxDim + maxp + 8 + 2 * kMaxDim) +
         sizeof(int) * (size_t)maxp + 64;
}
static int g_cx_max_lds = 65536;
void cx_set_max_lds(int bytes) {
  g_cx_max_lds = bytes;
  for (const void* f : {reinterpret_cast<const void*>(k_cx_base), reinterpret_cast<const void*>(k_cx_root),
                        reinterpret_cast<const void*>(k_cx_expand), reinterpret_cast<const void*>(k_cx_leaf)})
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
bool cx_fits(int base_p, int base_ld, int exp_n, int exp_p, int leaf_k, int leaf_r) {
  const size_t lim = (size_t)g_cx_max_lds;
  return cx_base_lds_bytes(base_p, base_ld) <= lim && cx_solve_lds_bytes(exp_n, exp_p) <= lim &&
         cx_solve_lds_bytes(leaf_k, leaf_r) <= lim && cx_solve_lds_bytes(kMaxDim, 2 * kMaxDim) <= lim;
}
void launch_cx_base(const DevEngine& c, const DevEngine& p, const int64_t* psbase, const Inputs& in, const double* x,
                    const double* u, Tols t, int32_t* status, int maxp, int ldw, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_base, dim3(c.nblocks), dim3(kBlock), cx_base_lds_bytes(maxp, ldw), s, c, p, psbase, in, x, u,
                     t, status, maxp, ldw);
}
void launch_cx_root(const DevEngine& c, const DevEngine& p, const int64_t* csbase, const int64_t* psbase, double* lam,
                    Tols t, int maxn, int maxp, hipStream_t s) {
  const int grid = c.B < 4096 ? c.B : 4096;
  hipLaunchKernelGGL(k_cx_root, dim3(grid > 0 ? grid : 1), dim3(kBlock), cx_solve_lds_bytes(maxn, maxp), s, c, p,
                     csbase, psbase, lam, t, maxn, maxp);
}
void launch_cx_expand(const DevEngine& c, const DevEngine& p, const int64_t* psbase, int64_t first, int64_t ntasks,
                      double* lam, Tols t, int32_t* status, int maxn, int maxp, hipStream_t s) {
  if (ntasks <= 0) return;
  const int grid = (int)(ntasks < c.nblocks ? ntasks : c.nblocks);
  hipLaunchKernelGGL(k_cx_expand, dim3(grid), dim3(kBlock), cx_solve_lds_bytes(maxn, maxp), s, c, p, psbase, first,
                     ntasks, lam, t, status, maxn, maxp);
}
void launch_cx_leaf(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                    double* mu, Tols t, int32_t* status, int maxk, int maxr, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_leaf, dim3(p.nblocks), dim3(kBlock), cx_solve_lds_bytes(maxk, maxr) + 2 * kMaxDim * 8, s, p,
                     in, x, u, lam, mu, t, status, maxk, maxr);
}

}  // namespace eclqr
