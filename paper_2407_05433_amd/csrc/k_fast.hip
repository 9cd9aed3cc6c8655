// Factor-reusing multiplier recovery (the fast route beside the contraction-
// expansion of Section VII, which the paper's implementation notes describe as
// algebraically equivalent).  It reuses what the primal pass already holds:
// the domains X_i = {H_i x + h_i = 0} (orthonormal rows H_i, null basis T_i),
// the value-function scan (suffix element of stage i: V_i(z) = 1/2 z'J_i z -
// eta_i'z) and the forward scan (z_i).
//
// With the objective gradients of eq. (objective-gradients) and the stage
// stationarity of eq. (stage-stationarity) (merged rows E_i x + F_i u + g_i = 0
// with multiplier mu_i):
//   * every multiplier has lambda_i = w_i + H_i' theta_i with w_i = T_i
//     lambda-bar_i, lambda-bar_i = J_i z_i - eta_i the costate of the reduced
//     problem (T_i' lambda_i is the gradient of the cost-to-go in z), and theta_i
//     in R^{r_i}, r_i = rank H_i;
//   * stage i's stationarity in the unknowns y = (mu_i, theta_{i+1}) reads
//       [E_i'  (H_{i+1} A_i)'] y = H_i' theta_i - g^x_i - A_i' w_{i+1} + w_i
//       [F_i'  (H_{i+1} B_i)'] y = - g^u_i - B_i' w_{i+1},
//     consistent for every theta_i (the rows of H_i span the projected
//     constraints of stage i).  A column-pivoted Householder QR of the
//     coefficient matrix and back substitution (free coordinates zero) give one
//     solution, affine in theta_i: theta_{i+1} = Pi_i theta_i + pi_i and
//     mu_i = Ym_i theta_i + ym_i;
//   * theta_0 = 0 (lambda_0 = -alpha then has no component normal to X_0);
//     a forward scan of the affine maps gives every theta_i;
//   * terminal stationarity (eq. (terminal-stationarity)):
//       E_N' mu_N = H_N' theta_N + w_N - g^x_N.
// Under LICQ the multipliers are unique and equal those of the minimum-norm
// route; otherwise this is one valid representative.  The route is linear in
// the vector data for fixed matrices, so refinement corrections add up.
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "scratch.hpp"

namespace eclqr {

namespace {

// Reduced dims of the domain normal: r_s = n_s - n-bar_s.
__device__ __forceinline__ int rdim(const DevEngine& e, int s) { return e.st[s].n - e.nbar[s]; }

// w = T (J z - eta) of stage s into out (LDS, n entries); tmp: LDS, >= n-bar.
__device__ __forceinline__ void reduced_costate(const DevEngine& e, int64_t s, double* out, double* tmp) {
  const StageInfo& st = e.st[s];
  const int n = st.n, nb = e.nbar[s];
  const RicLayout rl = ric_layout(n, 0);
  const double* V = slot_ptr(e, SCAN_RIC, st.suf[SCAN_RIC]);
  const double* J = V + rl.J;
  const double* eta = V + rl.eta;
  const double* z = slot_ptr(e, SCAN_FWD, st.suf[SCAN_FWD]);
  for (int j = ECLQR_TID; j < nb; j += ECLQR_NT) tmp[j] = lane_chain<false>(-eta[j], J + j * nb, 1, z, 1, nb);
  lds_sync();
  const Arena ar = arena_layout(n, st.np, st.m, st.k);
  const double* T = e.arena + st.ws + ar.T;
  for (int a = ECLQR_TID; a < n; a += ECLQR_NT) out[a] = lane_chain<false>(0.0, T + a * nb, 1, tmp, 1, nb);
  lds_sync();
}

}  // namespace

// One wavefront per stage.  LDS: W (maxrow x ldw) | tau | qr scratch | perm |
// w_i | w_{i+1} | gx | gu | tmp.
__global__ void __launch_bounds__(kBlock) k_mult_local(DevEngine e, Inputs in, const double* x, const double* u,
                                                       Tols t, int32_t* status, int maxrow, int ldw) {
  extern __shared__ double lds[];
  double* W = lds;
  double* tau = W + (int64_t)maxrow * ldw;
  double* qd = tau + 2 * kMaxDim;
  int* perm = (int*)(qd + 2 * kMaxDim + 8);
  double* wi = (double*)(perm + 2 * kMaxDim);
  double* w1 = wi + kMaxDim;
  double* gx = w1 + kMaxDim;
  double* gu = gx + kMaxDim;
  double* tmp = gu + kMaxDim;
  if (none_live(e)) return;
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, m = st.terminal ? 0 : st.m, k = st.k;
    const Arena ar = arena_layout(n, st.np, st.m, st.k);
    double* base = e.arena + st.ws;
    const int ri = rdim(e, (int)s);
    const double* Hi = slot_ptr(e, SCAN_REL, st.suf[SCAN_REL]);  // r_i x (n + 1)
    reduced_costate(e, s, wi, tmp);
    for (int a = ECLQR_TID; a < n; a += ECLQR_NT) base[ar.wl + a] = wi[a];
    // objective gradients, eq. (objective-gradients)
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
      for (int b = ECLQR_TID; b < m; b += ECLQR_NT) {
        double v = lane_chain<false>(in.f[IN_r][st.in[IN_r] + b], R + b * m, 1, us, 1, m);
        if (Mm) v = lane_chain<false>(v, Mm + b, m, xs, 1, n);
        gu[b] = v;
      }
    }
    lds_sync();
    const double* E = in.f[IN_E] + st.in[IN_E];
    int r1 = 0, n1 = 0;
    const double* H1 = nullptr;
    if (!st.terminal) {
      reduced_costate(e, s + 1, w1, tmp);
      r1 = rdim(e, (int)s + 1);
      n1 = e.st[s + 1].n;
      H1 = slot_ptr(e, SCAN_REL, e.st[s + 1].suf[SCAN_REL]);  // r1 x (n1 + 1)
    }
    // W = [coefficients (q columns) | H_i' (r_i columns) | constant], rows: x (n), u (m)
    const int q = k + r1, rows = n + m, c = q + ri + 1, ld = c | 1;
    const double* A = st.terminal ? nullptr : in.f[IN_A] + st.in[IN_A];
    const double* B = st.terminal ? nullptr : in.f[IN_B] + st.in[IN_B];
    const double* F = st.terminal ? nullptr : in.f[IN_F] + st.in[IN_F];
    for (int idx = ECLQR_TID; idx < rows * c; idx += ECLQR_NT) {
      const int row = idx / c, col = idx - (idx / c) * c;
      const bool xr = row < n;
      const int a = xr ? row : row - n;
      double v = 0.0;
      if (col < k) {
        v = xr ? E[col * n + a] : F[col * m + a];
      } else if (col < q) {  // (H_{i+1} A_i)' or (H_{i+1} B_i)'
        const int l = col - k;
        v = xr ? lane_chain<false>(0.0, H1 + l * (n1 + 1), 1, A + a, n, n1)
               : lane_chain<false>(0.0, H1 + l * (n1 + 1), 1, B + a, m, n1);
      } else if (col < q + ri) {
        v = xr ? Hi[(col - q) * (n + 1) + a] : 0.0;
      } else if (xr) {
        v = wi[a] - gx[a];
        if (!st.terminal) v = lane_chain<true>(v, A + a, n, w1, 1, n1);
      } else {
        v = lane_chain<true>(-gu[a], B + a, m, w1, 1, n1);
      }
      W[row * ld + col] = v;
    }
    wg_sync();
    const int rho = wg_qr_colpiv(W, ld, rows, c, 0, q, t.rank, tau, QRScratch{qd, perm});
    // Per right-hand side (one lane each): consistency -- the part outside
    // the range of the coefficients, rows rho.. of Q'rhs, against the column
    // norm (Q is orthogonal) -- then back substitution R11 y = (Q'rhs)[0:rho].
    bool bad = false;
    for (int col = q + ECLQR_TID; col < c; col += ECLQR_NT) {
      double res = 0.0, tot = 0.0;
      for (int row = 0; row < rows; ++row) {
        const double v = W[row * ld + col];
        tot = fma(v, v, tot);
        if (row >= rho) res = fma(v, v, res);
      }
      if (!(sqrt(res) <= t.cons * fmax(1.0, sqrt(tot)))) bad = true;
      for (int j = rho - 1; j >= 0; --j) {
        double v = W[j * ld + col];
        for (int l = j + 1; l < rho; ++l) v = fma(-W[j * ld + l], W[l * ld + col], v);
        W[j * ld + col] = v / W[j * ld + j];
      }
    }
    if (bad) flag(status, st.inst, ECLQR_RANK_INCONSISTENT);
    wg_sync();
    // y[perm[j]] = solution row j (j < rho), free coordinates 0
    double* Ymu = base + ar.Ym;
    double* ymu = base + ar.ym;
    double* Fth = st.terminal ? nullptr : e.theta + e.slot_off[SCAN_FWD * e.nslots + st.elem[SCAN_FWD]];
    for (int idx = ECLQR_TID; idx < q * (ri + 1); idx += ECLQR_NT) {
      const int yr = idx / (ri + 1), cc = idx - (idx / (ri + 1)) * (ri + 1);
      // position of unknown yr among the pivots
      int pos = -1;
      for (int j = 0; j < rho; ++j)
        if (perm[j] == yr) pos = j;
      const double v = (pos >= 0) ? W[pos * ld + q + cc] : 0.0;
      if (yr < k) {
        if (cc < ri) Ymu[yr * n + cc] = v;
        else ymu[yr] = v;
      } else {
        const int l = yr - k;  // theta_{i+1} row: map (r1 x r_i, ld r_i), constant at np * n
        if (cc < ri) Fth[l * ri + cc] = v;
        else Fth[(int64_t)st.np * n + l] = v;
      }
    }
    if (st.i == 0) {  // theta_0 = 0: the constant leaf of the scan
      double* th0 = e.theta + e.slot_off[SCAN_FWD * e.nslots + st.suf[SCAN_FWD]];
      for (int j = ECLQR_TID; j < ri; j += ECLQR_NT) th0[j] = 0.0;
    }
    wg_sync();
  }
}

// Forward scan of the theta maps: k_fwd_combine on the theta arena with the
// normal dims r_s.
__global__ void __launch_bounds__(kBlock) k_theta_combine(DevEngine e, int64_t first, int64_t ntasks) {
  if (none_live(e)) return;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * (first + ti)];
    const int bsl = e.tasks[3 * (first + ti) + 1];
    const int o = e.tasks[3 * (first + ti) + 2];
    const int so = slot_a(e, 1, a), smid = slot_b(e, 1, a), sin_ = slot_b(e, 1, bsl);
    if (gated(e, e.st[so].inst)) continue;
    const int dout = rdim(e, so), dmid = rdim(e, smid), din = (sin_ >= 0) ? rdim(e, sin_) : 0;
    const int nout = e.st[so].n, nmid = e.st[smid].n, nin = (sin_ >= 0) ? e.st[sin_].n : 0;
    const double* F1 = e.theta + e.slot_off[SCAN_FWD * e.nslots + a];
    const double* f1 = F1 + (int64_t)nout * nmid;
    const double* F2 = e.theta + e.slot_off[SCAN_FWD * e.nslots + bsl];
    const double* f2 = F2 + (int64_t)nmid * nin;
    double* Fo = e.theta + e.slot_off[SCAN_FWD * e.nslots + o];
    double* fo = Fo + (int64_t)nout * nin;
    if (sin_ >= 0) wg_gemm(Fo, din, F1, dmid, false, F2, din, false, dout, din, dmid, 1.0, 0.0);
    for (int i = ECLQR_TID; i < dout; i += ECLQR_NT) fo[i] = lane_chain<false>(f1[i], F1 + i * dmid, 1, f2, 1, dmid);
    wg_sync();
  }
}

// lambda_i = w_i + H_i' theta_i, mu_i = Ym_i theta_i + ym_i; written, or added
// to the values present (refinement corrections).
__global__ void __launch_bounds__(kBlock) k_mult_final(DevEngine e, double* lam, double* mu, int accumulate) {
  if (none_live(e)) return;
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, k = st.k;
    const Arena ar = arena_layout(n, st.np, st.m, st.k);
    const double* base = e.arena + st.ws;
    const int ri = rdim(e, (int)s);
    const double* Hi = slot_ptr(e, SCAN_REL, st.suf[SCAN_REL]);
    const double* th = e.theta + e.slot_off[SCAN_FWD * e.nslots + st.suf[SCAN_FWD]];
    for (int a = ECLQR_TID; a < n; a += ECLQR_NT) {
      const double v = lane_chain<false>(base[ar.wl + a], Hi + a, n + 1, th, 1, ri);
      lam[st.in[IN_q] + a] = accumulate ? lam[st.in[IN_q] + a] + v : v;
    }
    for (int j = ECLQR_TID; j < k; j += ECLQR_NT) {
      const double v = lane_chain<false>(base[ar.ym + j], base + ar.Ym + j * n, 1, th, 1, ri);
      mu[st.in[IN_g] + j] = accumulate ? mu[st.in[IN_g] + j] + v : v;
    }
  }
}

static int g_fast_max_lds = 65536;
void fast_set_max_lds(int bytes) {
  g_fast_max_lds = bytes;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_mult_local), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
}
size_t mult_local_lds_bytes(int maxrow, int ldw) {
  return sizeof(double) * ((size_t)maxrow * ldw + 2 * kMaxDim + 2 * kMaxDim + 8 + 5 * kMaxDim) +
         sizeof(int) * 2 * kMaxDim + 64;
}
bool launch_mult_local(const DevEngine& e, const Inputs& in, const double* x, const double* u, Tols t,
                       int32_t* status, int maxrow, int ldw, hipStream_t s) {
  const size_t lds = mult_local_lds_bytes(maxrow, ldw);
  if (lds > (size_t)g_fast_max_lds) return false;
  const int grid = task_grid(e, e.S);
  hipLaunchKernelGGL(k_mult_local, dim3(grid), dim3(kBlock), lds, s, e, in, x, u, t, status, maxrow, ldw);
  return true;
}
void launch_theta_combine(const DevEngine& e, int64_t first, int64_t ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  const int grid = (int)(ntasks < e.nblocks ? ntasks : e.nblocks);
  hipLaunchKernelGGL(k_theta_combine, dim3(grid), dim3(kBlock), 0, s, e, first, ntasks);
}
void launch_mult_final(const DevEngine& e, double* lam, double* mu, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_mult_final, dim3(e.nblocks), dim3(kBlock), 0, s, e, lam, mu, accumulate);
}


// ---------------------------------------------------------------------------
// Minimum-norm multipliers from the same domains and scans.
//
// Every valid multiplier vector is lambda_i = w_i + H_i' theta_i with
// (mu_i, theta_{i+1}) solving stage i's local system M_i y = [H_i'; 0] theta_i
// + c_i (see above).  With the minimum-norm solution of that system and an
// orthonormal basis N_i of null(M_i),
//   (mu_i, theta_{i+1}) = Y_i theta_i + y_i + N_i omega_i,   N_i'Y_i = 0, N_i'y_i = 0,
// and ||lambda_i||^2 = ||w_i||^2 + ||theta_i||^2 (w_i = T_i lambda-bar_i is
// orthogonal to the rows of H_i).  So the minimum-norm multiplier minimises
//   1/2 ||theta_0||^2 + sum_{i<N} [1/2 ||Y_i theta_i + y_i||^2 + 1/2 ||omega_i||^2]
//   + 1/2 ||Y_N theta_N + y_N||^2
// over theta_0 and omega subject to theta_{i+1} = Y_i^theta theta_i + N_i^theta
// omega_i + y_i^theta (the theta rows of the maps; each stage's term carries
// 1/2 ||theta_{i+1}||^2), a reduced LQR in the form the value-function scan
// solves: stage cost Q = Y'Y, q = Y'y, R = I, no cross term; dynamics
// A = Y^theta, B = N^theta, c = y^theta; terminal Q = Y_N'Y_N, q = Y_N'y_N;
// element A_e = A, b_e = c, C_e = B B', J_e = Q, eta_e = -q.  The free initial
// state is theta_0 = (I + J_0)^{-1} eta_0 from the scan's value function at
// stage 0.  The minimum-norm local solution comes from a Householder QR of
// M_i' with column pivoting (rows of M_i), as in Lemma 2 with the
// Moore-Penrose inverse: M_i' P = Q [R11 R12], y = Q1 R11^{-T} (P'b)_{1:rho},
// N_i = Q[:, rho:].
//
// The theta engine shares the primal schedule; its stage arena (input
// capacity k_i + n_{i+1}) holds: Y (q x r, ld r), y (q), Z = N (q x f, ld f)
// (the terminal stage: Ym, ym), the reduced LQR data Ab Bb cb Qb Mb Rb qb rb,
// the gains, and wl = w_i.

// LDS: W (maxq x max(ldw, maxr + 1)) | Qg (maxq x maxq) | X (maxq x (maxr+1)) |
// tau (maxq) | qd (ldw + 8) | cr (ldw) | perm (ldw ints) | wi w1 gx gu tmp (kMaxDim each).
// Yl = Q1 X (q x (r_i + 1)) is formed in W's place once the factorization
// in W has been read for the last time (the plan sizes the tile with a
// separate Yl block, an upper bound of this).
__host__ __device__ inline int64_t theta_w_doubles(int maxq, int ldw, int maxr) {
  return (int64_t)maxq * (ldw > maxr + 1 ? ldw : maxr + 1);
}
size_t theta_local_lds_bytes(int maxq, int ldw, int maxr) {
  return 8 * (theta_w_doubles(maxq, ldw, maxr) + (int64_t)maxq * maxq + (int64_t)maxq * (maxr + 1) + maxq +
              2 * (int64_t)ldw + 8 + 5 * kMaxDim) +
         4 * (int64_t)(ldw + 1) + 64;
}

// kMode 0: full pass.  kMode 1: vector-only pass for new vectors with the
// same matrices (refinement corrections, the adjoint, the solution after a
// matrix pass): a stage other than the terminal one reuses the factors the
// last full or matrix pass kept (pivots, R11, Q1) and recomputes only y and
// the vector parts of its element; with `status` it also checks the vector
// column of the local system, M_i y_i = c_i at the minimum-norm y_i (the part
// of the full pass's consistency test that depends on the vectors).
// kMode 2: matrix pass: the full pass with every vector zero (no read of the
// primal solution or of its value-function and forward scans, so it can run
// beside them once the domains are known); the vector pass completes it.
template <int kMode>
__global__ void __launch_bounds__(kBlock) k_theta_local(DevEngine p, DevEngine th, Inputs in, const double* x,
                                                        const double* u, Tols t, int32_t* status, int maxq, int ldw,
                                                        int maxr, int64_t first, int64_t count) {
  constexpr bool kVec = kMode == 1;
  constexpr bool kMat = kMode == 2;
  extern __shared__ double lds[];
  double* W = lds;
  double* Qg = W + theta_w_doubles(maxq, ldw, maxr);
  double* X = Qg + (int64_t)maxq * maxq;
  double* const Yl = W;  // after the last read of the factorization in W
  double* tau = X + (int64_t)maxq * (maxr + 1);
  double* qd = tau + maxq;
  double* cr = qd + ldw + 8;
  double* wi = cr + ldw;
  double* w1 = wi + kMaxDim;
  double* gx = w1 + kMaxDim;
  double* gu = gx + kMaxDim;
  double* tmp = gu + kMaxDim;
  int* perm = (int*)(tmp + kMaxDim);
  if (none_live(p)) return;
  for (int64_t ti = blockIdx.x; ti < count; ti += gridDim.x) {
    const int64_t s = stage_at(p, first, ti);
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    const StageInfo ts = th.st[s];
    const bool term = st.terminal;
    const int n = st.n, m = term ? 0 : st.m, k = st.k;
    const int ri = rdim(p, (int)s);
    const double* Hi = slot_ptr(p, SCAN_REL, st.suf[SCAN_REL]);  // r_i x (n + 1)
    if constexpr (kMat) {
      for (int a = ECLQR_TID; a < n; a += ECLQR_NT) {
        wi[a] = 0.0;
        gx[a] = 0.0;
      }
      for (int b = ECLQR_TID; b < m; b += ECLQR_NT) gu[b] = 0.0;
    } else {
      reduced_costate(p, s, wi, tmp);
      const double* Q = in.f[IN_Q] + st.in[IN_Q];
      const double* xs = x + st.in[IN_q];
      const double* us = term ? nullptr : u + st.in[IN_r];
      const double* Mm = (in.f[IN_M] && !term) ? in.f[IN_M] + st.in[IN_M] : nullptr;
      for (int a = ECLQR_TID; a < n; a += ECLQR_NT) {
        double v = lane_chain<false>(in.f[IN_q][st.in[IN_q] + a], Q + a * n, 1, xs, 1, n);
        if (Mm) v = lane_chain<false>(v, Mm + a * m, 1, us, 1, m);
        gx[a] = v;
      }
      if (!term) {
        const double* R = in.f[IN_R] + st.in[IN_R];
        for (int b = ECLQR_TID; b < m; b += ECLQR_NT) {
          double v = lane_chain<false>(in.f[IN_r][st.in[IN_r] + b], R + b * m, 1, us, 1, m);
          if (Mm) v = lane_chain<false>(v, Mm + b, m, xs, 1, n);
          gu[b] = v;
        }
      }
    }
    lds_sync();
    int r1 = 0, n1 = 0;
    const double* H1 = nullptr;
    if (!term) {
      r1 = rdim(p, (int)s + 1);
      n1 = p.st[s + 1].n;
      H1 = slot_ptr(p, SCAN_REL, p.st[s + 1].suf[SCAN_REL]);  // r1 x (n1 + 1)
      if constexpr (kMat) {
        for (int a = ECLQR_TID; a < n1; a += ECLQR_NT) w1[a] = 0.0;
        lds_sync();
      } else {
        reduced_costate(p, s + 1, w1, tmp);
      }
    }
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* A = term ? nullptr : in.f[IN_A] + st.in[IN_A];
    const double* B = term ? nullptr : in.f[IN_B] + st.in[IN_B];
    const double* F = term ? nullptr : in.f[IN_F] + st.in[IN_F];
    const int q = k + r1, Rr = n + m;
    // constant right-hand side: [w_i - g^x - A'w_{i+1}; -g^u - B'w_{i+1}]
    for (int row = ECLQR_TID; row < Rr; row += ECLQR_NT) {
      double v;
      if (row < n) {
        v = wi[row] - gx[row];
        if (!term) v = lane_chain<true>(v, A + row, n, w1, 1, n1);
      } else {
        v = lane_chain<true>(-gu[row - n], B + (row - n), m, w1, 1, n1);
      }
      cr[row] = v;
    }
    if (kVec && !term) {
      const Arena at = arena_layout(ts.n, ts.np, ts.m, ts.k);
      double* tb = th.arena + ts.ws;
      const int f = th.mbar[s], rho = q - f;
      // Yl: the q <= 64 multiplier values in the front of the tile (sized
      // for the terminal stages this pass factors: at least 16 x 17 doubles)
      lds_sync();
      // z = R11^{-T} (P'c)_{1:rho}, y = Q1 z
      const int lane = ECLQR_TID;
      double zv = (lane < rho) ? cr[(int)tb[at.prm + lane]] : 0.0;
      zv = lane_trsv_upper_t(tb + at.R11, rho, zv, rho);
      if (lane < rho) tmp[lane] = zv;
      lds_sync();
      for (int i = lane; i < q; i += ECLQR_NT) Yl[i] = lane_chain<false>(0.0, tb + at.Q1 + i * rho, 1, tmp, 1, rho);
      lds_sync();
      for (int i = lane; i < q; i += ECLQR_NT) tb[at.y + i] = Yl[i];
      for (int a = lane; a < n; a += ECLQR_NT) tb[at.wl + a] = wi[a];
      const RicLayout rl = ric_layout(ts.n, ts.np);
      double* ric = slot_ptr(th, SCAN_RIC, ts.elem[SCAN_RIC]);
      for (int l = lane; l < r1; l += ECLQR_NT) {
        tb[at.cb + l] = Yl[k + l];
        ric[rl.b + l] = Yl[k + l];
      }
      for (int c = lane; c < ri; c += ECLQR_NT) {
        const double v = lane_chain<false>(0.0, tb + at.Y + c, ri, Yl, 1, q);
        tb[at.qb + c] = v;
        ric[rl.eta + c] = -v;
      }
      if (status) {
        // M_i y = c_i: [E' y_mu + A'(H_{i+1}' y_theta); F' y_mu + B'(H_{i+1}' y_theta)] = c,
        // each row against its own terms' magnitudes
        for (int j = lane; j < n1; j += ECLQR_NT) tmp[j] = lane_chain<false>(0.0, H1 + j, n1 + 1, Yl + k, 1, r1);
        lds_sync();
        bool bad = false;
        for (int row = lane; row < Rr; row += ECLQR_NT) {
          const bool xr = row < n;
          const int a = xr ? row : row - n;
          const double* G = xr ? E + a : F + a;
          const double* D = xr ? A + a : B + a;
          const int ldg = xr ? n : m;
          double e = -cr[row], mag = fabs(cr[row]);
          for (int c = 0; c < k; ++c) {
            const double tl = G[c * ldg] * Yl[c];
            e += tl;
            mag += fabs(tl);
          }
          for (int j = 0; j < n1; ++j) {
            const double tl = D[j * ldg] * tmp[j];
            e += tl;
            mag += fabs(tl);
          }
          if (!(fabs(e) <= t.cons * fmax(1.0, mag))) bad = true;
        }
        if (bad) flag(status, st.inst, ECLQR_RANK_INCONSISTENT);
      }
      wg_sync();
      continue;
    }
    // W = M' (q x Rr): row col of W is column col of M (a multiplier unknown)
    for (int idx = ECLQR_TID; idx < q * Rr; idx += ECLQR_NT) {
      const int col = idx / Rr, row = idx - (idx / Rr) * Rr;
      const bool xr = row < n;
      const int a = xr ? row : row - n;
      double v;
      if (col < k) {
        v = xr ? E[col * n + a] : F[col * m + a];
      } else {
        const int l = col - k;
        v = xr ? lane_chain<false>(0.0, H1 + l * (n1 + 1), 1, A + a, n, n1)
               : lane_chain<false>(0.0, H1 + l * (n1 + 1), 1, B + a, m, n1);
      }
      W[col * ldw + row] = v;
    }
    wg_sync();
    const int rho = wg_qr_colpiv(W, ldw, q, Rr, 0, Rr, t.rank, tau, QRScratch{qd, perm});
    const int f = q - rho;
    const int nc = ri + 1;
    wg_identity(Qg, q, q);
    wg_apply_q(W, ldw, q, 0, rho, tau, Qg, q, q);
    // X = (P' [H_i' | c])_{1:rho}, then X <- R11^{-T} X
    for (int idx = ECLQR_TID; idx < rho * nc; idx += ECLQR_NT) {
      const int j = idx / nc, c = idx - (idx / nc) * nc;
      const int row = perm[j];
      X[idx] = (c < ri) ? ((row < n) ? Hi[c * (n + 1) + row] : 0.0) : cr[row];
    }
    wg_sync();
    wg_trsm_upper_t(W, ldw, 0, X, nc, rho, nc);
    // consistency: rows rho.. of P'b against R12' X (one lane per (row, column))
    {
      bool bad = false;
      for (int idx = ECLQR_TID; idx < (Rr - rho) * nc; idx += ECLQR_NT) {
        const int jj = rho + idx / nc, c = idx - (idx / nc) * nc;
        const int row = perm[jj];
        const double bv = (c < ri) ? ((row < n) ? Hi[c * (n + 1) + row] : 0.0) : cr[row];
        double e = -bv, mag = fabs(bv);
        for (int l = 0; l < rho; ++l) {
          const double tl = W[l * ldw + jj] * X[l * nc + c];
          e += tl;
          mag += fabs(tl);
        }
        if (!(fabs(e) <= t.cons * fmax(1.0, mag))) bad = true;
      }
      if (bad) flag(status, st.inst, ECLQR_RANK_INCONSISTENT);
    }
    // theta engine arena
    const Arena at = arena_layout(ts.n, ts.np, ts.m, ts.k);
    double* tb = th.arena + ts.ws;
    if (!term)  // R11 of the minimum-norm solve, read before Yl takes W's place
      for (int idx = ECLQR_TID; idx < rho * rho; idx += ECLQR_NT) {
        const int i = idx / rho, j = idx - (idx / rho) * rho;
        tb[at.R11 + idx] = (j >= i) ? W[i * ldw + j] : 0.0;
      }
    wg_sync();
    // Yl = Q1 X (q x (r_i + 1)): [Y | y]
    wg_gemm(Yl, nc, Qg, q, false, X, nc, false, q, nc, rho, 1.0, 0.0);
    // [Y | y] in the fields Y, y (capacity k + n') of a stage, Ym, ym (k x n) at the terminal
    double* Ya = tb + (term ? at.Ym : at.Y);
    double* ya = tb + (term ? at.ym : at.y);
    for (int idx = ECLQR_TID; idx < q * ri; idx += ECLQR_NT) Ya[idx] = Yl[(idx / ri) * nc + idx % ri];
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) ya[j] = Yl[j * nc + ri];
    if (!term) {
      double* Na = tb + at.Z;
      for (int idx = ECLQR_TID; idx < q * f; idx += ECLQR_NT) Na[idx] = Qg[(idx / f) * q + rho + idx % f];
      // factors of the minimum-norm solve, for the vector-only passes
      for (int j = ECLQR_TID; j < rho; j += ECLQR_NT) tb[at.prm + j] = (double)perm[j];
      for (int idx = ECLQR_TID; idx < q * rho; idx += ECLQR_NT) tb[at.Q1 + idx] = Qg[(idx / rho) * q + idx % rho];
    }
    for (int a = ECLQR_TID; a < n; a += ECLQR_NT) tb[at.wl + a] = wi[a];
    // reduced LQR data and the value-function element
    double* Qb = tb + at.Qb;
    double* qb = tb + at.qb;
    wg_gemm(Qb, ri, Yl, nc, true, Yl, nc, false, ri, ri, q, 1.0, 0.0);
    for (int c = ECLQR_TID; c < ri; c += ECLQR_NT) qb[c] = lane_chain<false>(0.0, Yl + c, nc, Yl + ri, nc, q);
    wg_sync();
    wg_symmetrize(Qb, ri, ri);
    double* ric = slot_ptr(th, SCAN_RIC, ts.elem[SCAN_RIC]);
    if (term) {
      const RicLayout rl = ric_layout(ts.n, 0);
      wg_copy(ric + rl.J, ri, Qb, ri, ri, ri);
      for (int c = ECLQR_TID; c < ri; c += ECLQR_NT) ric[rl.eta + c] = -qb[c];
      if (ECLQR_TID == 0) {
        th.nbar[s] = ri;
        th.mbar[s] = 0;
      }
      wg_sync();
      continue;
    }
    double* Ab = tb + at.Ab;
    double* Bb = tb + at.Bb;
    double* cb = tb + at.cb;
    for (int idx = ECLQR_TID; idx < r1 * ri; idx += ECLQR_NT) Ab[idx] = Yl[(k + idx / ri) * nc + idx % ri];
    for (int idx = ECLQR_TID; idx < r1 * f; idx += ECLQR_NT) Bb[idx] = Qg[(k + idx / f) * q + rho + idx % f];
    for (int l = ECLQR_TID; l < r1; l += ECLQR_NT) cb[l] = Yl[(k + l) * nc + ri];
    wg_fill(tb + at.Mb, f, ri, f, 0.0);
    wg_identity(tb + at.Rb, f, f);
    for (int j = ECLQR_TID; j < f; j += ECLQR_NT) tb[at.rb + j] = 0.0;
    wg_sync();
    const RicLayout rl = ric_layout(ts.n, ts.np);
    wg_copy(ric + rl.A, ri, Ab, ri, r1, ri);
    for (int l = ECLQR_TID; l < r1; l += ECLQR_NT) ric[rl.b + l] = cb[l];
    wg_gemm(ric + rl.C, r1, Bb, f, false, Bb, f, true, r1, r1, f, 1.0, 0.0);
    wg_symmetrize(ric + rl.C, r1, r1);
    wg_copy(ric + rl.J, ri, Qb, ri, ri, ri);
    for (int c = ECLQR_TID; c < ri; c += ECLQR_NT) ric[rl.eta + c] = -qb[c];
    if (ECLQR_TID == 0) {
      th.nbar[s] = ri;
      th.mbar[s] = f;
    }
    wg_sync();
  }
}

// theta_0 = (I + J_0)^{-1} eta_0: the free initial state of the theta LQR,
// written as the constant leaf of its forward scan.
__global__ void __launch_bounds__(kBlock) k_theta_init(DevEngine th) {
  __shared__ double S0[kMaxDim * kMaxDim];
  __shared__ double sh[16];
  if (none_live(th)) return;
  for (int64_t s = blockIdx.x; s < th.S; s += gridDim.x) {
    const StageInfo ts = th.st[s];
    if (ts.i != 0 || gated(th, ts.inst)) continue;
    const int r0 = th.nbar[s];
    const RicLayout rl = ric_layout(ts.n, 0);
    const double* V = slot_ptr(th, SCAN_RIC, ts.suf[SCAN_RIC]);
    for (int idx = ECLQR_TID; idx < r0 * r0; idx += ECLQR_NT) {
      const int i = idx / r0, j = idx - (idx / r0) * r0;
      S0[idx] = V[rl.J + idx] + ((i == j) ? 1.0 : 0.0);
    }
    lds_sync();
    wg_cholesky<true>(S0, r0, r0, sh, 0.0);
    const int lane = ECLQR_TID;
    double v = (lane < r0) ? V[rl.eta + lane] : 0.0;
    v = lane_trsv_lower(S0, r0, v, r0);
    v = lane_trsv_lower_t(S0, r0, v, r0);
    double* th0 = slot_ptr(th, SCAN_FWD, ts.suf[SCAN_FWD]);
    if (lane < r0) th0[lane] = v;
    lds_sync();
  }
}

// lambda_i = w_i + H_i' theta_i; omega_i = K_i theta_i + k_i;
// mu_i = (Y_i theta_i + y_i + N_i omega_i)_{1:k_i} (terminal: Y_N theta_N + y_N);
// written, or added to the values present (refinement corrections).
__global__ void __launch_bounds__(kBlock) k_theta_final(DevEngine p, DevEngine th, double* lam, double* mu,
                                                        int accumulate) {
  __shared__ double om[kMaxDim];
  if (none_live(p)) return;
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    const StageInfo ts = th.st[s];
    const int n = st.n, k = st.k;
    const int ri = th.nbar[s], f = st.terminal ? 0 : th.mbar[s];
    const Arena at = arena_layout(ts.n, ts.np, ts.m, ts.k);
    const double* tb = th.arena + ts.ws;
    const double* Hi = slot_ptr(p, SCAN_REL, st.suf[SCAN_REL]);
    const double* tv = slot_ptr(th, SCAN_FWD, ts.suf[SCAN_FWD]);
    for (int a = ECLQR_TID; a < n; a += ECLQR_NT) {
      const double v = lane_chain<false>(tb[at.wl + a], Hi + a, n + 1, tv, 1, ri);
      lam[st.in[IN_q] + a] = accumulate ? lam[st.in[IN_q] + a] + v : v;
    }
    for (int j = ECLQR_TID; j < f; j += ECLQR_NT) om[j] = lane_chain<false>(tb[at.kk + j], tb + at.K + j * ri, 1, tv, 1, ri);
    lds_sync();
    const int64_t oY = st.terminal ? at.Ym : at.Y, oy = st.terminal ? at.ym : at.y;
    for (int j = ECLQR_TID; j < k; j += ECLQR_NT) {
      double v = lane_chain<false>(tb[oy + j], tb + oY + j * ri, 1, tv, 1, ri);
      if (f > 0) v = lane_chain<false>(v, tb + at.Z + j * f, 1, om, 1, f);
      mu[st.in[IN_g] + j] = accumulate ? mu[st.in[IN_g] + j] + v : v;
    }
    lds_sync();
  }
}

static int g_theta_max_lds = 65536;
void theta_set_max_lds(int bytes) {
  g_theta_max_lds = bytes;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_theta_local<0>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_theta_local<1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_theta_local<2>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
bool launch_theta_local(const DevEngine& p, const DevEngine& th, const Inputs& in, const double* x, const double* u,
                        Tols t, int32_t* status, int maxq, int ldw, int maxr, int mode, int64_t first,
                        int64_t count, hipStream_t s) {
  const size_t lds = theta_local_lds_bytes(maxq, ldw, maxr);
  if (lds > (size_t)g_theta_max_lds) return false;
  if (count <= 0) return true;
  const int grid = task_grid(p, count);
  if (mode == 1)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_theta_local<1>), dim3(grid), dim3(kBlock), lds, s, p, th, in, x, u, t, status,
                       maxq, ldw, maxr, first, count);
  else if (mode == 2)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_theta_local<2>), dim3(grid), dim3(kBlock), lds, s, p, th, in, x, u, t, status,
                       maxq, ldw, maxr, first, count);
  else
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_theta_local<0>), dim3(grid), dim3(kBlock), lds, s, p, th, in, x, u, t, status,
                       maxq, ldw, maxr, first, count);
  return true;
}
void launch_theta_init(const DevEngine& th, hipStream_t s) {
  hipLaunchKernelGGL(k_theta_init, dim3(th.nblocks), dim3(kBlock), 0, s, th);
}
void launch_theta_final(const DevEngine& p, const DevEngine& th, double* lam, double* mu, int accumulate,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_theta_final, dim3(p.nblocks), dim3(kBlock), 0, s, p, th, lam, mu, accumulate);
}

}  // namespace eclqr
