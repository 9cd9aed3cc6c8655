// Stage-parallel constraint elimination (paper Section V) and the
// conditional value-function element of each reduced stage.
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "scratch.hpp"

namespace eclqr {

// Bump allocator over the workgroup's global scratch.
struct Bump {
  double* p;
  __device__ double* take(int64_t n) {
    double* r = p;
    p += rup4(n);
    return r;
  }
};

// Stage i < N: with x_i = T_i z + t_i and the successor constrained to
// X_{i+1} = {H_{i+1} x + h_{i+1} = 0} (eq. (local-control-system)):
//   Gamma = [F; H' B],  Phi = [E; H' A] T,  gamma = [E t + g; H'(A t + c) + h']
// (rows scaled by the norms of [Gamma, Psi]).  Lemma 2 with the Moore-Penrose
// inverse: a pivoted Householder QR of Gamma^T gives rank rho, the null-space
// basis Z = Q[:, rho:], and Y = -Q1 R11^{-T} P^T Phi, y = -Q1 R11^{-T} P^T gamma.
// Reduced data: eqs. (reduced-dynamics-data), (state-cost-data),
// (reduced-cost-data); the stage constant of eq. (stage-constant) is not
// formed, since no solution, multiplier or gradient depends on it.  The
// value-function element of the
// reduced stage (cross term removed with R-bar = L L^T):
//   A_e = A-bar - W^T V, b_e = c-bar - W^T w, C_e = W^T W,
//   J_e = Q-bar - V^T V, eta_e = -(q-bar - V^T w),
// W = L^{-1} B-bar^T, V = L^{-1} M-bar^T, w = L^{-1} r-bar.
// Terminal stage: Q-bar_N = T^T Q_N T, q-bar_N = T^T (Q_N t + q_N)
// (eq. (terminal-cost-data)), element J = Q-bar_N, eta = -q-bar_N.
// LDS: W (maxm x maxq) | tau | qr scratch | perm | Lc (maxm x maxm) | sh | reduction buffer
// [| the stage's working arrays, kLS: they live in LDS instead of the
// workgroup's global scratch (every dependent access then waits on LDS, not
// on L2)]
template <bool kLS>
__global__ void __launch_bounds__(kBlock, kLS ? 1 : 4) k_eliminate(DevEngine e, Inputs in, Tols t, int32_t* status, int maxm,
                                                      int maxq, int64_t first, int64_t count) {
  extern __shared__ double lds[];
  double* Wq = lds;
  double* tau = Wq + (int64_t)maxm * maxq;
  double* qd = tau + kMaxDim;
  int* perm = (int*)(qd + 2 * kMaxDim + 8);
  double* Lc = (double*)(perm + 2 * kMaxDim);
  double* sh = Lc + (int64_t)maxm * maxm;
  double* red = sh + 16;
  double* lscr = red + kBlock;
  for (int64_t ti = blockIdx.x; ti < count; ti += gridDim.x) {
    const int64_t s = stage_at(e, first, ti);
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const Arena ar = arena_layout(n, np, m, st.k);
    double* base = e.arena + st.ws;
    const int nb = e.nbar[s];
    const double* T = base + ar.T;
    const double* tv = base + ar.t;
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* qv = in.f[IN_q] + st.in[IN_q];
    // working arrays: one region, reused phase by phase (QR and maps; reduced
    // dynamics; reduced costs; value-function element), each phase starting
    // after a barrier that ends the previous one's reads
    double* const scr0 = kLS ? lscr : block_scratch(e);
    Bump bump{scr0};
    double* ric = slot_ptr(e, SCAN_RIC, st.elem[SCAN_RIC]);
    if (st.terminal) {
      const RicLayout rl = ric_layout(n, 0);
      double* QT = bump.take((int64_t)n * nb);
      double* v = bump.take(n);
      wg_gemm(QT, nb, Q, n, false, T, nb, false, n, nb, n, 1.0, 0.0);
      wg_gemm(ric + rl.J, nb, T, nb, true, QT, nb, false, nb, nb, n, 1.0, 0.0);
      wg_symmetrize(ric + rl.J, nb, nb);
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
        double a = qv[i];
        a = lane_chain<false>(a, Q + i * n, 1, tv, 1, n);
        v[i] = a;
      }
      wg_sync();
      wg_gemv(ric + rl.eta, T, nb, true, v, nb, n, -1.0, 0.0);
      continue;
    }
    const int inst = st.inst;
    const StageInfo& st1 = e.st[s + 1];
    const Arena ar1 = arena_layout(st1.n, st1.np, st1.m, st1.k);
    const double* T1 = e.arena + st1.ws + ar1.T;
    const double* t1 = e.arena + st1.ws + ar1.t;
    const int nb1 = e.nbar[s + 1];
    const int suf1 = st1.suf[SCAN_REL];
    const int r1 = e.slot_rows[suf1];
    const double* H1 = slot_ptr(e, SCAN_REL, suf1);  // r1 x (np + 1)
    const int ldh = np + 1;
    const double* A = in.f[IN_A] + st.in[IN_A];
    const double* B = in.f[IN_B] + st.in[IN_B];
    const double* cv = in.f[IN_c] + st.in[IN_c];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* F = in.f[IN_F] + st.in[IN_F];
    const double* g = in.f[IN_g] + st.in[IN_g];
    const double* R = in.f[IN_R] + st.in[IN_R];
    const double* Mm = in.f[IN_M] ? in.f[IN_M] + st.in[IN_M] : nullptr;
    const double* rv = in.f[IN_r] + st.in[IN_r];
    const int q = k + r1;

    double* Gs = bump.take((int64_t)q * m);
    double* Ps = bump.take((int64_t)q * n);
    double* gs = bump.take(q);
    double* Phi = bump.take((int64_t)q * n);
    double* gam = bump.take(q);
    // Q of the QR of Gamma^T is formed in LDS, in the Cholesky factor's
    // place (that factor is first needed by the value-function element): its
    // reflector updates then wait on LDS instead of global memory
    double* Qg = Lc;
    double* X = bump.take((int64_t)m * (n + 1));
    double* rsc = bump.take(q);

    // Gamma = [F; H' B], Psi = [E; H' A], gamma~ = [g; H' c + h']
    wg_copy(Gs, m, F, m, k, m);
    wg_copy(Ps, n, E, n, k, n);
    for (int j = ECLQR_TID; j < k; j += ECLQR_NT) gs[j] = g[j];
    wg_gemm(Gs + (int64_t)k * m, m, H1, ldh, false, B, m, false, r1, m, np, 1.0, 0.0);
    wg_gemm(Ps + (int64_t)k * n, n, H1, ldh, false, A, n, false, r1, n, np, 1.0, 0.0);
    for (int j = ECLQR_TID; j < r1; j += ECLQR_NT) {
      double a = H1[j * ldh + np];
      a = lane_chain<false>(a, H1 + j * ldh, 1, cv, 1, np);
      gs[k + j] = a;
    }
    wg_sync();
    // row scaling by the norms of [Gamma, Psi]
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) {
      double a = 0.0;
      a = lane_chain<false>(a, Gs + j * m, 1, Gs + j * m, 1, m);
      a = lane_chain<false>(a, Ps + j * n, 1, Ps + j * n, 1, n);
      rsc[j] = (a > 0.0) ? 1.0 / sqrt(a) : 1.0;
    }
    wg_sync();
    for (int idx = ECLQR_TID; idx < q * m; idx += ECLQR_NT) Gs[idx] *= rsc[idx / m];
    for (int idx = ECLQR_TID; idx < q * n; idx += ECLQR_NT) Ps[idx] *= rsc[idx / n];
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) gs[j] *= rsc[j];
    wg_sync();
    // Phi = Psi T, gamma = Psi t + gamma~
    wg_gemm(Phi, nb, Ps, n, false, T, nb, false, q, nb, n, 1.0, 0.0);
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) {
      double a = gs[j];
      a = lane_chain<false>(a, Ps + j * n, 1, tv, 1, n);
      gam[j] = a;
    }
    // Gamma^T in LDS, pivoted QR
    for (int idx = ECLQR_TID; idx < q * m; idx += ECLQR_NT) {
      const int j = idx / m, l = idx % m;
      Wq[l * q + j] = Gs[idx];
    }
    wg_sync();
    const int rho = wg_qr_colpiv(Wq, q, m, q, 0, q, t.rank, tau, QRScratch{qd, perm});
    const int mb = m - rho;
    wg_identity(Qg, m, m);
    wg_apply_q(Wq, q, m, 0, rho, tau, Qg, m, m);
    // X = R11^{-T} (P^T [Phi gamma])_{1:rho}
    for (int idx = ECLQR_TID; idx < rho * (nb + 1); idx += ECLQR_NT) {
      const int j = idx / (nb + 1), l = idx % (nb + 1);
      const int row = perm[j];
      X[idx] = (l < nb) ? Phi[row * nb + l] : gam[row];
    }
    wg_sync();
    // factors kept for the vector-only pass: row scales, pivots, R11, Q1
    for (int j = ECLQR_TID; j < q; j += ECLQR_NT) base[ar.rsc + j] = rsc[j];
    for (int j = ECLQR_TID; j < rho; j += ECLQR_NT) base[ar.prm + j] = (double)perm[j];
    for (int idx = ECLQR_TID; idx < rho * rho; idx += ECLQR_NT) {
      const int i = idx / rho, j = idx % rho;
      base[ar.R11 + idx] = (j >= i) ? Wq[i * q + j] : 0.0;
    }
    for (int idx = ECLQR_TID; idx < m * rho; idx += ECLQR_NT) {
      const int i = idx / rho, j = idx % rho;
      base[ar.Q1 + idx] = Qg[i * m + j];
    }
    wg_trsm_upper_t(Wq, q, 0, X, nb + 1, rho, nb + 1);
    double* Y = base + ar.Y;
    double* Z = base + ar.Z;
    double* y = base + ar.y;
    wg_gemm(Y, nb, Qg, m, false, X, nb + 1, false, m, nb, rho, -1.0, 0.0);
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double a = 0.0;
      a = lane_chain<false>(a, Qg + i * m, 1, X + nb, (nb + 1), rho);
      y[i] = -a;
    }
    for (int idx = ECLQR_TID; idx < m * mb; idx += ECLQR_NT) {
      const int i = idx / mb, j = idx % mb;
      Z[idx] = Qg[i * m + rho + j];
    }
    if (ECLQR_TID == 0) e.mbar[s] = mb;
    wg_sync();
    // consistency of the rank decisions: Gamma Y + Phi = 0, Gamma y + gamma = 0
    if (t.check_lemma2) {
      double mres = 0.0, mphi = 0.0, mres2 = 0.0, mg = 0.0;
      for (int idx = ECLQR_TID; idx < q * (nb + 1); idx += ECLQR_NT) {
        const int j = idx / (nb + 1), l = idx % (nb + 1);
        double a = (l < nb) ? Phi[j * nb + l] : gam[j];
        if (l < nb) mphi = fmax(mphi, fabs(a)); else mg = fmax(mg, fabs(a));
        a = (l < nb) ? lane_chain<false>(a, Gs + j * m, 1, Y + l, nb, m) : lane_chain<false>(a, Gs + j * m, 1, y, 1, m);
        if (l < nb) mres = fmax(mres, fabs(a)); else mres2 = fmax(mres2, fabs(a));
      }
      mres = wg_reduce_max(mres, red);
      mphi = wg_reduce_max(mphi, red);
      mres2 = wg_reduce_max(mres2, red);
      mg = wg_reduce_max(mg, red);
      if (ECLQR_TID == 0 && (mres > t.cons * fmax(1.0, mphi) || mres2 > t.cons * fmax(1.0, mg)))
        flag_at(e, status, inst, ECLQR_RANK_INCONSISTENT, st.i);
      wg_sync();
    }

    // ---- reduced dynamics ---------------------------------------------------
    wg_sync();
    bump.p = scr0;
    double* Ab = base + ar.Ab;
    double* Bb = base + ar.Bb;
    double* cb = base + ar.cb;
    double* AT = bump.take((int64_t)np * n);
    double* BZ = bump.take((int64_t)np * m);
    double* cvv = bump.take(np);
    wg_gemm(AT, nb, A, n, false, T, nb, false, np, nb, n, 1.0, 0.0);
    wg_gemm(AT, nb, B, m, false, Y, nb, false, np, nb, m, 1.0, 1.0);
    wg_gemm(Ab, nb, T1, nb1, true, AT, nb, false, nb1, nb, np, 1.0, 0.0);
    wg_gemm(BZ, mb, B, m, false, Z, mb, false, np, mb, m, 1.0, 0.0);
    wg_gemm(Bb, mb, T1, nb1, true, BZ, mb, false, nb1, mb, np, 1.0, 0.0);
    for (int i = ECLQR_TID; i < np; i += ECLQR_NT) {
      double a = cv[i] - t1[i];
      a = lane_chain<false>(a, A + i * n, 1, tv, 1, n);
      a = lane_chain<false>(a, B + i * m, 1, y, 1, m);
      cvv[i] = a;
    }
    wg_sync();
    wg_gemv(cb, T1, nb1, true, cvv, nb1, np, 1.0, 0.0);

    // ---- reduced costs --------------------------------------------------------
    bump.p = scr0;  // wg_gemv ends with a barrier
    double* QT = bump.take((int64_t)n * n);
    double* Mz = bump.take((int64_t)n * m);
    double* RY = bump.take((int64_t)m * n);
    double* RZ = bump.take((int64_t)m * m);
    double* MzY = bump.take((int64_t)n * n);
    double* w = bump.take(m);
    double* qz = bump.take(n);
    double* rz = bump.take(m);
    double* Qb = base + ar.Qb;
    double* Mb = base + ar.Mb;
    double* Rb = base + ar.Rb;
    double* qb = base + ar.qb;
    double* rb = base + ar.rb;
    wg_gemm(QT, nb, Q, n, false, T, nb, false, n, nb, n, 1.0, 0.0);
    wg_gemm(Qb, nb, T, nb, true, QT, nb, false, nb, nb, n, 1.0, 0.0);  // Q^z
    if (Mm) {
      wg_gemm(Mz, m, T, nb, true, Mm, m, false, nb, m, n, 1.0, 0.0);
    } else {
      wg_fill(Mz, m, nb, m, 0.0);
    }
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double a = rv[i];
      if (Mm)
        a = lane_chain<false>(a, Mm + i, m, tv, 1, n);
      rz[i] = a;
    }
    wg_sync();
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double a = rz[i];
      a = lane_chain<false>(a, R + i * m, 1, y, 1, m);
      w[i] = a;
    }
    wg_sync();
    wg_gemm(RY, nb, R, m, false, Y, nb, false, m, nb, m, 1.0, 0.0);
    wg_gemm(RZ, mb, R, m, false, Z, mb, false, m, mb, m, 1.0, 0.0);
    wg_gemm(MzY, nb, Mz, m, false, Y, nb, false, nb, nb, m, 1.0, 0.0);
    // Q-bar = Q^z + Mz Y + (Mz Y)^T + Y^T R Y
    wg_gemm(Qb, nb, Y, nb, true, RY, nb, false, nb, nb, m, 1.0, 1.0);
    for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) {
      const int i = idx / nb, j = idx % nb;
      Qb[idx] += MzY[i * nb + j] + MzY[j * nb + i];
    }
    wg_sync();
    wg_symmetrize(Qb, nb, nb);
    // M-bar = Mz Z + Y^T R Z ; R-bar = Z^T R Z
    wg_gemm(Mb, mb, Mz, m, false, Z, mb, false, nb, mb, m, 1.0, 0.0);
    wg_gemm(Mb, mb, Y, nb, true, RZ, mb, false, nb, mb, m, 1.0, 1.0);
    wg_gemm(Rb, mb, Z, mb, true, RZ, mb, false, mb, mb, m, 1.0, 0.0);
    wg_symmetrize(Rb, mb, mb);
    // q^z = T^T (Q t + q); q-bar = q^z + Mz y + Y^T w ; r-bar = Z^T w
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double a = qv[i];
      a = lane_chain<false>(a, Q + i * n, 1, tv, 1, n);
      QT[i] = a;  // reuse as a vector
    }
    wg_sync();
    wg_gemv(qz, T, nb, true, QT, nb, n, 1.0, 0.0);
    for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
      double a = qz[i];
      a = lane_chain<false>(a, Mz + i * m, 1, y, 1, m);
      a = lane_chain<false>(a, Y + i, nb, w, 1, m);
      qb[i] = a;
    }
    wg_gemv(rb, Z, mb, true, w, mb, m, 1.0, 0.0);

    // ---- value-function element -----------------------------------------------
    const RicLayout rl = ric_layout(n, np);
    bump.p = scr0;  // after the barrier above
    // [W | V | w] side by side (ld lv), so that one triangular solve, one
    // chain of dependent rows, serves all three
    const int lv = nb1 + nb + 1;
    double* Wt = bump.take((int64_t)m * lv);
    double* V = Wt + nb1;
    double* w2 = Wt + nb1 + nb;
    wg_copy(Lc, mb, Rb, mb, mb, mb);
    if (wg_cholesky(Lc, mb, mb, sh + 8)) {
      if (ECLQR_TID == 0) flag_at(e, status, inst, ECLQR_NOT_CONVEX, st.i);
      wg_sync();
      continue;
    }
    wg_copy(base + ar.Lc, mb, Lc, mb, mb, mb);
    wg_copy_t(Wt, lv, Bb, mb, nb1, mb);  // Wt = Bb^T  (mb x nb1)
    wg_copy_t(V, lv, Mb, mb, nb, mb);    // V = Mb^T  (mb x nb)
    for (int i = ECLQR_TID; i < mb; i += ECLQR_NT) w2[(int64_t)i * lv] = rb[i];
    wg_sync();
    wg_trsm_lower(Lc, mb, Wt, lv, mb, lv);
    double* Ae = ric + rl.A;
    double* be = ric + rl.b;
    double* Ce = ric + rl.C;
    double* ee = ric + rl.eta;
    double* Je = ric + rl.J;
    wg_copy(Ae, nb, Ab, nb, nb1, nb);
    wg_gemm(Ae, nb, Wt, lv, true, V, lv, false, nb1, nb, mb, -1.0, 1.0);
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double a = cb[i];
      a = lane_chain<true>(a, Wt + i, lv, w2, lv, mb);
      be[i] = a;
    }
    wg_gemm(Ce, nb1, Wt, lv, true, Wt, lv, false, nb1, nb1, mb, 1.0, 0.0);
    wg_symmetrize(Ce, nb1, nb1);
    wg_copy(Je, nb, Qb, nb, nb, nb);
    wg_gemm(Je, nb, V, lv, true, V, lv, false, nb, nb, mb, -1.0, 1.0);
    wg_symmetrize(Je, nb, nb);
    for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) {
      double a = qb[i];
      a = lane_chain<true>(a, V + i, lv, w2, lv, mb);
      ee[i] = -a;
    }
    wg_sync();
  }
}

static int g_elim_max_lds = 65536;
void eliminate_set_max_lds(int bytes) {
  g_elim_max_lds = bytes;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_eliminate<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_eliminate<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

size_t elim_lds_bytes(int maxm, int maxq) {
  return sizeof(double) * ((size_t)maxm * maxq + kMaxDim + 2 * kMaxDim + 8 + (size_t)maxm * maxm + 16 + kBlock) +
         sizeof(int) * 2 * kMaxDim + 64;
}

void launch_eliminate(const DevEngine& e, const Inputs& in, Tols t, int32_t* status, int maxm, int maxq, int maxn,
                      int maxk, int64_t first, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  const size_t base = elim_lds_bytes(maxm, maxq);
  const size_t with = base + sizeof(double) * (size_t)elim_scratch(maxn, maxn, maxm, maxk);
  // LDS only while a workgroup needs at most 20 KiB: above that the lost
  // occupancy costs more than the faster accesses gain (measured: 26 KiB
  // tiles, six workgroups per compute unit, 13.8 ms against 11.1 ms in global
  // scratch at four waves per SIMD; tiles up to 13 KiB faster in LDS)
  if (e.elim_lds == 1 && with <= 20480 && with <= (size_t)g_elim_max_lds) {
    const int grid = task_grid(e, count);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eliminate<true>), dim3(grid), dim3(kBlock), with, s, e, in, t, status, maxm,
                       maxq, first, count);
  } else {
    const int grid =
        fit_grid(reinterpret_cast<const void*>(k_eliminate<false>), kBlock, base, count < e.nblocks ? count : e.nblocks);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eliminate<false>), dim3(grid), dim3(kBlock), base, s, e, in, t, status, maxm,
                       maxq, first, count);
  }
}

}  // namespace eclqr
