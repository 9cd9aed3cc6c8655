// Sequential dynamic-programming solve of the reduced LQR for the instances
// the scan route cannot take: costs that are not positive definite stage by
// stage.  Section II (the paragraph after eq. (convexity)) holds the
// reduction valid for any symmetric costs; a minimiser exists exactly when
// the Hessian in minimal coordinates of the feasible trajectories is
// positive semidefinite with the linear term orthogonal to its null space,
// and it is unique exactly when that Hessian is positive definite.
//
// The reduced problem (stage arenas written by the elimination: A-bar,
// B-bar, c-bar, Q-bar, M-bar, R-bar, q-bar, r-bar in the minimal coordinates
// z_i, v_i of Section V) is solved backwards: with the cost-to-go
// V_{i+1}(z) = 1/2 z'P z + p'z,
//   H_uu = R + B'P B,  H_ux = M' + B'P A,  h_u = r + B'(P c + p),
//   H_xx = Q + A'P A,  h_x = q + A'(P c + p),
// the stage's input is minimised out.  These H_uu are the pivots of a block
// elimination of the reduced Hessian in the order N-1, ..., 0, so:
//   * every H_uu positive definite: the minimiser is unique (solved here);
//   * an H_uu with a negative eigenvalue: for every z_i the cost falls without
//     bound along that input direction -- no minimiser;
//   * an H_uu with a zero eigenvalue along n: the cost is linear along n with
//     slope n'(h_u + H_ux z_i); if n'H_ux = 0 and n'h_u = 0 the direction is
//     flat (a minimiser exists but is not unique; the pseudo-inverse picks
//     the one without that component), if n'H_ux = 0 and n'h_u != 0 there is
//     no minimiser, and if n'H_ux != 0 the answer depends on which z_i are
//     reachable, which this pass does not decide.
// The eigenvalues come from cyclic Jacobi rotations.  One wavefront per
// instance; the stage loop is sequential (this is a fallback for the
// instances the scan rejects, not a fast path).
#include <math.h>

#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "kernels.hpp"

namespace eclqr {

namespace {

constexpr double kEigTol = 1e-9;  // eigenvalue counted as zero within kEigTol * max(1, |largest|)

enum DpKind { kDpUnique = 0, kDpNotUnique = 1, kDpUndecided = 2, kDpNoMin = 3 };

// Y (r x c, ldy) = op(X) (r x k) times W (k x c), accumulated into Y when acc;
// one output entry per lane and round, each an FMA chain in ascending k.
__device__ inline void mm(double* Y, int ldy, const double* X, int ldx, bool tx, const double* W, int ldw, int r,
                          int c, int k, bool acc) {
  for (int idx = ECLQR_TID; idx < r * c; idx += ECLQR_NT) {
    const int i = idx / c, j = idx % c;
    double v = acc ? Y[i * ldy + j] : 0.0;
    if (tx) v = lane_chain<false>(v, X + i, ldx, W + j, ldw, k);
    else v = lane_chain<false>(v, X + i * ldx, 1, W + j, ldw, k);
    Y[i * ldy + j] = v;
  }
  wg_sync();
}

__device__ inline void sym(double* S, int ld, int n) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int i = idx / n, j = idx % n;
    if (i < j) {
      const double v = 0.5 * (S[i * ld + j] + S[j * ld + i]);
      S[i * ld + j] = v;
      S[j * ld + i] = v;
    }
  }
  wg_sync();
}

// Eigen-decomposition of the symmetric n x n matrix A (overwritten by a
// nearly diagonal matrix whose diagonal holds the eigenvalues) with the
// eigenvectors in the columns of V, by cyclic Jacobi rotations.
__device__ inline void jacobi_eig(double* A, int n, double* V) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  wg_sync();
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
      const double a = A[idx];
      tot += a * a;
      if (idx / n != idx % n) off += a * a;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if (!(off > 1e-32 * tot)) break;
    for (int p = 0; p + 1 < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        wg_sync();
        for (int k = ECLQR_TID; k < n; k += ECLQR_NT) {  // columns p, q of A and V
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
        wg_sync();
        for (int k = ECLQR_TID; k < n; k += ECLQR_NT) {  // rows p, q of A
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        wg_sync();
      }
  }
}

}  // namespace

// Instances eligible: ECLQR_NOT_CONVEX set, no outcome of the domains or the
// data (those leave no valid reduced problem).
constexpr int32_t kDpHard = ECLQR_INFEASIBLE_SUFFIX | ECLQR_INFEASIBLE_INITIAL | ECLQR_RANK_INCONSISTENT |
                            ECLQR_INVALID_INPUT | ECLQR_CAPACITY | ECLQR_TIMEOUT;

__global__ void __launch_bounds__(kBlock) k_dp_fallback(DevEngine e, Inputs in, const int64_t* sbase, double* x,
                                                        double* u, int32_t* status, int32_t* info, int32_t* dpflag,
                                                        double* scratch, int64_t stride, int maxn, int maxm) {
  __shared__ double zs[kMaxDim], vs[kMaxDim], z1[kMaxDim];
  double* w = scratch + (int64_t)blockIdx.x * stride;
  const int64_t nn = (int64_t)maxn * maxn, mm2 = (int64_t)maxm * maxm, nm = (int64_t)maxn * maxm;
  double* P = w;           // maxn^2  cost-to-go Hessian of stage i+1
  double* Pn = P + nn;     // maxn^2  H_xx, then the new P
  double* PA = Pn + nn;    // maxn^2  P A
  double* PB = PA + nn;    // maxn*maxm  P B
  double* Hux = PB + nm;   // maxm*maxn
  double* Wm = Hux + nm;   // maxm*maxn  V'H_ux scaled
  double* Huu = Wm + nm;   // maxm^2
  double* Vm = Huu + mm2;  // maxm^2
  double* pv = Vm + mm2;   // maxn  p
  double* pc = pv + maxn;  // maxn  P c + p
  double* hx = pc + maxn;  // maxn
  double* hu = hx + maxn;  // maxm
  double* wv = hu + maxm;  // maxm
  for (int b = blockIdx.x; b < e.B; b += gridDim.x) {
    if (ECLQR_TID == 0) dpflag[b] = 0;
    const int32_t sv = status[b];
    if (!(sv & ECLQR_NOT_CONVEX) || (sv & kDpHard)) continue;
    const int64_t s0 = sbase[b];
    const int N = e.st[s0].N;
    // terminal: P = Q-bar_N, p = q-bar_N (the elimination leaves them as the
    // terminal leaf J = Q-bar_N, eta = -q-bar_N of the value-function scan)
    {
      const StageInfo& st = e.st[s0 + N];
      const int nb = e.nbar[s0 + N];
      const RicLayout rl = ric_layout(st.n, 0);
      const double* leaf = slot_ptr(e, SCAN_RIC, st.elem[SCAN_RIC]);
      for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) P[idx] = leaf[rl.J + idx];
      for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) pv[i] = -leaf[rl.eta + i];
      wg_sync();
      sym(P, nb, nb);
      double* Vs = slot_ptr(e, SCAN_RIC, st.suf[SCAN_RIC]);
      for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) Vs[rl.J + idx] = P[idx];
      for (int i = ECLQR_TID; i < nb; i += ECLQR_NT) Vs[rl.eta + i] = -pv[i];
    }
    int kind = kDpUnique, fail = -1;
    for (int i = N - 1; i >= 0; --i) {
      const int64_t s = s0 + i;
      const StageInfo& st = e.st[s];
      const Arena ar = arena_layout(st.n, st.np, st.m, st.k);
      double* base = e.arena + st.ws;
      const int nb = e.nbar[s], nb1 = e.nbar[s + 1], mb = e.mbar[s];
      const double *Ab = base + ar.Ab, *Bb = base + ar.Bb, *cb = base + ar.cb, *Qb = base + ar.Qb;
      const double *Mb = base + ar.Mb, *Rb = base + ar.Rb, *qb = base + ar.qb, *rb = base + ar.rb;
      mm(PA, nb, P, nb1, false, Ab, nb, nb1, nb, nb1, false);  // P A  (nb1 x nb)
      mm(PB, mb, P, nb1, false, Bb, mb, nb1, mb, nb1, false);  // P B  (nb1 x mb)
      for (int r = ECLQR_TID; r < nb1; r += ECLQR_NT) pc[r] = lane_chain<false>(pv[r], P + r * nb1, 1, cb, 1, nb1);
      wg_sync();
      // H_xx = Q + A'PA, h_x = q + A'pc ; H_uu = R + B'PB ; H_ux = M' + B'PA ; h_u = r + B'pc
      for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) Pn[idx] = Qb[idx];
      for (int idx = ECLQR_TID; idx < mb * mb; idx += ECLQR_NT) Huu[idx] = Rb[idx];
      for (int idx = ECLQR_TID; idx < mb * nb; idx += ECLQR_NT) Hux[idx] = Mb[(idx % nb) * mb + idx / nb];
      wg_sync();
      mm(Pn, nb, Ab, nb, true, PA, nb, nb, nb, nb1, true);
      mm(Huu, mb, Bb, mb, true, PB, mb, mb, mb, nb1, true);
      mm(Hux, nb, Bb, mb, true, PA, nb, mb, nb, nb1, true);
      for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) hx[r] = lane_chain<false>(qb[r], Ab + r, nb, pc, 1, nb1);
      for (int r = ECLQR_TID; r < mb; r += ECLQR_NT) hu[r] = lane_chain<false>(rb[r], Bb + r, mb, pc, 1, nb1);
      wg_sync();
      sym(Pn, nb, nb);
      sym(Huu, mb, mb);
      if (mb > 0) {
        jacobi_eig(Huu, mb, Vm);
        double lmax = 0.0, lmin = HUGE_VAL;
        for (int j = 0; j < mb; ++j) {
          const double l = Huu[j * mb + j];
          lmax = fmax(lmax, fabs(l));
          lmin = fmin(lmin, l);
        }
        const double tol = kEigTol * fmax(1.0, lmax);
        int k = kDpUnique;
        if (lmin < -tol) k = kDpNoMin;
        // Wm = V'H_ux, wv = V'h_u; rows of zero eigenvalues tested, the others scaled by 1/lambda
        mm(Wm, nb, Vm, mb, true, Hux, nb, mb, nb, mb, false);
        for (int j = ECLQR_TID; j < mb; j += ECLQR_NT) wv[j] = lane_chain<false>(0.0, Vm + j, mb, hu, 1, mb);
        wg_sync();
        if (k == kDpUnique) {
          double hn = 0.0, gn = 0.0;
          for (int idx = ECLQR_TID; idx < mb * nb; idx += ECLQR_NT) hn += Hux[idx] * Hux[idx];
          for (int j = ECLQR_TID; j < mb; j += ECLQR_NT) gn += hu[j] * hu[j];
          hn = sqrt(wave_sum(hn));
          gn = sqrt(wave_sum(gn));
          for (int j = 0; j < mb && k != kDpNoMin; ++j) {
            if (fabs(Huu[j * mb + j]) > tol) continue;
            double r1 = 0.0;
            for (int c = ECLQR_TID; c < nb; c += ECLQR_NT) r1 += Wm[j * nb + c] * Wm[j * nb + c];
            r1 = sqrt(wave_sum(r1));
            if (r1 > kEigTol * fmax(1.0, hn)) {
              k = (k > kDpUndecided) ? k : kDpUndecided;
            } else if (fabs(wv[j]) > kEigTol * fmax(1.0, gn)) {
              k = kDpNoMin;
            } else if (k < kDpNotUnique) {
              k = kDpNotUnique;
            }
          }
        }
        if (k >= kDpUndecided) {
          kind = k;
          fail = i;
          break;
        }
        if (k > kind) kind = k;
        // K = -V Lambda^+ V'H_ux, k = -V Lambda^+ V'h_u (zero eigenvalues dropped)
        for (int idx = ECLQR_TID; idx < mb * nb; idx += ECLQR_NT) {
          const double l = Huu[(idx / nb) * mb + idx / nb];
          Wm[idx] = (fabs(l) > tol) ? Wm[idx] / l : 0.0;
        }
        for (int j = ECLQR_TID; j < mb; j += ECLQR_NT) {
          const double l = Huu[j * mb + j];
          wv[j] = (fabs(l) > tol) ? wv[j] / l : 0.0;
        }
        wg_sync();
        double* K = base + ar.K;
        double* kk = base + ar.kk;
        for (int idx = ECLQR_TID; idx < mb * nb; idx += ECLQR_NT) {
          const int r = idx / nb, c = idx % nb;
          K[idx] = -lane_chain<false>(0.0, Vm + r * mb, 1, Wm + c, nb, mb);
        }
        for (int r = ECLQR_TID; r < mb; r += ECLQR_NT) kk[r] = -lane_chain<false>(0.0, Vm + r * mb, 1, wv, 1, mb);
        wg_sync();
        // P = H_xx + H_ux'K, p = h_x + H_ux'k
        mm(Pn, nb, Hux, nb, true, K, nb, nb, nb, mb, true);
        for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) hx[r] = lane_chain<false>(hx[r], Hux + r, nb, kk, 1, mb);
        wg_sync();
      }
      sym(Pn, nb, nb);
      for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) P[idx] = Pn[idx];
      for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) pv[r] = hx[r];
      wg_sync();
      const RicLayout rl = ric_layout(st.n, 0);
      double* Vs = slot_ptr(e, SCAN_RIC, st.suf[SCAN_RIC]);
      for (int idx = ECLQR_TID; idx < nb * nb; idx += ECLQR_NT) Vs[rl.J + idx] = P[idx];
      for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) Vs[rl.eta + r] = -pv[r];
      wg_sync();
    }
    if (kind >= kDpUndecided) {
      if (ECLQR_TID == 0) {
        if (kind == kDpNoMin) status[b] = sv | ECLQR_NO_MINIMIZER;
        if (info) info[b] = fail;
      }
      continue;
    }
    // forward: z_0 = T_0'(x0 - t_0); v_i = K z_i + k; z_{i+1} = A z + B v + c;
    // x_i = T z + t, u_i = Y z + Z v + y
    {
      const StageInfo& st = e.st[s0];
      const Arena ar = arena_layout(st.n, st.np, st.m, st.k);
      const double* base = e.arena + st.ws;
      const int nb = e.nbar[s0];
      for (int c = ECLQR_TID; c < st.n; c += ECLQR_NT) z1[c] = in.x0[st.x0 + c] - base[ar.t + c];
      wg_sync();
      for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) zs[r] = lane_chain<false>(0.0, base + ar.T + r, nb, z1, 1, st.n);
      wg_sync();
    }
    for (int i = 0; i <= N; ++i) {
      const int64_t s = s0 + i;
      const StageInfo& st = e.st[s];
      const Arena ar = arena_layout(st.n, st.np, st.m, st.k);
      const double* base = e.arena + st.ws;
      const int nb = e.nbar[s];
      double* zslot = slot_ptr(e, SCAN_FWD, st.suf[SCAN_FWD]);
      for (int r = ECLQR_TID; r < nb; r += ECLQR_NT) zslot[r] = zs[r];
      for (int r = ECLQR_TID; r < st.n; r += ECLQR_NT)
        x[st.in[IN_q] + r] = lane_chain<false>(base[ar.t + r], base + ar.T + r * nb, 1, zs, 1, nb);
      if (i == N) break;
      const int nb1 = e.nbar[s + 1], mb = e.mbar[s];
      for (int r = ECLQR_TID; r < mb; r += ECLQR_NT)
        vs[r] = lane_chain<false>(base[ar.kk + r], base + ar.K + r * nb, 1, zs, 1, nb);
      wg_sync();
      for (int r = ECLQR_TID; r < st.m; r += ECLQR_NT) {
        double v = lane_chain<false>(base[ar.y + r], base + ar.Y + r * nb, 1, zs, 1, nb);
        u[st.in[IN_r] + r] = lane_chain<false>(v, base + ar.Z + r * mb, 1, vs, 1, mb);
      }
      for (int r = ECLQR_TID; r < nb1; r += ECLQR_NT) {
        double v = lane_chain<false>(base[ar.cb + r], base + ar.Ab + r * nb, 1, zs, 1, nb);
        z1[r] = lane_chain<false>(v, base + ar.Bb + r * mb, 1, vs, 1, mb);
      }
      wg_sync();
      for (int r = ECLQR_TID; r < nb1; r += ECLQR_NT) zs[r] = z1[r];
      wg_sync();
    }
    if (ECLQR_TID == 0) {
      status[b] = (kind == kDpNotUnique) ? ECLQR_NOT_UNIQUE : 0;
      dpflag[b] = 1;
      if (info) info[b] = -1;
    }
    wg_sync();
  }
}

// The fallback's instances skip refinement: their gate goes to the state of
// an instance accepted after the first pass.
__global__ void k_dp_hold(const int32_t* dpflag, int32_t* gate, int32_t B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x)
    if (dpflag[b]) gate[b] = kGateFinal;
}

__global__ void k_flag_where(const int32_t* flag, int32_t* out, int32_t bit, int32_t B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x)
    if (flag[b]) out[b] |= bit;
}

void launch_dp_fallback(const DevEngine& e, const Inputs& in, const int64_t* sbase, double* x, double* u,
                        int32_t* status, int32_t* info, int32_t* dpflag, double* scratch, int64_t stride,
                        int32_t blocks, int maxn, int maxm, hipStream_t s) {
  hipLaunchKernelGGL(k_dp_fallback, dim3(blocks), dim3(kBlock), 0, s, e, in, sbase, x, u, status, info, dpflag,
                     scratch, stride, maxn, maxm);
}
void launch_dp_hold(const int32_t* dpflag, int32_t* gate, int32_t B, hipStream_t s) {
  const int grid = (B + 255) / 256;
  hipLaunchKernelGGL(k_dp_hold, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, dpflag, gate, B);
}
void launch_flag_where(const int32_t* flag, int32_t* out, int32_t bit, int32_t B, hipStream_t s) {
  const int grid = (B + 255) / 256;
  hipLaunchKernelGGL(k_flag_where, dim3(grid > 0 ? grid : 1), dim3(256), 0, s, flag, out, bit, B);
}
}  // namespace eclqr
