// Multipliers (paper Section VII), refinement, residual (Section IX) and the
// adjoint gradient assembly.  All kernels are stage-parallel and memory-bound.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"

namespace eclqr {


// ---------------------------------------------------------------------------
// Matrices of the reversed-time stationarity problem:
//   stage 0:       A = [] (n_N x 0), B = E_N^T, R = I_{k_N}
//   stage j=1..N:  A = A_i^T, B = E_i^T, E = B_i^T, F = F_i^T, Q = I, R = I  (i = N - j)
//   terminal:      Q = I_{n_0}
// and zero linear terms.  x0 of the reversed problem is empty.
__global__ void __launch_bounds__(kBlock) k_dual_matrices(DevEngine p, Inputs in, DevEngine d, DualPtrs dp) {
  for (int64_t ds = blockIdx.x; ds < d.S; ds += gridDim.x) {
    const StageInfo sd = d.st[ds];
    const int b = sd.inst;
    const int N = sd.N - 1;
    const int64_t s0 = dp.pbase[b];
    const int ip = (sd.i == 0) ? N : ((sd.i <= N) ? N - sd.i : 0);
    const StageInfo sp = p.st[s0 + ip];
    double* Qd = dp.f[IN_Q] + sd.in[IN_Q];
    double* qd = dp.f[IN_q] + sd.in[IN_q];
    for (int idx = ECLQR_TID; idx < sd.n * sd.n; idx += ECLQR_NT) Qd[idx] = (idx / sd.n == idx % sd.n) ? 1.0 : 0.0;
    for (int idx = ECLQR_TID; idx < sd.n; idx += ECLQR_NT) qd[idx] = 0.0;
    if (sd.terminal) continue;
    double* Rd = dp.f[IN_R] + sd.in[IN_R];
    double* rd = dp.f[IN_r] + sd.in[IN_r];
    for (int idx = ECLQR_TID; idx < sd.m * sd.m; idx += ECLQR_NT) Rd[idx] = (idx / sd.m == idx % sd.m) ? 1.0 : 0.0;
    for (int idx = ECLQR_TID; idx < sd.m; idx += ECLQR_NT) rd[idx] = 0.0;
    double* Ad = dp.f[IN_A] + sd.in[IN_A];
    double* Bd = dp.f[IN_B] + sd.in[IN_B];
    double* Ed = dp.f[IN_E] + sd.in[IN_E];
    double* Fd = dp.f[IN_F] + sd.in[IN_F];
    const double* Ep = in.f[IN_E] + sp.in[IN_E];  // k x n
    // B^D = E^T  (n_i x k_i), also for the terminal block at dual stage 0
    for (int idx = ECLQR_TID; idx < sp.k * sp.n; idx += ECLQR_NT) {
      const int r = idx / sp.n, c = idx % sp.n;
      Bd[c * sp.k + r] = Ep[idx];
    }
    if (sd.i >= 1) {
      const double* Ap = in.f[IN_A] + sp.in[IN_A];  // np x n
      const double* Bp = in.f[IN_B] + sp.in[IN_B];  // np x m
      const double* Fp = in.f[IN_F] + sp.in[IN_F];  // k x m
      for (int idx = ECLQR_TID; idx < sp.np * sp.n; idx += ECLQR_NT) {
        const int r = idx / sp.n, c = idx % sp.n;
        Ad[c * sp.np + r] = Ap[idx];
      }
      for (int idx = ECLQR_TID; idx < sp.np * sp.m; idx += ECLQR_NT) {
        const int r = idx / sp.m, c = idx % sp.m;
        Ed[c * sp.np + r] = Bp[idx];
      }
      for (int idx = ECLQR_TID; idx < sp.k * sp.m; idx += ECLQR_NT) {
        const int r = idx / sp.m, c = idx % sp.m;
        Fd[c * sp.k + r] = Fp[idx];
      }
    }
    __syncthreads();
  }
}

// Offsets of the reversed-time problem: c^D_j = g^x_i, g^D_j = g^u_i at (x, u)
// (eq. (objective-gradients)); c^D_0 = g^x_N.
__global__ void __launch_bounds__(kBlock) k_dual_vectors(DevEngine p, Inputs in, const double* x, const double* u,
                                                         DevEngine d, DualPtrs dp) {
  if (none_live(p)) return;
  for (int64_t ds = blockIdx.x; ds < d.S; ds += gridDim.x) {
    const StageInfo sd = d.st[ds];
    if (sd.terminal || gated(d, sd.inst)) continue;
    const int b = sd.inst;
    const int N = sd.N - 1;
    const int64_t s0 = dp.pbase[b];
    const int ip = (sd.i == 0) ? N : N - sd.i;
    const StageInfo sp = p.st[s0 + ip];
    const double* xs = x + sp.in[IN_q];
    const double* Q = in.f[IN_Q] + sp.in[IN_Q];
    const double* q = in.f[IN_q] + sp.in[IN_q];
    double* cd = dp.f[IN_c] + sd.in[IN_c];
    const double* M = (in.f[IN_M] && !sp.terminal) ? in.f[IN_M] + sp.in[IN_M] : nullptr;
    const double* us = sp.terminal ? nullptr : u + sp.in[IN_r];
    for (int i = ECLQR_TID; i < sp.n; i += ECLQR_NT) {
      double v = q[i];
      v = lane_chain<false>(v, Q + i * sp.n, 1, xs, 1, sp.n);
      if (M)
        v = lane_chain<false>(v, M + i * sp.m, 1, us, 1, sp.m);
      cd[i] = v;
    }
    if (!sp.terminal) {
      const double* R = in.f[IN_R] + sp.in[IN_R];
      const double* r = in.f[IN_r] + sp.in[IN_r];
      double* gd = dp.f[IN_g] + sd.in[IN_g];
      for (int i = ECLQR_TID; i < sp.m; i += ECLQR_NT) {
        double v = r[i];
        v = lane_chain<false>(v, R + i * sp.m, 1, us, 1, sp.m);
        if (M)
          v = lane_chain<false>(v, M + i, sp.m, xs, 1, sp.n);
        gd[i] = v;
      }
    }
    __syncthreads();
  }
}

// lambda_i = x^D_{N-i+1}, mu_i = u^D_{N-i}.
__global__ void __launch_bounds__(kBlock) k_dual_extract(DevEngine p, DevEngine d, const double* dx, const double* du,
                                                         double* lam, double* mu, DualPtrs dp) {
  if (none_live(p)) return;
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo sp = p.st[s];
    if (gated(p, sp.inst)) continue;
    const int N = sp.N;
    const int64_t d0 = dp.dbase[sp.inst];
    const StageInfo& sx = d.st[d0 + (N - sp.i + 1)];
    const StageInfo& su = d.st[d0 + (N - sp.i)];
    for (int i = ECLQR_TID; i < sp.n; i += ECLQR_NT) lam[sp.in[IN_q] + i] = dx[sx.in[IN_q] + i];
    for (int i = ECLQR_TID; i < sp.k; i += ECLQR_NT) mu[sp.in[IN_g] + i] = du[su.in[IN_r] + i];
  }
}

// Correction problem of one refinement step: the same constrained LQR with
//   q <- stationarity residual of x (including -lambda_i + A'lambda_{i+1} + E'mu_i),
//   r <- stationarity residual of u, c <- dynamics residual, g <- row residual,
//   x0 <- x0 - x_0.
__global__ void __launch_bounds__(kBlock) k_correction(DevEngine p, Inputs in, const double* x, const double* u,
                                                       const double* lam, const double* mu, CorrPtrs cp) {
  if (none_live(p)) return;
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const double* xs = x + st.in[IN_q];
    const double* ls = lam + st.in[IN_q];
    const double* ms = mu + st.in[IN_g];
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* q = in.f[IN_q] + st.in[IN_q];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* g = in.f[IN_g] + st.in[IN_g];
    double* qo = cp.q + st.in[IN_q];
    double* go = cp.g + st.in[IN_g];
    if (st.terminal) {
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
        double v = q[i] - ls[i];
        v = lane_chain<false>(v, Q + i * n, 1, xs, 1, n);
        v = lane_chain<false>(v, E + i, n, ms, 1, k);
        qo[i] = v;
      }
      for (int i = ECLQR_TID; i < k; i += ECLQR_NT) {
        double v = g[i];
        v = lane_chain<false>(v, E + i * n, 1, xs, 1, n);
        go[i] = v;
      }
      __syncthreads();
      continue;
    }
    const StageInfo& st1 = p.st[s + 1];
    const double* x1 = x + st1.in[IN_q];
    const double* l1 = lam + st1.in[IN_q];
    const double* us = u + st.in[IN_r];
    const double* R = in.f[IN_R] + st.in[IN_R];
    const double* r = in.f[IN_r] + st.in[IN_r];
    const double* M = in.f[IN_M] ? in.f[IN_M] + st.in[IN_M] : nullptr;
    const double* A = in.f[IN_A] + st.in[IN_A];
    const double* B = in.f[IN_B] + st.in[IN_B];
    const double* c = in.f[IN_c] + st.in[IN_c];
    const double* F = in.f[IN_F] + st.in[IN_F];
    double* ro = cp.r + st.in[IN_r];
    double* co = cp.c + st.in[IN_c];
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double v = q[i] - ls[i];
      v = lane_chain<false>(v, Q + i * n, 1, xs, 1, n);
      if (M)
        v = lane_chain<false>(v, M + i * m, 1, us, 1, m);
      v = lane_chain<false>(v, A + i, n, l1, 1, np);
      v = lane_chain<false>(v, E + i, n, ms, 1, k);
      qo[i] = v;
    }
    for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
      double v = r[i];
      v = lane_chain<false>(v, R + i * m, 1, us, 1, m);
      if (M)
        v = lane_chain<false>(v, M + i, m, xs, 1, n);
      v = lane_chain<false>(v, B + i, m, l1, 1, np);
      v = lane_chain<false>(v, F + i, m, ms, 1, k);
      ro[i] = v;
    }
    for (int i = ECLQR_TID; i < np; i += ECLQR_NT) {
      double v = c[i] - x1[i];
      v = lane_chain<false>(v, A + i * n, 1, xs, 1, n);
      v = lane_chain<false>(v, B + i * m, 1, us, 1, m);
      co[i] = v;
    }
    for (int i = ECLQR_TID; i < k; i += ECLQR_NT) {
      double v = g[i];
      v = lane_chain<false>(v, E + i * n, 1, xs, 1, n);
      v = lane_chain<false>(v, F + i * m, 1, us, 1, m);
      go[i] = v;
    }
    if (st.i == 0)
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) cp.x0[st.x0 + i] = in.x0[st.x0 + i] - xs[i];
    __syncthreads();
  }
}

// x += dx, u += du for instances still refining; per stage, the squared norms
// of the correction and of the updated iterate (one wavefront per stage).
__global__ void __launch_bounds__(kBlock) k_refine_update(DevEngine p, double* x, double* u, const double* dx,
                                                          const double* du, double* norms) {
  if (none_live(p)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  for (int64_t s = (int64_t)blockIdx.x * waves + wave; s < p.S; s += (int64_t)gridDim.x * waves) {
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    double d2 = 0.0, w2 = 0.0;
    for (int i = lane; i < st.n; i += 64) {
      const double d = dx[st.in[IN_q] + i];
      const double w = x[st.in[IN_q] + i] + d;
      x[st.in[IN_q] + i] = w;
      d2 = fma(d, d, d2);
      w2 = fma(w, w, w2);
    }
    if (!st.terminal)
      for (int i = lane; i < st.m; i += 64) {
        const double d = du[st.in[IN_r] + i];
        const double w = u[st.in[IN_r] + i] + d;
        u[st.in[IN_r] + i] = w;
        d2 = fma(d, d, d2);
        w2 = fma(w, w, w2);
      }
    d2 = wave_sum(d2);
    w2 = wave_sum(w2);
    if (lane == 0) {
      norms[2 * s] = d2;
      norms[2 * s + 1] = w2;
    }
  }
}

// One workgroup per instance: fixed-order sums of the stage norms; an instance
// still refining becomes final when ||correction|| <= tol ||iterate|| or on the
// last step.
__global__ void __launch_bounds__(kBlock) k_refine_decide(DevEngine p, const int64_t* sbase, const double* norms,
                                                          double tol, int last, int32_t* gate, int32_t* steps) {
  if (none_live(p)) return;
  __shared__ double sd[kBlock], sw[kBlock];
  for (int b = blockIdx.x; b < p.B; b += gridDim.x) {
    if (gate[b] != kGateActive) continue;
    const int64_t s0 = sbase[b];
    const int L = p.st[s0].N + 1;
    double d2 = 0.0, w2 = 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
      d2 += norms[2 * (s0 + j)];
      w2 += norms[2 * (s0 + j) + 1];
    }
    sd[threadIdx.x] = d2;
    sw[threadIdx.x] = w2;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        sd[threadIdx.x] += sd[threadIdx.x + h];
        sw[threadIdx.x] += sw[threadIdx.x + h];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      steps[b] += 1;
      if (last || sd[0] <= tol * tol * sw[0]) gate[b] = kGateFinal;
    }
    __syncthreads();
  }
}

// The share of one lane of an 8-lane row group of v += sum_l a[l sa] b[l],
// mag += sum_l |a[l sa] b[l]|, an += sum_l |a[l sa]|: the terms l = c, c + 8,
// ... (c the lane's place in its group), so the group's loads of one step
// are 8 consecutive elements of a row-major row, or of 8 rows at one column.
// part_load fetches a share's first four terms (every row of up to 32 terms)
// so that the loads of all of a row's families are in flight together;
// part_acc adds them, then any further terms, in ascending l.  Masked terms
// are zeros, which leave the sums' bits unchanged.
struct Part4 {
  double a[4], b[4];
};

__device__ __forceinline__ Part4 part_load(const double* a, int sa, const double* b, int n, int c) {
  Part4 P;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int l = c + 8 * t;
    const bool ok = l < n;
    P.a[t] = ok ? a[l * sa] : 0.0;
    P.b[t] = ok ? b[l] : 0.0;
  }
  return P;
}

__device__ __forceinline__ void part_acc(const Part4& P, const double* a, int sa, const double* b, int n, int c,
                                         double& v, double& mag, double& an) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double tt = P.a[t] * P.b[t];
    v += tt;
    mag += fabs(tt);
    an += fabs(P.a[t]);
  }
  for (int l = c + 32; l < n; l += 8) {
    const double av = a[l * sa];
    const double tt = av * b[l];
    v += tt;
    mag += fabs(tt);
    an += fabs(av);
  }
}

// Sum over the 8 lanes of a row group (every lane ends with the group's sum).
__device__ __forceinline__ double group8_sum(double v) {
  v += __shfl_xor(v, 4, 8);
  v += __shfl_xor(v, 2, 8);
  v += __shfl_xor(v, 1, 8);
  return v;
}

// Largest |entry| of x, u, lambda, mu per instance (the scale of the
// unknowns), max-accumulated on the bit patterns of non-negative doubles.
__global__ void __launch_bounds__(kBlock) k_unknown_scale(DevEngine p, const double* x, const double* u,
                                                          const double* lam, const double* mu,
                                                          unsigned long long* wmax) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    double w = 0.0;
    for (int i = ECLQR_TID; i < st.n; i += ECLQR_NT)
      w = fmax(w, fmax(fabs(x[st.in[IN_q] + i]), fabs(lam[st.in[IN_q] + i])));
    if (!st.terminal)
      for (int i = ECLQR_TID; i < st.m; i += ECLQR_NT) w = fmax(w, fabs(u[st.in[IN_r] + i]));
    for (int i = ECLQR_TID; i < st.k; i += ECLQR_NT) w = fmax(w, fabs(mu[st.in[IN_g] + i]));
    w = wave_max(w);
    if (ECLQR_TID == 0) atomicMax(wmax + st.inst, (unsigned long long)__double_as_longlong(w));
  }
}

// Backward error of the KKT system at (x, u, lambda, mu), over stationarity
// in x and u, dynamics, equality rows and the initial condition: per row
// |residual| / (sum of |terms|), the componentwise measure, except on rows
// whose componentwise scale is negligible next to their normwise scale
// ||row||_1 ||unknowns||_inf + |offset| (below 1000 (terms) eps times it),
// which take the normwise measure instead -- the two-category backward error
// of Arioli, Demmel and Duff (SIAM J. Matrix Anal. Appl. 10(2), 1989).  Rows
// whose data and solution are near zero (an offset of rounding size, as in a
// Newton step at a feasible point) would otherwise demand a relative accuracy
// no solver reaches.  The maximum over rows; one wavefront per stage, eight
// rows at a time, each split over 8 lanes (coalesced 8-element segments of
// the row-major blocks instead of a row per lane); the
// per-instance maximum is accumulated with an integer atomic max on the bit
// pattern (order independent, so deterministic).
__global__ void __launch_bounds__(kBlock) k_backward_error(DevEngine p, Inputs in, const double* x, const double* u,
                                                           const double* lam, const double* mu,
                                                           const unsigned long long* wmax,
                                                           unsigned long long* omega) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int g = lane >> 3, c = lane & 7;  // row group (a row per group at a time), place in the group
  constexpr double kEps = 2.220446049250313e-16;
  for (int64_t s = (int64_t)blockIdx.x * waves + wave; s < p.S; s += (int64_t)gridDim.x * waves) {
    const StageInfo st = p.st[s];
    if (gated(p, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const double W = __longlong_as_double((long long)wmax[st.inst]);
    const double* xs = x + st.in[IN_q];
    const double* ls = lam + st.in[IN_q];
    const double* ms = mu + st.in[IN_g];
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* q = in.f[IN_q] + st.in[IN_q];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* gv = in.f[IN_g] + st.in[IN_g];
    const bool term = st.terminal;
    const double* us = term ? nullptr : u + st.in[IN_r];
    const double* F = term ? nullptr : in.f[IN_F] + st.in[IN_F];
    const double* M = (!term && in.f[IN_M]) ? in.f[IN_M] + st.in[IN_M] : nullptr;
    const double* A = term ? nullptr : in.f[IN_A] + st.in[IN_A];
    const double* B = term ? nullptr : in.f[IN_B] + st.in[IN_B];
    const double* R = term ? nullptr : in.f[IN_R] + st.in[IN_R];
    const double* r = term ? nullptr : in.f[IN_r] + st.in[IN_r];
    const double* cv = term ? nullptr : in.f[IN_c] + st.in[IN_c];
    const double* x1 = term ? nullptr : x + p.st[s + 1].in[IN_q];
    const double* l1 = term ? nullptr : lam + p.st[s + 1].in[IN_q];
    double w = 0.0;
    // res: residual, mag: sum of |terms|, an: sum of |coefficients|, b: the
    // row's offset, len: its number of terms
    auto acc = [&](double res, double mag, double an, double b, int len) {
      const double nrm = an * W + fabs(b);
      const double den = (mag > 1000.0 * len * kEps * nrm) ? mag : nrm;
      const double e = (den > 0.0) ? fabs(res) / den : (res == 0.0 ? 0.0 : HUGE_VAL);
      w = (e > w || e != e) ? e : w;
    };
    // every family of rows: each row group takes rows g, g + 8, ...; its 8
    // lanes split the row's terms, then sum them (all lanes of the wave run
    // the group sums)
    for (int i0 = 0; i0 < n; i0 += 8) {  // stationarity in x_i
      const int i = i0 + g;
      double v = 0.0, a = 0.0, an = 0.0;
      if (i < n) {
        const Part4 p0 = part_load(Q + i * n, 1, xs, n, c);
        const Part4 p1 = part_load(E + i, n, ms, k, c);
        const Part4 p2 = (!term && M) ? part_load(M + i * m, 1, us, m, c) : Part4{};
        const Part4 p3 = !term ? part_load(A + i, n, l1, np, c) : Part4{};
        part_acc(p0, Q + i * n, 1, xs, n, c, v, a, an);
        part_acc(p1, E + i, n, ms, k, c, v, a, an);
        if (!term) {
          if (M) part_acc(p2, M + i * m, 1, us, m, c, v, a, an);
          part_acc(p3, A + i, n, l1, np, c, v, a, an);
        }
      }
      v = group8_sum(v);
      a = group8_sum(a);
      an = group8_sum(an);
      if (i < n)
        acc((q[i] - ls[i]) + v, (fabs(q[i]) + fabs(ls[i])) + a, 1.0 + an, q[i],
            2 + n + k + (term ? 0 : (M ? m : 0) + np));
    }
    for (int i0 = 0; i0 < k; i0 += 8) {  // equality rows
      const int i = i0 + g;
      double v = 0.0, a = 0.0, an = 0.0;
      if (i < k) {
        const Part4 p0 = part_load(E + i * n, 1, xs, n, c);
        const Part4 p1 = !term ? part_load(F + i * m, 1, us, m, c) : Part4{};
        part_acc(p0, E + i * n, 1, xs, n, c, v, a, an);
        if (!term) part_acc(p1, F + i * m, 1, us, m, c, v, a, an);
      }
      v = group8_sum(v);
      a = group8_sum(a);
      an = group8_sum(an);
      if (i < k) acc(gv[i] + v, fabs(gv[i]) + a, an, gv[i], 1 + n + (term ? 0 : m));
    }
    if (!term) {
      for (int i0 = 0; i0 < m; i0 += 8) {  // stationarity in u_i
        const int i = i0 + g;
        double v = 0.0, a = 0.0, an = 0.0;
        if (i < m) {
          const Part4 p0 = part_load(R + i * m, 1, us, m, c);
          const Part4 p1 = M ? part_load(M + i, m, xs, n, c) : Part4{};
          const Part4 p2 = part_load(B + i, m, l1, np, c);
          const Part4 p3 = part_load(F + i, m, ms, k, c);
          part_acc(p0, R + i * m, 1, us, m, c, v, a, an);
          if (M) part_acc(p1, M + i, m, xs, n, c, v, a, an);
          part_acc(p2, B + i, m, l1, np, c, v, a, an);
          part_acc(p3, F + i, m, ms, k, c, v, a, an);
        }
        v = group8_sum(v);
        a = group8_sum(a);
        an = group8_sum(an);
        if (i < m) acc(r[i] + v, fabs(r[i]) + a, an, r[i], 1 + m + (M ? n : 0) + np + k);
      }
      for (int i0 = 0; i0 < np; i0 += 8) {  // dynamics
        const int i = i0 + g;
        double v = 0.0, a = 0.0, an = 0.0;
        if (i < np) {
          const Part4 p0 = part_load(A + i * n, 1, xs, n, c);
          const Part4 p1 = part_load(B + i * m, 1, us, m, c);
          part_acc(p0, A + i * n, 1, xs, n, c, v, a, an);
          part_acc(p1, B + i * m, 1, us, m, c, v, a, an);
        }
        v = group8_sum(v);
        a = group8_sum(a);
        an = group8_sum(an);
        if (i < np) acc((cv[i] - x1[i]) + v, (fabs(cv[i]) + fabs(x1[i])) + a, 1.0 + an, cv[i], 2 + n + m);
      }
    }
    if (st.i == 0)
      for (int i = lane; i < n; i += 64)
        acc(xs[i] - in.x0[st.x0 + i], fabs(xs[i]) + fabs(in.x0[st.x0 + i]), 1.0, in.x0[st.x0 + i], 2);
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(w, off, 64);
      w = (o > w || o != o) ? o : w;
    }
    if (lane == 0) {
      const double wv = (w != w) ? HUGE_VAL : w;
      atomicMax(omega + st.inst, (unsigned long long)__double_as_longlong(wv));
    }
  }
}

// Before the backward error of the returned point: an instance that took a
// refinement step is measured again (active, its scale and error cleared);
// the others are skipped and keep the first pass's figures, which are those
// of their unchanged solution.
__global__ void k_gate_refined(const int32_t* steps, int32_t* gate, unsigned long long* wmax,
                               unsigned long long* omega, int32_t B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
    if (steps[i] > 0) {
      gate[i] = kGateActive;
      wmax[i] = 0ull;
      omega[i] = 0ull;
    } else {
      gate[i] = kGateDone;
    }
  }
}

// Instances still refining whose backward error is <= tol and whose
// reversed-time solve succeeded are final without a refinement step.
__global__ void k_accept(const unsigned long long* omega, const int32_t* dstatus, double tol, int32_t* gate,
                         int32_t B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x)
    if (gate[i] == kGateActive && dstatus[i] == 0 && __longlong_as_double((long long)omega[i]) <= tol)
      gate[i] = kGateFinal;
}

__global__ void k_merge_dual_bits(int32_t* status, const int32_t* other, int32_t bit, int32_t mask, int32_t B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x)
    if (other[i] & mask) status[i] |= bit | ((other[i] & 0xff) << 8);
}

__global__ void k_flag_unconverged(const unsigned long long* omega, const int32_t* steps, double tol,
                                   int32_t* status, int32_t bit, int32_t B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x)
    if (steps[i] > 0 && !(__longlong_as_double((long long)omega[i]) <= tol)) status[i] |= bit;
}

// One workgroup: FINAL -> DONE, and the count of instances still ACTIVE.
__global__ void k_gate_advance(int32_t* gate, int32_t* live, int32_t B) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < B; i += blockDim.x) {
    int g = gate[i];
    if (g == kGateFinal) {
      g = kGateDone;
      gate[i] = g;
    }
    c += (g == kGateActive) ? 1 : 0;
  }
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) *live = cnt;
}
__global__ void k_fill(double* y, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void k_fill_u64(unsigned long long* y, unsigned long long v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void k_fill_i32(int32_t* y, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
// A failed reversed-time solve sets `bit` and keeps its own outcome bits in bits 8..15.
__global__ void k_merge_status(int32_t* status, const int32_t* other, int32_t bit, int32_t B, const int32_t* gate,
                               int32_t want) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x)
    if (other[i] != 0 && (!gate || gate[i] == want)) status[i] |= bit | ((other[i] & 0xff) << 8);
}

// Outputs of an instance whose status is not OK become NaN.
__global__ void __launch_bounds__(kBlock) k_finalize(DevEngine p, const int32_t* status, double* x, double* u,
                                                     double* lam, double* mu) {
  const double nan = __builtin_nan("");
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    if ((status[st.inst] & ~ECLQR_NOT_UNIQUE) == 0) continue;  // a minimiser, not unique, is kept
    for (int i = ECLQR_TID; i < st.n; i += ECLQR_NT) {
      x[st.in[IN_q] + i] = nan;
      if (lam) lam[st.in[IN_q] + i] = nan;
    }
    for (int i = ECLQR_TID; i < st.m; i += ECLQR_NT) u[st.in[IN_r] + i] = nan;
    if (mu)
      for (int i = ECLQR_TID; i < st.k; i += ECLQR_NT) mu[st.in[IN_g] + i] = nan;
  }
}

// KKT residual of Section IX, per stage: [initial, dynamics, equalities
// (rows / max(1, |coefficients|, |offset|)), stationarity], infinity norms.
__global__ void __launch_bounds__(kBlock) k_kkt_residual(DevEngine p, Inputs in, const double* x, const double* u,
                                                         const double* lam, const double* mu) {
  __shared__ double red[kBlock];
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const double* xs = x + st.in[IN_q];
    const double* ls = lam + st.in[IN_q];
    const double* ms = mu + st.in[IN_g];
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* q = in.f[IN_q] + st.in[IN_q];
    const double* E = in.f[IN_E] + st.in[IN_E];
    const double* g = in.f[IN_g] + st.in[IN_g];
    const double* us = st.terminal ? nullptr : u + st.in[IN_r];
    const double* F = st.terminal ? nullptr : in.f[IN_F] + st.in[IN_F];
    const double* M = (!st.terminal && in.f[IN_M]) ? in.f[IN_M] + st.in[IN_M] : nullptr;
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
    if (st.i == 0)
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) r0 = fmax(r0, fabs(xs[i] - in.x0[st.x0 + i]));
    for (int i = ECLQR_TID; i < k; i += ECLQR_NT) {
      double v = g[i], den = fmax(1.0, fabs(g[i]));
      for (int l = 0; l < n; ++l) {
        v = fma(E[i * n + l], xs[l], v);
        den = fmax(den, fabs(E[i * n + l]));
      }
      if (F)
        for (int l = 0; l < m; ++l) {
          v = fma(F[i * m + l], us[l], v);
          den = fmax(den, fabs(F[i * m + l]));
        }
      r2 = fmax(r2, fabs(v) / den);
    }
    if (st.terminal) {
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
        double v = q[i] - ls[i];
        v = lane_chain<false>(v, Q + i * n, 1, xs, 1, n);
        v = lane_chain<false>(v, E + i, n, ms, 1, k);
        r3 = fmax(r3, fabs(v));
      }
    } else {
      const StageInfo& st1 = p.st[s + 1];
      const double* x1 = x + st1.in[IN_q];
      const double* l1 = lam + st1.in[IN_q];
      const double* R = in.f[IN_R] + st.in[IN_R];
      const double* r = in.f[IN_r] + st.in[IN_r];
      const double* A = in.f[IN_A] + st.in[IN_A];
      const double* B = in.f[IN_B] + st.in[IN_B];
      const double* c = in.f[IN_c] + st.in[IN_c];
      for (int i = ECLQR_TID; i < np; i += ECLQR_NT) {
        double v = c[i] - x1[i];
        v = lane_chain<false>(v, A + i * n, 1, xs, 1, n);
        v = lane_chain<false>(v, B + i * m, 1, us, 1, m);
        r1 = fmax(r1, fabs(v));
      }
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
        double v = q[i] - ls[i];
        v = lane_chain<false>(v, Q + i * n, 1, xs, 1, n);
        if (M)
          v = lane_chain<false>(v, M + i * m, 1, us, 1, m);
        v = lane_chain<false>(v, A + i, n, l1, 1, np);
        v = lane_chain<false>(v, E + i, n, ms, 1, k);
        r3 = fmax(r3, fabs(v));
      }
      for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
        double v = r[i];
        v = lane_chain<false>(v, R + i * m, 1, us, 1, m);
        if (M)
          v = lane_chain<false>(v, M + i, m, xs, 1, n);
        v = lane_chain<false>(v, B + i, m, l1, 1, np);
        v = lane_chain<false>(v, F + i, m, ms, 1, k);
        r3 = fmax(r3, fabs(v));
      }
    }
    r0 = wg_reduce_max(r0, red);
    r1 = wg_reduce_max(r1, red);
    r2 = wg_reduce_max(r2, red);
    r3 = wg_reduce_max(r3, red);
    if (ECLQR_TID == 0) {
      p.resid[4 * s + 0] = r0;
      p.resid[4 * s + 1] = r1;
      p.resid[4 * s + 2] = r2;
      p.resid[4 * s + 3] = r3;
    }
    __syncthreads();
  }
}

__global__ void k_resid_reduce(DevEngine p, const int64_t* sbase, double* out) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < p.B; b += gridDim.x * blockDim.x) {
    const int64_t s0 = sbase[b];
    const int N = p.st[s0].N;
    double r[4] = {0, 0, 0, 0};
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j < 4; ++j) r[j] = fmax(r[j], p.resid[4 * (s0 + i) + j]);
    for (int j = 0; j < 4; ++j) out[4 * b + j] = r[j];
  }
}

// Gradients from the forward solution (x, u, lambda, mu) and the adjoint
// solution (a_x, a_u, a_lambda, a_mu) -- outer products of implicit
// differentiation of the KKT system.
__global__ void __launch_bounds__(kBlock) k_grad_assemble(DevEngine p, const double* x, const double* u,
                                                          const double* lam, const double* mu, const double* ax,
                                                          const double* au, const double* al, const double* am,
                                                          GradPtrs g, const int32_t* gstatus) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    if (gstatus[st.inst] != 0) {  // not differentiable (or failed): every gradient block of the stage is NaN
      const double nan = __builtin_nan("");
      const int n = st.n, np = st.np, m = st.m, k = st.k;
      const int64_t sz[IN_COUNT] = {(int64_t)n * n, n, (int64_t)m * m, m, (int64_t)n * m, (int64_t)np * n,
                                    (int64_t)np * m, np, (int64_t)k * n, (int64_t)k * m, k};
      for (int f = 0; f < IN_COUNT; ++f) {
        if (!g.f[f]) continue;
        for (int64_t j = ECLQR_TID; j < sz[f]; j += ECLQR_NT) g.f[f][st.in[f] + j] = nan;
      }
      if (st.i == 0)
        for (int i = ECLQR_TID; i < n; i += ECLQR_NT) g.x0[st.x0 + i] = nan;
      continue;
    }
    const int n = st.n, np = st.np, m = st.m, k = st.k;
    const double* xs = x + st.in[IN_q];
    const double* axs = ax + st.in[IN_q];
    const double* ms = mu + st.in[IN_g];
    const double* ams = am + st.in[IN_g];
    for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
      const int i = idx / n, j = idx % n;
      g.f[IN_Q][st.in[IN_Q] + idx] = 0.5 * (axs[i] * xs[j] + xs[i] * axs[j]);
    }
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) g.f[IN_q][st.in[IN_q] + i] = axs[i];
    for (int idx = ECLQR_TID; idx < k * n; idx += ECLQR_NT) {
      const int i = idx / n, j = idx % n;
      g.f[IN_E][st.in[IN_E] + idx] = ms[i] * axs[j] + ams[i] * xs[j];
    }
    for (int i = ECLQR_TID; i < k; i += ECLQR_NT) g.f[IN_g][st.in[IN_g] + i] = ams[i];
    if (st.i == 0)
      for (int i = ECLQR_TID; i < n; i += ECLQR_NT) g.x0[st.x0 + i] = al[st.in[IN_q] + i];
    if (!st.terminal) {
      const StageInfo& st1 = p.st[s + 1];
      const double* us = u + st.in[IN_r];
      const double* aus = au + st.in[IN_r];
      const double* l1 = lam + st1.in[IN_q];
      const double* al1 = al + st1.in[IN_q];
      for (int idx = ECLQR_TID; idx < m * m; idx += ECLQR_NT) {
        const int i = idx / m, j = idx % m;
        g.f[IN_R][st.in[IN_R] + idx] = 0.5 * (aus[i] * us[j] + us[i] * aus[j]);
      }
      for (int i = ECLQR_TID; i < m; i += ECLQR_NT) g.f[IN_r][st.in[IN_r] + i] = aus[i];
      if (g.f[IN_M])
        for (int idx = ECLQR_TID; idx < n * m; idx += ECLQR_NT) {
          const int i = idx / m, j = idx % m;
          g.f[IN_M][st.in[IN_M] + idx] = axs[i] * us[j] + xs[i] * aus[j];
        }
      for (int idx = ECLQR_TID; idx < np * n; idx += ECLQR_NT) {
        const int i = idx / n, j = idx % n;
        g.f[IN_A][st.in[IN_A] + idx] = l1[i] * axs[j] + al1[i] * xs[j];
      }
      for (int idx = ECLQR_TID; idx < np * m; idx += ECLQR_NT) {
        const int i = idx / m, j = idx % m;
        g.f[IN_B][st.in[IN_B] + idx] = l1[i] * aus[j] + al1[i] * us[j];
      }
      for (int i = ECLQR_TID; i < np; i += ECLQR_NT) g.f[IN_c][st.in[IN_c] + i] = al1[i];
      for (int idx = ECLQR_TID; idx < k * m; idx += ECLQR_NT) {
        const int i = idx / m, j = idx % m;
        g.f[IN_F][st.in[IN_F] + idx] = ms[i] * aus[j] + ams[i] * us[j];
      }
    }
  }
}

// One wavefront per instance: the rows of its constraint Jacobian (x_0 = x0,
// dynamics, stage rows, terminal rows) number n_0 + sum (n_{i+1} + k_i) + k_N
// and its variables sum n_i + sum m_i; the feasible set found by the forward
// pass has dimension sum m-bar_i (z_0 is fixed and every free input
// coordinate is independent), so rank = dim(w) - sum m-bar_i, and the rows are
// independent exactly when sum_{i<N} (m_i - m-bar_i) - sum_{i<=N} k_i = 0.
__global__ void __launch_bounds__(kBlock) k_licq(DevEngine p, const int64_t* sbase, const int32_t* fstatus,
                                                 int32_t* gstatus) {
  for (int b = blockIdx.x; b < p.B; b += gridDim.x) {
    const int64_t s0 = sbase[b];
    const int N = p.st[s0].N;
    long long def = 0;
    for (int i = threadIdx.x; i <= N; i += kBlock) {
      const StageInfo& st = p.st[s0 + i];
      def += st.terminal ? -(long long)st.k : (long long)(st.m - p.mbar[s0 + i] - st.k);
    }
    const double tot = wave_sum((double)def);
    if (threadIdx.x == 0) gstatus[b] = fstatus[b] | ((tot != 0.0) ? ECLQR_NOT_DIFFERENTIABLE : 0);
  }
}

__global__ void __launch_bounds__(kBlock) k_adjoint_offsets(DevEngine p, const double* dlam, double* c, double* x0) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo& st = p.st[s];
    if (!st.terminal) {
      const StageInfo& st1 = p.st[s + 1];
      for (int i = threadIdx.x; i < st.np; i += kBlock) c[st.in[IN_c] + i] = dlam[st1.in[IN_q] + i];
    }
    if (st.i == 0)
      for (int i = threadIdx.x; i < st.n; i += kBlock) x0[st.x0 + i] = dlam[st.in[IN_q] + i];
  }
}

// ---------------------------------------------------------------------------
static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

int fit_grid(const void* fn, int block, size_t lds, int64_t want) {
  if (want < 1) return 1;
  const int cap_want = (int)std::min<int64_t>(want, 1 << 30);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return cap_want;
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int> cache;
  const auto key = std::make_tuple(dev, fn, block, lds);
  int cap = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) cap = it->second;
  }
  if (cap == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds) != hipSuccess || per_cu < 1 ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
      (void)hipGetLastError();
      return cap_want;
    }
    cap = per_cu * cus;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = cap;
  }
  return std::min(cap_want, cap);
}

void launch_dual_matrices(const DevEngine& p, const Inputs& in, const DevEngine& d, const DualPtrs& dp,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_dual_matrices, dim3(d.nblocks), dim3(kBlock), 0, s, p, in, d, dp);
}
void launch_dual_vectors(const DevEngine& p, const Inputs& in, const double* x, const double* u, const DevEngine& d,
                         const DualPtrs& dp, hipStream_t s) {
  hipLaunchKernelGGL(k_dual_vectors, dim3(d.nblocks), dim3(kBlock), 0, s, p, in, x, u, d, dp);
}
void launch_dual_extract(const DevEngine& p, const DevEngine& d, const double* dx, const double* du, double* lam,
                         double* mu, const DualPtrs& dp, hipStream_t s) {
  hipLaunchKernelGGL(k_dual_extract, dim3(p.nblocks), dim3(kBlock), 0, s, p, d, dx, du, lam, mu, dp);
}
void launch_correction(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                       const double* mu, const CorrPtrs& cp, hipStream_t s) {
  hipLaunchKernelGGL(k_correction, dim3(p.nblocks), dim3(kBlock), 0, s, p, in, x, u, lam, mu, cp);
}
void launch_refine_update(const DevEngine& p, double* x, double* u, const double* dx, const double* du,
                          double* norms, hipStream_t s) {
  const int64_t g = std::min<int64_t>(4096, std::max<int64_t>(1, (p.S + 3) / 4));
  hipLaunchKernelGGL(k_refine_update, dim3((unsigned)g), dim3(kBlock), 0, s, p, x, u, dx, du, norms);
}
void launch_refine_decide(const DevEngine& p, const int64_t* sbase, const double* norms, double tol, int last,
                          int32_t* gate, int32_t* steps, hipStream_t s) {
  const int g = std::min(4096, std::max(1, p.B));
  hipLaunchKernelGGL(k_refine_decide, dim3(g), dim3(kBlock), 0, s, p, sbase, norms, tol, last, gate, steps);
}
void launch_backward_error(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                           const double* mu, unsigned long long* wmax, unsigned long long* omega, hipStream_t s,
                           bool clear) {
  if (clear) launch_fill_u64(wmax, 0ull, p.B, s);
  hipLaunchKernelGGL(k_unknown_scale, dim3(p.nblocks), dim3(kBlock), 0, s, p, x, u, lam, mu, wmax);
  hipLaunchKernelGGL(k_backward_error, dim3(p.nblocks), dim3(kBlock), 0, s, p, in, x, u, lam, mu, wmax, omega);
}
void launch_gate_refined(const int32_t* steps, int32_t* gate, unsigned long long* wmax, unsigned long long* omega,
                         int32_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_gate_refined, dim3(grid_for(B)), dim3(256), 0, s, steps, gate, wmax, omega, B);
}
void launch_accept(const unsigned long long* omega, const int32_t* dstatus, double tol, int32_t* gate, int32_t B,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_accept, dim3(grid_for(B)), dim3(256), 0, s, omega, dstatus, tol, gate, B);
}
void launch_fill_u64(unsigned long long* y, unsigned long long v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, s, y, v, n);
}
void launch_merge_dual_bits(int32_t* status, const int32_t* other, int32_t bit, int32_t mask, int32_t B,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_merge_dual_bits, dim3(grid_for(B)), dim3(256), 0, s, status, other, bit, mask, B);
}
void launch_flag_unconverged(const unsigned long long* omega, const int32_t* steps, double tol, int32_t* status,
                             int32_t bit, int32_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_unconverged, dim3(grid_for(B)), dim3(256), 0, s, omega, steps, tol, status, bit, B);
}
void launch_gate_advance(int32_t* gate, int32_t* live, int32_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_gate_advance, dim3(1), dim3(256), 0, s, gate, live, B);
}
void launch_fill(double* y, double v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, y, v, n);
}
void launch_fill_i32(int32_t* y, int32_t v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, y, v, n);
}
void launch_merge_status(int32_t* status, const int32_t* other, int32_t bit, int32_t B, const int32_t* gate,
                         int32_t want, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_status, dim3(grid_for(B)), dim3(256), 0, s, status, other, bit, B, gate, want);
}
void launch_finalize(const DevEngine& p, const int32_t* status, double* x, double* u, double* lam, double* mu,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(p.nblocks), dim3(kBlock), 0, s, p, status, x, u, lam, mu);
}
void launch_kkt_residual(const DevEngine& p, const Inputs& in, const double* x, const double* u, const double* lam,
                         const double* mu, const int64_t* sbase, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_kkt_residual, dim3(p.nblocks), dim3(kBlock), 0, s, p, in, x, u, lam, mu);
  hipLaunchKernelGGL(k_resid_reduce, dim3(grid_for(p.B)), dim3(256), 0, s, p, sbase, out);
}
void launch_grad_assemble(const DevEngine& p, const double* x, const double* u, const double* lam, const double* mu,
                          const double* ax, const double* au, const double* al, const double* am, const GradPtrs& g,
                          const int32_t* gstatus, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_assemble, dim3(p.nblocks), dim3(kBlock), 0, s, p, x, u, lam, mu, ax, au, al, am, g,
                     gstatus);
}
void launch_licq(const DevEngine& p, const int64_t* sbase, const int32_t* fstatus, int32_t* gstatus, hipStream_t s) {
  const int grid = p.B < 4096 ? p.B : 4096;
  hipLaunchKernelGGL(k_licq, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, s, p, sbase, fstatus, gstatus);
}
void launch_adjoint_offsets(const DevEngine& p, const double* dlam, double* c, double* x0, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_offsets, dim3(p.nblocks), dim3(kBlock), 0, s, p, dlam, c, x0);
}

}  // namespace eclqr
