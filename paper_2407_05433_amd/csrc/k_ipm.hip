// Elementwise kernels of the interior-point driver for bound-constrained
// problems (the use that motivates the method in Section I: a sequence of
// equality-constrained LQR problems of fixed structure whose diagonal
// weights change).  Each linear system of Mehrotra's predictor-corrector
// method is one solve of the same plan; these kernels form its data from the
// current iterate, choose the step and take it.
//
// Bounds lo <= v <= hi apply to the inputs u_i and to the states x_i, i >= 1
// (x_0 is fixed); an absent side (null array or infinite entry) is no bound.
// With d_lo = v - lo, d_hi = hi - v, bound multipliers z_lo, z_hi and
// complementarity targets t_lo, t_hi, the Newton problem has Hessian diagonal
// S = z_lo/d_lo + z_hi/d_hi added to Q, R, linear terms
// grad f - t_lo/d_lo + t_hi/d_hi, and offsets equal to the current equality
// residuals; its solution is the step dv and its multipliers the new equality
// multipliers; then
//   dz_lo = t_lo/d_lo - z_lo - (z_lo/d_lo) dv,
//   dz_hi = t_hi/d_hi - z_hi + (z_hi/d_hi) dv.
// The predictor takes zero targets; the corrector takes
//   t_lo = sigma mu - dz_lo_aff dv_aff,   t_hi = sigma mu + dz_hi_aff dv_aff
// from the predictor's step (aff), with sigma = min(1, (mu_aff/mu)^3).
#include <math.h>

#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "kernels.hpp"

namespace eclqr {

namespace {

struct Bound {
  double lo, hi;
  bool fl, fh;
};
__device__ inline Bound bound_at(const double* lo, const double* hi, int64_t j) {
  Bound b;
  b.lo = lo ? lo[j] : -HUGE_VAL;
  b.hi = hi ? hi[j] : HUGE_VAL;
  b.fl = isfinite(b.lo);
  b.fh = isfinite(b.hi);
  return b;
}

// The bounded variables of a stage, numbered j < nu + nx: inputs first
// (offset in the layout of r), then states (layout of q; stage 0 has none).
struct Blocks {
  int64_t uo, xo;
  int nu, nx;
};
__device__ inline Blocks blocks_of(const StageInfo& st) {
  Blocks b;
  b.uo = st.in[IN_r];
  b.xo = st.in[IN_q];
  b.nu = st.terminal ? 0 : st.m;
  b.nx = (st.i == 0) ? 0 : st.n;
  return b;
}

// One bounded variable at the current iterate.
struct Var {
  Bound b;
  int64_t o;      // element offset (layout of r for inputs, of q for states)
  bool isu;
  double v, zl, zh, dl, dh;  // value, multipliers, distances to the bounds (1 where absent)
};
__device__ inline Var var_at(const IpmBounds& bd, const double* x, const double* u, const IpmDuals& z,
                             const Blocks& bl, int j) {
  Var w;
  w.isu = j < bl.nu;
  w.o = w.isu ? bl.uo + j : bl.xo + (j - bl.nu);
  w.b = w.isu ? bound_at(bd.u_lo, bd.u_hi, w.o) : bound_at(bd.x_lo, bd.x_hi, w.o);
  w.v = w.isu ? u[w.o] : x[w.o];
  w.zl = w.b.fl ? (w.isu ? z.ul[w.o] : z.xl[w.o]) : 0.0;
  w.zh = w.b.fh ? (w.isu ? z.uh[w.o] : z.xh[w.o]) : 0.0;
  w.dl = w.b.fl ? w.v - w.b.lo : 1.0;
  w.dh = w.b.fh ? w.b.hi - w.v : 1.0;
  return w;
}
__device__ inline double step_of(const Var& w, const double* dx, const double* du) {
  return w.isu ? du[w.o] : dx[w.o];
}

// Complementarity targets of one variable: zero without a predictor step
// (ax, au null), else the corrector's second-order targets.
struct Targets {
  double tl, th;
};
__device__ inline Targets targets_of(const Var& w, const double* ax, const double* au, double smu) {
  Targets t{0.0, 0.0};
  if (!ax) return t;
  const double da = step_of(w, ax, au);
  if (w.b.fl) t.tl = smu - (-w.zl - w.zl / w.dl * da) * da;
  if (w.b.fh) t.th = smu + (-w.zh + w.zh / w.dh * da) * da;
  return t;
}
__device__ inline double dz_lo(const Var& w, const Targets& t, double dv) {
  return w.b.fl ? t.tl / w.dl - w.zl - w.zl / w.dl * dv : 0.0;
}
__device__ inline double dz_hi(const Var& w, const Targets& t, double dv) {
  return w.b.fh ? t.th / w.dh - w.zh + w.zh / w.dh * dv : 0.0;
}

__device__ inline bool active(const int32_t* act, int inst) { return act[inst] != 0; }

__device__ inline double wave_min(double v) { return -wave_max(-v); }

__device__ inline double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }

}  // namespace

// Start-solve outcome: the status of the equality-constrained solve; only
// the instances it solved take Newton steps.
__global__ void k_ipm_start(const int32_t* nstatus, int32_t* status, int32_t* act, int32_t* steps, int32_t B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const int32_t v = nstatus[b];
    status[b] = v;
    act[b] = v == 0;
    steps[b] = 0;
  }
}

// Starting point: the equality-constrained solution moved inside the bounds
// (at least `interior` of a two-sided gap, or of max(1, |bound|) from a
// one-sided bound), z = mu0 / distance.  A NaN bound or lo >= hi flags the
// instance.  One wavefront per stage.
__global__ void __launch_bounds__(kBlock) k_ipm_init(DevEngine p, IpmBounds bd, double* x, double* u, IpmDuals z,
                                                     double mu0, double interior, int32_t* status, int32_t* act) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo& st = p.st[s];
    const Blocks bl = blocks_of(st);
    bool bad = false;
    for (int j = ECLQR_TID; j < bl.nu + bl.nx; j += ECLQR_NT) {
      const bool isu = j < bl.nu;
      const int64_t o = isu ? bl.uo + j : bl.xo + (j - bl.nu);
      const Bound b = isu ? bound_at(bd.u_lo, bd.u_hi, o) : bound_at(bd.x_lo, bd.x_hi, o);
      double* v = isu ? u + o : x + o;
      const bool two = b.fl && b.fh;
      if (isnan(b.lo) || isnan(b.hi) || (two && !(b.lo < b.hi))) bad = true;
      const double gap = two ? b.hi - b.lo : 0.0;
      const double offl = two ? interior * gap : interior * fmax(1.0, fabs(b.fl ? b.lo : 0.0));
      const double offh = two ? interior * gap : interior * fmax(1.0, fabs(b.fh ? b.hi : 0.0));
      double w = *v;
      if (b.fl) w = fmax(w, b.lo + offl);
      if (b.fh) w = fmin(w, b.hi - offh);
      *v = w;
      (isu ? z.ul : z.xl)[o] = b.fl ? mu0 / (w - b.lo) : 0.0;
      (isu ? z.uh : z.xh)[o] = b.fh ? mu0 / (b.hi - w) : 0.0;
    }
    if (st.i == 0)  // x_0 carries no bound
      for (int j = ECLQR_TID; j < st.n; j += ECLQR_NT) {
        z.xl[st.in[IN_q] + j] = 0.0;
        z.xh[st.in[IN_q] + j] = 0.0;
      }
    if (__any(bad) && ECLQR_TID == 0) {
      atomicOr(status + st.inst, ECLQR_INVALID_INPUT);
      act[st.inst] = 0;
    }
  }
}

// Per stage: the sum of complementarity products (part[2 s]) and the count of
// finite bounds (part[2 s + 1]), at the iterate or, with ax non-null, after
// the predictor step of length alpha[instance] (zero targets).
__global__ void __launch_bounds__(kBlock) k_ipm_partial(DevEngine p, IpmBounds bd, const double* x, const double* u,
                                                        IpmDuals z, const double* ax, const double* au,
                                                        const unsigned long long* alpha, double* part) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo& st = p.st[s];
    const Blocks bl = blocks_of(st);
    const double a = ax ? bits_to_double(alpha[st.inst]) : 0.0;
    const Targets t{0.0, 0.0};
    double prod = 0.0, cnt = 0.0;
    for (int j = ECLQR_TID; j < bl.nu + bl.nx; j += ECLQR_NT) {
      const Var w = var_at(bd, x, u, z, bl, j);
      const double dv = ax ? step_of(w, ax, au) : 0.0;
      if (w.b.fl) {
        prod += (w.zl + a * dz_lo(w, t, dv)) * (w.dl + a * dv);
        cnt += 1.0;
      }
      if (w.b.fh) {
        prod += (w.zh + a * dz_hi(w, t, dv)) * (w.dh - a * dv);
        cnt += 1.0;
      }
    }
    prod = wave_sum(prod);
    cnt = wave_sum(cnt);
    if (ECLQR_TID == 0) {
      part[2 * s] = prod;
      part[2 * s + 1] = cnt;
    }
  }
}

// Per instance, from the stage sums in stage order (deterministic):
// mode 0: mu = sum / count; an active instance whose mu is below mu_stop
// stops.  mode 1: mu_aff = sum / count and smu = min(1, (mu_aff/mu)^3) mu.
__global__ void __launch_bounds__(kBlock) k_ipm_mu(DevEngine p, const int64_t* sbase, const double* part, int mode,
                                                   double mu_stop, double* mu, double* smu, int32_t* act) {
  for (int b = blockIdx.x; b < p.B; b += gridDim.x) {
    const int64_t s0 = sbase[b];
    const int N = p.st[s0].N;
    double prod = 0.0, cnt = 0.0;
    for (int i = ECLQR_TID; i <= N; i += ECLQR_NT) {
      prod += part[2 * (s0 + i)];
      cnt += part[2 * (s0 + i) + 1];
    }
    prod = wave_sum(prod);
    cnt = wave_sum(cnt);
    if (ECLQR_TID == 0) {
      const double m = prod / fmax(cnt, 1.0);
      if (mode == 0) {
        mu[b] = m;
        if (!(m >= mu_stop)) act[b] = 0;
      } else {
        const double r = m / mu[b];
        smu[b] = fmin(1.0, r * r * r) * mu[b];
      }
    }
  }
}

// Data of the Newton problem at the current iterate.  Matrices not written
// (M, A, B, E, F) are the problem's own.  vectors_only: the corrector, whose
// matrices and offsets are the predictor's; only q and r change.
__global__ void __launch_bounds__(kBlock) k_ipm_newton(DevEngine p, Inputs in, IpmBounds bd, const double* x,
                                                       const double* u, IpmDuals z, const double* ax,
                                                       const double* au, const double* smu, int vectors_only,
                                                       IpmNewton nw) {
  __shared__ double gx[kMaxDim], gu[kMaxDim];
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo st = p.st[s];
    const int n = st.n, np = st.np, m = st.terminal ? 0 : st.m, k = st.k;
    const double sm = ax ? smu[st.inst] : 0.0;
    const Blocks bl = blocks_of(st);
    const double* Q = in.f[IN_Q] + st.in[IN_Q];
    const double* xs = x + st.in[IN_q];
    const double* us = st.terminal ? nullptr : u + st.in[IN_r];
    const double* Mm = (in.f[IN_M] && !st.terminal) ? in.f[IN_M] + st.in[IN_M] : nullptr;
    // objective gradient: g^x = Q x + M u + q, g^u = R u + M' x + r
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
    if (!vectors_only) {
      double* Qn = nw.Q + st.in[IN_Q];
      for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) Qn[idx] = Q[idx];
      if (!st.terminal) {
        const double* R = in.f[IN_R] + st.in[IN_R];
        double* Rn = nw.R + st.in[IN_R];
        for (int idx = ECLQR_TID; idx < m * m; idx += ECLQR_NT) Rn[idx] = R[idx];
      }
    }
    wg_sync();
    // the linear terms of every variable, bounded or not, and the diagonal S
    // of the bounded ones (x_0 has no bound)
    for (int j = ECLQR_TID; j < m + n; j += ECLQR_NT) {
      const bool isu = j < m;
      const int c = isu ? j : j - m;
      double S = 0.0, gb = 0.0;
      if (isu || st.i > 0) {
        const Var w = var_at(bd, x, u, z, bl, isu ? c : bl.nu + c);
        const Targets t = targets_of(w, ax, au, sm);
        if (w.b.fl) {
          S += w.zl / w.dl;
          gb -= t.tl / w.dl;
        }
        if (w.b.fh) {
          S += w.zh / w.dh;
          gb += t.th / w.dh;
        }
      }
      if (isu) {
        nw.r[st.in[IN_r] + c] = gu[c] + gb;
        if (!vectors_only) nw.R[st.in[IN_R] + c * m + c] += S;
      } else {
        nw.q[st.in[IN_q] + c] = gx[c] + gb;
        if (!vectors_only) nw.Q[st.in[IN_Q] + c * n + c] += S;
      }
    }
    if (!vectors_only) {
      // E x + F u + g (offsets of the Newton rows)
      const double* E = in.f[IN_E] + st.in[IN_E];
      const double* F = st.terminal ? nullptr : in.f[IN_F] + st.in[IN_F];
      const double* g = in.f[IN_g] + st.in[IN_g];
      for (int r = ECLQR_TID; r < k; r += ECLQR_NT) {
        double v = lane_chain<false>(g[r], E + r * n, 1, xs, 1, n);
        if (F) v = lane_chain<false>(v, F + r * m, 1, us, 1, m);
        nw.g[st.in[IN_g] + r] = v;
      }
      if (st.i == 0)
        for (int a = ECLQR_TID; a < n; a += ECLQR_NT) nw.x0[st.x0 + a] = in.x0[st.x0 + a] - xs[a];
      if (!st.terminal) {
        // A x + B u + c - x' (the dynamics residual)
        const double* A = in.f[IN_A] + st.in[IN_A];
        const double* B = in.f[IN_B] + st.in[IN_B];
        const double* cv = in.f[IN_c] + st.in[IN_c];
        const double* x1 = x + p.st[s + 1].in[IN_q];
        for (int r = ECLQR_TID; r < np; r += ECLQR_NT) {
          double v = cv[r] - x1[r];
          v = lane_chain<false>(v, A + r * n, 1, xs, 1, n);
          v = lane_chain<false>(v, B + r * m, 1, us, 1, m);
          nw.c[st.in[IN_c] + r] = v;
        }
      }
    }
    wg_sync();
  }
}

// Largest step alpha <= 1 of each instance with v + alpha dv inside the
// bounds and z + alpha dz >= 0, each ratio scaled by tau (1 for the
// predictor, the fraction to the boundary for the corrector).  alpha holds
// the bits of non-negative doubles, min-accumulated from 1.
__global__ void __launch_bounds__(kBlock) k_ipm_alpha(DevEngine p, IpmBounds bd, const double* x, const double* u,
                                                      IpmDuals z, const double* dx, const double* du,
                                                      const double* ax, const double* au, const double* smu,
                                                      double tau, unsigned long long* alpha, const int32_t* act) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo& st = p.st[s];
    if (!active(act, st.inst)) continue;
    const Blocks bl = blocks_of(st);
    const double sm = ax ? smu[st.inst] : 0.0;
    double a = 1.0;
    for (int j = ECLQR_TID; j < bl.nu + bl.nx; j += ECLQR_NT) {
      const Var w = var_at(bd, x, u, z, bl, j);
      const Targets t = targets_of(w, ax, au, sm);
      const double dv = step_of(w, dx, du);
      if (w.b.fl) {
        const double dz = dz_lo(w, t, dv);
        if (dv < 0.0) a = fmin(a, tau * (w.dl / -dv));
        if (dz < 0.0) a = fmin(a, tau * (w.zl / -dz));
      }
      if (w.b.fh) {
        const double dz = dz_hi(w, t, dv);
        if (dv > 0.0) a = fmin(a, tau * (w.dh / dv));
        if (dz < 0.0) a = fmin(a, tau * (w.zh / -dz));
      }
    }
    a = wave_min(a);
    if (ECLQR_TID == 0) atomicMin(alpha + st.inst, (unsigned long long)__double_as_longlong(a));
  }
}

// The step of the active instances: v += alpha dv, z += alpha dz,
// (lam, mu) += alpha (new - old); steps counts it.
__global__ void __launch_bounds__(kBlock) k_ipm_update(DevEngine p, IpmBounds bd, double* x, double* u, double* lam,
                                                       double* mu_eq, IpmDuals z, const double* dx, const double* du,
                                                       const double* lam_new, const double* mu_new, const double* ax,
                                                       const double* au, const double* smu,
                                                       const unsigned long long* alpha, const int32_t* act,
                                                       int32_t* steps) {
  for (int64_t s = blockIdx.x; s < p.S; s += gridDim.x) {
    const StageInfo& st = p.st[s];
    if (!active(act, st.inst)) continue;
    const Blocks bl = blocks_of(st);
    const double sm = smu[st.inst];
    const double a = bits_to_double(alpha[st.inst]);
    if (st.i == 0 && ECLQR_TID == 0) steps[st.inst] += 1;
    for (int j = ECLQR_TID; j < bl.nu + bl.nx; j += ECLQR_NT) {
      const Var w = var_at(bd, x, u, z, bl, j);
      const Targets t = targets_of(w, ax, au, sm);
      const double dv = step_of(w, dx, du);
      if (w.b.fl) (w.isu ? z.ul : z.xl)[w.o] = w.zl + a * dz_lo(w, t, dv);
      if (w.b.fh) (w.isu ? z.uh : z.xh)[w.o] = w.zh + a * dz_hi(w, t, dv);
    }
    // every variable moves, x_0 included (it reaches x0 with a full step)
    for (int j = ECLQR_TID; j < (st.terminal ? 0 : st.m); j += ECLQR_NT) u[st.in[IN_r] + j] += a * du[st.in[IN_r] + j];
    for (int j = ECLQR_TID; j < st.n; j += ECLQR_NT) {
      const int64_t o = st.in[IN_q] + j;
      x[o] += a * dx[o];
      lam[o] += a * (lam_new[o] - lam[o]);
    }
    for (int j = ECLQR_TID; j < st.k; j += ECLQR_NT) {
      const int64_t o = st.in[IN_g] + j;
      mu_eq[o] += a * (mu_new[o] - mu_eq[o]);
    }
  }
}

// Newton outcome: an active instance whose predictor or corrector solve
// failed stops and reports those bits in status (cstatus: the corrector's
// own outcome when it was a full solve, else null).
__global__ void k_ipm_newton_status(const int32_t* nstatus, const int32_t* cstatus, int32_t* status, int32_t* act,
                                    int32_t B) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const int32_t v = nstatus[b] | (cstatus ? cstatus[b] : 0);
    if (act[b] && v != 0) {
      status[b] |= v;
      act[b] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
namespace {
constexpr unsigned long long kOneBits = 0x3FF0000000000000ull;  // bits of 1.0
int small_grid(int32_t n) { return n > 0 ? (n + 255) / 256 : 1; }
int instance_grid(int32_t B) { return B < 1 ? 1 : (B < 4096 ? B : 4096); }
}  // namespace

void launch_ipm_start(const int32_t* nstatus, int32_t* status, int32_t* act, int32_t* steps, int32_t B,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_start, dim3(small_grid(B)), dim3(256), 0, s, nstatus, status, act, steps, B);
}
void launch_ipm_init(const DevEngine& p, const IpmBounds& bd, double* x, double* u, const IpmDuals& z, double mu0,
                     double interior, int32_t* status, int32_t* act, hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_init, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, z, mu0, interior, status, act);
}
void launch_ipm_mu(const DevEngine& p, const int64_t* sbase, const IpmBounds& bd, const double* x, const double* u,
                   const IpmDuals& z, double* part, double mu_stop, double* mu, int32_t* act, hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_partial, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, z, nullptr, nullptr, nullptr,
                     part);
  hipLaunchKernelGGL(k_ipm_mu, dim3(instance_grid(p.B)), dim3(kBlock), 0, s, p, sbase, part, 0, mu_stop, mu, nullptr,
                     act);
}
void launch_ipm_newton(const DevEngine& p, const Inputs& in, const IpmBounds& bd, const double* x, const double* u,
                       const IpmDuals& z, const double* ax, const double* au, const double* smu, int vectors_only,
                       const IpmNewton& nw, hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_newton, dim3(p.nblocks), dim3(kBlock), 0, s, p, in, bd, x, u, z, ax, au, smu, vectors_only,
                     nw);
}
void launch_ipm_centering(const DevEngine& p, const int64_t* sbase, const IpmBounds& bd, const double* x,
                          const double* u, const IpmDuals& z, const double* ax, const double* au,
                          unsigned long long* alpha, double* part, double* mu, double* smu, const int32_t* act,
                          hipStream_t s) {
  launch_fill_u64(alpha, kOneBits, p.B, s);
  hipLaunchKernelGGL(k_ipm_alpha, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, z, ax, au, nullptr, nullptr,
                     nullptr, 1.0, alpha, act);
  hipLaunchKernelGGL(k_ipm_partial, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, z, ax, au, alpha, part);
  hipLaunchKernelGGL(k_ipm_mu, dim3(instance_grid(p.B)), dim3(kBlock), 0, s, p, sbase, part, 1, 0.0, mu, smu,
                     nullptr);
}
void launch_ipm_step(const DevEngine& p, const IpmBounds& bd, double* x, double* u, double* lam, double* mu_eq,
                     const IpmDuals& z, const double* dx, const double* du, const double* lam_new,
                     const double* mu_new, const double* ax, const double* au, const double* smu,
                     const int32_t* nstatus, const int32_t* cstatus, int32_t* status, double tau,
                     unsigned long long* alpha, int32_t* act, int32_t* steps, hipStream_t s) {
  hipLaunchKernelGGL(k_ipm_newton_status, dim3(small_grid(p.B)), dim3(256), 0, s, nstatus, cstatus, status, act,
                     p.B);
  launch_fill_u64(alpha, kOneBits, p.B, s);
  hipLaunchKernelGGL(k_ipm_alpha, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, z, dx, du, ax, au, smu, tau,
                     alpha, act);
  hipLaunchKernelGGL(k_ipm_update, dim3(p.nblocks), dim3(kBlock), 0, s, p, bd, x, u, lam, mu_eq, z, dx, du, lam_new,
                     mu_new, ax, au, smu, alpha, act, steps);
}

}  // namespace eclqr
