// Register-resident small dense routines (one wavefront, n <= NMAX <= 64):
// a row (Cholesky) or a column (triangular solves) of the operand per lane,
// every loop unrolled to NMAX with the runtime size as a uniform guard.  The
// arithmetic of each routine is exactly that of its LDS counterpart in
// dense.hpp (same operations in the same order), so the two give the same
// bits and either may serve any task.
#pragma once

#include "dense.hpp"

namespace eclqr {

// wg_cholesky on S (LDS, n x n, ld): lane i holds row i; column j is handed
// to every lane through colbuf (LDS, >= NMAX doubles).  Returns 1 (S
// unchanged) if a pivot is not above floor.
template <int NMAX>
__device__ __forceinline__ int reg_cholesky(double* S, int ld, int n, double floor, double* colbuf) {
  const int lane = ECLQR_TID;
  const bool mine = lane < n;
  double r[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) r[k] = (mine && k < n) ? S[lane * ld + k] : 0.0;
  int fail = 0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n && !fail) {
      const double d = wave_bcast(r[j], j);
      if (!(d > floor)) {
        fail = 1;
      } else {
        const double dj = sqrt(d);
        if (lane > j) r[j] = r[j] / dj;
        if (lane == j) r[j] = dj;
        if (mine) colbuf[lane] = r[j];
        lds_sync();
        const double al = -r[j];
#pragma unroll
        for (int c = j + 1; c < NMAX; ++c) {
          if (c < n) {
            const double lc = colbuf[c];
            if (lane >= c) r[c] = fma(al, lc, r[c]);
          }
        }
        lds_sync();
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!fail && mine) {
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (k < n) S[lane * ld + k] = (k <= lane) ? r[k] : 0.0;
  }
  lds_sync();
  return fail;
}

// wg_trsm_lower: L X = B in place on X (n x nc), column per lane.
template <int NMAX>
__device__ __forceinline__ void reg_trsm_lower(const double* L, int ld, double* X, int ldx, int n, int nc) {
  for (int c0 = 0; c0 < nc; c0 += ECLQR_NT) {
    const int col = c0 + ECLQR_TID;
    const bool mine = col < nc;
    double x[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) x[k] = (mine && k < n) ? X[k * ldx + col] : 0.0;
    const double rdl = (ECLQR_TID < n) ? 1.0 / L[ECLQR_TID * ld + ECLQR_TID] : 0.0;  // 1 / L(i,i) in lane i
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n) {
        const double rd = wave_bcast(rdl, i);
        double acc = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc = fma(-L[i * ld + k], x[k], acc);
        x[i] = acc * rd;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (mine) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < n) X[k * ldx + col] = x[k];
    }
  }
  lds_sync();
}

// wg_trsm_lower_t: L' X = B in place on X (n x nc), column per lane.
template <int NMAX>
__device__ __forceinline__ void reg_trsm_lower_t(const double* L, int ld, double* X, int ldx, int n, int nc) {
  for (int c0 = 0; c0 < nc; c0 += ECLQR_NT) {
    const int col = c0 + ECLQR_TID;
    const bool mine = col < nc;
    double x[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) x[k] = (mine && k < n) ? X[k * ldx + col] : 0.0;
    const double rdl = (ECLQR_TID < n) ? 1.0 / L[ECLQR_TID * ld + ECLQR_TID] : 0.0;  // 1 / L(i,i) in lane i
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
      if (i < n) {
        const double rd = wave_bcast(rdl, i);
        double acc = x[i];
#pragma unroll
        for (int k = i + 1; k < NMAX; ++k)
          if (k < n) acc = fma(-L[k * ld + i], x[k], acc);
        x[i] = acc * rd;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (mine) {
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < n) X[k * ldx + col] = x[k];
    }
  }
  lds_sync();
}

// wg_pchol on S (LDS, read only): lane i holds row i of K; the pivot row is
// handed to every lane through rowbuf (LDS, >= NMAX doubles).
template <int NMAX>
__device__ __forceinline__ int reg_pchol(const double* S, int ld, int n, double tol, double* K, int ldk, double* rowbuf) {
  const int lane = ECLQR_TID;
  const bool row = lane < n;
  double kr[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) kr[k] = 0.0;
  double rm = row ? S[lane * ld + lane] : 0.0;
  bool done = !row;
  const double ref = wave_max(row ? rm : 0.0);
  int r = 0;
  bool stop = false;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n && !stop) {
      double bv = done ? 0.0 : rm;
      int best = done ? -1 : lane;
      wave_argmax(bv, best);
      if (!(best >= 0 && bv > tol * ref && bv > 0.0)) {
        stop = true;
      } else {
        const int p = best;
        const double dp = sqrt(bv);
        if (lane == p) {
#pragma unroll
          for (int l = 0; l < j; ++l) rowbuf[l] = kr[l];
        }
        lds_sync();
        double v = 0.0;
        if (row) {
          if (lane == p) {
            v = dp;
          } else if (!done) {
            double acc = S[lane * ld + p];
#pragma unroll
            for (int l = 0; l < j; ++l) acc = fma(-kr[l], rowbuf[l], acc);
            v = acc / dp;
          }
        }
        kr[j] = v;
        if (lane == p) done = true;
        if (!done) rm = fma(-v, v, rm);
        r = j + 1;
        lds_sync();
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (row) {
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (k < r) K[lane * ldk + k] = kr[k];
  }
  lds_sync();
  return r;
}

}  // namespace eclqr
