// Register-resident small dense routines (one wavefront, n <= NMAX <= 64):
// a row (Cholesky, pivoted Cholesky) or a column (triangular solves) of the
// operand per lane, every loop unrolled to NMAX with the runtime size as a
// uniform guard.  Loads are unconditional at clamped (in-bounds) indices and
// issued together, and lane-dependent updates are selects, so no load waits
// inside a divergent branch.  The arithmetic of each routine is exactly that
// of its LDS counterpart in dense.hpp (same operations in the same order), so
// the two give the same bits and either may serve any task.
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
  const int rl = mine ? lane : 0;
  double r[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    const double v = S[rl * ld + (k < n ? k : 0)];
    r[k] = (mine && k < n) ? v : 0.0;
  }
  int fail = 0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n && !fail) {
      const double d = wave_bcast(r[j], j);
      if (!(d > floor)) {
        fail = 1;
      } else {
        const double dj = sqrt(d);
        const double sc = r[j] / dj;
        r[j] = (lane > j) ? sc : ((lane == j) ? dj : r[j]);
        colbuf[lane] = r[j];
        lds_sync();
        double lc[NMAX];
#pragma unroll
        for (int c = j + 1; c < NMAX; ++c) lc[c] = colbuf[c];
        const double al = -r[j];
#pragma unroll
        for (int c = j + 1; c < NMAX; ++c) {
          const double nv = fma(al, lc[c], r[c]);
          r[c] = (c < n && lane >= c) ? nv : r[c];
        }
        lds_sync();
      }
    }
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
  const int lane = ECLQR_TID;
  const double rdl = 1.0 / L[(lane < n ? lane : 0) * (ld + 1)];  // 1 / L(i,i) in lane i
  for (int c0 = 0; c0 < nc; c0 += ECLQR_NT) {
    const int col = c0 + lane;
    const bool mine = col < nc;
    const int cl = mine ? col : c0;
    double x[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) x[k] = X[(k < n ? k : 0) * ldx + cl];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < n) {
        const double rd = wave_bcast(rdl, i);
        double lr[NMAX];
#pragma unroll
        for (int k = 0; k < i; ++k) lr[k] = L[i * ld + k];
        double acc = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc = fma(-lr[k], x[k], acc);
        x[i] = acc * rd;
      }
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
  const int lane = ECLQR_TID;
  const double rdl = 1.0 / L[(lane < n ? lane : 0) * (ld + 1)];
  for (int c0 = 0; c0 < nc; c0 += ECLQR_NT) {
    const int col = c0 + lane;
    const bool mine = col < nc;
    const int cl = mine ? col : c0;
    double x[NMAX];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) x[k] = X[(k < n ? k : 0) * ldx + cl];
#pragma unroll
    for (int i = NMAX - 1; i >= 0; --i) {
      if (i < n) {
        const double rd = wave_bcast(rdl, i);
        double lc[NMAX];
#pragma unroll
        for (int k = i + 1; k < NMAX; ++k) lc[k] = L[(k < n ? k : i) * ld + i];
        double acc = x[i];
#pragma unroll
        for (int k = i + 1; k < NMAX; ++k) {
          const double nv = fma(-lc[k], x[k], acc);
          acc = (k < n) ? nv : acc;
        }
        x[i] = acc * rd;
      }
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
__device__ __forceinline__ int reg_pchol(const double* S, int ld, int n, double tol, double* K, int ldk,
                                         double* rowbuf) {
  const int lane = ECLQR_TID;
  const bool row = lane < n;
  const int rl = row ? lane : 0;
  double kr[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) kr[k] = 0.0;
  double rm = row ? S[rl * ld + rl] : 0.0;
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
        double kp[NMAX];
#pragma unroll
        for (int l = 0; l < j; ++l) kp[l] = rowbuf[l];
        double acc = S[rl * ld + p];
#pragma unroll
        for (int l = 0; l < j; ++l) acc = fma(-kr[l], kp[l], acc);
        const double q = acc / dp;
        const double v = !row ? 0.0 : ((lane == p) ? dp : (done ? 0.0 : q));
        kr[j] = v;
        if (lane == p) done = true;
        rm = done ? rm : fma(-v, v, rm);
        r = j + 1;
        lds_sync();
      }
    }
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
