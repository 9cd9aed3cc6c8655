// Small dense routines on an 8 x 8 lane grid (one wavefront, n <= NMAX = 8 NB
// <= 64): lane (gr, gc) = (lane / 8, lane % 8) holds the elements (gr + 8a,
// gc + 8b) of the operand in registers, so every instruction of a step works
// on up to 64 elements instead of one row or column per lane.  Loops are
// unrolled to the bound with the runtime size as a uniform guard; loads are
// unconditional at clamped (in-bounds) indices, and lane-dependent updates are
// selects.  The arithmetic of each routine is exactly that of its LDS
// counterpart in dense.hpp (the same operations on every element in the same
// order), so the two give the same bits and either may serve any task.
#pragma once

#include "dense.hpp"

namespace eclqr {

// wg_cholesky on S (LDS, n x n, ld).  buf: LDS, >= 64 doubles.  Returns 1 (S
// unchanged) if a pivot is not above floor.
template <int NB>
__device__ __forceinline__ int reg_cholesky(double* S, int ld, int n, double floor, double* buf) {
  constexpr int NMAX = 8 * NB;
  const int lane = ECLQR_TID, gr = lane >> 3, gc = lane & 7;
  double t[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = gr + 8 * a, c = gc + 8 * b;
      const double v = S[(i < n ? i : 0) * ld + (c < n ? c : 0)];
      t[a][b] = (i < n && c < n) ? v : 0.0;
    }
  int fail = 0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n && !fail) {
      const int jb = j >> 3, jr = j & 7;
      const double d = wave_bcast(t[jb][jb], 9 * jr);
      if (!(d > floor)) {
        fail = 1;
      } else {
        const double dj = sqrt(d);
        // column j: lanes of grid column jr hold (i, j); scale rows i > j
        if (gc == jr) {
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            const int i = gr + 8 * a;
            const double sc = t[a][jb] / dj;
            t[a][jb] = (i > j) ? sc : ((i == j) ? dj : t[a][jb]);
            if (i < NMAX) buf[i] = t[a][jb];
          }
        }
        lds_sync();
        double li[NB], lc[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) li[a] = buf[gr + 8 * a];
#pragma unroll
        for (int b = 0; b < NB; ++b) lc[b] = buf[gc + 8 * b];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int i = gr + 8 * a, c = gc + 8 * b;
            const double nv = fma(-li[a], lc[b], t[a][b]);
            t[a][b] = (j < c && c <= i && i < n) ? nv : t[a][b];
          }
        lds_sync();
      }
    }
  }
  if (!fail) {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = gr + 8 * a, c = gc + 8 * b;
        if (i < n && c < n) S[i * ld + c] = (c <= i) ? t[a][b] : 0.0;
      }
  }
  lds_sync();
  return fail;
}

// wg_trsm_lower (L X = B in place on X, n x nc, nc <= 8 NBC): step k scales
// row k by 1 / L(k,k), then every row i > k takes fma(-L(i,k), x_k, x_i).
template <int NB, int NBC>
__device__ __forceinline__ void reg_trsm_lower(const double* L, int ld, double* X, int ldx, int n, int nc,
                                               double* buf) {
  constexpr int NMAX = 8 * NB;
  const int lane = ECLQR_TID, gr = lane >> 3, gc = lane & 7;
  double x[NB][NBC];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NBC; ++b) {
      const int i = gr + 8 * a, c = gc + 8 * b;
      x[a][b] = X[(i < n ? i : 0) * ldx + (c < nc ? c : 0)];
    }
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      const int kb = k >> 3, kr = k & 7;
      const double rd = 1.0 / L[k * ld + k];
      if (gr == kr) {
#pragma unroll
        for (int b = 0; b < NBC; ++b) {
          x[kb][b] = x[kb][b] * rd;
          buf[gc + 8 * b] = x[kb][b];
        }
      }
      lds_sync();
      double xk[NBC], lk[NB];
#pragma unroll
      for (int b = 0; b < NBC; ++b) xk[b] = buf[gc + 8 * b];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = gr + 8 * a;
        lk[a] = L[(i < n ? i : 0) * ld + k];
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) {
          const int i = gr + 8 * a;
          const double nv = fma(-lk[a], xk[b], x[a][b]);
          x[a][b] = (i > k && i < n) ? nv : x[a][b];
        }
      lds_sync();
    }
  }
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NBC; ++b) {
      const int i = gr + 8 * a, c = gc + 8 * b;
      if (i < n && c < nc) X[i * ldx + c] = x[a][b];
    }
  lds_sync();
}

// wg_trsm_lower_t (L' X = B in place on X): step k (descending) scales row k,
// then every row i < k takes fma(-L(k,i), x_k, x_i).
template <int NB, int NBC>
__device__ __forceinline__ void reg_trsm_lower_t(const double* L, int ld, double* X, int ldx, int n, int nc,
                                                 double* buf) {
  constexpr int NMAX = 8 * NB;
  const int lane = ECLQR_TID, gr = lane >> 3, gc = lane & 7;
  double x[NB][NBC];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NBC; ++b) {
      const int i = gr + 8 * a, c = gc + 8 * b;
      x[a][b] = X[(i < n ? i : 0) * ldx + (c < nc ? c : 0)];
    }
#pragma unroll
  for (int k = NMAX - 1; k >= 0; --k) {
    if (k < n) {
      const int kb = k >> 3, kr = k & 7;
      const double rd = 1.0 / L[k * ld + k];
      if (gr == kr) {
#pragma unroll
        for (int b = 0; b < NBC; ++b) {
          x[kb][b] = x[kb][b] * rd;
          buf[gc + 8 * b] = x[kb][b];
        }
      }
      lds_sync();
      double xk[NBC], lk[NB];
#pragma unroll
      for (int b = 0; b < NBC; ++b) xk[b] = buf[gc + 8 * b];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = gr + 8 * a;
        lk[a] = L[k * ld + (i < n ? i : 0)];
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NBC; ++b) {
          const int i = gr + 8 * a;
          const double nv = fma(-lk[a], xk[b], x[a][b]);
          x[a][b] = (i < k) ? nv : x[a][b];
        }
      lds_sync();
    }
  }
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NBC; ++b) {
      const int i = gr + 8 * a, c = gc + 8 * b;
      if (i < n && c < nc) X[i * ldx + c] = x[a][b];
    }
  lds_sync();
}

}  // namespace eclqr
