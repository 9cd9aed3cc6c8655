// Workgroup-cooperative dense FP64 routines for small row-major matrices.
//
// Every routine is called by all threads of the workgroup with identical
// arguments and returns after a barrier.  Matrices live in LDS or global
// memory (row-major, leading dimension ld); outputs never alias inputs unless
// stated.  Threads own columns in the Householder routines (each thread
// updates whole columns, the reflector is broadcast from LDS), which keeps
// the only cross-thread traffic to one vector and one reduction per step.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace eclqr {

#define ECLQR_TID ((int)threadIdx.x)
#define ECLQR_NT ((int)blockDim.x)

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// Maximum of one value per thread over the workgroup; buf holds blockDim.x doubles.
__device__ inline double wg_reduce_max(double v, double* buf) {
  buf[ECLQR_TID] = v;
  wg_sync();
  for (int w = ECLQR_NT / 2; w > 0; w >>= 1) {
    if (ECLQR_TID < w) buf[ECLQR_TID] = fmax(buf[ECLQR_TID], buf[ECLQR_TID + w]);
    wg_sync();
  }
  const double r = buf[0];
  wg_sync();
  return r;
}

// C(MxN) = alpha * op(A) * op(B) + beta * C.  op(A) is MxK, op(B) is KxN.
// beta == 0 never reads C.
__device__ inline void wg_gemm(double* C, int ldc, const double* A, int lda, bool tA, const double* B, int ldb,
                               bool tB, int M, int N, int K, double alpha, double beta) {
  for (int idx = ECLQR_TID; idx < M * N; idx += ECLQR_NT) {
    const int i = idx / N, j = idx - (idx / N) * N;
    double acc = 0.0;
    if (!tA && !tB) {
      for (int k = 0; k < K; ++k) acc = fma(A[i * lda + k], B[k * ldb + j], acc);
    } else if (tA && !tB) {
      for (int k = 0; k < K; ++k) acc = fma(A[k * lda + i], B[k * ldb + j], acc);
    } else if (!tA && tB) {
      for (int k = 0; k < K; ++k) acc = fma(A[i * lda + k], B[j * ldb + k], acc);
    } else {
      for (int k = 0; k < K; ++k) acc = fma(A[k * lda + i], B[j * ldb + k], acc);
    }
    const double prev = (beta == 0.0) ? 0.0 : beta * C[i * ldc + j];
    C[i * ldc + j] = alpha * acc + prev;
  }
  wg_sync();
}

// y(M) = alpha * op(A) x + beta * y.   op(A) is MxK.
__device__ inline void wg_gemv(double* y, const double* A, int lda, bool tA, const double* x, int M, int K,
                               double alpha, double beta) {
  for (int i = ECLQR_TID; i < M; i += ECLQR_NT) {
    double acc = 0.0;
    if (!tA) {
      for (int k = 0; k < K; ++k) acc = fma(A[i * lda + k], x[k], acc);
    } else {
      for (int k = 0; k < K; ++k) acc = fma(A[k * lda + i], x[k], acc);
    }
    const double prev = (beta == 0.0) ? 0.0 : beta * y[i];
    y[i] = alpha * acc + prev;
  }
  wg_sync();
}

__device__ inline void wg_copy(double* dst, int ldd, const double* src, int lds, int rows, int cols) {
  for (int idx = ECLQR_TID; idx < rows * cols; idx += ECLQR_NT) {
    const int i = idx / cols, j = idx - (idx / cols) * cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
  wg_sync();
}

__device__ inline void wg_copy_t(double* dst, int ldd, const double* src, int lds, int rows, int cols) {
  // dst (cols x rows) = src(rows x cols)^T
  for (int idx = ECLQR_TID; idx < rows * cols; idx += ECLQR_NT) {
    const int i = idx / cols, j = idx - (idx / cols) * cols;
    dst[j * ldd + i] = src[i * lds + j];
  }
  wg_sync();
}

__device__ inline void wg_fill(double* dst, int ldd, int rows, int cols, double v) {
  for (int idx = ECLQR_TID; idx < rows * cols; idx += ECLQR_NT) {
    const int i = idx / cols, j = idx - (idx / cols) * cols;
    dst[i * ldd + j] = v;
  }
  wg_sync();
}

__device__ inline void wg_identity(double* dst, int ldd, int n) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    dst[i * ldd + j] = (i == j) ? 1.0 : 0.0;
  }
  wg_sync();
}

// Symmetrise a square matrix in place: S = (S + S^T)/2.
__device__ inline void wg_symmetrize(double* S, int ld, int n) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    if (i < j) {
      const double v = 0.5 * (S[i * ld + j] + S[j * ld + i]);
      S[i * ld + j] = v;
      S[j * ld + i] = v;
    }
  }
  wg_sync();
}

// Scratch needed by wg_qr_colpiv: (cp + 8) doubles and cp ints.
struct QRScratch {
  double* d;  // >= cp + 8
  int* perm;  // >= cp (original column index of each pivot position)
};

// Householder QR with column pivoting of the p x c row-major matrix W; the
// pivot candidates are the cp columns [c0, c0 + cp), the reflectors are
// applied to every column.  Stops when the largest remaining candidate norm is
// <= thr * max(1, first pivot norm).  On exit the pivot columns are permuted
// in place (perm[j] = original candidate index), W[j][c0+j] = R_jj, rows
// below the diagonal of pivot column j hold the Householder vector (v_j = 1
// implicit) and tau[j] its scalar.  Returns the numerical rank.
__device__ inline int wg_qr_colpiv(double* W, int ld, int p, int c, int c0, int cp, double thr, double* tau,
                                   QRScratch sc) {
  double* norms = sc.d;
  double* sh = sc.d + cp;  // sh[0] stop flag, sh[1] pivot, sh[2] ref, sh[3] beta, sh[4] tau, sh[5] scale
  for (int j = ECLQR_TID; j < cp; j += ECLQR_NT) sc.perm[j] = j;
  wg_sync();
  const int steps = (p < cp) ? p : cp;
  int r = 0;
  for (int j = 0; j < steps; ++j) {
    for (int col = j + ECLQR_TID; col < cp; col += ECLQR_NT) {
      double s = 0.0;
      for (int row = j; row < p; ++row) {
        const double v = W[row * ld + c0 + col];
        s = fma(v, v, s);
      }
      norms[col] = s;
    }
    wg_sync();
    if (ECLQR_TID == 0) {
      int best = j;
      double bv = norms[j];
      for (int col = j + 1; col < cp; ++col)
        if (norms[col] > bv) {
          bv = norms[col];
          best = col;
        }
      const double nrm = sqrt(bv);
      if (j == 0) sh[2] = fmax(1.0, nrm);
      sh[0] = (nrm <= thr * sh[2]) ? 1.0 : 0.0;
      sh[1] = (double)best;
      if (sh[0] == 0.0) {
        const int pc = best;
        // swap the pivot column into place (column entries handled below)
        const int tp = sc.perm[j];
        sc.perm[j] = sc.perm[pc];
        sc.perm[pc] = tp;
        const double x0 = (pc == j) ? W[j * ld + c0 + j] : W[j * ld + c0 + pc];
        const double beta = -copysign(nrm, x0);
        sh[3] = beta;
        sh[4] = (beta - x0) / beta;
        sh[5] = 1.0 / (x0 - beta);
      }
    }
    wg_sync();
    if (sh[0] != 0.0) break;
    const int pc = (int)sh[1];
    if (pc != j) {
      for (int row = ECLQR_TID; row < p; row += ECLQR_NT) {
        const double a = W[row * ld + c0 + j];
        W[row * ld + c0 + j] = W[row * ld + c0 + pc];
        W[row * ld + c0 + pc] = a;
      }
      wg_sync();
    }
    const double scale = sh[5];
    const double tj = sh[4];
    for (int row = j + 1 + ECLQR_TID; row < p; row += ECLQR_NT) W[row * ld + c0 + j] *= scale;
    if (ECLQR_TID == 0) tau[j] = tj;
    wg_sync();
    for (int col = ECLQR_TID; col < c; col += ECLQR_NT) {
      // skip this and the earlier pivot columns (they hold reflectors below the diagonal)
      if (col >= c0 && col <= c0 + j) continue;
      double w = W[j * ld + col];
      for (int row = j + 1; row < p; ++row) w = fma(W[row * ld + c0 + j], W[row * ld + col], w);
      w *= tj;
      W[j * ld + col] -= w;
      for (int row = j + 1; row < p; ++row) W[row * ld + col] = fma(-w, W[row * ld + c0 + j], W[row * ld + col]);
    }
    wg_sync();
    if (ECLQR_TID == 0) W[j * ld + c0 + j] = sh[3];
    wg_sync();
    r = j + 1;
  }
  return r;
}

// Apply Q = H_0 H_1 ... H_{r-1} (reflectors stored by wg_qr_colpiv in the
// pivot columns [c0, c0 + r) of W, rows j+1.. of column c0+j) to the p x nc
// matrix X (row-major, ldx) from the left: X <- Q X.
__device__ inline void wg_apply_q(const double* W, int ld, int p, int c0, int r, const double* tau, double* X,
                                  int ldx, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int j = r - 1; j >= 0; --j) {
      double w = X[j * ldx + col];
      for (int row = j + 1; row < p; ++row) w = fma(W[row * ld + c0 + j], X[row * ldx + col], w);
      w *= tau[j];
      X[j * ldx + col] -= w;
      for (int row = j + 1; row < p; ++row) X[row * ldx + col] = fma(-w, W[row * ld + c0 + j], X[row * ldx + col]);
    }
  }
  wg_sync();
}

// Orthonormal row basis (Section VIII items 3-4) of the equations
//   W[row][k0 .. k0+kc) . z + W[row][k0+kc] = 0,   rows [r0, p).
// Row-pivoted Gram-Schmidt: the remaining row of largest coefficient norm is
// re-orthogonalised against the rows already chosen, normalised (offset
// included) and projected out of the remaining rows.  Chosen rows end up in
// rows [r0, r0 + rank).  Rows whose coefficient norm falls to
// <= thr * max(1, first norm) are dependent; any of them with
// |offset| > cons_thr makes the system inconsistent (*bad = 1).
__device__ inline int wg_row_basis(double* W, int ld, int r0, int p, int k0, int kc, double thr, double cons_thr,
                                   int* bad, double* scr /* >= 2*(p - r0) + 8 + 64 */) {
  const int rows = p - r0;
  double* nrm = scr;           // rows
  double* dots = scr + rows;   // max(rows, 64)
  double* sh = dots + (rows > 64 ? rows : 64);
  if (ECLQR_TID == 0) {
    sh[0] = 0.0;
    sh[4] = 0.0;
  }
  wg_sync();
  int sel = 0;
  while (sel < rows) {
    const int base = r0 + sel;
    for (int rr = base + ECLQR_TID; rr < p; rr += ECLQR_NT) {
      double s = 0.0;
      for (int cc = 0; cc < kc; ++cc) {
        const double v = W[rr * ld + k0 + cc];
        s = fma(v, v, s);
      }
      nrm[rr - r0] = s;
    }
    wg_sync();
    if (ECLQR_TID == 0) {
      int best = base;
      double bv = nrm[sel];
      for (int rr = base + 1; rr < p; ++rr)
        if (nrm[rr - r0] > bv) {
          bv = nrm[rr - r0];
          best = rr;
        }
      const double nv = sqrt(bv);
      if (sel == 0) sh[2] = fmax(1.0, nv);
      sh[1] = (double)best;
      sh[3] = (nv <= thr * sh[2]) ? 1.0 : 0.0;
    }
    wg_sync();
    if (sh[3] != 0.0) break;
    const int best = (int)sh[1];
    if (best != base) {
      for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT) {
        const double a = W[base * ld + k0 + cc];
        W[base * ld + k0 + cc] = W[best * ld + k0 + cc];
        W[best * ld + k0 + cc] = a;
      }
      wg_sync();
    }
    // re-orthogonalise the pivot row against the chosen rows (one pass)
    if (sel > 0) {
      for (int l = ECLQR_TID; l < sel; l += ECLQR_NT) {
        double d = 0.0;
        for (int cc = 0; cc < kc; ++cc) d = fma(W[(r0 + l) * ld + k0 + cc], W[base * ld + k0 + cc], d);
        dots[l] = d;
      }
      wg_sync();
      for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT) {
        double v = W[base * ld + k0 + cc];
        for (int l = 0; l < sel; ++l) v = fma(-dots[l], W[(r0 + l) * ld + k0 + cc], v);
        W[base * ld + k0 + cc] = v;
      }
      wg_sync();
    }
    // normalise
    if (ECLQR_TID == 0) {
      double s = 0.0;
      for (int cc = 0; cc < kc; ++cc) s = fma(W[base * ld + k0 + cc], W[base * ld + k0 + cc], s);
      sh[5] = 1.0 / sqrt(s);
    }
    wg_sync();
    const double inv = sh[5];
    for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT) W[base * ld + k0 + cc] *= inv;
    wg_sync();
    // project the pivot row out of the remaining rows
    for (int rr = base + 1 + ECLQR_TID; rr < p; rr += ECLQR_NT) {
      double d = 0.0;
      for (int cc = 0; cc < kc; ++cc) d = fma(W[rr * ld + k0 + cc], W[base * ld + k0 + cc], d);
      for (int cc = 0; cc <= kc; ++cc) W[rr * ld + k0 + cc] = fma(-d, W[base * ld + k0 + cc], W[rr * ld + k0 + cc]);
    }
    wg_sync();
    ++sel;
  }
  // consistency of the dependent rows
  for (int rr = r0 + sel + ECLQR_TID; rr < p; rr += ECLQR_NT) {
    if (fabs(W[rr * ld + k0 + kc]) > cons_thr) sh[4] = 1.0;
  }
  wg_sync();
  *bad = (sh[4] != 0.0) ? 1 : 0;
  wg_sync();
  return sel;
}

// In-place Cholesky S = L L^T of an n x n SPD matrix (lower triangle holds L,
// upper triangle zeroed).  Returns 0 on success, 1 if a pivot (before the
// square root) is not above `floor`.
__device__ inline int wg_cholesky(double* S, int ld, int n, double* sh /* 2 doubles */, double floor = 0.0) {
  if (ECLQR_TID == 0) sh[0] = 0.0;
  wg_sync();
  for (int j = 0; j < n; ++j) {
    if (ECLQR_TID == 0) {
      const double d = S[j * ld + j];
      if (!(d > floor)) {
        sh[0] = 1.0;
        sh[1] = 1.0;
      } else {
        sh[1] = sqrt(d);
      }
      S[j * ld + j] = sh[1];
    }
    wg_sync();
    if (sh[0] != 0.0) return 1;
    const double dj = sh[1];
    for (int i = j + 1 + ECLQR_TID; i < n; i += ECLQR_NT) S[i * ld + j] /= dj;
    wg_sync();
    // trailing update of the lower triangle
    const int m = n - j - 1;
    for (int idx = ECLQR_TID; idx < m * m; idx += ECLQR_NT) {
      const int a = j + 1 + idx / m, b = j + 1 + idx % m;
      if (b <= a) S[a * ld + b] = fma(-S[a * ld + j], S[b * ld + j], S[a * ld + b]);
    }
    wg_sync();
  }
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int a = idx / n, b = idx % n;
    if (b > a) S[a * ld + b] = 0.0;
  }
  wg_sync();
  return 0;
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix S
// (read only): K (n x r, row-major, ldk) with S ~= K K^T, rows in the original
// order, columns in pivot order.  Stops when the largest remaining diagonal is
// <= tol * (largest diagonal of S).  rem: n doubles, used: n ints.  Returns r.
__device__ inline int wg_pchol(const double* S, int ld, int n, double tol, double* K, int ldk, double* rem, int* used,
                               double* sh /* 2 doubles */) {
  for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
    rem[i] = S[i * ld + i];
    used[i] = 0;
  }
  wg_sync();
  double ref = 0.0;
  for (int i = 0; i < n; ++i) ref = fmax(ref, rem[i]);
  int r = 0;
  for (int j = 0; j < n; ++j) {
    if (ECLQR_TID == 0) {
      int best = -1;
      double bv = 0.0;
      for (int i = 0; i < n; ++i)
        if (!used[i] && (best < 0 || rem[i] > bv)) {
          best = i;
          bv = rem[i];
        }
      sh[0] = (best >= 0 && bv > tol * ref && bv > 0.0) ? (double)best : -1.0;
      if (best >= 0 && sh[0] >= 0.0) used[best] = 1;
    }
    wg_sync();
    const int p = (int)sh[0];
    if (p < 0) break;
    const double dp = sqrt(rem[p]);
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double v = 0.0;
      if (i == p) {
        v = dp;
      } else if (!used[i]) {
        v = S[i * ld + p];
        for (int l = 0; l < j; ++l) v = fma(-K[i * ldk + l], K[p * ldk + l], v);
        v /= dp;
      }
      K[i * ldk + j] = v;
    }
    wg_sync();
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT)
      if (!used[i]) rem[i] = fma(-K[i * ldk + j], K[i * ldk + j], rem[i]);
    r = j + 1;
    wg_sync();
  }
  return r;
}

// Solve L X = B (lower triangular L, n x n) in place on B (n x nc).
__device__ inline void wg_trsm_lower(const double* L, int ldl, double* X, int ldx, int n, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < n; ++i) {
      double v = X[i * ldx + col];
      for (int k = 0; k < i; ++k) v = fma(-L[i * ldl + k], X[k * ldx + col], v);
      X[i * ldx + col] = v / L[i * ldl + i];
    }
  }
  wg_sync();
}

// Solve L^T X = B (L lower triangular) in place on B (n x nc).
__device__ inline void wg_trsm_lower_t(const double* L, int ldl, double* X, int ldx, int n, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = n - 1; i >= 0; --i) {
      double v = X[i * ldx + col];
      for (int k = i + 1; k < n; ++k) v = fma(-L[k * ldl + i], X[k * ldx + col], v);
      X[i * ldx + col] = v / L[i * ldl + i];
    }
  }
  wg_sync();
}

// Solve U^T X = B with U upper triangular (r x r, diagonal U[j][c0+j] inside a
// wider matrix: U(i, j) = W[i*ld + c0 + j]) in place on X (r x nc).
__device__ inline void wg_trsm_upper_t(const double* W, int ld, int c0, double* X, int ldx, int r, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < r; ++i) {
      double v = X[i * ldx + col];
      for (int k = 0; k < i; ++k) v = fma(-W[k * ld + c0 + i], X[k * ldx + col], v);
      X[i * ldx + col] = v / W[i * ld + c0 + i];
    }
  }
  wg_sync();
}

// LU factorisation with partial pivoting of an n x n matrix in place;
// piv[i] = row swapped with row i at step i.
__device__ inline void wg_lu(double* Mt, int ld, int n, int* piv, double* sh) {
  for (int j = 0; j < n; ++j) {
    if (ECLQR_TID == 0) {
      int best = j;
      double bv = fabs(Mt[j * ld + j]);
      for (int i = j + 1; i < n; ++i) {
        const double v = fabs(Mt[i * ld + j]);
        if (v > bv) {
          bv = v;
          best = i;
        }
      }
      piv[j] = best;
      sh[0] = (double)best;
    }
    wg_sync();
    const int best = (int)sh[0];
    if (best != j) {
      for (int c = ECLQR_TID; c < n; c += ECLQR_NT) {
        const double a = Mt[j * ld + c];
        Mt[j * ld + c] = Mt[best * ld + c];
        Mt[best * ld + c] = a;
      }
      wg_sync();
    }
    const double d = Mt[j * ld + j];
    for (int i = j + 1 + ECLQR_TID; i < n; i += ECLQR_NT) Mt[i * ld + j] /= d;
    wg_sync();
    const int m = n - j - 1;
    for (int idx = ECLQR_TID; idx < m * m; idx += ECLQR_NT) {
      const int a = j + 1 + idx / m, b = j + 1 + idx % m;
      Mt[a * ld + b] = fma(-Mt[a * ld + j], Mt[j * ld + b], Mt[a * ld + b]);
    }
    wg_sync();
  }
}

// Solve (P L U) X = B in place on B (n x nc), factors from wg_lu.
__device__ inline void wg_lu_solve(const double* LU, int ld, int n, const int* piv, double* X, int ldx, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < n; ++i) {
      const int pi = piv[i];
      if (pi != i) {
        const double a = X[i * ldx + col];
        X[i * ldx + col] = X[pi * ldx + col];
        X[pi * ldx + col] = a;
      }
    }
    for (int i = 0; i < n; ++i) {
      double v = X[i * ldx + col];
      for (int k = 0; k < i; ++k) v = fma(-LU[i * ld + k], X[k * ldx + col], v);
      X[i * ldx + col] = v;
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = X[i * ldx + col];
      for (int k = i + 1; k < n; ++k) v = fma(-LU[i * ld + k], X[k * ldx + col], v);
      X[i * ldx + col] = v / LU[i * ld + i];
    }
  }
  wg_sync();
}

// Solve (P L U)^T X = B in place on B (n x nc):  U^T L^T P^T X = B.
__device__ inline void wg_lu_solve_t(const double* LU, int ld, int n, const int* piv, double* X, int ldx, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < n; ++i) {  // U^T y = b
      double v = X[i * ldx + col];
      for (int k = 0; k < i; ++k) v = fma(-LU[k * ld + i], X[k * ldx + col], v);
      X[i * ldx + col] = v / LU[i * ld + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T w = y (unit diagonal)
      double v = X[i * ldx + col];
      for (int k = i + 1; k < n; ++k) v = fma(-LU[k * ld + i], X[k * ldx + col], v);
      X[i * ldx + col] = v;
    }
    for (int i = n - 1; i >= 0; --i) {  // x = P w  (undo the swaps in reverse)
      const int pi = piv[i];
      if (pi != i) {
        const double a = X[i * ldx + col];
        X[i * ldx + col] = X[pi * ldx + col];
        X[pi * ldx + col] = a;
      }
    }
  }
  wg_sync();
}

}  // namespace eclqr
