// Reduced unconstrained LQR (paper Section VI: any LQR solver; here the
// logarithmic-depth associative scan over conditional value functions),
// feedback gains, the forward affine scan and the recovery maps
// (eq. (recovery-maps)).
// Every kernel here runs one wavefront per workgroup except the split
// value-function combine (two wavefronts, each running its own part of one
// combine): the dense routines count lanes within the wavefront.
#define ECLQR_TID ((int)(threadIdx.x & 63))
#define ECLQR_NT 64
#include "dense.hpp"
#include "device_util.hpp"
#include "eclqr.h"
#include "scratch.hpp"
#include "smallreg.hpp"

namespace eclqr {

// Element of an interval [s, e) of the reduced problem: the conditional value
//   V(x, y) = 1/2 x'J x - eta'x + sup_l [ l'(y - A x - b) - 1/2 l'C l ]
// (cost from reduced state x at s to y at e).  A unary element (end at the
// terminal stage) is V(x) = 1/2 x'J x - eta'x.  Combining [s, m) with [m, e):
//   A = A2 Minv A1,  b = A2 Minv (b1 + C1 eta2) + b2,  C = A2 Minv C1 A2' + C2,
//   eta = A1' Minv' (eta2 - J2 b1) + eta1,  J = A1' Minv' J2 A1 + J1,
// Minv = (I + C1 J2)^{-1}.
//
// Value functions of nearly uncontrollable reduced systems reach 1e11..1e14,
// where an LU factorisation of I + C1 J2 loses most digits.  With J2 = L L'
// (Cholesky) and G = I + L'C1 L = Rg Rg' (G >= I), I + J2 C1 = L G L^{-1}, so
//   J   = J1 + (Rg^{-1} L'A1)'(Rg^{-1} L'A1),
//   xi  = L^{-1} eta2,  d = G^{-1}(xi - L'b1),  eta = eta1 + A1' L d,
//   A   = A2 L^{-T} G^{-1} L'A1,  b = A2 L^{-T}(xi - d) + b2,
// and with C1 = K K' (pivoted Cholesky) and G2 = I + K'J2 K = R2 R2',
//   C   = C2 + (A2 K R2^{-T})(A2 K R2^{-T})'.
// Every factor is applied as a triangular or SPD solve; no difference of two
// large terms is formed.  When J2 is not numerically positive definite the
// LU form is used.
namespace {

// Routines of the combine: on the 8 x 8 lane grid when NMAX > 0 and the sizes
// fit (operands in LDS), else the LDS/global ones; both give the same bits.
template <bool kL, int NMAX>
__device__ __forceinline__ int d_cholesky(double* S, int ld, int n, double* sh, double floor, double* buf) {
  if constexpr (NMAX > 0)
    if (n <= NMAX) return reg_cholesky<NMAX / 8>(S, ld, n, floor, buf);
  return wg_cholesky<kL>(S, ld, n, sh, floor);
}
template <bool kL, int NMAX>
__device__ __forceinline__ void d_trsm_lower(const double* L, int ld, double* X, int ldx, int n, int nc,
                                             double* buf) {
  if constexpr (NMAX > 0)
    if (n <= NMAX && nc <= NMAX + 8) return reg_trsm_lower<NMAX / 8, NMAX / 8 + 1>(L, ld, X, ldx, n, nc, buf);
  wg_trsm_lower<kL>(L, ld, X, ldx, n, nc);
}
template <bool kL, int NMAX>
__device__ __forceinline__ void d_trsm_lower_t(const double* L, int ld, double* X, int ldx, int n, int nc,
                                               double* buf) {
  if constexpr (NMAX > 0)
    if (n <= NMAX && nc <= NMAX + 8) return reg_trsm_lower_t<NMAX / 8, NMAX / 8 + 1>(L, ld, X, ldx, n, nc, buf);
  wg_trsm_lower_t<kL>(L, ld, X, ldx, n, nc);
}
template <bool kL, int NMAX>
__device__ __forceinline__ int d_pchol(const double* S, int ld, int n, double tol, double* K, int ldk, double* rem,
                                       int* used, double* sh, double* buf) {
  (void)buf;
  return wg_pchol<kL>(S, ld, n, tol, K, ldk, rem, used, sh);
}

template <bool kL>
__device__ __forceinline__ void combine_lu(const double* A1, const double* b1, const double* C1, const double* et1, const double* J1,
                           const double* A2, const double* b2, const double* C2, const double* et2, const double* J2,
                           double* Eo, const RicLayout& lo, int ds, int dm, int de, bool binary, double* pool,
                           int* piv, double* sh, double* rlog) {
  double* Mt = pool;                                      // dm x dm
  double* X = Mt + rup4((int64_t)dm * dm);                // dm x (ds + 1 + dm)
  double* Yv = X + rup4((int64_t)dm * (ds + 1 + dm));     // dm x (dm + 1)
  double* T1 = Yv + rup4((int64_t)dm * (dm + 1));         // de x dm
  double* T2 = T1 + rup4((int64_t)de * dm);               // ds x dm
  const int lx = ds + 1 + dm, ly = dm + 1;
  wg_gemm<kL>(Mt, dm, C1, dm, false, J2, dm, false, dm, dm, dm, 1.0, 0.0);
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) Mt[i * dm + i] += 1.0;
  bsync<kL>();
  wg_lu<kL>(Mt, dm, dm, piv, sh);
  // log for the vector-only pass: flag 2, LU factors, pivots
  for (int idx = ECLQR_TID; idx < dm * dm; idx += ECLQR_NT) rlog[4 + idx] = Mt[idx];
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) rlog[4 + 2 * dm * dm + i] = (double)piv[i];
  if (ECLQR_TID == 0) rlog[0] = 2.0;
  for (int idx = ECLQR_TID; idx < dm * ly; idx += ECLQR_NT) {
    const int i = idx / ly, j = idx % ly;
    if (j < dm) {
      Yv[idx] = J2[i * dm + j];
    } else {
      Yv[idx] = lane_chain<true>(et2[i], J2 + i * dm, 1, b1, 1, dm);
    }
  }
  if (binary) {
    for (int idx = ECLQR_TID; idx < dm * lx; idx += ECLQR_NT) {
      const int i = idx / lx, j = idx % lx;
      double v;
      if (j < ds) {
        v = A1[i * ds + j];
      } else if (j == ds) {
        v = lane_chain<false>(b1[i], C1 + i * dm, 1, et2, 1, dm);
      } else {
        v = C1[i * dm + (j - ds - 1)];
      }
      X[idx] = v;
    }
  }
  bsync<kL>();
  wg_lu_solve_t<kL>(Mt, dm, dm, piv, Yv, ly, ly);
  wg_gemm<kL>(T2, dm, A1, ds, true, Yv, ly, false, ds, dm, dm, 1.0, 0.0);
  wg_gemm<kL>(Eo + lo.J, ds, T2, dm, false, A1, ds, false, ds, ds, dm, 1.0, 0.0);
  for (int idx = ECLQR_TID; idx < ds * ds; idx += ECLQR_NT) Eo[lo.J + idx] += J1[idx];
  for (int i = ECLQR_TID; i < ds; i += ECLQR_NT) Eo[lo.eta + i] = lane_chain<false>(et1[i], A1 + i, ds, Yv + dm, ly, dm);
  bsync<kL>();
  wg_symmetrize<kL>(Eo + lo.J, ds, ds);
  if (binary) {
    wg_lu_solve<kL>(Mt, dm, dm, piv, X, lx, lx);
    wg_gemm<kL>(Eo + lo.A, ds, A2, dm, false, X, lx, false, de, ds, dm, 1.0, 0.0);
    for (int i = ECLQR_TID; i < de; i += ECLQR_NT) Eo[lo.b + i] = lane_chain<false>(b2[i], A2 + i * dm, 1, X + ds, lx, dm);
    wg_gemm<kL>(T1, dm, A2, dm, false, X + ds + 1, lx, false, de, dm, dm, 1.0, 0.0);
    wg_gemm<kL>(Eo + lo.C, de, T1, dm, false, A2, dm, true, de, de, dm, 1.0, 0.0);
    for (int idx = ECLQR_TID; idx < de * de; idx += ECLQR_NT) Eo[lo.C + idx] += C2[idx];
    bsync<kL>();
    wg_symmetrize<kL>(Eo + lo.C, de, de);
  }
}

// Factored combine; returns false when J2, G or G2 is not numerically
// positive definite (outputs then incomplete: the caller redoes the combine in
// LU form).  kPart 0: everything; 1: all but C (J, eta, A, b and the log);
// 2: only C (binary combines) -- the two parts share no output or work array
// other than the read-only operands, so two wavefronts can run them at once.
template <bool kL, int NMAX, int kPart = 0>
__device__ __forceinline__ bool combine_factored(const double* A1, const double* b1, const double* C1, const double* et1,
                                 const double* J1, const double* A2, const double* b2, const double* C2,
                                 const double* et2, const double* J2, double* Eo, const RicLayout& lo, int ds, int dm,
                                 int de, bool binary, double* pool, int* used, double* sh, double* rlog, double* buf) {
  const int64_t dd = rup4((int64_t)dm * dm);
  double* Lj = pool;                          // dm x dm   L (J2 = L L')
  double* Gm = Lj + dd;                       // dm x dm   G, then Rg
  double* Tm = Gm + dd;                       // dm x dm   C1 L, later J2 K
  double* Mm = Tm + dd;                       // dm x dm   Rg^{-1} L', later R2^{-1} K'
  double* Km = Mm + dd;                       // dm x dm   K (C1 = K K')
  double* G2 = Km + dd;                       // dm x dm   G2, then R2
  double* Yb = G2 + dd;                       // dm x (ds + 1)
  double* AN = Yb + rup4((int64_t)dm * (ds + 1));  // de x dm
  double* xi = AN + rup4((int64_t)de * dm);   // dm
  double* tv = xi + rup4(dm);                 // dm
  double* wv = tv + rup4(dm);                 // dm
  double* rem = wv + rup4(dm);                // dm
  if constexpr (kPart != 2) {
  double mx = 0.0;
  for (int i = 0; i < dm; ++i) mx = fmax(mx, J2[i * dm + i]);
  if (!(mx > 0.0)) return false;
  wg_copy<kL>(Lj, dm, J2, dm, dm, dm);
  if (d_cholesky<kL, NMAX>(Lj, dm, dm, sh, 1e-15 * mx, buf)) return false;
  // G = I + L'(C1 L)
  wg_gemm<kL>(Tm, dm, C1, dm, false, Lj, dm, false, dm, dm, dm, 1.0, 0.0);
  wg_gemm<kL>(Gm, dm, Lj, dm, true, Tm, dm, false, dm, dm, dm, 1.0, 0.0);
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) Gm[i * dm + i] += 1.0;
  bsync<kL>();
  wg_symmetrize<kL>(Gm, dm, dm);
  if (d_cholesky<kL, NMAX>(Gm, dm, dm, sh, 0.0, buf)) return false;
  // log for the vector-only pass: flag 1, L, Rg
  for (int idx = ECLQR_TID; idx < dm * dm; idx += ECLQR_NT) {
    rlog[4 + idx] = Lj[idx];
    rlog[4 + dm * dm + idx] = Gm[idx];
  }
  if (ECLQR_TID == 0) rlog[0] = 1.0;
  // xi = L^{-1} eta2 ; tv = d = G^{-1}(xi - L'b1) ; wv = L d  (entry i in lane i)
  {
    const int lane = ECLQR_TID;
    double xv = (lane < dm) ? et2[lane] : 0.0;
    xv = lane_trsv_lower(Lj, dm, xv, dm);
    double dv = xv;
    if (lane < dm) dv = lane_chain<true>(dv, Lj + lane * dm + lane, dm, b1 + lane, 1, dm - lane);
    dv = lane_trsv_lower(Gm, dm, dv, dm);
    dv = lane_trsv_lower_t(Gm, dm, dv, dm);
    if (lane < dm) {
      xi[lane] = xv;
      tv[lane] = dv;
    }
  }
  bsync<kL>();
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) wv[i] = lane_chain<false>(0.0, Lj + i * dm, 1, tv, 1, i + 1);
  bsync<kL>();
  for (int i = ECLQR_TID; i < ds; i += ECLQR_NT) Eo[lo.eta + i] = lane_chain<false>(et1[i], A1 + i, ds, wv, 1, dm);
  // Mm = Rg^{-1} L' ; Yb[:, :ds] = Mm A1 ; J = J1 + Yb'Yb
  wg_copy_t<kL>(Mm, dm, Lj, dm, dm, dm);
  d_trsm_lower<kL, NMAX>(Gm, dm, Mm, dm, dm, dm, buf);
  const int ly = ds + 1;
  wg_gemm<kL>(Yb, ly, Mm, dm, false, A1, ds, false, dm, ds, dm, 1.0, 0.0);
  wg_gemm<kL>(Eo + lo.J, ds, Yb, ly, true, Yb, ly, false, ds, ds, dm, 1.0, 0.0);
  for (int idx = ECLQR_TID; idx < ds * ds; idx += ECLQR_NT) Eo[lo.J + idx] += J1[idx];
  bsync<kL>();
  wg_symmetrize<kL>(Eo + lo.J, ds, ds);
  if (!binary) return true;
  // Yb = L^{-T} [Rg^{-T} Mm A1 | xi - d] ; A = A2 Yb[:, :ds] ; b = A2 Yb[:, ds] + b2
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) Yb[i * ly + ds] = xi[i] - tv[i];
  bsync<kL>();
  d_trsm_lower_t<kL, NMAX>(Gm, dm, Yb, ly, dm, ds, buf);
  d_trsm_lower_t<kL, NMAX>(Lj, dm, Yb, ly, dm, ly, buf);
  wg_gemm<kL>(Eo + lo.A, ds, A2, dm, false, Yb, ly, false, de, ds, dm, 1.0, 0.0);
  for (int i = ECLQR_TID; i < de; i += ECLQR_NT) Eo[lo.b + i] = lane_chain<false>(b2[i], A2 + i * dm, 1, Yb + ds, ly, dm);
  }
  if constexpr (kPart == 1) return true;
  // C = C2 + (A2 K R2^{-T})(A2 K R2^{-T})'
  const int r = d_pchol<kL, NMAX>(C1, dm, dm, 1e-15, Km, dm, rem, used, sh, buf);
  if (r > 0) {
    wg_gemm<kL>(Tm, r, J2, dm, false, Km, dm, false, dm, r, dm, 1.0, 0.0);
    wg_gemm<kL>(G2, r, Km, dm, true, Tm, r, false, r, r, dm, 1.0, 0.0);
    for (int i = ECLQR_TID; i < r; i += ECLQR_NT) G2[i * r + i] += 1.0;
    bsync<kL>();
    wg_symmetrize<kL>(G2, r, r);
    if (d_cholesky<kL, NMAX>(G2, r, r, sh, 0.0, buf)) return false;
    wg_copy_t<kL>(Mm, dm, Km, dm, dm, r);           // K' (r x dm)
    d_trsm_lower<kL, NMAX>(G2, r, Mm, dm, r, dm, buf);
    wg_gemm<kL>(AN, r, A2, dm, false, Mm, dm, true, de, r, dm, 1.0, 0.0);
    wg_gemm<kL>(Eo + lo.C, de, AN, r, false, AN, r, true, de, de, r, 1.0, 0.0);
  } else {
    wg_fill<kL>(Eo + lo.C, de, de, de, 0.0);
  }
  for (int idx = ECLQR_TID; idx < de * de; idx += ECLQR_NT) Eo[lo.C + idx] += C2[idx];
  bsync<kL>();
  wg_symmetrize<kL>(Eo + lo.C, de, de);
  return true;
}


// ---- one lane per combine: reduced dims <= 4 ---------------------------------
// The factored combine above, with every matrix held in the registers of one
// lane (4 x 4 arrays; a block beyond the task's dims is identity on the
// diagonal of the factored matrices and zero elsewhere, which leaves the
// leading blocks exactly as at their own size).  64 small combines run side by
// side in one wavefront instead of one after another.  Same factorizations,
// same failure tests, same log (flag 1, L, Rg); a combine that fails a test is
// redone by the whole wavefront with the routines above (factored, else LU).
constexpr int kLD = 4;

// In-place Cholesky of the leading n x n block (identity beyond it); false
// when a leading pivot is not above floor.  rd: reciprocals of the diagonal
// of the factor, for the triangular solves below (a multiply per entry
// instead of a divide).
__device__ __forceinline__ bool lc_chol(double (&S)[kLD][kLD], int n, double floor, double (&rd)[kLD]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kLD; ++j) {
    double d = S[j][j];
#pragma unroll
    for (int p = 0; p < j; ++p) d = fma(-S[j][p], S[j][p], d);
    ok = ok && (j >= n || d > floor);
    const double lj = (j < n) ? sqrt(d) : 1.0;
    const double rl = 1.0 / lj;
    S[j][j] = lj;
    rd[j] = rl;
#pragma unroll
    for (int i = j + 1; i < kLD; ++i) {
      double v = S[i][j];
#pragma unroll
      for (int p = 0; p < j; ++p) v = fma(-S[i][p], S[j][p], v);
      S[i][j] = v * rl;
    }
#pragma unroll
    for (int i = 0; i < j; ++i) S[i][j] = 0.0;
  }
  return ok;
}
// x <- L^{-1} x, x <- L^{-T} x (rd: reciprocals of L's diagonal)
__device__ __forceinline__ void lc_fwd(const double (&L)[kLD][kLD], const double (&rd)[kLD], double (&x)[kLD]) {
#pragma unroll
  for (int i = 0; i < kLD; ++i) {
    double v = x[i];
#pragma unroll
    for (int p = 0; p < i; ++p) v = fma(-L[i][p], x[p], v);
    x[i] = v * rd[i];
  }
}
__device__ __forceinline__ void lc_bwd(const double (&L)[kLD][kLD], const double (&rd)[kLD], double (&x)[kLD]) {
#pragma unroll
  for (int i = kLD - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int p = i + 1; p < kLD; ++p) v = fma(-L[p][i], x[p], v);
    x[i] = v * rd[i];
  }
}
__device__ __forceinline__ void lc_sym(double (&S)[kLD][kLD]) {
#pragma unroll
  for (int i = 0; i < kLD; ++i)
#pragma unroll
    for (int j = i + 1; j < kLD; ++j) {
      const double v = 0.5 * (S[i][j] + S[j][i]);
      S[i][j] = v;
      S[j][i] = v;
    }
}
// r x c block of a row-major (ld) array, zero beyond (pad_id: identity
// diagonal).  Every lane issues all 16 loads unconditionally (indices clamped
// into the block, or to `safe` when the block is empty) and selects
// afterwards: a load under a lane-dependent branch would wait on its own.
__device__ __forceinline__ void lc_load(double (&M)[kLD][kLD], const double* src, int r, int c, int ld, bool pad_id,
                                        const double* safe) {
  const double* base = (r > 0 && c > 0) ? src : safe;
  double v[kLD][kLD];
#pragma unroll
  for (int i = 0; i < kLD; ++i)
#pragma unroll
    for (int j = 0; j < kLD; ++j) {
      const int ii = (i < r) ? i : 0, jj = (j < c) ? j : 0;
      v[i][j] = base[ii * ld + jj];
    }
#pragma unroll
  for (int i = 0; i < kLD; ++i)
#pragma unroll
    for (int j = 0; j < kLD; ++j) M[i][j] = (i < r && j < c) ? v[i][j] : ((pad_id && i == j) ? 1.0 : 0.0);
}
// first n entries of a vector, zero beyond (same load discipline)
__device__ __forceinline__ void lc_loadv(double (&x)[kLD], const double* src, int n, const double* safe) {
  const double* base = (n > 0) ? src : safe;
  double v[kLD];
#pragma unroll
  for (int i = 0; i < kLD; ++i) v[i] = base[(i < n) ? i : 0];
#pragma unroll
  for (int i = 0; i < kLD; ++i) x[i] = (i < n) ? v[i] : 0.0;
}
__device__ __forceinline__ void lc_store(double* dst, const double (&M)[kLD][kLD], int r, int c, int ld) {
#pragma unroll
  for (int i = 0; i < kLD; ++i)
#pragma unroll
    for (int j = 0; j < kLD; ++j)
      if (i < r && j < c) dst[i * ld + j] = M[i][j];
}

// Returns false when a factorization test fails (outputs then incomplete).
__device__ __forceinline__ bool lane_combine(const double* E1, const RicLayout& l1, const double* E2,
                                             const RicLayout& l2, double* Eo, const RicLayout& lo, int ds, int dm,
                                             int de, bool binary, double* rlog, const double* safe) {
  if (dm == 0) {  // empty middle: J = J1, eta = eta1, A = 0, b = b2, C = C2 (the LU form's result)
    double M[kLD][kLD];
    lc_load(M, E1 + l1.J, ds, ds, ds, false, safe);
    lc_store(Eo + lo.J, M, ds, ds, ds);
    double ev[kLD], bv[kLD];
    lc_loadv(ev, E1 + l1.eta, ds, safe);
    lc_loadv(bv, E2 + l2.b, de, safe);
#pragma unroll
    for (int i = 0; i < kLD; ++i)
      if (i < ds) Eo[lo.eta + i] = ev[i];
    if (binary) {
#pragma unroll
      for (int i = 0; i < kLD; ++i) {
        if (i < de) Eo[lo.b + i] = bv[i];
#pragma unroll
        for (int j = 0; j < kLD; ++j)
          if (i < de && j < ds) Eo[lo.A + i * ds + j] = 0.0;
      }
      lc_load(M, E2 + l2.C, de, de, de, false, safe);
      lc_store(Eo + lo.C, M, de, de, de);
    }
    rlog[0] = 2.0;
    return true;
  }
  double J2[kLD][kLD], L[kLD][kLD], Rg[kLD][kLD];
  lc_load(J2, E2 + l2.J, dm, dm, dm, true, safe);
  double mx = 0.0;
#pragma unroll
  for (int i = 0; i < kLD; ++i)
    if (i < dm) mx = fmax(mx, J2[i][i]);
  if (!(mx > 0.0)) return false;
#pragma unroll
  for (int i = 0; i < kLD; ++i)
#pragma unroll
    for (int j = 0; j < kLD; ++j) L[i][j] = J2[i][j];
  double rL[kLD], rR[kLD];
  if (!lc_chol(L, dm, 1e-15 * mx, rL)) return false;
  {
    // G = I + L'(C1 L)
    double C1[kLD][kLD], T[kLD][kLD];
    lc_load(C1, E1 + l1.C, dm, dm, dm, false, safe);
#pragma unroll
    for (int i = 0; i < kLD; ++i)
#pragma unroll
      for (int j = 0; j < kLD; ++j) {
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < kLD; ++p) v = fma(C1[i][p], L[p][j], v);
        T[i][j] = v;
      }
#pragma unroll
    for (int i = 0; i < kLD; ++i)
#pragma unroll
      for (int j = 0; j < kLD; ++j) {
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < kLD; ++p) v = fma(L[p][i], T[p][j], v);
        Rg[i][j] = v + ((i == j) ? 1.0 : 0.0);
      }
  }
  lc_sym(Rg);
  if (!lc_chol(Rg, dm, 0.0, rR)) return false;
  lc_store(rlog + 4, L, dm, dm, dm);
  lc_store(rlog + 4 + dm * dm, Rg, dm, dm, dm);
  rlog[0] = 1.0;
  // xi = L^{-1} eta2 ; d = G^{-1}(xi - L'b1) ; w = L d
  double xi[kLD], dv[kLD], wv[kLD];
  lc_loadv(xi, E2 + l2.eta, dm, safe);
  lc_fwd(L, rL, xi);
  {
    double b1[kLD];
    lc_loadv(b1, E1 + l1.b, dm, safe);
#pragma unroll
    for (int i = 0; i < kLD; ++i) {
      double v = xi[i];
#pragma unroll
      for (int j = i; j < kLD; ++j) v = fma(-L[j][i], b1[j], v);
      dv[i] = v;
    }
  }
  lc_fwd(Rg, rR, dv);
  lc_bwd(Rg, rR, dv);
#pragma unroll
  for (int i = 0; i < kLD; ++i) {
    double v = 0.0;
#pragma unroll
    for (int p = 0; p <= i; ++p) v = fma(L[i][p], dv[p], v);
    wv[i] = v;
  }
  double A1[kLD][kLD], Yb[kLD][kLD];
  lc_load(A1, E1 + l1.A, dm, ds, ds, false, safe);
  {
    double e1[kLD];
    lc_loadv(e1, E1 + l1.eta, ds, safe);
#pragma unroll
    for (int c = 0; c < kLD; ++c) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < kLD; ++j) v = fma(A1[j][c], wv[j], v);
      if (c < ds) Eo[lo.eta + c] = e1[c] + v;
    }
  }
  // Yb = Rg^{-1} L' A1 ; J = J1 + Yb'Yb
  {
    double Mm[kLD][kLD];
#pragma unroll
    for (int c = 0; c < kLD; ++c) {
      double col[kLD];
#pragma unroll
      for (int r = 0; r < kLD; ++r) col[r] = L[c][r];
      lc_fwd(Rg, rR, col);
#pragma unroll
      for (int r = 0; r < kLD; ++r) Mm[r][c] = col[r];
    }
#pragma unroll
    for (int i = 0; i < kLD; ++i)
#pragma unroll
      for (int c = 0; c < kLD; ++c) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kLD; ++j) v = fma(Mm[i][j], A1[j][c], v);
        Yb[i][c] = v;
      }
  }
  {
    double Jo[kLD][kLD];
    lc_load(Jo, E1 + l1.J, ds, ds, ds, false, safe);
#pragma unroll
    for (int a = 0; a < kLD; ++a)
#pragma unroll
      for (int b = 0; b < kLD; ++b) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < kLD; ++i) v = fma(Yb[i][a], Yb[i][b], v);
        Jo[a][b] += v;
      }
    lc_sym(Jo);
    lc_store(Eo + lo.J, Jo, ds, ds, ds);
  }
  if (!binary) return true;
  // [Yb | xi - d] <- L^{-T} [Rg^{-T} Yb | xi - d] ; A = A2 Yb ; b = b2 + A2 (.)
  double yv[kLD];
#pragma unroll
  for (int i = 0; i < kLD; ++i) yv[i] = xi[i] - dv[i];
#pragma unroll
  for (int c = 0; c < kLD; ++c) {
    double col[kLD];
#pragma unroll
    for (int r = 0; r < kLD; ++r) col[r] = Yb[r][c];
    lc_bwd(Rg, rR, col);
    lc_bwd(L, rL, col);
#pragma unroll
    for (int r = 0; r < kLD; ++r) Yb[r][c] = col[r];
  }
  lc_bwd(L, rL, yv);
  double A2[kLD][kLD], b2[kLD];
  lc_load(A2, E2 + l2.A, de, dm, dm, false, safe);
  lc_loadv(b2, E2 + l2.b, de, safe);
#pragma unroll
  for (int r = 0; r < kLD; ++r) {
#pragma unroll
    for (int c = 0; c < kLD; ++c) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < kLD; ++i) v = fma(A2[r][i], Yb[i][c], v);
      if (r < de && c < ds) Eo[lo.A + r * ds + c] = v;
    }
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kLD; ++i) v = fma(A2[r][i], yv[i], v);
    if (r < de) Eo[lo.b + r] = b2[r] + v;
  }
  // C = C2 + (A2 K R2^{-T})(A2 K R2^{-T})' with C1 = K K' (pivoted Cholesky, tol 1e-15)
  double K[kLD][kLD];
  int rk = 0;
  {
    double C1[kLD][kLD], rm[kLD];
    bool done[kLD];
    lc_load(C1, E1 + l1.C, dm, dm, dm, false, safe);
    double ref = 0.0;
#pragma unroll
    for (int i = 0; i < kLD; ++i) {
      rm[i] = C1[i][i];
      done[i] = i >= dm;
      if (i < dm) ref = fmax(ref, rm[i]);
#pragma unroll
      for (int j = 0; j < kLD; ++j) K[i][j] = 0.0;
    }
    bool go = true;
#pragma unroll
    for (int j = 0; j < kLD; ++j) {
      double bv = 0.0;
      int best = -1;
#pragma unroll
      for (int i = 0; i < kLD; ++i)
        if (!done[i] && (best < 0 || rm[i] > bv)) {
          bv = rm[i];
          best = i;
        }
      go = go && best >= 0 && bv > 1e-15 * ref && bv > 0.0;
      if (go) {
        const double dp = sqrt(bv);
        double kp[kLD];  // row `best` of K (columns < j)
#pragma unroll
        for (int l = 0; l < kLD; ++l) {
          double v = 0.0;
#pragma unroll
          for (int i = 0; i < kLD; ++i) v = (i == best) ? K[i][l] : v;
          kp[l] = v;
        }
#pragma unroll
        for (int i = 0; i < kLD; ++i) {
          double cib = 0.0;
#pragma unroll
          for (int q = 0; q < kLD; ++q) cib = (q == best) ? C1[i][q] : cib;
          double v = 0.0;
          if (i == best) {
            v = dp;
          } else if (!done[i]) {
            v = cib;
#pragma unroll
            for (int l = 0; l < j; ++l) v = fma(-K[i][l], kp[l], v);
            v = v / dp;
          }
          K[i][j] = v;
          done[i] = done[i] || (i == best);
          if (!done[i]) rm[i] = fma(-v, v, rm[i]);
        }
        rk = j + 1;
      }
    }
  }
  double Co[kLD][kLD];
  lc_load(Co, E2 + l2.C, de, de, de, false, safe);
  if (rk > 0) {
    // G2 = I + K' J2 K = R2 R2'
    double G2[kLD][kLD];
    {
      double T[kLD][kLD];
#pragma unroll
      for (int i = 0; i < kLD; ++i)
#pragma unroll
        for (int j = 0; j < kLD; ++j) {
          double v = 0.0;
#pragma unroll
          for (int p = 0; p < kLD; ++p)
            if (p < dm) v = fma(J2[i][p], K[p][j], v);
          T[i][j] = (i < dm) ? v : 0.0;
        }
#pragma unroll
      for (int i = 0; i < kLD; ++i)
#pragma unroll
        for (int j = 0; j < kLD; ++j) {
          double v = 0.0;
#pragma unroll
          for (int p = 0; p < kLD; ++p) v = fma(K[p][i], T[p][j], v);
          G2[i][j] = v + ((i == j) ? 1.0 : 0.0);
        }
    }
    lc_sym(G2);
    double r2[kLD];
    if (!lc_chol(G2, rk, 0.0, r2)) return false;
    // AN = A2 K R2^{-T} (rows of (R2^{-1} K')' ), C += AN AN'
    double AN[kLD][kLD];
#pragma unroll
    for (int r = 0; r < kLD; ++r) {
      double v[kLD];
#pragma unroll
      for (int j = 0; j < kLD; ++j) {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < kLD; ++i) a = fma(A2[r][i], K[i][j], a);
        v[j] = a;
      }
      lc_fwd(G2, r2, v);  // row r of A2 K times R2^{-T}: solve R2 y = (A2 K)_r'
#pragma unroll
      for (int j = 0; j < kLD; ++j) AN[r][j] = v[j];
    }
#pragma unroll
    for (int a = 0; a < kLD; ++a)
#pragma unroll
      for (int b = 0; b < kLD; ++b) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < kLD; ++j) v = fma(AN[a][j], AN[b][j], v);
        Co[a][b] += v;
      }
  }
  lc_sym(Co);
  lc_store(Eo + lo.C, Co, de, de, de);
  return true;
}

// The factored combine with A1, C1, J2 and A2 (read more than once) staged in
// LDS and the other operands read from global memory once; J and C are formed
// in the pool and written out once, so global data is only read, or written
// and not read back, and every barrier is LDS-only.  Same operations in the
// same order as combine_factored, so the same bits.  Pool, with d the largest
// dim of the task: P0 (d x d) L, then K, then the C update; P1 (d x d) G, then
// Rg, then G2, then R2; P2 (d x d) C1 L, then Rg^{-1} L', then the J update,
// then J2 K, then A2 K R2^{-T}; P3 (d x (d + 1)) Yb, then R2^{-1} K'; four
// vectors.
template <int NMAX>
__device__ __forceinline__ bool combine_staged(const double* A1, const double* b1, const double* C1, const double* et1,
                                               const double* J1, const double* A2, const double* b2, const double* C2,
                                               const double* et2, const double* J2, double* Eo, const RicLayout& lo,
                                               int ds, int dm, int de, bool binary, double* pool, int* used, double* sh,
                                               double* rlog, double* buf) {
  int d = ds > dm ? ds : dm;
  d = d > de ? d : de;
  const int64_t dd = rup4((int64_t)d * d);
  double* P0 = pool;
  double* P1 = P0 + dd;
  double* P2 = P1 + dd;
  double* P3 = P2 + dd;
  double* xi = P3 + rup4((int64_t)d * (d + 1));
  double* tv = xi + rup4(d);
  double* wv = tv + rup4(d);
  double* rem = wv + rup4(d);
  double mx = 0.0;
  for (int i = 0; i < dm; ++i) mx = fmax(mx, J2[i * dm + i]);
  if (!(mx > 0.0)) return false;
  double* Lj = P0;
  double* Gm = P1;
  wg_copy<true>(Lj, dm, J2, dm, dm, dm);
  if (d_cholesky<true, NMAX>(Lj, dm, dm, sh, 1e-15 * mx, buf)) return false;
  // G = I + L'(C1 L)
  wg_gemm<true>(P2, dm, C1, dm, false, Lj, dm, false, dm, dm, dm, 1.0, 0.0);
  wg_gemm<true>(Gm, dm, Lj, dm, true, P2, dm, false, dm, dm, dm, 1.0, 0.0);
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) Gm[i * dm + i] += 1.0;
  bsync<true>();
  wg_symmetrize<true>(Gm, dm, dm);
  if (d_cholesky<true, NMAX>(Gm, dm, dm, sh, 0.0, buf)) return false;
  for (int idx = ECLQR_TID; idx < dm * dm; idx += ECLQR_NT) {
    rlog[4 + idx] = Lj[idx];
    rlog[4 + dm * dm + idx] = Gm[idx];
  }
  if (ECLQR_TID == 0) rlog[0] = 1.0;
  {
    const int lane = ECLQR_TID;
    double xv = (lane < dm) ? et2[lane] : 0.0;
    xv = lane_trsv_lower(Lj, dm, xv, dm);
    double dv = xv;
    if (lane < dm) dv = lane_chain<true>(dv, Lj + lane * dm + lane, dm, b1 + lane, 1, dm - lane);
    dv = lane_trsv_lower(Gm, dm, dv, dm);
    dv = lane_trsv_lower_t(Gm, dm, dv, dm);
    if (lane < dm) {
      xi[lane] = xv;
      tv[lane] = dv;
    }
  }
  bsync<true>();
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) wv[i] = lane_chain<false>(0.0, Lj + i * dm, 1, tv, 1, i + 1);
  bsync<true>();
  for (int i = ECLQR_TID; i < ds; i += ECLQR_NT) Eo[lo.eta + i] = lane_chain<false>(et1[i], A1 + i, ds, wv, 1, dm);
  // Rg^{-1} L' ; Yb[:, :ds] = (Rg^{-1} L') A1 ; J = J1 + Yb'Yb
  double* Mm = P2;
  wg_copy_t<true>(Mm, dm, Lj, dm, dm, dm);
  d_trsm_lower<true, NMAX>(Gm, dm, Mm, dm, dm, dm, buf);
  const int ly = ds + 1;
  double* Yb = P3;
  wg_gemm<true>(Yb, ly, Mm, dm, false, A1, ds, false, dm, ds, dm, 1.0, 0.0);
  double* Jt = P2;
  wg_gemm<true>(Jt, ds, Yb, ly, true, Yb, ly, false, ds, ds, dm, 1.0, 0.0);
  for (int idx = ECLQR_TID; idx < ds * ds; idx += ECLQR_NT) Jt[idx] += J1[idx];
  bsync<true>();
  wg_symmetrize<true>(Jt, ds, ds);
  for (int idx = ECLQR_TID; idx < ds * ds; idx += ECLQR_NT) Eo[lo.J + idx] = Jt[idx];
  if (!binary) return true;
  // Yb = L^{-T} [Rg^{-T} Mm A1 | xi - d] ; A = A2 Yb[:, :ds] ; b = A2 Yb[:, ds] + b2
  for (int i = ECLQR_TID; i < dm; i += ECLQR_NT) Yb[i * ly + ds] = xi[i] - tv[i];
  bsync<true>();
  d_trsm_lower_t<true, NMAX>(Gm, dm, Yb, ly, dm, ds, buf);
  d_trsm_lower_t<true, NMAX>(Lj, dm, Yb, ly, dm, ly, buf);
  wg_gemm<true>(Eo + lo.A, ds, A2, dm, false, Yb, ly, false, de, ds, dm, 1.0, 0.0);
  for (int i = ECLQR_TID; i < de; i += ECLQR_NT) Eo[lo.b + i] = lane_chain<false>(b2[i], A2 + i * dm, 1, Yb + ds, ly, dm);
  bsync<true>();
  // C = C2 + (A2 K R2^{-T})(A2 K R2^{-T})'
  double* Km = P0;
  double* Ct = P0;
  const int r = d_pchol<true, NMAX>(C1, dm, dm, 1e-15, Km, dm, rem, used, sh, buf);
  if (r > 0) {
    double* G2 = P1;
    double* M2 = P3;
    wg_gemm<true>(P2, r, J2, dm, false, Km, dm, false, dm, r, dm, 1.0, 0.0);
    wg_gemm<true>(G2, r, Km, dm, true, P2, r, false, r, r, dm, 1.0, 0.0);
    for (int i = ECLQR_TID; i < r; i += ECLQR_NT) G2[i * r + i] += 1.0;
    bsync<true>();
    wg_symmetrize<true>(G2, r, r);
    if (d_cholesky<true, NMAX>(G2, r, r, sh, 0.0, buf)) return false;
    wg_copy_t<true>(M2, dm, Km, dm, dm, r);  // K' (r x dm)
    d_trsm_lower<true, NMAX>(G2, r, M2, dm, r, dm, buf);
    double* AN = P2;
    wg_gemm<true>(AN, r, A2, dm, false, M2, dm, true, de, r, dm, 1.0, 0.0);
    wg_gemm<true>(Ct, de, AN, r, false, AN, r, true, de, de, r, 1.0, 0.0);
  } else {
    wg_fill<true>(Ct, de, de, de, 0.0);
  }
  for (int idx = ECLQR_TID; idx < de * de; idx += ECLQR_NT) Ct[idx] += C2[idx];
  bsync<true>();
  wg_symmetrize<true>(Ct, de, de);
  for (int idx = ECLQR_TID; idx < de * de; idx += ECLQR_NT) Eo[lo.C + idx] = Ct[idx];
  return true;
}

}  // namespace

// Copy the used part of a value-function element with reduced dims (na, nb)
// between two layouts (fields A, b, C, eta, J, each contiguous); all loads of
// a round are issued before its stores.
__device__ __forceinline__ void ric_move(double* dst, const RicLayout& ld, const double* src, const RicLayout& ls, int na,
                                int nb) {
  const int64_t n0 = (int64_t)nb * na, n1 = n0 + nb, n2 = n1 + (int64_t)nb * nb, n3 = n2 + na,
                n4 = n3 + (int64_t)na * na;
  for (int64_t f0 = ECLQR_TID; f0 < n4; f0 += 8 * ECLQR_NT) {
    double v[8];
    int64_t od[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t f = f0 + (int64_t)t * ECLQR_NT;
      int64_t os = 0, o = -1;
      if (f < n0) {
        os = ls.A + f;
        o = ld.A + f;
      } else if (f < n1) {
        os = ls.b + (f - n0);
        o = ld.b + (f - n0);
      } else if (f < n2) {
        os = ls.C + (f - n1);
        o = ld.C + (f - n1);
      } else if (f < n3) {
        os = ls.eta + (f - n2);
        o = ld.eta + (f - n2);
      } else if (f < n4) {
        os = ls.J + (f - n3);
        o = ld.J + (f - n3);
      }
      od[t] = o;
      v[t] = (o >= 0) ? src[os] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (od[t] >= 0) dst[od[t]] = v[t];
  }
}

// Stage the operands of a combine that it reads more than once, compactly in
// LDS at S: A1 (dm x ds), C1 (dm x dm), J2 (dm x dm), A2 (de x dm); all loads
// of a round are issued before its stores.
__device__ __forceinline__ void ric_stage(double* S, const double* A1, const double* C1, const double* J2,
                                          const double* A2, int ds, int dm, int de) {
  const int64_t n0 = (int64_t)dm * ds, n1 = n0 + (int64_t)dm * dm, n2 = n1 + (int64_t)dm * dm,
                n3 = n2 + (int64_t)de * dm;
  for (int64_t f0 = ECLQR_TID; f0 < n3; f0 += 8 * ECLQR_NT) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t f = f0 + (int64_t)t * ECLQR_NT;
      const double* src = (f < n0) ? A1 + f : (f < n1) ? C1 + (f - n0) : (f < n2) ? J2 + (f - n1) : A2 + (f - n2);
      v[t] = (f < n3) ? *src : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t f = f0 + (int64_t)t * ECLQR_NT;
      if (f < n3) S[f] = v[t];
    }
  }
}

// Task of position t of a value-function combine launch (the plan's dim-bucket
// order, else the level's own order).
__device__ __forceinline__ int64_t ric_task(const DevEngine& e, int64_t t) { return e.ric_perm ? e.ric_perm[t] : t; }

// kMode 0: work pool in per-block global scratch; 1: pool in LDS; 2: both
// operands, the result and the pool in LDS (operands staged in, result
// written out in bulk), every barrier LDS-only; 3: the operands read more than
// once staged in LDS, a compact pool in LDS, the result written once to
// global memory (combine_staged), every barrier of the factored form LDS-only,
// the LU form in the global scratch.
// LDS: [operand 1 | operand 2 | result (mode 2); staged operands (mode 3)]
// [pool (modes 1, 2, 3)] | piv/used ints | sh
// NMAX > 0 (modes 2, 3): factorizations and solves of size <= NMAX run
// register-resident.  With NMAX = 16 (every dim <= 16, where LDS leaves room
// for several workgroups per compute unit) registers are capped for three
// waves per SIMD (at most 168 VGPRs; four would spill).
template <int kMode, int NMAX>
__global__ void __launch_bounds__(kBlock, (NMAX == 16) ? 3 : 1) k_ric_combine(DevEngine e, int64_t first, int64_t ntasks, int32_t* status,
                                                        int maxd) {
  extern __shared__ double lds[];
  const int64_t esz = (kMode == 2) ? ric_layout(maxd, maxd).size : 0;
  const int64_t head = (kMode == 3) ? ric_stage_size(maxd) : 3 * esz;
  const int64_t pool_sz = (kMode == 3) ? ric_pool_staged(maxd) : (kMode >= 1) ? ric_pool(maxd) : 0;
  double* S1 = lds;
  double* S2 = S1 + esz;
  double* So = S2 + esz;
  int* piv = (int*)(lds + head + pool_sz);
  double* sh = (double*)(piv + kMaxDim);
  double* buf = sh + 16;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * ric_task(e, first + ti)];
    const int bsl = e.tasks[3 * ric_task(e, first + ti) + 1];
    const int o = e.tasks[3 * ric_task(e, first + ti) + 2];
    const int sa = slot_a(e, 0, a), sm = slot_b(e, 0, a), se = slot_b(e, 0, bsl);
    if (gated(e, e.st[sa].inst)) continue;
    const int ds = e.nbar[sa], dm = e.nbar[sm], de = (se >= 0) ? e.nbar[se] : 0;
    const int ns = e.st[sa].n, nm = e.st[sm].n, ne = (se >= 0) ? e.st[se].n : 0;
    const RicLayout l1 = ric_layout(ns, nm), l2 = ric_layout(nm, ne), lo = ric_layout(ns, ne);
    const double* E1 = slot_ptr(e, SCAN_RIC, a);
    const double* E2 = slot_ptr(e, SCAN_RIC, bsl);
    double* Eo = slot_ptr(e, SCAN_RIC, o);
    const bool binary = se >= 0;
    double* rlog = e.ric_log + e.ric_log_off[o];
    if constexpr (kMode == 3) {
      double* St = lds;
      ric_stage(St, E1 + l1.A, E1 + l1.C, E2 + l2.J, E2 + l2.A, ds, dm, de);
      lds_sync();
      const double* A1s = St;
      const double* C1s = A1s + (int64_t)dm * ds;
      const double* J2s = C1s + (int64_t)dm * dm;
      const double* A2s = J2s + (int64_t)dm * dm;
      // the LU form, when a factorization fails, works in the block's global
      // scratch (the grid is capped at the plan's workgroups in this mode)
      if (!combine_staged<NMAX>(A1s, E1 + l1.b, C1s, E1 + l1.eta, E1 + l1.J, A2s, E2 + l2.b, E2 + l2.C, E2 + l2.eta,
                                J2s, Eo, lo, ds, dm, de, binary, lds + head, piv, sh, rlog, buf)) {
        wg_sync();
        combine_lu<false>(A1s, E1 + l1.b, C1s, E1 + l1.eta, E1 + l1.J, A2s, E2 + l2.b, E2 + l2.C, E2 + l2.eta, J2s, Eo,
                          lo, ds, dm, de, binary, block_scratch(e), piv, sh, rlog);
      }
      wg_sync();
    } else if constexpr (kMode == 2) {
      const RicLayout s1 = ric_layout(ds, dm), s2 = ric_layout(dm, de), so = ric_layout(ds, de);
      ric_move(S1, s1, E1, l1, ds, dm);
      ric_move(S2, s2, E2, l2, dm, de);
      lds_sync();
      const double *A1 = S1 + s1.A, *b1 = S1 + s1.b, *C1 = S1 + s1.C, *et1 = S1 + s1.eta, *J1 = S1 + s1.J;
      const double *A2 = S2 + s2.A, *b2 = S2 + s2.b, *C2 = S2 + s2.C, *et2 = S2 + s2.eta, *J2 = S2 + s2.J;
      double* pool = lds + 3 * esz;
      if (!combine_factored<true, NMAX>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, So, so, ds, dm, de, binary, pool,
                                        piv, sh, rlog, buf))
        combine_lu<true>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, So, so, ds, dm, de, binary, pool, piv, sh, rlog);
      lds_sync();
      ric_move(Eo, lo, So, so, ds, de);
      lds_sync();
    } else {
      const double *A1 = E1 + l1.A, *b1 = E1 + l1.b, *C1 = E1 + l1.C, *et1 = E1 + l1.eta, *J1 = E1 + l1.J;
      const double *A2 = E2 + l2.A, *b2 = E2 + l2.b, *C2 = E2 + l2.C, *et2 = E2 + l2.eta, *J2 = E2 + l2.J;
      double* pool = (kMode == 1) ? lds : block_scratch(e);
      if (!combine_factored<false, 0>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, Eo, lo, ds, dm, de, binary, pool,
                                      piv, sh, rlog, buf))
        combine_lu<false>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, Eo, lo, ds, dm, de, binary, pool, piv, sh, rlog);
    }
    (void)status;
  }
}

// Value-function combines of a level with two wavefronts per task: wavefront
// 0 computes J, eta, A, b (and the log), wavefront 1 the C update -- the two
// chains of the factored combine depend only on the operands.  Operands and
// result in LDS as in mode 2, one work pool per wavefront; the LU form, when a
// factorization fails, by wavefront 0.  Same operations in the same order as
// the one-wavefront kernel, so the same bits.
// LDS: S1 | S2 | So | pool 0 | pool 1 | piv 0, 1 | flags | sh, buf (x2)
template <int NMAX>
__global__ void __launch_bounds__(2 * kBlock, 1) k_ric_combine_split(DevEngine e, int64_t first, int64_t ntasks,
                                                                     int maxd) {
  extern __shared__ double lds[];
  const int64_t esz = ric_layout(maxd, maxd).size;
  const int64_t pool_sz = ric_pool(maxd);
  const int wave = threadIdx.x >> 6;
  double* S1 = lds;
  double* S2 = S1 + esz;
  double* So = S2 + esz;
  double* pool = So + esz + wave * pool_sz;
  int* pivs = (int*)(So + esz + 2 * pool_sz);
  int* piv = pivs + wave * kMaxDim;
  int* okf = pivs + 2 * kMaxDim;
  double* sh = (double*)(okf + 4) + wave * (16 + kMaxDim);
  double* buf = sh + 16;
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * ric_task(e, first + ti)];
    const int bsl = e.tasks[3 * ric_task(e, first + ti) + 1];
    const int o = e.tasks[3 * ric_task(e, first + ti) + 2];
    const int sa = slot_a(e, 0, a), sm = slot_b(e, 0, a), se = slot_b(e, 0, bsl);
    if (gated(e, e.st[sa].inst)) continue;  // the same for both wavefronts
    const int ds = e.nbar[sa], dm = e.nbar[sm], de = (se >= 0) ? e.nbar[se] : 0;
    const int ns = e.st[sa].n, nm = e.st[sm].n, ne = (se >= 0) ? e.st[se].n : 0;
    const RicLayout l1 = ric_layout(ns, nm), l2 = ric_layout(nm, ne), lo = ric_layout(ns, ne);
    const RicLayout s1 = ric_layout(ds, dm), s2 = ric_layout(dm, de), so = ric_layout(ds, de);
    const bool binary = se >= 0;
    double* rlog = e.ric_log + e.ric_log_off[o];
    if (wave == 0)
      ric_move(S1, s1, slot_ptr(e, SCAN_RIC, a), l1, ds, dm);
    else
      ric_move(S2, s2, slot_ptr(e, SCAN_RIC, bsl), l2, dm, de);
    __syncthreads();
    const double *A1 = S1 + s1.A, *b1 = S1 + s1.b, *C1 = S1 + s1.C, *et1 = S1 + s1.eta, *J1 = S1 + s1.J;
    const double *A2 = S2 + s2.A, *b2 = S2 + s2.b, *C2 = S2 + s2.C, *et2 = S2 + s2.eta, *J2 = S2 + s2.J;
    bool ok = true;
    if (wave == 0)
      ok = combine_factored<true, NMAX, 1>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, So, so, ds, dm, de, binary,
                                           pool, piv, sh, rlog, buf);
    else if (binary)
      ok = combine_factored<true, NMAX, 2>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, So, so, ds, dm, de, binary,
                                           pool, piv, sh, rlog, buf);
    if ((threadIdx.x & 63) == 0) okf[wave] = ok ? 1 : 0;
    __syncthreads();
    if (!(okf[0] && okf[1])) {  // read by both wavefronts after the barrier: uniform
      if (wave == 0) combine_lu<true>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, So, so, ds, dm, de, binary, pool, piv,
                                      sh, rlog);
      __syncthreads();
    }
    if (wave == 0) ric_move(slot_ptr(e, SCAN_RIC, o), lo, So, so, ds, de);
    __syncthreads();
  }
}

// One combine of a level by the whole wavefront, global work pool (factored,
// else LU): the tasks the lane kernel does not finish.
__device__ __forceinline__ void ric_combine_wave(const DevEngine& e, int64_t first, int64_t tj, int* piv, double* sh,
                                                 double* buf) {
  const int a = e.tasks[3 * (first + tj)];
  const int bsl = e.tasks[3 * (first + tj) + 1];
  const int o = e.tasks[3 * (first + tj) + 2];
  const int sa = slot_a(e, 0, a), sm = slot_b(e, 0, a), se = slot_b(e, 0, bsl);
  const int ds = e.nbar[sa], dm = e.nbar[sm], de = (se >= 0) ? e.nbar[se] : 0;
  const int ns = e.st[sa].n, nm = e.st[sm].n, ne = (se >= 0) ? e.st[se].n : 0;
  const RicLayout l1 = ric_layout(ns, nm), l2 = ric_layout(nm, ne), lo = ric_layout(ns, ne);
  const double* E1 = slot_ptr(e, SCAN_RIC, a);
  const double* E2 = slot_ptr(e, SCAN_RIC, bsl);
  double* Eo = slot_ptr(e, SCAN_RIC, o);
  const double *A1 = E1 + l1.A, *b1 = E1 + l1.b, *C1 = E1 + l1.C, *et1 = E1 + l1.eta, *J1 = E1 + l1.J;
  const double *A2 = E2 + l2.A, *b2 = E2 + l2.b, *C2 = E2 + l2.C, *et2 = E2 + l2.eta, *J2 = E2 + l2.J;
  double* rlog = e.ric_log + e.ric_log_off[o];
  double* pool = block_scratch(e);
  wg_sync();
  if (!combine_factored<false, 0>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, Eo, lo, ds, dm, de, se >= 0, pool, piv, sh,
                                  rlog, buf))
    combine_lu<false>(A1, b1, C1, et1, J1, A2, b2, C2, et2, J2, Eo, lo, ds, dm, de, se >= 0, pool, piv, sh, rlog);
  wg_sync();
}

// Value-function combines of a level, one lane per task where every reduced
// dim is <= 4 (lane_combine).  The tasks of a tile of 64 that do not qualify,
// or fail a factorization test there, are combined by the whole wavefront
// (global work pool) -- right away, or (defer_count non-null) appended to
// defer_list for k_ric_combine_deferred, so that a wide level's large tasks
// run one per wavefront instead of one after another.
__global__ void __launch_bounds__(kBlock) k_ric_combine_lane(DevEngine e, int64_t first, int64_t ntasks,
                                                             int32_t* defer_count, int32_t* defer_list) {
  __shared__ int piv[kMaxDim];
  __shared__ double sh[16];
  __shared__ double buf[kMaxDim];
  const int lane = ECLQR_TID;
  for (int64_t t0 = (int64_t)blockIdx.x * kBlock; t0 < ntasks; t0 += (int64_t)gridDim.x * kBlock) {
    const int64_t ti = t0 + lane;
    bool need = false;
    if (ti < ntasks) {
      const int a = e.tasks[3 * (first + ti)];
      const int bsl = e.tasks[3 * (first + ti) + 1];
      const int o = e.tasks[3 * (first + ti) + 2];
      const int sa = slot_a(e, 0, a), sm = slot_b(e, 0, a), se = slot_b(e, 0, bsl);
      if (!gated(e, e.st[sa].inst)) {
        const int ds = e.nbar[sa], dm = e.nbar[sm], de = (se >= 0) ? e.nbar[se] : 0;
        need = true;
        if (ds <= kLD && dm <= kLD && de <= kLD) {
          const int ns = e.st[sa].n, nm = e.st[sm].n, ne = (se >= 0) ? e.st[se].n : 0;
          const RicLayout l1 = ric_layout(ns, nm), l2 = ric_layout(nm, ne), lo = ric_layout(ns, ne);
          need = !lane_combine(slot_ptr(e, SCAN_RIC, a), l1, slot_ptr(e, SCAN_RIC, bsl), l2, slot_ptr(e, SCAN_RIC, o),
                               lo, ds, dm, de, se >= 0, e.ric_log + e.ric_log_off[o], e.arena);
        }
      }
    }
    unsigned long long rest = __ballot(need);
    if (defer_count) {  // append the rest to the deferred list
      if (rest) {
        int base = 0;
        if (lane == 0) base = atomicAdd(defer_count, __popcll(rest));
        base = wave_bcast_i(base, 0);
        if (need) defer_list[base + __popcll(rest & ((1ull << lane) - 1ull))] = (int32_t)ti;
      }
      continue;
    }
    // the rest, one task at a time by the whole wavefront
    while (rest) {
      const int l = __ffsll((long long)rest) - 1;
      rest &= rest - 1;
      ric_combine_wave(e, first, t0 + l, piv, sh, buf);
    }
  }
}

// The deferred tasks of a level (count and task indices from the lane
// kernel), one per wavefront.
__global__ void __launch_bounds__(kBlock) k_ric_combine_deferred(DevEngine e, int64_t first, const int32_t* count,
                                                                 const int32_t* list) {
  __shared__ int piv[kMaxDim];
  __shared__ double sh[16];
  __shared__ double buf[kMaxDim];
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) ric_combine_wave(e, first, list[i], piv, sh, buf);
}

// Feedback of stage i from the value function of stage i+1 (P', p' = J, -eta
// of the suffix element):  H_uu = R-bar + B-bar'P'B-bar,
// H_ux = M-bar' + B-bar'P'A-bar, h_u = r-bar + B-bar'(P'c-bar + p'),
// K = -H_uu^{-1} H_ux, k = -H_uu^{-1} h_u, and the closed-loop map
// z' = (A-bar + B-bar K) z + (B-bar k + c-bar) as the forward-scan leaf.
// LDS: Huu (maxm x maxm) | sh [| working arrays, kLS: in LDS instead of the
// workgroup's global scratch]
template <bool kLS>
__global__ void __launch_bounds__(kBlock) k_gains(DevEngine e, int32_t* status, int maxm, int64_t first,
                                                  int64_t count) {
  extern __shared__ double lds[];
  double* Huu = lds;
  double* sh = Huu + (int64_t)maxm * maxm;
  double* lscr = sh + 16;
  for (int64_t ti = blockIdx.x; ti < count; ti += gridDim.x) {
    const int64_t s = stage_at(e, first, ti);
    const StageInfo st = e.st[s];
    if (st.terminal || gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m;
    const Arena ar = arena_layout(n, np, m, st.k);
    double* base = e.arena + st.ws;
    const int nb = e.nbar[s], nb1 = e.nbar[s + 1], mb = e.mbar[s];
    const StageInfo& st1 = e.st[s + 1];
    const RicLayout l1 = ric_layout(st1.n, 0);
    const double* P1 = slot_ptr(e, SCAN_RIC, st1.suf[SCAN_RIC]) + l1.J;
    const double* et1 = slot_ptr(e, SCAN_RIC, st1.suf[SCAN_RIC]) + l1.eta;
    const double *Ab = base + ar.Ab, *Bb = base + ar.Bb, *cb = base + ar.cb;
    const double *Mb = base + ar.Mb, *Rb = base + ar.Rb, *rb = base + ar.rb;
    double* K = base + ar.K;
    double* kk = base + ar.kk;
    double* s0 = kLS ? lscr : block_scratch(e);
    double* PB = s0;                                   // nb1 x mb
    double* PA = PB + rup4((int64_t)nb1 * mb);         // nb1 x nb
    double* Hux = PA + rup4((int64_t)nb1 * nb);        // mb x nb
    double* pc = Hux + rup4((int64_t)mb * nb);         // nb1
    double* hu = pc + rup4(nb1);                       // mb
    wg_gemm<false, true>(PB, mb, P1, nb1, false, Bb, mb, false, nb1, mb, nb1, 1.0, 0.0);
    wg_gemm<false, true>(PA, nb, P1, nb1, false, Ab, nb, false, nb1, nb, nb1, 1.0, 0.0);
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double v = -et1[i];
      v = lane_chain<false>(v, P1 + i * nb1, 1, cb, 1, nb1);
      pc[i] = v;
    }
    wg_copy(Huu, mb, Rb, mb, mb, mb);
    wg_gemm<false, true>(Huu, mb, Bb, mb, true, PB, mb, false, mb, mb, nb1, 1.0, 1.0);
    wg_symmetrize(Huu, mb, mb);
    wg_copy_t(Hux, nb, Mb, mb, nb, mb);
    wg_gemm<false, true>(Hux, nb, Bb, mb, true, PA, nb, false, mb, nb, nb1, 1.0, 1.0);
    for (int i = ECLQR_TID; i < mb; i += ECLQR_NT) {
      double v = rb[i];
      v = lane_chain<false>(v, Bb + i, mb, pc, 1, nb1);
      hu[i] = v;
    }
    wg_sync();
    if (wg_cholesky(Huu, mb, mb, sh)) {
      if (ECLQR_TID == 0) flag_at(e, status, st.inst, ECLQR_NOT_CONVEX, st.i);
      wg_sync();
      continue;
    }
    wg_copy(base + ar.Hc, mb, Huu, mb, mb, mb);
    // K = -Huu^{-1} Hux ; k = -Huu^{-1} hu
    wg_trsm_lower(Huu, mb, Hux, nb, mb, nb);
    wg_trsm_lower_t(Huu, mb, Hux, nb, mb, nb);
    wg_trsm_lower(Huu, mb, hu, 1, mb, 1);
    wg_trsm_lower_t(Huu, mb, hu, 1, mb, 1);
    for (int idx = ECLQR_TID; idx < mb * nb; idx += ECLQR_NT) K[idx] = -Hux[idx];
    for (int i = ECLQR_TID; i < mb; i += ECLQR_NT) kk[i] = -hu[i];
    wg_sync();
    // closed loop: F = A-bar + B-bar K (nb1 x nb), f = B-bar k + c-bar
    double* Fs = slot_ptr(e, SCAN_FWD, st.elem[SCAN_FWD]);
    double* fs = Fs + (int64_t)np * n;
    wg_copy(Fs, nb, Ab, nb, nb1, nb);
    wg_gemm<false, true>(Fs, nb, Bb, mb, false, K, nb, false, nb1, nb, mb, 1.0, 1.0);
    for (int i = ECLQR_TID; i < nb1; i += ECLQR_NT) {
      double v = cb[i];
      v = lane_chain<false>(v, Bb + i * mb, 1, kk, 1, mb);
      fs[i] = v;
    }
    wg_sync();
  }
}

// Forward scan: composition of affine maps of the reduced state.  The left
// operand maps mid -> out, the right operand maps in -> mid (or is the
// constant z at mid); result F = F1 F2, f = F1 f2 + f1.
__global__ void __launch_bounds__(kBlock) k_fwd_combine(DevEngine e, int64_t first, int64_t ntasks) {
  for (int64_t ti = blockIdx.x; ti < ntasks; ti += gridDim.x) {
    const int a = e.tasks[3 * (first + ti)];
    const int bsl = e.tasks[3 * (first + ti) + 1];
    const int o = e.tasks[3 * (first + ti) + 2];
    const int so = slot_a(e, 1, a), smid = slot_b(e, 1, a), sin_ = slot_b(e, 1, bsl);
    if (gated(e, e.st[so].inst)) continue;
    const int dout = e.nbar[so], dmid = e.nbar[smid], din = (sin_ >= 0) ? e.nbar[sin_] : 0;
    const int nout = e.st[so].n, nmid = e.st[smid].n, nin = (sin_ >= 0) ? e.st[sin_].n : 0;
    const double* F1 = slot_ptr(e, SCAN_FWD, a);
    const double* f1 = F1 + (int64_t)nout * nmid;
    const double* F2 = slot_ptr(e, SCAN_FWD, bsl);
    const double* f2 = F2 + (int64_t)nmid * nin;
    double* Fo = slot_ptr(e, SCAN_FWD, o);
    double* fo = Fo + (int64_t)nout * nin;
    if (sin_ >= 0) wg_gemm(Fo, din, F1, dmid, false, F2, din, false, dout, din, dmid, 1.0, 0.0);
    for (int i = ECLQR_TID; i < dout; i += ECLQR_NT) {
      double v = f1[i];
      v = lane_chain<false>(v, F1 + i * dmid, 1, f2, 1, dmid);
      fo[i] = v;
    }
    wg_sync();
  }
}

// Recovery (eq. (recovery-maps)): v_i = K_i z_i + k_i, x_i = T_i z_i + t_i,
// u_i = Y_i z_i + Z_i v_i + y_i.
__global__ void __launch_bounds__(kBlock) k_recover(DevEngine e, double* x, double* u) {
  if (none_live(e)) return;
  __shared__ double vsh[kMaxDim];
  for (int64_t s = blockIdx.x; s < e.S; s += gridDim.x) {
    const StageInfo st = e.st[s];
    if (gated(e, st.inst)) continue;
    const int n = st.n, np = st.np, m = st.m;
    const Arena ar = arena_layout(n, np, m, st.k);
    const double* base = e.arena + st.ws;
    const int nb = e.nbar[s];
    const double* z = slot_ptr(e, SCAN_FWD, st.suf[SCAN_FWD]);
    double* xo = x + st.in[IN_q];
    const double* T = base + ar.T;
    const double* tv = base + ar.t;
    for (int i = ECLQR_TID; i < n; i += ECLQR_NT) {
      double v = tv[i];
      v = lane_chain<false>(v, T + i * nb, 1, z, 1, nb);
      xo[i] = v;
    }
    if (!st.terminal) {
      const int mb = e.mbar[s];
      const double *K = base + ar.K, *kk = base + ar.kk, *Y = base + ar.Y, *Z = base + ar.Z, *y = base + ar.y;
      for (int i = ECLQR_TID; i < mb; i += ECLQR_NT) {
        double v = kk[i];
        v = lane_chain<false>(v, K + i * nb, 1, z, 1, nb);
        vsh[i] = v;
      }
      __syncthreads();
      double* uo = u + st.in[IN_r];
      for (int i = ECLQR_TID; i < m; i += ECLQR_NT) {
        double v = y[i];
        v = lane_chain<false>(v, Y + i * nb, 1, z, 1, nb);
        v = lane_chain<false>(v, Z + i * mb, 1, vsh, 1, mb);
        uo[i] = v;
      }
    }
    __syncthreads();
  }
}

static int g_lqr_max_lds = 65536;

void lqr_set_max_lds(int bytes) {
  g_lqr_max_lds = bytes;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine<1, 0>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine<2, 0>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine<2, 16>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine<2, 32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine_split<16>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_ric_combine_split<32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gains<false>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gains<true>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
}

// LDS bytes of a value-function combine launch in mode m at middle dim bound d.
static size_t ric_mode_bytes(int m, int d) {
  const size_t head = (m == 3) ? (size_t)ric_stage_size(d) : (m == 2) ? 3 * (size_t)ric_layout(d, d).size : 0;
  const size_t pool = (m == 3) ? (size_t)ric_pool_staged(d) : (m >= 1) ? (size_t)ric_pool(d) : 0;
  return sizeof(double) * (head + pool + 16 + kMaxDim) + sizeof(int) * kMaxDim + 64;
}
// Mode actually used for a requested mode: the largest one <= requested whose
// LDS fits.
static int ric_mode(int want, int d) {
  for (int m = want; m > 0; --m)
    if (ric_mode_bytes(m, d) <= (size_t)g_lqr_max_lds) return m;
  return 0;
}
size_t ric_lds_bytes(int maxd) { return ric_mode_bytes(ric_mode(2, maxd), maxd); }
size_t gains_lds_bytes(int maxm) { return sizeof(double) * ((size_t)maxm * maxm + 16) + 64; }

static int g_lds_per_cu = 160 * 1024, g_num_cu = 256;
void lqr_set_device(int lds_per_cu, int num_cu) {
  if (lds_per_cu > 0) g_lds_per_cu = lds_per_cu;
  if (num_cu > 0) g_num_cu = num_cu;
}
static size_t ric_split_bytes(int d) {
  return sizeof(double) * (3 * (size_t)ric_layout(d, d).size + 2 * (size_t)ric_pool(d) + 2 * (16 + kMaxDim)) +
         sizeof(int) * (2 * kMaxDim + 4) + 64;
}

void launch_ric_combine(const DevEngine& e, int64_t first, int64_t ntasks, int32_t* status, int maxd,
                        hipStream_t s) {
  if (ntasks <= 0) return;
  const int grid = task_grid(e, ntasks);  // modes 1 and 2 and the split kernel keep their pool in LDS
  const int mode = ric_mode(e.pool_lds, maxd);
  // two wavefronts per combine while the level still fits the device at once
  if (e.split_combine && mode >= 2 && maxd <= 32) {
    const size_t lds = ric_split_bytes(maxd);
    const int64_t per_cu = (int64_t)g_lds_per_cu / (int64_t)lds;
    if (lds <= (size_t)g_lqr_max_lds && ntasks <= per_cu * g_num_cu) {
      if (maxd <= 16)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ric_combine_split<16>), dim3(grid), dim3(2 * kBlock), lds, s, e, first,
                           ntasks, maxd);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ric_combine_split<32>), dim3(grid), dim3(2 * kBlock), lds, s, e, first,
                           ntasks, maxd);
      return;
    }
  }
  const size_t lds = ric_mode_bytes(mode, maxd);
  const void* fn = (mode == 3 && maxd <= 16)   ? reinterpret_cast<const void*>(k_ric_combine<3, 16>)
                   : (mode == 3 && maxd <= 32) ? reinterpret_cast<const void*>(k_ric_combine<3, 32>)
                   : (mode == 3)               ? reinterpret_cast<const void*>(k_ric_combine<3, 0>)
                   : (mode == 2 && maxd <= 16) ? reinterpret_cast<const void*>(k_ric_combine<2, 16>)
                   : (mode == 2 && maxd <= 32) ? reinterpret_cast<const void*>(k_ric_combine<2, 32>)
                   : (mode == 2)               ? reinterpret_cast<const void*>(k_ric_combine<2, 0>)
                   : (mode == 1)               ? reinterpret_cast<const void*>(k_ric_combine<1, 0>)
                                               : reinterpret_cast<const void*>(k_ric_combine<0, 0>);
  // modes 0 and 3 use the per-workgroup global scratch (nblocks of them): as
  // the pool, or for the LU form
  const int g = (mode == 0 || mode == 3) ? fit_grid(fn, kBlock, lds, ntasks < e.nblocks ? ntasks : e.nblocks) : grid;
  DevEngine ev = e;
  void* args[] = {&ev, &first, &ntasks, &status, &maxd};
  (void)hipLaunchKernel(fn, dim3(g), dim3(kBlock), args, lds, s);
}

void launch_ric_combine_lane(const DevEngine& e, int64_t first, int64_t ntasks, int32_t* defer_count,
                             int32_t* defer_list, hipStream_t s) {
  if (ntasks <= 0) return;
  const int64_t tiles = (ntasks + kBlock - 1) / kBlock;
  const int grid = (int)(tiles < e.nblocks ? tiles : e.nblocks);
  hipLaunchKernelGGL(k_ric_combine_lane, dim3(grid), dim3(kBlock), 0, s, e, first, ntasks, defer_count, defer_list);
  if (defer_count) {
    const int g2 = (int)(ntasks < e.nblocks ? ntasks : e.nblocks);
    hipLaunchKernelGGL(k_ric_combine_deferred, dim3(g2), dim3(kBlock), 0, s, e, first, defer_count, defer_list);
  }
}

void launch_gains(const DevEngine& e, int32_t* status, int maxm, int maxn, int64_t first, int64_t count,
                  hipStream_t s) {
  if (count <= 0) return;
  const size_t base = gains_lds_bytes(maxm);
  const size_t with = base + sizeof(double) * (size_t)gains_scratch(maxn, maxn, maxm);
  if (e.elim_lds && with <= 32768 && with <= (size_t)g_lqr_max_lds) {
    const int grid = task_grid(e, count);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gains<true>), dim3(grid), dim3(kBlock), with, s, e, status, maxm, first,
                       count);
  } else {
    const int grid =
        fit_grid(reinterpret_cast<const void*>(k_gains<false>), kBlock, base, count < e.nblocks ? count : e.nblocks);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gains<false>), dim3(grid), dim3(kBlock), base, s, e, status, maxm, first,
                       count);
  }
}

void launch_fwd_combine(const DevEngine& e, int64_t first, int64_t ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  const int grid = (int)(ntasks < e.nblocks ? ntasks : e.nblocks);
  hipLaunchKernelGGL(k_fwd_combine, dim3(grid), dim3(kBlock), 0, s, e, first, ntasks);
}

void launch_recover(const DevEngine& e, double* x, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_recover, dim3(e.nblocks), dim3(kBlock), 0, s, e, x, u);
}

}  // namespace eclqr
