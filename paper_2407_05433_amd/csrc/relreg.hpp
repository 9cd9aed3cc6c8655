// Register-resident factorization of a stacked relation system (one
// wavefront): the same two steps as wg_qr_colpiv + wg_row_basis (Lemma 1, then
// an orthonormal row basis, Section VIII items 1-4), with the matrix held in
// VGPRs instead of LDS so that every step is a few unrolled FMA sweeps.
//
//   phase 1  one stacked column per lane (NC columns per lane, PR rows):
//            Householder QR with column pivoting over the first nb columns,
//            applied to every column.  No columns move; the pivot column of
//            each step is broadcast through LDS.
//   phase 2  one remaining row per lane (KC coefficient columns + offset):
//            row-pivoted Gram-Schmidt with one re-orthogonalisation pass of
//            each pivot against the chosen rows (kept in LDS).
//
// Replay log (RelLog layout, header word 3 = 2): reflectors and tau as for
// the LDS routines; Gram-Schmidt records hold the pivot as an index into the
// phase-2 rows, 1/norm, the re-orthogonalisation coefficients and, for every
// row still unchosen at that step, its projection coefficient.
#pragma once

#include "common.hpp"
#include "dense.hpp"

namespace eclqr {

// vbuf, vs: LDS, PR doubles each.
template <int PR, int NC>
__device__ __forceinline__ int rr_phase1(double (&col)[NC][PR], int p, int c, int nb, double thr, double* vbuf,
                                         double* vs, double* Vlog, int P, double* taulog, int R) {
  const int lane = ECLQR_TID;
  bool used[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) used[t] = false;
  double ref = 1.0;
  int rho = 0;
  const int steps = (p < nb) ? p : nb;
  for (int j = 0; j < steps; ++j) {
    double bv = 0.0;
    int best = -1;
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int cl = lane + 64 * t;
      if (cl < nb && !used[t]) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < PR; r0 += 8) {
          if (r0 + 8 > j) {  // uniform: blocks of rows above the pivot row add exact zeros
#pragma unroll
            for (int r = r0; r < r0 + 8; r += 2) {
              const double a0 = (r >= j) ? col[t][r] : 0.0;
              const double a1 = (r + 1 >= j) ? col[t][r + 1] : 0.0;
              s0 = fma(a0, a0, s0);
              s1 = fma(a1, a1, s1);
            }
          }
        }
        const double s = s0 + s1;
        if (best < 0 || s > bv) {
          bv = s;
          best = cl;
        }
      }
    }
    wave_argmax(bv, best);
    if (best < 0) break;
    const double nrm = sqrt(bv);
    if (j == 0) ref = fmax(1.0, nrm);
    if (nrm <= thr * ref) break;
    const int owner = best & 63, town = best >> 6;
    if (lane == owner) {
#pragma unroll
      for (int t = 0; t < NC; ++t)
        if (t == town) {
#pragma unroll
          for (int r = 0; r < PR; ++r) vbuf[r] = col[t][r];
          used[t] = true;
        }
    }
    lds_sync();
    const double x0 = vbuf[j];
    const double beta = -copysign(nrm, x0);
    const double tj = (beta - x0) / beta;
    const double scale = 1.0 / (x0 - beta);
    // the scaled reflector, entry r in lane r (implicit 1 at row j), once
    for (int r = lane; r < PR; r += 64) {
      const double v = (r > j && r < p) ? vbuf[r] * scale : ((r == j) ? 1.0 : 0.0);
      vs[r] = v;
      if (j < R && r < p) Vlog[(int64_t)j * P + r] = (r > j) ? v : 0.0;
    }
    if (j < R && lane == 0) taulog[j] = tj;
    lds_sync();
    double vr[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) vr[r] = vs[r];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int cl = lane + 64 * t;
      if (cl < c && !used[t]) {
        double w0 = 0.0, w1 = 0.0;
#pragma unroll
        for (int r0 = 0; r0 < PR; r0 += 8) {
          if (r0 + 8 > j) {
#pragma unroll
            for (int r = r0; r < r0 + 8; r += 2) {
              w0 = fma(vr[r], col[t][r], w0);
              w1 = fma(vr[r + 1], col[t][r + 1], w1);
            }
          }
        }
        const double w = (w0 + w1) * tj;
#pragma unroll
        for (int r0 = 0; r0 < PR; r0 += 8) {
          if (r0 + 8 > j) {
#pragma unroll
            for (int r = r0; r < r0 + 8; ++r) col[t][r] = fma(-w, vr[r], col[t][r]);
          }
        }
      }
    }
    lds_sync();
    rho = j + 1;
  }
  return rho;
}

// Phase 2 on the rows held one per lane (lane < q).  Q: LDS, >= C x (KC + 1)
// (chosen rows with their offsets), pb: LDS KC + 1, dots: LDS C.  Returns the
// rows chosen; *over = 1 when more than C rows are independent.
// Columns >= kc of every row are zero; the unrolled sweeps skip those blocks.
template <int KC>
__device__ __forceinline__ int rr_phase2(double (&row)[KC], double& off, int q, int kc, double thr, double cons_thr,
                                         double* Q, double* pb, double* dots, int C, double* gslog, int64_t gstep,
                                         int* bad, int* over) {
  const int lane = ECLQR_TID;
  bool chosen = lane >= q;
  int sel = 0;
  double ref = 1.0;
  *over = 0;
  while (sel < q) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k0 = 0; k0 < KC; k0 += 8) {
      if (k0 < kc) {
#pragma unroll
        for (int k = k0; k < k0 + 8; k += 2) {
          s0 = fma(row[k], row[k], s0);
          s1 = fma(row[k + 1], row[k + 1], s1);
        }
      }
    }
    double bv = chosen ? 0.0 : s0 + s1;
    int best = chosen ? -1 : lane;
    wave_argmax(bv, best);
    if (best < 0) break;
    const double nv = sqrt(bv);
    if (sel == 0) ref = fmax(1.0, nv);
    if (nv <= thr * ref) break;
    if (sel >= C) {
      *over = 1;
      break;
    }
    double* rec = gslog + (int64_t)sel * gstep;
    if (lane == best) {
#pragma unroll
      for (int k = 0; k < KC; ++k) pb[k] = row[k];
      pb[KC] = off;
      chosen = true;
      rec[0] = (double)best;
    }
    lds_sync();
    if (sel > 0) {
      for (int l = lane; l < sel; l += 64) {
        const double d = lane_dot(Q + (int64_t)l * (KC + 1), 1, pb, 1, kc);
        dots[l] = d;
        rec[2 + l] = d;
      }
      lds_sync();
      for (int k = lane; k <= KC; k += 64) pb[k] -= lane_dot(dots, 1, Q + k, KC + 1, sel);
      lds_sync();
    }
    double part = 0.0;
    for (int k = lane; k < KC; k += 64) part = fma(pb[k], pb[k], part);
    const double inv = 1.0 / sqrt(wave_sum(part));
    if (lane == 0) rec[1] = inv;
    double* qs = Q + (int64_t)sel * (KC + 1);
    for (int k = lane; k <= KC; k += 64) qs[k] = pb[k] * inv;
    lds_sync();
    double qv[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) qv[k] = qs[k];
    if (!chosen) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int k0 = 0; k0 < KC; k0 += 8) {
        if (k0 < kc) {
#pragma unroll
          for (int k = k0; k < k0 + 8; k += 2) {
            d0 = fma(row[k], qv[k], d0);
            d1 = fma(row[k + 1], qv[k + 1], d1);
          }
        }
      }
      const double d = d0 + d1;
#pragma unroll
      for (int k0 = 0; k0 < KC; k0 += 8) {
        if (k0 < kc) {
#pragma unroll
          for (int k = k0; k < k0 + 8; ++k) row[k] = fma(-d, qv[k], row[k]);
        }
      }
      off = fma(-d, qs[KC], off);
      rec[2 + C + lane] = d;
    }
    ++sel;
  }
  const double any = (!chosen && fabs(off) > cons_thr) ? 1.0 : 0.0;
  *bad = (wave_max(any) != 0.0) ? 1 : 0;
  lds_sync();
  return sel;
}

}  // namespace eclqr
