// Per-workgroup global scratch sizes (doubles), shared by host and device so
// the host can size the workspace exactly.
#pragma once

#include "common.hpp"

namespace eclqr {

ECLQR_HD inline int64_t rup4(int64_t x) { return (x + 3) & ~int64_t(3); }

// stage elimination: dims of the stage (n, n', m, k) at capacity.  The
// kernel reuses one region phase by phase, so the size is the largest phase.
ECLQR_HD inline int64_t elim_scratch(int n, int np, int m, int k) {
  const int64_t q = k + np;
  // QR of Gamma^T and the maps Y, y, Z: Gs Ps gs Phi gam X rsc (Q in LDS)
  const int64_t p1 = rup4(q * m) + rup4(q * n) + rup4(q) + rup4(q * n) + rup4(q) + rup4((int64_t)m * (n + 1)) +
                     rup4(q);
  const int64_t p2 = rup4((int64_t)np * n) + rup4((int64_t)np * m) + rup4(np);  // AT BZ cv
  // QT Mz RY RZ MzY w qz rz (the terminal stage's QT and v fit in it)
  const int64_t p3 = rup4((int64_t)n * n) + rup4((int64_t)n * m) + rup4((int64_t)m * n) + rup4((int64_t)m * m) +
                     rup4((int64_t)n * n) + rup4(m) + rup4(n) + rup4(m);
  const int64_t p4 = rup4((int64_t)m * (np + n + 1));  // [Wt V w2]
  int64_t s = p1 > p2 ? p1 : p2;
  s = s > p3 ? s : p3;
  s = s > p4 ? s : p4;
  return s + 64;
}

// Working pool of one value-function combine with every endpoint dim <= d:
// the factored path uses six d x d blocks, d x (d+1), d x d and four vectors;
// the LU fallback fits in the same pool.
ECLQR_HD inline int64_t ric_pool(int d) {
  const int64_t dd = rup4((int64_t)d * d);
  return 7 * dd + rup4((int64_t)d * (d + 1)) + 4 * rup4(d) + 64;
}

// Value-function combine with staged operands (every endpoint dim <= d): the
// operands read more than once (four d x d blocks at most), and a pool that
// holds the factored form (three d x d blocks, d x (d + 1), four vectors; the
// LU fallback uses the global scratch).
ECLQR_HD inline int64_t ric_stage_size(int d) { return rup4(4 * (int64_t)d * d); }
ECLQR_HD inline int64_t ric_pool_staged(int d) {
  const int64_t dd = rup4((int64_t)d * d);
  return 3 * dd + rup4((int64_t)d * (d + 1)) + 4 * rup4(d) + 64;
}

// Work arrays of one instance of the sequential fallback (doubles).
ECLQR_HD inline int64_t dp_stride(int maxn, int maxm) {
  const int64_t nn = (int64_t)maxn * maxn, mm2 = (int64_t)maxm * maxm, nm = (int64_t)maxn * maxm;
  return 3 * nn + 3 * nm + 2 * mm2 + 3 * (int64_t)maxn + 2 * (int64_t)maxm + 16;
}

// gains: dims at capacity (n, n', m)
ECLQR_HD inline int64_t gains_scratch(int n, int np, int m) {
  int64_t s = 0;
  s += rup4((int64_t)np * m) + rup4((int64_t)m * m) + rup4((int64_t)np * n) + rup4((int64_t)m * n);
  s += rup4(np) + rup4(m) + 64;
  return s;
}

// LDS per workgroup on gfx950 (the only target): plans decide at creation
// which kernels' tiles fit, and a device that reports less is rejected at
// solve time rather than launched past its limit.
constexpr int64_t kDeviceLdsBytes = 160 * 1024;

// Stacked systems of relation compositions whose LDS tile would exceed this
// run in a per-workgroup tile of global memory instead (measured on the
// 512-instance batch: tiles of up to 56 KiB at two workgroups per compute
// unit, 4.8 ms of compositions in LDS against 4.4 in global memory).
constexpr int64_t kRelComposeLds = 24 * 1024;

// LDS bytes of the minimum-norm local systems of the theta route
// (k_theta_local): the stacked system maxq x ldw, its Q factor, two
// maxq x (maxr + 1) blocks, vectors and pivots.
ECLQR_HD inline int64_t theta_local_lds(int maxq, int ldw, int maxr) {
  return 8 * ((int64_t)maxq * ldw + (int64_t)maxq * maxq + 2 * (int64_t)maxq * (maxr + 1) + maxq + 2 * (int64_t)ldw +
              8 + 5 * kMaxDim) +
         4 * (int64_t)(ldw + 1) + 64;
}

}  // namespace eclqr
