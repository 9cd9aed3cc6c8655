// Shared host/device definitions: per-stage descriptors, workspace arenas and
// slot layouts of the three associative scans.
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#define ECLQR_HD __host__ __device__
#else
#define ECLQR_HD
#endif

namespace eclqr {

constexpr int kMaxDim = 64;  // largest n_i, m_i, k_i handled by the kernels

// Offsets of the caller's fields (elements), order of the ECLQR_F_* enum minus x0.
enum InField { IN_Q = 0, IN_q, IN_R, IN_r, IN_M, IN_A, IN_B, IN_c, IN_E, IN_F, IN_g, IN_COUNT };

// Scan kinds.  REL: affine endpoint relations (feasible-domain scan, Section IV).
// RIC: conditional value-function elements of the reduced LQR.  FWD: affine
// closed-loop maps of the reduced state (forward pass).
enum ScanKind { SCAN_REL = 0, SCAN_RIC = 1, SCAN_FWD = 2, SCAN_COUNT = 3 };

struct StageInfo {
  int32_t n, np, m, k;   // n_i, n_{i+1} (0 at the terminal stage), m_i (0 at terminal), k_i
  int32_t inst, i, N;    // instance, stage index, horizon of the instance
  int32_t terminal;      // 1 for i == N
  int64_t in[IN_COUNT];  // element offsets into the caller's arrays
  int64_t x0;            // element offset of x0 (valid on stage 0)
  int64_t ws;            // base of the stage arena (doubles)
  int32_t elem[SCAN_COUNT];  // slot id of this stage's scan element
  int32_t suf[SCAN_COUNT];   // slot id of this stage's suffix result
};

// Stage arena: everything the stage-parallel kernels produce, sized by the
// stage's own (n, n', m, k) -- reduced dims are at most these.  The last
// block keeps the factors that a vector-only pass reuses: row scales,
// pivot order, Q1 and R11 of the QR of Gamma^T, the Cholesky factors of
// R-bar and of H_uu.
struct Arena {
  int64_t T, t, Y, Z, y, Ab, Bb, cb, Qb, Mb, Rb, qb, rb, K, kk, v;
  int64_t rsc, prm, Q1, R11, Lc, Hc, wl, Ym, ym, size;
};

ECLQR_HD inline Arena arena_layout(int n, int np, int m, int k) {
  Arena a;
  int64_t o = 0;
  a.T = o; o += (int64_t)n * n;
  a.t = o; o += n;
  a.Y = o; o += (int64_t)m * n;
  a.Z = o; o += (int64_t)m * m;
  a.y = o; o += m;
  a.Ab = o; o += (int64_t)np * n;
  a.Bb = o; o += (int64_t)np * m;
  a.cb = o; o += np;
  a.Qb = o; o += (int64_t)n * n;
  a.Mb = o; o += (int64_t)n * m;
  a.Rb = o; o += (int64_t)m * m;
  a.qb = o; o += n;
  a.rb = o; o += m;
  a.K = o; o += (int64_t)m * n;
  a.kk = o; o += m;
  a.v = o; o += m;
  a.rsc = o; o += k + np;
  a.prm = o; o += m;
  a.Q1 = o; o += (int64_t)m * m;
  a.R11 = o; o += (int64_t)m * m;
  a.Lc = o; o += (int64_t)m * m;
  a.Hc = o; o += (int64_t)m * m;
  a.wl = o; o += n;                // fast multipliers: T lambda-bar
  a.Ym = o; o += (int64_t)k * n;   // mu = Ym theta + ym (k x r, ld n)
  a.ym = o; o += k;
  a.size = (o + 3) & ~int64_t(3);  // 32-byte multiple
  return a;
}

// Log of a relation factorization (base relation or composition), replayed on
// new offsets by the vector-only pass.  P = row capacity of the stacked
// system, R = most Householder steps (min(eliminated dim, P)), C = row
// capacity of the result.  Layout: header (p, rho, rr) | row scales (P) |
// tau (R) | reflectors (R columns of P) | one record per Gram-Schmidt step:
// pivot row, 1/norm, re-orthogonalisation coefficients (C), projection
// coefficients by row (P).
struct RelLog {
  int64_t hdr, scale, tau, V, gs, step, size;
};
ECLQR_HD inline RelLog rel_log_layout(int P, int R, int C) {
  RelLog l;
  int64_t o = 0;
  l.hdr = o; o += 4;
  l.scale = o; o += P;
  l.tau = o; o += R;
  l.V = o; o += (int64_t)P * R;
  l.gs = o;
  l.step = 2 + (int64_t)C + P;
  o += (int64_t)C * l.step;
  l.size = (o + 3) & ~int64_t(3);
  return l;
}

// Log of a value-function combine over a middle dim d: flag (1 factored,
// 2 LU) | L or LU (d x d) | Rg (d x d) | pivots (d).
ECLQR_HD inline int64_t ric_log_size(int d) { return (4 + 2 * (int64_t)d * d + d + 3) & ~int64_t(3); }

// REL slot: rows x (na + nb + 1), row-major, coefficient columns of the left
// endpoint, then of the right endpoint, then the offset.
ECLQR_HD inline int64_t rel_slot_size(int cap, int na, int nb) {
  return (((int64_t)cap * (na + nb + 1)) + 3) & ~int64_t(3);
}

// RIC slot over endpoints (start, end) with dims (na, nb): [A nb x na | b nb |
// C nb x nb | eta na | J na x na]; a unary slot (nb = 0) holds only eta, J.
struct RicLayout {
  int64_t A, b, C, eta, J, size;
};
ECLQR_HD inline RicLayout ric_layout(int na, int nb) {
  RicLayout r;
  int64_t o = 0;
  r.A = o; o += (int64_t)nb * na;
  r.b = o; o += nb;
  r.C = o; o += (int64_t)nb * nb;
  r.eta = o; o += na;
  r.J = o; o += (int64_t)na * na;
  r.size = (o + 3) & ~int64_t(3);
  return r;
}

// FWD slot: affine map from the input side (nb) to the output side (na):
// [F na x nb | f na]; a unary slot (nb = 0) is the constant f.
ECLQR_HD inline int64_t fwd_slot_size(int na, int nb) {
  return (((int64_t)na * nb + na) + 3) & ~int64_t(3);
}

}  // namespace eclqr
