// Workgroup-cooperative dense FP64 routines for small row-major matrices.
//
// A workgroup is exactly one wavefront (64 lanes): reductions and pivot
// searches are register shuffles whose result every lane holds, and barriers
// only order LDS traffic inside the wave.  Every routine is called by all
// lanes with identical arguments and returns after a barrier.  Matrices live in LDS or global
// memory (row-major, leading dimension ld); outputs never alias inputs unless
// stated.  Threads own columns in the Householder routines (each thread
// updates whole columns, the reflector is broadcast from LDS), which keeps
// the only cross-thread traffic to one vector and one reduction per step.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace eclqr {

// Lane id and lane count of the routines; a file whose workgroups hold
// several wavefronts that each run routines on their own data defines them
// per wavefront before including this header.
#ifndef ECLQR_TID
#define ECLQR_TID ((int)threadIdx.x)
#endif
#ifndef ECLQR_NT
#define ECLQR_NT ((int)blockDim.x)
#endif

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// Orders LDS traffic between the lanes of the one-wavefront workgroup.  The
// LDS instructions of a wave execute in issue order, so it is enough that the
// compiler moves no memory operation across this point; unlike wg_sync it
// does not wait for outstanding global stores.  Only for code whose
// cross-lane data lives in LDS or registers (global memory written in the
// section is not read back in it).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_wave_barrier();
  __asm__ volatile("" ::: "memory");
}

// Barrier selected at compile time: routines called on LDS-resident operands
// only (kL) need no wait for outstanding global stores.
template <bool kL>
__device__ __forceinline__ void bsync() {
  if constexpr (kL) lds_sync();
  else wg_sync();
}

// Wave reductions by DPP lane moves (VALU, no LDS traffic).  Within each row
// of 16 lanes, quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and
// row_mirror pair every lane with a partner holding a disjoint partial, so
// after four steps all 16 lanes hold the row's result.  row_bcast15 (rows 1,
// 3 take lane 15 of the row below) and row_bcast31 (rows 2, 3 take lane 31)
// leave the wave's result in lane 63, which v_readlane hands to every lane:
// all lanes end with the same bits.  Called by all 64 lanes (full EXEC).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, kCtrl, kRowMask, 0xF, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_d(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = dpp_i<kCtrl, kRowMask>((int)(o & 0xffffffffll), (int)(x & 0xffffffffll));
  const int hi = dpp_i<kCtrl, kRowMask>((int)(o >> 32), (int)(x >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// Value of `v` in lane `lane` (wave-uniform lane index).
__device__ __forceinline__ double wave_bcast(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ int wave_bcast_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

constexpr int kDppX1 = 0xB1, kDppX2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140, kDppBcast15 = 0x142,
              kDppBcast31 = 0x143;

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppX1, 0xF>(0.0, v);
  v += dpp_d<kDppX2, 0xF>(0.0, v);
  v += dpp_d<kDppHalfMirror, 0xF>(0.0, v);
  v += dpp_d<kDppMirror, 0xF>(0.0, v);
  v += dpp_d<kDppBcast15, 0xA>(0.0, v);
  v += dpp_d<kDppBcast31, 0xC>(0.0, v);
  return wave_bcast(v, 63);
}
__device__ __forceinline__ double wave_max(double v) {
  const double lo = -HUGE_VAL;
  v = fmax(v, dpp_d<kDppX1, 0xF>(lo, v));
  v = fmax(v, dpp_d<kDppX2, 0xF>(lo, v));
  v = fmax(v, dpp_d<kDppHalfMirror, 0xF>(lo, v));
  v = fmax(v, dpp_d<kDppMirror, 0xF>(lo, v));
  v = fmax(v, dpp_d<kDppBcast15, 0xA>(lo, v));
  v = fmax(v, dpp_d<kDppBcast31, 0xC>(lo, v));
  return wave_bcast(v, 63);
}
// Largest value and its index over the lanes (idx < 0: lane has no
// candidate); the lowest index wins ties, as in an ascending serial scan.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void argmax_step(double& v, int& idx) {
  const double ov = dpp_d<kCtrl, kRowMask>(v, v);
  const int oi = dpp_i<kCtrl, kRowMask>(-1, idx);
  if (oi >= 0 && (idx < 0 || ov > v || (ov == v && oi < idx))) {
    v = ov;
    idx = oi;
  }
}
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  argmax_step<kDppX1, 0xF>(v, idx);
  argmax_step<kDppX2, 0xF>(v, idx);
  argmax_step<kDppHalfMirror, 0xF>(v, idx);
  argmax_step<kDppMirror, 0xF>(v, idx);
  argmax_step<kDppBcast15, 0xA>(v, idx);
  argmax_step<kDppBcast31, 0xC>(v, idx);
  v = wave_bcast(v, 63);
  idx = wave_bcast_i(idx, 63);
}

// Triangular solves with the vector held one entry per lane (lane i holds
// entry i, n <= 64; lanes >= n keep their value).  Each step hands the newly
// solved entry to every lane by v_readlane; diagonals are inverted up front so
// the chain carries a multiply rather than a divide.
// L y = x, L lower triangular.
__device__ __forceinline__ double lane_trsv_lower(const double* L, int ld, double v, int n) {
  const int lane = ECLQR_TID;
  const double rd = (lane < n) ? 1.0 / L[lane * ld + lane] : 0.0;
  for (int i = 0; i < n; ++i) {
    if (lane == i) v *= rd;
    const double xi = wave_bcast(v, i);
    if (lane > i && lane < n) v = fma(-L[lane * ld + i], xi, v);
  }
  return v;
}
// L' y = x, L lower triangular.
__device__ __forceinline__ double lane_trsv_lower_t(const double* L, int ld, double v, int n) {
  const int lane = ECLQR_TID;
  const double rd = (lane < n) ? 1.0 / L[lane * ld + lane] : 0.0;
  for (int i = n - 1; i >= 0; --i) {
    if (lane == i) v *= rd;
    const double yi = wave_bcast(v, i);
    if (lane < i) v = fma(-L[i * ld + lane], yi, v);
  }
  return v;
}
// lane_trsv_lower and lane_trsv_lower_t for n <= NM with the lane's row
// (column) of L loaded into registers before the first step, so the solve
// waits on memory once instead of once a step (L in global memory).  Same
// operations in the same order, so the same bits.
template <int NM>
__device__ __forceinline__ double lane_trsv_lower_pre(const double* L, int ld, double v, int n) {
  const int lane = ECLQR_TID;
  const int r = (lane < n) ? lane : 0;
  double row[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) row[i] = L[r * ld + ((i < n) ? i : 0)];
  const double rd = (lane < n) ? 1.0 / L[lane * ld + lane] : 0.0;
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    if (i < n) {
      if (lane == i) v *= rd;
      const double xi = wave_bcast(v, i);
      if (lane > i && lane < n) v = fma(-row[i], xi, v);
    }
  }
  return v;
}
template <int NM>
__device__ __forceinline__ double lane_trsv_lower_t_pre(const double* L, int ld, double v, int n) {
  const int lane = ECLQR_TID;
  const int cl = (lane < n) ? lane : 0;
  double col[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) col[i] = L[((i < n) ? i : 0) * ld + cl];
  const double rd = (lane < n) ? 1.0 / L[lane * ld + lane] : 0.0;
#pragma unroll
  for (int i = NM - 1; i >= 0; --i) {
    if (i < n) {
      if (lane == i) v *= rd;
      const double yi = wave_bcast(v, i);
      if (lane < i) v = fma(-col[i], yi, v);
    }
  }
  return v;
}
// Dispatch on n: preloaded for n <= 32, else the plain form.
__device__ __forceinline__ double lane_trsv_lower_any(const double* L, int ld, double v, int n) {
  if (n <= 16) return lane_trsv_lower_pre<16>(L, ld, v, n);
  if (n <= 32) return lane_trsv_lower_pre<32>(L, ld, v, n);
  return lane_trsv_lower(L, ld, v, n);
}
__device__ __forceinline__ double lane_trsv_lower_t_any(const double* L, int ld, double v, int n) {
  if (n <= 16) return lane_trsv_lower_t_pre<16>(L, ld, v, n);
  if (n <= 32) return lane_trsv_lower_t_pre<32>(L, ld, v, n);
  return lane_trsv_lower_t(L, ld, v, n);
}
// U' y = x, U upper triangular.
__device__ __forceinline__ double lane_trsv_upper_t(const double* U, int ld, double v, int n) {
  const int lane = ECLQR_TID;
  const double rd = (lane < n) ? 1.0 / U[lane * ld + lane] : 0.0;
  for (int i = 0; i < n; ++i) {
    if (lane == i) v *= rd;
    const double xi = wave_bcast(v, i);
    if (lane > i && lane < n) v = fma(-U[i * ld + lane], xi, v);
  }
  return v;
}

// Maximum of one value per lane (buf unused, kept for call sites).
__device__ __forceinline__ double wg_reduce_max(double v, double* /*buf*/) { return wave_max(v); }

// Per-lane strided kernels.  LDS and global loads of a later iteration cannot
// move above an earlier store the compiler cannot prove disjoint, so in-place
// updates load a batch of operands into registers before storing it, and dot
// products keep four independent accumulators.
// The tails of these loops run as at most one 4-, one 2- and one 1-element
// step, each issuing its loads before its arithmetic (a plain remainder loop
// waits on every load in turn); the arithmetic order is that of a plain loop.
__device__ __forceinline__ double lane_dot(const double* a, int sa, const double* b, int sb, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    s0 = fma(a[i * sa], b[i * sb], s0);
    s1 = fma(a[(i + 1) * sa], b[(i + 1) * sb], s1);
    s2 = fma(a[(i + 2) * sa], b[(i + 2) * sb], s2);
    s3 = fma(a[(i + 3) * sa], b[(i + 3) * sb], s3);
  }
  if (i + 2 <= n) {
    const double a0 = a[i * sa], b0 = b[i * sb], a1 = a[(i + 1) * sa], b1 = b[(i + 1) * sb];
    s0 = fma(a1, b1, fma(a0, b0, s0));
    i += 2;
  }
  if (i < n) s0 = fma(a[i * sa], b[i * sb], s0);
  return (s0 + s1) + (s2 + s3);
}

// acc + sgn * sum_{k<n} a[k] b[k] as one FMA chain in ascending k.
template <bool kNeg>
__device__ __forceinline__ double lane_chain(double acc, const double* a, int sa, const double* b, int sb, int n) {
  int k = 0;
  for (; k + 8 <= n; k += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      av[t] = a[(k + t) * sa];
      bv[t] = b[(k + t) * sb];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) acc = fma(kNeg ? -av[t] : av[t], bv[t], acc);
  }
  if (k + 4 <= n) {
    double av[4], bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      av[t] = a[(k + t) * sa];
      bv[t] = b[(k + t) * sb];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = fma(kNeg ? -av[t] : av[t], bv[t], acc);
    k += 4;
  }
  if (k + 2 <= n) {
    const double a0 = a[k * sa], b0 = b[k * sb], a1 = a[(k + 1) * sa], b1 = b[(k + 1) * sb];
    acc = fma(kNeg ? -a0 : a0, b0, acc);
    acc = fma(kNeg ? -a1 : a1, b1, acc);
    k += 2;
  }
  if (k < n) acc = fma(kNeg ? -a[k * sa] : a[k * sa], b[k * sb], acc);
  return acc;
}

// y[i] += alpha x[i], i < n (x and y disjoint).
__device__ __forceinline__ void lane_axpy(double* y, int sy, const double* x, int sx, int n, double alpha) {
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    double xv[8], yv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      xv[t] = x[(i + t) * sx];
      yv[t] = y[(i + t) * sy];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) y[(i + t) * sy] = fma(alpha, xv[t], yv[t]);
  }
  if (i + 4 <= n) {
    double xv[4], yv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      xv[t] = x[(i + t) * sx];
      yv[t] = y[(i + t) * sy];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) y[(i + t) * sy] = fma(alpha, xv[t], yv[t]);
    i += 4;
  }
  if (i + 2 <= n) {
    const double x0 = x[i * sx], y0 = y[i * sy], x1 = x[(i + 1) * sx], y1 = y[(i + 1) * sy];
    y[i * sy] = fma(alpha, x0, y0);
    y[(i + 1) * sy] = fma(alpha, x1, y1);
    i += 2;
  }
  if (i < n) y[i * sy] = fma(alpha, x[i * sx], y[i * sy]);
}

// wg_gemm for outputs of at least 8 x 8: lanes on an 8 x 8 grid, lane (gr, gc)
// computing the R x R outputs (gr + 8a, gc + 8b) of each 8R x 8R tile, so a k
// step loads R values of op(A) and R of op(B) for R * R FMAs (instead of two
// loads per FMA).  Every output is the same FMA chain in ascending k as in
// wg_gemm's other form, with the same final expression, so the same bits.
template <int R>
__device__ __forceinline__ void wg_gemm_grid(double* C, int ldc, const double* A, int lda, bool tA, const double* B,
                                             int ldb, bool tB, int M, int N, int K, double alpha, double beta) {
  const int gr = ECLQR_TID >> 3, gc = ECLQR_TID & 7;
  const int sa = tA ? lda : 1, sb = tB ? 1 : ldb;  // k strides
  const int ra = tA ? 1 : lda, cb = tB ? ldb : 1;  // strides between rows of op(A), columns of op(B)
  for (int i0 = 0; i0 < M; i0 += 8 * R)
    for (int j0 = 0; j0 < N; j0 += 8 * R) {
      const double* ap[R];
      const double* bp[R];
      bool rv[R], cv[R];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const int i = i0 + gr + 8 * a;
        rv[a] = i < M;
        ap[a] = A + (int64_t)(rv[a] ? i : 0) * ra;  // rows past M read row 0 and are dropped
      }
#pragma unroll
      for (int b = 0; b < R; ++b) {
        const int j = j0 + gc + 8 * b;
        cv[b] = j < N;
        bp[b] = B + (int64_t)(cv[b] ? j : 0) * cb;
      }
      double acc[R][R];
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) acc[a][b] = 0.0;
      int k = 0;
      for (; k + 2 <= K; k += 2) {
        double av[R][2], bv[R][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int a = 0; a < R; ++a) av[a][q] = ap[a][(k + q) * sa];
#pragma unroll
          for (int b = 0; b < R; ++b) bv[b][q] = bp[b][(k + q) * sb];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) acc[a][b] = fma(av[a][q], bv[b][q], acc[a][b]);
      }
      for (; k < K; ++k) {
        double av[R], bv[R];
#pragma unroll
        for (int a = 0; a < R; ++a) av[a] = ap[a][k * sa];
#pragma unroll
        for (int b = 0; b < R; ++b) bv[b] = bp[b][k * sb];
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
          for (int b = 0; b < R; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
          if (rv[a] && cv[b]) {
            const int co = (i0 + gr + 8 * a) * ldc + (j0 + gc + 8 * b);
            const double prev = (beta != 0.0) ? beta * C[co] : 0.0;
            C[co] = alpha * acc[a][b] + prev;
          }
        }
    }
}

// C(MxN) = alpha * op(A) * op(B) + beta * C.  op(A) is MxK, op(B) is KxN.
// beta == 0 never reads C.  With kGrid (default: operands in LDS), outputs of
// at least 8 x 8 go to wg_gemm_grid; its accumulators and operand registers
// raise a kernel's VGPR count, which costs the latency-bound kernels on
// global memory more occupancy than the fewer loads gain them (the stage
// elimination: 139 -> 169 VGPRs, 11.5 -> 12.2 ms).  Otherwise each lane computes
// up to four outputs per round with their
// accumulations interleaved (the loads of four k steps of all four are
// independent and in flight together).  Either way every output is one FMA
// chain in ascending k.
template <bool kL = false, bool kGrid = kL>
__device__ __forceinline__ void wg_gemm(double* C, int ldc, const double* A, int lda, bool tA, const double* B, int ldb,
                               bool tB, int M, int N, int K, double alpha, double beta) {
  if (kGrid && M >= 8 && N >= 8) {
    if (M <= 16 && N <= 16)
      wg_gemm_grid<2>(C, ldc, A, lda, tA, B, ldb, tB, M, N, K, alpha, beta);
    else
      wg_gemm_grid<3>(C, ldc, A, lda, tA, B, ldb, tB, M, N, K, alpha, beta);
    bsync<kL>();
    return;
  }
  const int sa = tA ? lda : 1, sb = tB ? 1 : ldb;
  const int total = M * N;
  for (int r0 = ECLQR_TID; r0 < total; r0 += 4 * ECLQR_NT) {
    const double* ap[4];
    const double* bp[4];
    int co[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int want = r0 + t * ECLQR_NT;
      const int idx = (want < total) ? want : r0;  // surplus slots recompute a valid output and drop it
      const int i = idx / N, j = idx - (idx / N) * N;
      ap[t] = tA ? A + i : A + (int64_t)i * lda;
      bp[t] = tB ? B + (int64_t)j * ldb : B + j;
      co[t] = (want < total) ? i * ldc + j : -1;
    }
    int k = 0;
    for (; k + 2 <= K; k += 2) {
      double av[4][2], bv[4][2];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          av[t][q] = ap[t][(k + q) * sa];
          bv[t][q] = bp[t][(k + q) * sb];
        }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[t] = fma(av[t][q], bv[t][q], acc[t]);
    }
    for (; k < K; ++k)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = fma(ap[t][k * sa], bp[t][k * sb], acc[t]);
    double prev[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) prev[t] = (co[t] >= 0 && beta != 0.0) ? beta * C[co[t]] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (co[t] >= 0) C[co[t]] = alpha * acc[t] + prev[t];
  }
  bsync<kL>();
}

// y(M) = alpha * op(A) x + beta * y.   op(A) is MxK.  Each entry is one FMA
// chain in ascending k (lane_chain: eight k steps' loads in flight).
template <bool kL = false>
__device__ __forceinline__ void wg_gemv(double* y, const double* A, int lda, bool tA, const double* x, int M, int K,
                               double alpha, double beta) {
  for (int i = ECLQR_TID; i < M; i += ECLQR_NT) {
    const double acc = tA ? lane_chain<false>(0.0, A + i, lda, x, 1, K)
                          : lane_chain<false>(0.0, A + (int64_t)i * lda, 1, x, 1, K);
    const double prev = (beta == 0.0) ? 0.0 : beta * y[i];
    y[i] = alpha * acc + prev;
  }
  bsync<kL>();
}

template <bool kL = false>
__device__ __forceinline__ void wg_copy(double* dst, int ldd, const double* src, int lds, int rows, int cols) {
  const int total = rows * cols;
  for (int r0 = ECLQR_TID; r0 < total; r0 += 4 * ECLQR_NT) {
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = r0 + t * ECLQR_NT;
      const int i = idx / cols, j = idx - (idx / cols) * cols;
      v[t] = (idx < total) ? src[i * lds + j] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = r0 + t * ECLQR_NT;
      const int i = idx / cols, j = idx - (idx / cols) * cols;
      if (idx < total) dst[i * ldd + j] = v[t];
    }
  }
  bsync<kL>();
}

template <bool kL = false>
__device__ __forceinline__ void wg_copy_t(double* dst, int ldd, const double* src, int lds, int rows, int cols) {
  // dst (cols x rows) = src(rows x cols)^T
  const int total = rows * cols;
  for (int r0 = ECLQR_TID; r0 < total; r0 += 4 * ECLQR_NT) {
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = r0 + t * ECLQR_NT;
      const int i = idx / cols, j = idx - (idx / cols) * cols;
      v[t] = (idx < total) ? src[i * lds + j] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int idx = r0 + t * ECLQR_NT;
      const int i = idx / cols, j = idx - (idx / cols) * cols;
      if (idx < total) dst[j * ldd + i] = v[t];
    }
  }
  bsync<kL>();
}

template <bool kL = false>
__device__ __forceinline__ void wg_fill(double* dst, int ldd, int rows, int cols, double v) {
  for (int idx = ECLQR_TID; idx < rows * cols; idx += ECLQR_NT) {
    const int i = idx / cols, j = idx - (idx / cols) * cols;
    dst[i * ldd + j] = v;
  }
  bsync<kL>();
}

template <bool kL = false>
__device__ __forceinline__ void wg_identity(double* dst, int ldd, int n) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    dst[i * ldd + j] = (i == j) ? 1.0 : 0.0;
  }
  bsync<kL>();
}

// Symmetrise a square matrix in place: S = (S + S^T)/2.
template <bool kL = false>
__device__ __forceinline__ void wg_symmetrize(double* S, int ld, int n) {
  for (int idx = ECLQR_TID; idx < n * n; idx += ECLQR_NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    if (i < j) {
      const double v = 0.5 * (S[i * ld + j] + S[j * ld + i]);
      S[i * ld + j] = v;
      S[j * ld + i] = v;
    }
  }
  bsync<kL>();
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
__device__ __forceinline__ int wg_qr_colpiv(double* W, int ld, int p, int c, int c0, int cp, double thr, double* tau,
                                   QRScratch sc) {
  for (int j = ECLQR_TID; j < cp; j += ECLQR_NT) sc.perm[j] = j;
  lds_sync();
  const int steps = (p < cp) ? p : cp;
  int r = 0;
  double ref = 1.0;
  for (int j = 0; j < steps; ++j) {
    double bv = 0.0;
    int best = -1;
    for (int col = j + ECLQR_TID; col < cp; col += ECLQR_NT) {
      const double* cv = W + j * ld + c0 + col;
      const double s = lane_dot(cv, ld, cv, ld, p - j);
      if (best < 0 || s > bv) {
        bv = s;
        best = col;
      }
    }
    wave_argmax(bv, best);
    const double nrm = sqrt(bv);
    if (j == 0) ref = fmax(1.0, nrm);
    if (nrm <= thr * ref) break;
    const int pc = best;
    const double x0 = W[j * ld + c0 + pc];
    const double beta = -copysign(nrm, x0);
    const double tj = (beta - x0) / beta;
    const double scale = 1.0 / (x0 - beta);
    lds_sync();
    if (ECLQR_TID == 0) {
      const int tp = sc.perm[j];
      sc.perm[j] = sc.perm[pc];
      sc.perm[pc] = tp;
    }
    if (pc != j) {
      for (int row = ECLQR_TID; row < p; row += ECLQR_NT) {
        const double a = W[row * ld + c0 + j];
        W[row * ld + c0 + j] = W[row * ld + c0 + pc];
        W[row * ld + c0 + pc] = a;
      }
      lds_sync();
    }
    for (int row = j + 1 + ECLQR_TID; row < p; row += ECLQR_NT) W[row * ld + c0 + j] *= scale;
    if (ECLQR_TID == 0) tau[j] = tj;
    lds_sync();
    for (int col = ECLQR_TID; col < c; col += ECLQR_NT) {
      // skip this and the earlier pivot columns (they hold reflectors below the diagonal)
      if (col >= c0 && col <= c0 + j) continue;
      const double* v = W + (j + 1) * ld + c0 + j;
      double* y = W + (j + 1) * ld + col;
      const double w = (W[j * ld + col] + lane_dot(v, ld, y, ld, p - j - 1)) * tj;
      W[j * ld + col] -= w;
      lane_axpy(y, ld, v, ld, p - j - 1, -w);
    }
    lds_sync();
    if (ECLQR_TID == 0) W[j * ld + c0 + j] = beta;
    lds_sync();
    r = j + 1;
  }
  return r;
}

// Copy the r reflectors left by wg_qr_colpiv (rows below the diagonal of the
// pivot columns [c0, c0 + r)) and their scalars to a log: V[j * P + row].
__device__ __forceinline__ void wg_log_reflectors(const double* W, int ld, int p, int c0, int r, const double* tau, double* V,
                                         int P, double* tlog) {
  for (int idx = ECLQR_TID; idx < r * p; idx += ECLQR_NT) {
    const int j = idx / p, row = idx - (idx / p) * p;
    V[(int64_t)j * P + row] = (row > j) ? W[row * ld + c0 + j] : 0.0;
  }
  for (int j = ECLQR_TID; j < r; j += ECLQR_NT) tlog[j] = tau[j];
  lds_sync();
}

// Apply Q = H_0 H_1 ... H_{r-1} (reflectors stored by wg_qr_colpiv in the
// pivot columns [c0, c0 + r) of W, rows j+1.. of column c0+j) to the p x nc
// matrix X (row-major, ldx) from the left: X <- Q X.
__device__ __forceinline__ void wg_apply_q(const double* W, int ld, int p, int c0, int r, const double* tau, double* X,
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
// When glog is given, every step is recorded for replay on a new offset
// column: glog[s * gstep + 0] = pivot row, [1] = 1/norm, [2 + l] = the
// re-orthogonalisation coefficient of chosen row l, [2 + gcap + row] = the
// projection coefficient of each later row (steps s < gcap only).
__device__ __forceinline__ int wg_row_basis(double* W, int ld, int r0, int p, int k0, int kc, double thr, double cons_thr,
                                   int* bad, double* scr /* >= 2*(p - r0) + 8 + 64 */, double* glog = nullptr,
                                   int64_t gstep = 0, int gcap = 0) {
  const int rows = p - r0;
  double* dots = scr;  // >= rows
  int sel = 0;
  double ref = 1.0;
  while (sel < rows) {
    const int base = r0 + sel;
    double bv = 0.0;
    int best = -1;
    for (int rr = base + ECLQR_TID; rr < p; rr += ECLQR_NT) {
      const double* rv = W + rr * ld + k0;
      const double s = lane_dot(rv, 1, rv, 1, kc);
      if (best < 0 || s > bv) {
        bv = s;
        best = rr;
      }
    }
    wave_argmax(bv, best);
    const double nv = sqrt(bv);
    if (sel == 0) ref = fmax(1.0, nv);
    if (nv <= thr * ref) break;
    double* rec = (glog && sel < gcap) ? glog + (int64_t)sel * gstep : nullptr;
    if (rec && ECLQR_TID == 0) rec[0] = (double)best;
    if (best != base) {
      for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT) {
        const double a = W[base * ld + k0 + cc];
        W[base * ld + k0 + cc] = W[best * ld + k0 + cc];
        W[best * ld + k0 + cc] = a;
      }
      lds_sync();
    }
    // re-orthogonalise the pivot row against the chosen rows (one pass)
    if (sel > 0) {
      for (int l = ECLQR_TID; l < sel; l += ECLQR_NT) {
        const double d = lane_dot(W + (r0 + l) * ld + k0, 1, W + base * ld + k0, 1, kc);
        dots[l] = d;
        if (rec) rec[2 + l] = d;
      }
      lds_sync();
      for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT)
        W[base * ld + k0 + cc] -= lane_dot(dots, 1, W + r0 * ld + k0 + cc, ld, sel);
      lds_sync();
    }
    // normalise (offset included)
    double s = 0.0;
    for (int cc = ECLQR_TID; cc < kc; cc += ECLQR_NT) s = fma(W[base * ld + k0 + cc], W[base * ld + k0 + cc], s);
    const double inv = 1.0 / sqrt(wave_sum(s));
    if (rec && ECLQR_TID == 0) rec[1] = inv;
    lds_sync();
    for (int cc = ECLQR_TID; cc <= kc; cc += ECLQR_NT) W[base * ld + k0 + cc] *= inv;
    lds_sync();
    // project the pivot row out of the remaining rows
    for (int rr = base + 1 + ECLQR_TID; rr < p; rr += ECLQR_NT) {
      double* row = W + rr * ld + k0;
      const double* piv = W + base * ld + k0;
      const double d = lane_dot(row, 1, piv, 1, kc);
      lane_axpy(row, 1, piv, 1, kc + 1, -d);
      if (rec) rec[2 + gcap + rr] = d;
    }
    lds_sync();
    ++sel;
  }
  // consistency of the dependent rows
  double any = 0.0;
  for (int rr = r0 + sel + ECLQR_TID; rr < p; rr += ECLQR_NT)
    if (fabs(W[rr * ld + k0 + kc]) > cons_thr) any = 1.0;
  *bad = (wave_max(any) != 0.0) ? 1 : 0;
  lds_sync();
  return sel;
}

// In-place Cholesky S = L L^T of an n x n SPD matrix (lower triangle holds L,
// upper triangle zeroed).  Returns 0 on success, 1 if a pivot (before the
// square root) is not above `floor`.  Right-looking, one row per lane for the
// column scaling and the trailing update (lane_axpy: batched, predicated).
template <bool kL = false>
__device__ __forceinline__ int wg_cholesky(double* S, int ld, int n, double* sh /* unused */, double floor = 0.0) {
  (void)sh;
  for (int j = 0; j < n; ++j) {
    const double d = S[j * ld + j];
    if (!(d > floor)) {
      bsync<kL>();
      return 1;
    }
    const double dj = sqrt(d);
    for (int i = j + 1 + ECLQR_TID; i < n; i += ECLQR_NT) S[i * ld + j] /= dj;
    if (ECLQR_TID == 0) S[j * ld + j] = dj;
    bsync<kL>();
    // trailing update of the lower triangle, one row per lane
    for (int a2 = j + 1 + ECLQR_TID; a2 < n; a2 += ECLQR_NT)
      lane_axpy(S + a2 * ld + j + 1, 1, S + (j + 1) * ld + j, ld, a2 - j, -S[a2 * ld + j]);
    bsync<kL>();
  }
  for (int a2 = ECLQR_TID; a2 < n; a2 += ECLQR_NT)
    for (int b = a2 + 1; b < n; ++b) S[a2 * ld + b] = 0.0;
  bsync<kL>();
  return 0;
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix S
// (read only, n <= 64): K (n x r, row-major, ldk) with S ~= K K^T, rows in the
// original order, columns in pivot order.  Stops when the largest remaining
// diagonal is <= tol * (largest diagonal of S).  Row i is lane i: its
// remaining diagonal and "used" flag live in registers.  rem, used, sh unused.
template <bool kL = false>
__device__ __forceinline__ int wg_pchol(const double* S, int ld, int n, double tol, double* K, int ldk, double* rem, int* used,
                               double* sh) {
  (void)rem;
  (void)used;
  (void)sh;
  const int lane = ECLQR_TID;
  const bool row = lane < n;
  double rm = row ? S[lane * ld + lane] : 0.0;
  bool done = !row;
  const double ref = wave_max(row ? rm : 0.0);
  int r = 0;
  for (int j = 0; j < n; ++j) {
    double bv = done ? 0.0 : rm;
    int best = done ? -1 : lane;
    wave_argmax(bv, best);
    if (!(best >= 0 && bv > tol * ref && bv > 0.0)) break;
    const int p = best;
    const double dp = sqrt(bv);
    double v = 0.0;
    if (row) {
      if (lane == p) {
        v = dp;
      } else if (!done) {
        v = lane_chain<true>(S[lane * ld + p], K + lane * ldk, 1, K + p * ldk, 1, j) / dp;
      }
      K[lane * ldk + j] = v;
    }
    if (lane == p) done = true;
    if (!done) rm = fma(-v, v, rm);
    r = j + 1;
    bsync<kL>();
  }
  return r;
}

// Solve L X = B (lower triangular L, n x n) in place on B (n x nc); one
// column per lane, each entry one FMA chain in ascending k times the
// reciprocal of the diagonal (which does not depend on the solve, so its
// latency overlaps the chain).
template <bool kL = false>
__device__ __forceinline__ void wg_trsm_lower(const double* L, int ldl, double* X, int ldx, int n, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < n; ++i) {
      const double rd = 1.0 / L[i * ldl + i];
      X[i * ldx + col] = lane_chain<true>(X[i * ldx + col], L + i * ldl, 1, X + col, ldx, i) * rd;
    }
  }
  bsync<kL>();
}

// Solve L^T X = B (L lower triangular) in place on B (n x nc).
template <bool kL = false>
__device__ __forceinline__ void wg_trsm_lower_t(const double* L, int ldl, double* X, int ldx, int n, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = n - 1; i >= 0; --i) {
      const double rd = 1.0 / L[i * ldl + i];
      // updates in descending k (the order of the right-looking form)
      X[i * ldx + col] =
          lane_chain<true>(X[i * ldx + col], L + (n - 1) * ldl + i, -ldl, X + (n - 1) * ldx + col, -ldx, n - i - 1) * rd;
    }
  }
  bsync<kL>();
}

// Solve U^T X = B with U upper triangular (r x r, diagonal U[j][c0+j] inside a
// wider matrix: U(i, j) = W[i*ld + c0 + j]) in place on X (r x nc).
template <bool kL = false>
__device__ __forceinline__ void wg_trsm_upper_t(const double* W, int ld, int c0, double* X, int ldx, int r, int nc) {
  for (int col = ECLQR_TID; col < nc; col += ECLQR_NT) {
    for (int i = 0; i < r; ++i)
      X[i * ldx + col] = (X[i * ldx + col] - lane_dot(W + c0 + i, ld, X + col, ldx, i)) / W[i * ld + c0 + i];
  }
  bsync<kL>();
}

// LU factorisation with partial pivoting of an n x n matrix in place;
// piv[i] = row swapped with row i at step i.
template <bool kL = false>
__device__ __forceinline__ void wg_lu(double* Mt, int ld, int n, int* piv, double* sh) {
  (void)sh;
  for (int j = 0; j < n; ++j) {
    double bv = 0.0;
    int best = -1;
    for (int i = j + ECLQR_TID; i < n; i += ECLQR_NT) {
      const double v = fabs(Mt[i * ld + j]);
      if (best < 0 || v > bv) {
        bv = v;
        best = i;
      }
    }
    wave_argmax(bv, best);
    if (ECLQR_TID == 0) piv[j] = best;
    bsync<kL>();
    if (best != j) {
      for (int c = ECLQR_TID; c < n; c += ECLQR_NT) {
        const double a = Mt[j * ld + c];
        Mt[j * ld + c] = Mt[best * ld + c];
        Mt[best * ld + c] = a;
      }
      bsync<kL>();
    }
    const double d = Mt[j * ld + j];
    for (int i = j + 1 + ECLQR_TID; i < n; i += ECLQR_NT) Mt[i * ld + j] /= d;
    bsync<kL>();
    // trailing update, one row per lane
    for (int a = j + 1 + ECLQR_TID; a < n; a += ECLQR_NT)
      lane_axpy(Mt + a * ld + j + 1, 1, Mt + j * ld + j + 1, 1, n - j - 1, -Mt[a * ld + j]);
    bsync<kL>();
  }
}

// Solve (P L U) X = B in place on B (n x nc), factors from wg_lu.
template <bool kL = false>
__device__ __forceinline__ void wg_lu_solve(const double* LU, int ld, int n, const int* piv, double* X, int ldx, int nc) {
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
  bsync<kL>();
}

// Solve (P L U)^T X = B in place on B (n x nc):  U^T L^T P^T X = B.
template <bool kL = false>
__device__ __forceinline__ void wg_lu_solve_t(const double* LU, int ld, int n, const int* piv, double* X, int ldx, int nc) {
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
  bsync<kL>();
}

}  // namespace eclqr
