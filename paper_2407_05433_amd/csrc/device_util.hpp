// Device-side accessors for the engine tables.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace eclqr {

// One wavefront per workgroup: the dense helpers reduce with lane shuffles.
constexpr int kBlock = 64;

__device__ __forceinline__ double* slot_ptr(const DevEngine& e, int kind, int slot) {
  return e.scan[kind] + e.slot_off[(int64_t)kind * e.nslots + slot];
}
// variant 0: REL / RIC endpoints, variant 1: FWD endpoints
__device__ __forceinline__ int slot_a(const DevEngine& e, int var, int slot) { return e.slot_sa[var * e.nslots + slot]; }
__device__ __forceinline__ int slot_b(const DevEngine& e, int var, int slot) { return e.slot_sb[var * e.nslots + slot]; }

__device__ __forceinline__ void flag(int32_t* status, int inst, int32_t bit) {
  if (status) atomicOr(status + inst, bit);
}

// Outcome bit of a failure detected at stage `stage` of instance `inst` by a
// kernel of the problem's own pass: info (when the engine has it) keeps the
// largest such stage.  Algorithm 1 sweeps from the terminal stage backwards,
// so that is the first failure in its order.
__device__ __forceinline__ void flag_at(const DevEngine& e, int32_t* status, int inst, int32_t bit, int stage) {
  if (status) {
    atomicOr(status + inst, bit);
    if (e.info) atomicMax(e.info + inst, stage);
  }
}

// true when the instance has finished refining and must not be touched
__device__ __forceinline__ bool gated(const DevEngine& e, int inst) { return e.gate && e.gate[inst] == kGateDone; }

// true when no instance is refining: every task of a refinement-step kernel
// would be gated, so the kernel returns before reading its task list
__device__ __forceinline__ bool none_live(const DevEngine& e) { return e.live && *e.live == 0; }

// Stage at position t of a stage-kernel launch over [first, first + count) of
// the plan's size order.
__device__ __forceinline__ int64_t stage_at(const DevEngine& e, int64_t first, int64_t t) {
  return e.stage_perm ? (int64_t)e.stage_perm[first + t] : first + t;
}

__device__ __forceinline__ double* block_scratch(const DevEngine& e) {
  return e.scratch + (int64_t)blockIdx.x * e.scratch_per_block;
}

}  // namespace eclqr
