// Device-side helpers shared by the library's kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlu.h"

namespace rlu {

// ---------------------------------------------------------------------------
// Counter-based parameters of the projections.  mix64 is the SplitMix64
// output function (Steele, Lea & Flood 2014, Stafford's variant 13).
// ---------------------------------------------------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kStreamSem = 1;
constexpr int kStreamSigns = 2;
constexpr int kStreamSelect = 3;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t stream_key(uint64_t seed, int t) {
  return mix64(seed + (uint64_t)t * kGamma);
}
__host__ __device__ inline uint64_t draw(uint64_t key, uint64_t i) {
  return mix64(key + (i + 1) * kGamma);
}

// Packed column code used by the sketch kernels: bucket in the low 16 bits
// (s <= 65536), bit 31 set when the folded sign sgn(j) * d[h(j)] is -1.
// Folding the +-1 FFT diagonal into the SEM sign is exact: flipping the sign
// of every summand of a bucket flips the rounded sum.
__device__ inline uint32_t code_bucket(uint32_t c) { return c & 0xFFFFu; }
__device__ inline double code_apply(uint32_t c, double v) { return (c >> 31) ? -v : v; }

// ---------------------------------------------------------------------------
// Device-wide barrier for cooperative (co-resident) launches.
//
// Monotonic counter: barrier number b completes when the counter reaches
// b * nblocks.  Every wave issues an agent-scope release fence before the
// block barrier (the block barrier alone does not wait for other waves'
// stores to leave the CU, and L2s of different XCDs are not coherent), so
// that everything the block wrote is visible device-wide before thread 0
// arrives.  Waiting is bounded: after `timeout_ticks` of the 100 MHz
// real-time counter, or when another block has raised the abort flag, the
// wait fails and the caller must leave the kernel.
// ---------------------------------------------------------------------------
struct GridSync {
  uint32_t *counter;
  int32_t *abort_flag;
  uint32_t nblocks;
  uint64_t timeout_ticks;
};

__device__ inline void grid_arrive(const GridSync &gs) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(gs.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true when barrier `number` (1-based) completed for every block.
__device__ inline bool grid_wait(const GridSync &gs, uint32_t number, int *lds_flag) {
  if (threadIdx.x == 0) {
    const uint32_t target = number * gs.nblocks;
    int ok = 1;
    uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(gs.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(gs.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
      if (__builtin_amdgcn_s_memrealtime() - t0 > gs.timeout_ticks) {
        __hip_atomic_store(gs.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_flag = ok;
  }
  __syncthreads();
  return *lds_flag != 0;
}

// ---------------------------------------------------------------------------
// Pivot candidates: larger magnitude wins, ties go to the smaller position.
// ---------------------------------------------------------------------------
struct Cand {
  double v;     // |value|; -1 for a non-finite value, -2 for "no candidate"
  int32_t pos;  // current position of the row
  int32_t idx;  // row index (original numbering) or slot number
};

__device__ inline bool cand_better(double v1, int p1, double v2, int p2) {
  return (v1 > v2) || (v1 == v2 && p1 < p2);
}

__device__ inline Cand wave_argmax(Cand c) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double v = __shfl_xor(c.v, off, 64);
    int p = __shfl_xor(c.pos, off, 64);
    int i = __shfl_xor(c.idx, off, 64);
    if (cand_better(v, p, c.v, c.pos)) { c.v = v; c.pos = p; c.idx = i; }
  }
  return c;
}

}  // namespace rlu
