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
constexpr int kStreamSem2 = 4;     // the same three draws of Omega_2 (Algorithm 1 step 4)
constexpr int kStreamSigns2 = 5;
constexpr int kStreamSelect2 = 6;

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
// Tagged words: 32 bits of data and a 32-bit tag in one 64-bit word, written
// and read with agent-scope atomic stores / loads.  A reader that sees the
// expected tag also sees the data that came with it, so blocks exchange
// values without read-modify-write atomics and without cache-wide fences
// (a counter that every block increments serialises at the memory side;
// one word per block, polled by all, does not).  Buffers are zeroed before
// each launch and tags start at 1.
// ---------------------------------------------------------------------------
__device__ inline void tw_put(uint64_t *w, uint32_t data, uint32_t tag) {
  __hip_atomic_store(w, (uint64_t)data | ((uint64_t)tag << 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t tw_get(const uint64_t *w) {
  return __hip_atomic_load(const_cast<uint64_t *>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t tw_tag(uint64_t v) { return (uint32_t)(v >> 32); }
__device__ inline uint32_t tw_data(uint64_t v) { return (uint32_t)v; }
__device__ inline void tw_put_f64(uint64_t *w, double x, uint32_t tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  tw_put(w, (uint32_t)b, tag);
  tw_put(w + 1, (uint32_t)(b >> 32), tag);
}
__device__ inline double tw_f64(uint64_t lo, uint64_t hi) {
  return __longlong_as_double((long long)(((uint64_t)tw_data(hi) << 32) | tw_data(lo)));
}

// Bounded poll helper: true while the deadline has not passed and no block
// raised the abort flag; raises the flag on time-out.
__device__ inline bool poll_ok(uint64_t t0, uint64_t timeout_ticks, int32_t *abort_flag) {
  if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
  if (__builtin_amdgcn_s_memrealtime() - t0 > timeout_ticks) {
    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  return true;
}

// Flag barrier over the blocks of a cooperative launch: every block stores
// its own tag (128 bytes apart), every block polls all of them.  Data
// written before the barrier with plain stores is published by the
// agent-scope release fence of every wave and picked up by the acquire
// fence after the wait.
struct FlagBar {
  uint64_t *flags;     // nblocks x 16 words, zeroed before the launch
  int32_t *abort_flag;
  int nblocks;
  uint64_t timeout_ticks;
};

__device__ inline void fbar_arrive(const FlagBar &fb, uint32_t tag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) tw_put(fb.flags + (size_t)blockIdx.x * 16, 0u, tag);
}

__device__ inline bool fbar_wait(const FlagBar &fb, uint32_t tag, int *lds_flag) {
  if (threadIdx.x < 64) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    int ok = 1;
    for (;;) {
      int all = 1;
      for (int g = threadIdx.x; g < fb.nblocks; g += 64) all &= (tw_tag(tw_get(fb.flags + (size_t)g * 16)) >= tag);
      if (__all(all)) break;
      if (!poll_ok(t0, fb.timeout_ticks, fb.abort_flag)) { ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *lds_flag = ok;
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
  // bitwise, so that it compiles to straight-line compares and mask logic
  return (v1 > v2) | ((v1 == v2) & (p1 < p2));
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
