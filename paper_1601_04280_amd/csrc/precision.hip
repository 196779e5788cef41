// Reduced-precision forms of the least-squares contraction.
//
// Corollary 3.2's product B = L_y^+ P A is formed as G^{-1} Lhat^T A with
// Lhat = P^T L_y and G = Lhat^T Lhat; its one large term is the contraction
// W^T = A^T Lhat (n x l, K = m).  These forms change only that term: the
// pivot searches, G, its Cholesky factor and inverse, and the l x l products
// stay in FP64.
//
// BF16 with one refinement step (in the transposed orientation the library
// keeps B in):
//   W0^T = bf16(A)^T bf16(Lhat)        BF16 MFMA, FP32 accumulation
//   X0^T = W0^T G^{-1}                 FP64
//   R    = A - Lhat X0                 Lhat X0 from the three leading products
//                                      of the hi/lo BF16 splits (hi.hi + hi.lo
//                                      + lo.hi, each split exact to ~2^-17),
//                                      FP32 accumulation, A - (.) in A's type,
//                                      stored rounded to BF16
//   dW^T = bf16(R)^T bf16(Lhat)        BF16 MFMA
//   B^T  = X0^T + dW^T G^{-1}          FP64
// After the step the error of B is about 2^-8 ||R|| (the BF16 rounding of R
// and of the correction's operands) instead of 2^-8 ||A||; R is only as
// large as the part of A outside Im(Lhat) plus the first pass's error, so
// the step recovers most of the lost accuracy when A is close to rank l.
// R must be formed to about 2^-16 of ||A|| for this to hold, hence the split
// products rather than a plain BF16 product.
//
// FP32: W^T = A^T fp32(Lhat) in one pass on FP32 MFMA (the GEMM of
// gemm_f64.hip with FP32 compute), then B^T = W^T G^{-1} in FP64.
//
// BF16 MFMA operand layouts (v_mfma_f32_16x16x32_bf16): lane l supplies
// A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. 8(l/16)+7][l%16]; element v
// of the result in lane l is D[4(l/16) + v][l%16].
#include <type_traits>

#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// 16 bytes as a native vector (HIP's u32x4 is a struct, which selects and
// arrays of keep in scratch memory)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Round to nearest even, two values packed low-first.  (__bf16) of a float is
// gfx950's v_cvt_pk_bf16_f32; of a double, a single correctly rounded step.
__device__ inline uint32_t pack_bf16(float a, float b) {
  bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ inline uint32_t pack_bf16(double a, double b) {
  bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ inline uint32_t pack_bf16(uint16_t a, uint16_t b) { return (uint32_t)a | ((uint32_t)b << 16); }

__device__ inline uint16_t bf16_of(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline uint16_t bf16_of(double x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline double double_of_bf16(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

// Consecutive hardware block ids are dealt to the eight XCDs in turn.  Give
// each XCD a contiguous range of logical tiles, so that blocks sharing an
// operand tile read it through the same L2.
__device__ inline int64_t xcd_tile(int64_t per_xcd) {
  return (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}
static unsigned xcd_grid(int64_t tiles, int64_t *per_xcd) {
  *per_xcd = ceil_div(tiles, 8);
  return (unsigned)(8 * *per_xcd);
}

// ---------------------------------------------------------------------------
// hi = bf16(x), lo = bf16(x - hi) (lo optional) of an FP64 matrix, written
// rows x ldo with zeros in the padding columns.
// ---------------------------------------------------------------------------
__global__ void k_split_bf16(int64_t rows, int cols, const double *__restrict__ x, int64_t ldx,
                             uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int ldo) {
  const int64_t total = rows * ldo;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ldo;
    const int c = (int)(e - r * ldo);
    uint16_t h = 0, q = 0;
    if (c < cols) {
      const double v = x[r * ldx + c];
      h = bf16_of(v);
      q = bf16_of(v - double_of_bf16(h));
    }
    hi[e] = h;
    if (lo) lo[e] = q;
  }
}

// out (cols_p x rows_p, ld rows_p) = in^T for in (rows x cols, ld ldi, BF16),
// zero outside; 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_bf16(int64_t rows, int cols, const uint16_t *__restrict__ in,
                                                        int64_t ldi, uint16_t *__restrict__ out, int64_t rows_p) {
  __shared__ uint16_t t[64][66];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i;
    const int c = c0 + tx;
    t[i][tx] = (r < rows && c < cols) ? in[r * ldi + c] : (uint16_t)0;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) out[(int64_t)(c0 + i) * rows_p + r0 + tx] = t[tx][i];
}

__global__ void k_to_f32(int64_t rows, int cols, const double *__restrict__ x, int64_t ldx, float *__restrict__ y,
                         int ldo) {
  const int64_t total = rows * ldo;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ldo;
    const int c = (int)(e - r * ldo);
    y[e] = c < cols ? (float)x[r * ldx + c] : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// C (M x N) = X^T Lb over K, Lb given transposed: LbT (N_p x K_p BF16,
// K-contiguous, zero padded to a multiple of 128 rows and 64 columns).
//   XT = false: X is K x M row major (ldx) in FP32 or FP64, read coalesced
//     along its rows and transposed into LDS while being rounded to BF16.
//   XT = true:  X is given transposed, XT (M x K_p BF16, K-contiguous, zero
//     padded), read in 16-byte chunks like LbT.
// LDS tiles hold [col][k] rows of 8 consecutive k per 16-byte word (the
// MFMA operand shape).  Block tile (32 WM) x (32 WN) over four waves in a
// 2 x 2 grid; K advances 64 at a time through a double-buffered LDS tile,
// the next stage's loads in flight during the current stage's MFMAs.  Loads
// are unconditional from in-bounds addresses; out-of-range values are zeroed
// when the stage is written to LDS.  With splits > 1, FP32 partial sums per
// K range (multiples of 64) go to `parts` and are summed in FP64 in a fixed
// order afterwards.
// ---------------------------------------------------------------------------
struct Bf16Tn {
  int64_t M, N, K;
  const void *X;
  int64_t ldx;
  const uint16_t *LbT;
  int64_t ldl;
  double *C;
  int64_t ldc;
  float *parts;
  int64_t Kc;
  int ntm, ntn;
  int64_t tiles, per_xcd;
};

template <typename TX, bool XT, int WM, int WN>
__global__ __launch_bounds__(256) void k_bf16_tn(Bf16Tn p) {
  constexpr int BM = 32 * WM, BN = 32 * WN, BK = 64, LS = BK + 8;  // 144-byte rows: conflict-free 16-byte reads
  constexpr int CX = BM / 32;  // transposing loader: columns per thread
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][BM * LS];
  __shared__ __attribute__((aligned(16))) uint16_t Ls[2][BN * LS];
  const int64_t t = xcd_tile(p.per_xcd);
  if (t >= p.tiles) return;
  const int tn = (int)(t % p.ntn);
  const int64_t rest = t / p.ntn;
  const int tm = (int)(rest % p.ntm);
  const int z = (int)(rest / p.ntm);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t kb = (int64_t)z * p.Kc, ke = min(p.K, kb + p.Kc);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int cg = tid & 31, kg = tid >> 5;  // transposing loader: columns cg + 32 c, k rows 8 kg .. 8 kg + 7

  TX rx[XT ? 1 : CX][8];
  u32x4 rxq[XT ? WM : 1];
  u32x4 rlq[WN];
  auto load = [&](int64_t k0) {
    if constexpr (XT) {
      const uint16_t *Xb = reinterpret_cast<const uint16_t *>(p.X);
#pragma unroll
      for (int q = 0; q < WM; ++q) {
        const int e = tid + 256 * q, r = e >> 3, kc = e & 7;
        const int64_t row = m0 + r < p.M ? m0 + r : m0;
        rxq[q] = *reinterpret_cast<const u32x4 *>(Xb + row * p.ldx + k0 + kc * 8);
      }
    } else {
      const TX *X = reinterpret_cast<const TX *>(p.X);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + kg * 8 + e;
#pragma unroll
        for (int c = 0; c < CX; ++c) {
          const int64_t col = m0 + cg + 32 * c;
          const bool ok = k < ke && col < p.M;
          rx[c][e] = X[(ok ? k : kb) * p.ldx + (ok ? col : m0)];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < WN; ++q) {
      const int e = tid + 256 * q, r = e >> 3, kc = e & 7;
      rlq[q] = *reinterpret_cast<const u32x4 *>(p.LbT + (n0 + r) * p.ldl + k0 + kc * 8);
    }
  };
  auto store = [&](int buf, int64_t k0) {
    if constexpr (XT) {
#pragma unroll
      for (int q = 0; q < WM; ++q) {
        const int e = tid + 256 * q, r = e >> 3, kc = e & 7;
        const u32x4 zero = {0u, 0u, 0u, 0u};
        *reinterpret_cast<u32x4 *>(&Xs[buf][r * LS + kc * 8]) = m0 + r < p.M ? rxq[q] : zero;
      }
    } else {
#pragma unroll
      for (int c = 0; c < CX; ++c) {
        const bool cok = m0 + cg + 32 * c < p.M;
        TX v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (cok && k0 + kg * 8 + e < ke) ? rx[c][e] : (TX)0;
        u32x4 w;
        w.x = pack_bf16(v[0], v[1]);
        w.y = pack_bf16(v[2], v[3]);
        w.z = pack_bf16(v[4], v[5]);
        w.w = pack_bf16(v[6], v[7]);
        *reinterpret_cast<u32x4 *>(&Xs[buf][(cg + 32 * c) * LS + kg * 8]) = w;
      }
    }
#pragma unroll
    for (int q = 0; q < WN; ++q) {
      const int e = tid + 256 * q, r = e >> 3, kc = e & 7;
      *reinterpret_cast<u32x4 *>(&Ls[buf][r * LS + kc * 8]) = rlq[q];
    }
  };

  f32x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0, kb);
    __syncthreads();
  }
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    const bool more = k0 + BK < ke;
    if (more) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ko = ks * 32 + 8 * (lane >> 4);
      bf16x8 a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i)
        a[i] = *reinterpret_cast<const bf16x8 *>(&Xs[buf][(wm * 16 * WM + i * 16 + (lane & 15)) * LS + ko]);
#pragma unroll
      for (int j = 0; j < WN; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(&Ls[buf][(wn * 16 * WN + j * 16 + (lane & 15)) * LS + ko]);
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store(buf ^ 1, k0 + BK);
      __syncthreads();
      buf ^= 1;
    }
  }

#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 16 * WM + i * 16 + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn * 16 * WN + j * 16 + (lane & 15);
        if (row < p.M && col < p.N) {
          if (p.parts) p.parts[(int64_t)z * p.M * p.N + row * p.N + col] = acc[i][j][v];
          else p.C[row * p.ldc + col] = (double)acc[i][j][v];
        }
      }
}

// ---------------------------------------------------------------------------
// Wide form of the same product for 128 < N <= 576 (N = l): one block spans
// all N columns, so X (A, or R^T) is read from memory once instead of once
// per 128-column tile; only Lb^T, the small operand, is read again by every
// row tile.  K is split into `splits` ranges laid out so that each XCD works
// on one range, whose slice of Lb^T then stays in that XCD's L2.  Eight waves
// in a 2 x 4 grid, wave tile 64 x (16 WN), block tile 128 x (64 WN); K
// advances 32 per stage (v_mfma_f32_16x16x32_bf16).  FP32 partial sums per
// K range go to `parts` (summed in FP64 afterwards, in a fixed order) or,
// with one range, straight to C.
//
// Loads run two stages ahead.  Every 16-byte K-contiguous
// operand (Lb^T, and X^T when given transposed) goes from global memory
// straight to LDS (global_load_lds_dwordx4: lane i's 16 bytes land at the
// wavefront's LDS base + 16 i) into a ring of three stages, issued two
// stages ahead, so two stages of loads are in flight while a third is
// multiplied; FP32 / FP64 X goes through registers, two stages ahead in two
// register sets, and is rounded and transposed into a double-buffered LDS
// tile.  The ring rows are 64 bytes (32 k) with the four 16-byte chunks of
// row r permuted by chunk ^ ((r >> 1) & 3), so that the fragment reads of
// 16 consecutive rows spread over the banks.
// ---------------------------------------------------------------------------
__device__ inline int ring_sw(int r) { return (r >> 1) & 3; }

__device__ inline void lds_direct16(const void *g, uint16_t *lds) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

template <typename TX, bool XT, int WN>
__global__ __launch_bounds__(512) void k_bf16_tn_pipe(Bf16Tn p) {
  constexpr int BM = 128, BN = 64 * WN, BK = 32, LS = BK + 8;
  constexpr int NPL = 128 * ((WN + 1) / 2);  // rows of Lb^T per stage (Lb^T is padded to 128 rows)
  constexpr int LIW = NPL / 16 / 8;          // its direct loads per wavefront per stage
  // The ring's three stages are three LDS arrays, addressed statically (the
  // stage loop is unrolled by six), so that the compiler can tell a fragment
  // read of one stage from the loads in flight into another and does not
  // wait for those.
  __shared__ __attribute__((aligned(16))) uint16_t Ls0[NPL * 32], Ls1[NPL * 32], Ls2[NPL * 32];
  __shared__ __attribute__((aligned(16))) uint16_t Xr0[XT ? BM * 32 : 8], Xr1[XT ? BM * 32 : 8], Xr2[XT ? BM * 32 : 8];
  __shared__ __attribute__((aligned(16))) uint16_t Xd0[XT ? 8 : BM * LS], Xd1[XT ? 8 : BM * LS];
  const int64_t t = xcd_tile(p.per_xcd);
  if (t >= p.tiles) return;
  const int tm = (int)(t % p.ntm);
  const int z = (int)(t / p.ntm);  // K range: consecutive tiles (one XCD) share it
  const int64_t m0 = (int64_t)tm * BM;
  const int64_t kb = (int64_t)z * p.Kc, ke = min(p.K, kb + p.Kc);
  const int nst = (int)ceil_div(ke - kb, BK);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int xc = tid & 127, xk = tid >> 7;  // FP32 / FP64 loader: column xc, k rows 8 xk .. 8 xk + 7
  const int q = lane >> 4;

  auto lring = [&](auto c) -> uint16_t * {
    constexpr int C = decltype(c)::value;
    if constexpr (C == 0) return Ls0;
    else if constexpr (C == 1) return Ls1;
    else return Ls2;
  };
  auto xring = [&](auto c) -> uint16_t * {
    constexpr int C = decltype(c)::value;
    if constexpr (C == 0) return Xr0;
    else if constexpr (C == 1) return Xr1;
    else return Xr2;
  };
  auto xdbl = [&](auto c) -> uint16_t * {
    if constexpr (decltype(c)::value == 0) return Xd0;
    else return Xd1;
  };

  auto issue = [&](auto slot, int s) {  // direct loads of stage s into ring slot `slot`
    const int64_t k0 = kb + (int64_t)s * BK;
    uint16_t *ls = lring(slot);
#pragma unroll
    for (int i = 0; i < LIW; ++i) {
      const int r0 = (wave * LIW + i) * 16;
      const int r = r0 + (lane >> 2), kc = (lane & 3) ^ ring_sw(r);
      lds_direct16(p.LbT + (int64_t)r * p.ldl + k0 + kc * 8, ls + r0 * 32);
    }
    if constexpr (XT) {
      const uint16_t *Xb = reinterpret_cast<const uint16_t *>(p.X);
      const int r0 = wave * 16;
      const int r = r0 + (lane >> 2), kc = (lane & 3) ^ ring_sw(r);
      const int64_t row = m0 + r < p.M ? m0 + r : m0;  // rows past M: a copy of row m0, never stored
      lds_direct16(Xb + row * p.ldx + k0 + kc * 8, xring(slot) + r0 * 32);
    }
  };
  auto load_x = [&](TX (&rx)[8], int s) {  // FP32 / FP64 X of stage s into registers
    const TX *X = reinterpret_cast<const TX *>(p.X);
    const int64_t k0 = kb + (int64_t)s * BK, col = m0 + xc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = k0 + xk * 8 + e;
      const bool ok = k < ke && col < p.M;
      rx[e] = X[(ok ? k : kb) * p.ldx + (ok ? col : m0)];
    }
  };
  auto store_x = [&](const TX (&rx)[8], auto par, int s) {  // ... rounded and transposed into an Xd tile
    const int64_t k0 = kb + (int64_t)s * BK;
    const bool cok = m0 + xc < p.M;
    TX v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (cok && k0 + xk * 8 + e < ke) ? rx[e] : (TX)0;
    u32x4 w;
    w.x = pack_bf16(v[0], v[1]);
    w.y = pack_bf16(v[2], v[3]);
    w.z = pack_bf16(v[4], v[5]);
    w.w = pack_bf16(v[6], v[7]);
    *reinterpret_cast<u32x4 *>(xdbl(par) + xc * LS + xk * 8) = w;
  };

  f32x4 acc[4][WN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto read_stage = [&](auto slot, auto par, bf16x8 (&a)[4], bf16x8 (&b)[WN]) {  // this wavefront's fragments
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + (lane & 15);
      if constexpr (XT) a[i] = *reinterpret_cast<const bf16x8 *>(xring(slot) + r * 32 + ((q ^ ring_sw(r)) * 8));
      else a[i] = *reinterpret_cast<const bf16x8 *>(xdbl(par) + r * LS + q * 8);
    }
    const uint16_t *ls = lring(slot);
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int r = wn * 16 * WN + j * 16 + (lane & 15);
      b[j] = *reinterpret_cast<const bf16x8 *>(ls + r * 32 + ((q ^ ring_sw(r)) * 8));
    }
  };
  auto mfma_stage = [&](const bf16x8 (&a)[4], const bf16x8 (&b)[WN]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };

  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  TX rx[8];
  if (nst > 0) {
    if constexpr (!XT) load_x(rx, 0);
    issue(I0{}, 0);
    if (nst > 1) issue(I1{}, 1);
    if constexpr (!XT) store_x(rx, I0{}, 0);
    if (nst > 1) asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(LIW + (XT ? 1 : 0)) : "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
  }
  // Stage s (ring slot s % 3, X parity s % 2): the loads of stage s + 1's X
  // (registers) and stage s + 2's ring copies, this wavefront's fragments of
  // stage s (with X^T in the ring: first, so that a wait the compiler places
  // before these reads, for copies into this slot, cannot cover the copies
  // issued next), the MFMAs of stage s, and stage s + 1 made ready: its X
  // rounded into LDS, its copies waited for (stage s + 2's left in flight),
  // a bare barrier (__syncthreads' workgroup fence would also wait for stage
  // s + 2's copies).
  auto step = [&](auto slot, auto par, int s) {
    using Ahead = std::integral_constant<int, (decltype(slot)::value + 2) % 3>;
    using NPar = std::integral_constant<int, 1 - decltype(par)::value>;
    const bool next = s + 1 < nst, ahead = s + 2 < nst;
    bf16x8 fa[4], fb[WN];
    if constexpr (XT) {
      read_stage(slot, par, fa, fb);
      if (ahead) issue(Ahead{}, s + 2);
    } else {
      // X's loads before the copies (the wait below then leaves only the
      // copies in flight), and the fragments after them: read first they
      // would stay live across the loads' address arithmetic, beyond the
      // register budget of the widest tile
      if (next) load_x(rx, s + 1);
      if (ahead) issue(Ahead{}, s + 2);
      read_stage(slot, par, fa, fb);
    }
    mfma_stage(fa, fb);
    if (next) {
      if constexpr (!XT) store_x(rx, NPar{}, s + 1);
      if (ahead) asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(LIW + (XT ? 1 : 0)) : "memory");
      else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
      __builtin_amdgcn_s_barrier();
    }
  };
  for (int s = 0; s < nst; s += 6) {
    step(I0{}, I0{}, s);
    if (s + 1 < nst) step(I1{}, I1{}, s + 1);
    if (s + 2 < nst) step(I2{}, I0{}, s + 2);
    if (s + 3 < nst) step(I0{}, I1{}, s + 3);
    if (s + 4 < nst) step(I1{}, I0{}, s + 4);
    if (s + 5 < nst) step(I2{}, I1{}, s + 5);
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t col = wn * 16 * WN + j * 16 + (lane & 15);
        if (row < p.M && col < p.N) {
          if (p.parts) p.parts[(int64_t)z * p.M * p.N + row * p.N + col] = acc[i][j][v];
          else p.C[row * p.ldc + col] = (double)acc[i][j][v];
        }
      }
}

__global__ void k_sum_parts(int64_t M, int64_t N, int splits, const float *__restrict__ parts, double *__restrict__ C,
                            int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += (double)parts[(int64_t)z * total + e];
    const int64_t r = e / N;
    C[r * ldc + (e - r * N)] = s;
  }
}

// ---------------------------------------------------------------------------
// R^T (N x M_p BF16, ld ldr) with R = A - (Lh Xh^T + Lh Xl^T + Ll Xh^T) for
// A (M x N), Lh, Ll (M x K) and Xh, Xl (N x K) BF16, K-contiguous with row
// stride K (a multiple of 32, zero padded); columns M .. M_p - 1 of R^T are
// written as zeros.  Each product term is exact in FP32; the sum is
// accumulated in FP32 and subtracted from A in A's storage type.  Block tile
// (32 WM) x (32 WN), K advancing 32 at a time through a double-buffered LDS
// tile.
// ---------------------------------------------------------------------------
constexpr int kResidSub = 8;  // column tiles of one sub-band (their X operands: 2.2 MB at K = 544)

struct Bf16Resid {
  int64_t M, N, Mp;
  int K;
  const void *A;
  int64_t lda;
  const uint16_t *Lh, *Ll, *Xh, *Xl;
  uint16_t *RT;
  int64_t ldr;
  int ntn;
  int64_t ntm;
  int64_t tiles, per_xcd;
};

template <typename TA, int WM, int WN>
__global__ __launch_bounds__(256) void k_bf16_resid(Bf16Resid p) {
  constexpr int BM = 32 * WM, BN = 32 * WN, BK = 32, LS = BK + 8;  // 80-byte rows
  constexpr int QM = BM / 64, QN = BN / 64;                      // 16-byte chunks per thread per operand
  static_assert(QM >= 1 && QN >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) uint16_t Lhs[2][BM * LS], Lls[2][BM * LS], Xhs[2][BN * LS],
      Xls[2][BN * LS];
  // Column tiles by XCD: XCD x owns a band of nb = ceil(ntn / 8) column
  // tiles and walks every row tile over sub-bands of kResidSub of them, so
  // the X operands of a sub-band stay in that XCD's L2 while the row tiles'
  // L operands stream through it (hardware block ids go to the XCDs in turn).
  const int xcd = (int)(blockIdx.x & 7);
  const int64_t j = blockIdx.x >> 3;
  const int nb = (int)ceil_div(p.ntn, 8);
  const int64_t per_sub = p.ntm * kResidSub;
  const int sub = (int)(j / per_sub);
  const int64_t rem = j - (int64_t)sub * per_sub;
  const int64_t tm = rem / kResidSub;
  const int tl = sub * kResidSub + (int)(rem % kResidSub);  // column tile within the band
  const int tn = xcd * nb + tl;
  if (tl >= nb || tn >= p.ntn || tm >= p.ntm) return;
  const int64_t m0 = tm * BM, n0 = (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  u32x4 rlh[QM], rll[QM], rxh[QN], rxl[QN];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int e = tid + 256 * q, r = e >> 2, kc = e & 3;
      const int64_t gr = m0 + r < p.M ? m0 + r : m0;
      rlh[q] = *reinterpret_cast<const u32x4 *>(p.Lh + gr * p.K + k0 + kc * 8);
      rll[q] = *reinterpret_cast<const u32x4 *>(p.Ll + gr * p.K + k0 + kc * 8);
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int e = tid + 256 * q, r = e >> 2, kc = e & 3;
      const int64_t gr = n0 + r < p.N ? n0 + r : n0;
      rxh[q] = *reinterpret_cast<const u32x4 *>(p.Xh + gr * p.K + k0 + kc * 8);
      rxl[q] = *reinterpret_cast<const u32x4 *>(p.Xl + gr * p.K + k0 + kc * 8);
    }
  };
  auto store = [&](int buf) {
    const u32x4 zero = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int e = tid + 256 * q, r = e >> 2, kc = e & 3;
      const bool ok = m0 + r < p.M;
      *reinterpret_cast<u32x4 *>(&Lhs[buf][r * LS + kc * 8]) = ok ? rlh[q] : zero;
      *reinterpret_cast<u32x4 *>(&Lls[buf][r * LS + kc * 8]) = ok ? rll[q] : zero;
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int e = tid + 256 * q, r = e >> 2, kc = e & 3;
      const bool ok = n0 + r < p.N;
      *reinterpret_cast<u32x4 *>(&Xhs[buf][r * LS + kc * 8]) = ok ? rxh[q] : zero;
      *reinterpret_cast<u32x4 *>(&Xls[buf][r * LS + kc * 8]) = ok ? rxl[q] : zero;
    }
  };

  f32x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  int buf = 0;
  load(0);
  store(0);
  __syncthreads();
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    const bool more = k0 + BK < p.K;
    if (more) load(k0 + BK);
    const int ko = 8 * (lane >> 4);
    bf16x8 ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const int r = (wm * 16 * WM + i * 16 + (lane & 15)) * LS + ko;
      ah[i] = *reinterpret_cast<const bf16x8 *>(&Lhs[buf][r]);
      al[i] = *reinterpret_cast<const bf16x8 *>(&Lls[buf][r]);
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int r = (wn * 16 * WN + j * 16 + (lane & 15)) * LS + ko;
      bh[j] = *reinterpret_cast<const bf16x8 *>(&Xhs[buf][r]);
      bl[j] = *reinterpret_cast<const bf16x8 *>(&Xls[buf][r]);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (more) {
      store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // A values first (clamped, unconditional), then R^T: lane holds rows
  // i .. i+3 of column j, i.e. four consecutive entries of row j of R^T.
  const TA *A = reinterpret_cast<const TA *>(p.A);
  TA av[WM][WN][4];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 16 * WM + i * 16 + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn * 16 * WN + j * 16 + (lane & 15);
        const bool ok = row < p.M && col < p.N;
        av[i][j][v] = __builtin_nontemporal_load(A + (ok ? row : m0) * p.lda + (ok ? col : n0));  // read once
      }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int64_t row = m0 + wm * 16 * WM + i * 16 + 4 * (lane >> 4);
      const int64_t col = n0 + wn * 16 * WN + j * 16 + (lane & 15);
      if (col < p.N && row < p.Mp) {
        uint16_t h[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) h[v] = row + v < p.M ? bf16_of((TA)(av[i][j][v] - (TA)acc[i][j][v])) : (uint16_t)0;
        u32x2 w;
        w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        *reinterpret_cast<u32x2 *>(p.RT + col * p.ldr + row) = w;
      }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename T>
static T *at(void *base, size_t off) { return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off); }

constexpr int kRowPad = 128;  // rows of LbT padded to the widest N tile
constexpr int kKPad = 64;     // K padding of the K-contiguous operands

constexpr int kWideMaxN = 576;  // the wide product's widest block (WN = 9)
constexpr int kWideSplits = 8;  // one K range per XCD

static void bf16_tn_shape(int64_t M, int64_t N, int64_t K, int num_cu, int *wm, int *wn, int *splits, int64_t *Kc) {
  if (N > 128 && N <= kWideMaxN) {  // the wide form: wn = WN (block tile 64 WN columns), wm = 0 marks it
    *wm = 0;
    *wn = (int)ceil_div(N, 64);
    int64_t s = std::max<int64_t>(1, std::min<int64_t>(kWideSplits, K / 1024));
    int64_t kc = ceil_div(std::max<int64_t>(K, 1), s);
    kc = ceil_div(kc, kKPad) * kKPad;
    *Kc = kc;
    *splits = (int)ceil_div(std::max<int64_t>(K, 1), kc);
    return;
  }
  *wm = M > 64 ? 4 : 2;
  *wn = N > 64 ? 4 : 2;
  const int64_t tiles = ceil_div(M, 32 * *wm) * ceil_div(N, 32 * *wn);
  int64_t s = ceil_div(2 * (int64_t)num_cu, tiles);
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / 512));
  s = std::max<int64_t>(1, std::min<int64_t>(s, 64));
  int64_t kc = ceil_div(std::max<int64_t>(K, 1), s);
  kc = ceil_div(kc, kKPad) * kKPad;
  *Kc = kc;
  *splits = (int)ceil_div(std::max<int64_t>(K, 1), kc);
}

bool plan_precision(int64_t m, int64_t n, int l, int precision, int num_cu, PrecPlan *pp) {
  *pp = PrecPlan{};
  pp->precision = precision;
  pp->lp = (int)ceil_div(l, 32) * 32;
  pp->mp = ceil_div(m, kKPad) * kKPad;
  pp->np_rows = ceil_div(l, kRowPad) * kRowPad;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  if (precision == RLU_PREC_F32) {
    pp->lf = take((size_t)m * l * 4);
  } else if (precision == RLU_PREC_BF16_REFINED) {
    bf16_tn_shape(n, l, m, num_cu, &pp->wm, &pp->wn, &pp->splits, &pp->Kc);
    pp->lhi = take((size_t)m * pp->lp * 2);
    pp->llo = take((size_t)m * pp->lp * 2);
    pp->lht = take((size_t)pp->np_rows * pp->mp * 2);
    pp->xhi = take((size_t)n * pp->lp * 2);
    pp->xlo = take((size_t)n * pp->lp * 2);
    pp->r = take((size_t)n * pp->mp * 2);
    pp->parts = take(pp->splits > 1 ? (size_t)pp->splits * n * l * 4 : 0);
  } else {
    return false;
  }
  pp->total = off;
  return true;
}

static unsigned ew_blocks(int64_t total) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, ceil_div(total, 256))); }

template <typename TX, bool XT>
static hipError_t launch_tn_wide(const Bf16Tn &k, int wn, unsigned grid, hipStream_t st) {
  if (k.ntn < 128 * ((wn + 1) / 2)) return hipErrorInvalidValue;  // rows of Lb^T the ring loads
  switch (wn) {
#define RLU_WIDE(W)                                                                          \
  case W:                                                                                    \
    hipLaunchKernelGGL((k_bf16_tn_pipe<TX, XT, W>), dim3(grid), dim3(512), 0, st, k);         \
    break;
    RLU_WIDE(3) RLU_WIDE(4) RLU_WIDE(5) RLU_WIDE(6) RLU_WIDE(7) RLU_WIDE(8) RLU_WIDE(9)
#undef RLU_WIDE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TX, bool XT>
static hipError_t launch_tn_t(const Bf16Tn &k, int wm, int wn, unsigned grid, hipStream_t st) {
  if (wm == 4 && wn == 4) hipLaunchKernelGGL((k_bf16_tn<TX, XT, 4, 4>), dim3(grid), dim3(256), 0, st, k);
  else if (wm == 4 && wn == 2) hipLaunchKernelGGL((k_bf16_tn<TX, XT, 4, 2>), dim3(grid), dim3(256), 0, st, k);
  else if (wm == 2 && wn == 4) hipLaunchKernelGGL((k_bf16_tn<TX, XT, 2, 4>), dim3(grid), dim3(256), 0, st, k);
  else if (wm == 2 && wn == 2) hipLaunchKernelGGL((k_bf16_tn<TX, XT, 2, 2>), dim3(grid), dim3(256), 0, st, k);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// C (M x N, FP64) = X^T Lb over K (LbT: N_p x K_p, ld ldl).  X: K x M (ldx) in
// FP32 / FP64 (xt = false) or X^T: M x K_p BF16 (ldx) (xt = true).  parts must
// hold splits x M x N floats when splits > 1.
static hipError_t bf16_tn(int64_t M, int64_t N, int64_t K, const void *X, int x_dtype, bool xt, int64_t ldx,
                          const uint16_t *LbT, int64_t ldl, int64_t lb_rows, double *C, int64_t ldc, int wm, int wn,
                          int splits, int64_t Kc, float *parts, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (wm == 0) {  // wide form: one block spans all N columns, K ranges by XCD
    Bf16Tn k{};
    k.M = M; k.N = N; k.K = K;
    k.X = X; k.ldx = ldx; k.LbT = LbT; k.ldl = ldl;
    k.C = C; k.ldc = ldc;
    k.parts = splits > 1 ? parts : nullptr;
    k.Kc = splits > 1 ? Kc : ceil_div(std::max<int64_t>(K, 1), kKPad) * kKPad;
    k.ntm = (int)ceil_div(M, 128);
    k.ntn = (int)lb_rows;  // rows of Lb^T that may be read
    const int used = splits > 1 ? (int)ceil_div(K, Kc) : 1;
    k.tiles = (int64_t)k.ntm * used;
    const unsigned grid = xcd_grid(k.tiles, &k.per_xcd);
    hipError_t e;
    if (xt) e = launch_tn_wide<uint16_t, true>(k, wn, grid, st);
    else if (x_dtype == RLU_F32) e = launch_tn_wide<float, false>(k, wn, grid, st);
    else if (x_dtype == RLU_F64) e = launch_tn_wide<double, false>(k, wn, grid, st);
    else return hipErrorInvalidValue;
    if (e != hipSuccess || used <= 1) return e;
    hipLaunchKernelGGL(k_sum_parts, dim3(ew_blocks(M * N)), dim3(256), 0, st, M, N, used, (const float *)parts, C,
                       ldc);
    return hipGetLastError();
  }
  Bf16Tn k{};
  k.M = M; k.N = N; k.K = K;
  k.X = X; k.ldx = ldx; k.LbT = LbT; k.ldl = ldl;
  k.C = C; k.ldc = ldc;
  k.parts = splits > 1 ? parts : nullptr;
  k.Kc = splits > 1 ? Kc : ceil_div(std::max<int64_t>(K, 1), kKPad) * kKPad;
  k.ntm = (int)ceil_div(M, 32 * wm);
  k.ntn = (int)ceil_div(N, 32 * wn);
  const int used = splits > 1 ? (int)ceil_div(K, Kc) : 1;
  k.tiles = (int64_t)k.ntm * k.ntn * used;
  const unsigned grid = xcd_grid(k.tiles, &k.per_xcd);
  hipError_t e;
  if (xt) e = launch_tn_t<uint16_t, true>(k, wm, wn, grid, st);
  else if (x_dtype == RLU_F32) e = launch_tn_t<float, false>(k, wm, wn, grid, st);
  else if (x_dtype == RLU_F64) e = launch_tn_t<double, false>(k, wm, wn, grid, st);
  else return hipErrorInvalidValue;
  if (e != hipSuccess || used <= 1) return e;
  hipLaunchKernelGGL(k_sum_parts, dim3(ew_blocks(M * N)), dim3(256), 0, st, M, N, used, (const float *)parts, C, ldc);
  return hipGetLastError();
}

static hipError_t bf16_resid(int64_t M, int64_t N, int64_t Mp, int K, const void *A, int a_dtype, int64_t lda,
                             const uint16_t *Lh, const uint16_t *Ll, const uint16_t *Xh, const uint16_t *Xl,
                             uint16_t *RT, int64_t ldr, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int w = (M > 64 && N > 64) ? 4 : 2;
  Bf16Resid k{};
  k.M = M; k.N = N; k.Mp = Mp; k.K = K;
  k.A = A; k.lda = lda;
  k.Lh = Lh; k.Ll = Ll; k.Xh = Xh; k.Xl = Xl;
  k.RT = RT; k.ldr = ldr;
  k.ntn = (int)ceil_div(N, 32 * w);
  k.ntm = ceil_div(Mp, 32 * w);  // row tiles cover the zero columns of R^T too
  k.tiles = k.ntm * k.ntn;
  const int64_t nb = ceil_div(k.ntn, 8), subs = ceil_div(nb, kResidSub);
  const unsigned grid = (unsigned)(8 * subs * k.ntm * kResidSub);
  if (a_dtype == RLU_F32) {
    if (w == 4) hipLaunchKernelGGL((k_bf16_resid<float, 4, 4>), dim3(grid), dim3(256), 0, st, k);
    else hipLaunchKernelGGL((k_bf16_resid<float, 2, 2>), dim3(grid), dim3(256), 0, st, k);
  } else if (a_dtype == RLU_F64) {
    if (w == 4) hipLaunchKernelGGL((k_bf16_resid<double, 4, 4>), dim3(grid), dim3(256), 0, st, k);
    else hipLaunchKernelGGL((k_bf16_resid<double, 2, 2>), dim3(grid), dim3(256), 0, st, k);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t precision_contract(const PrecPlan &pp, const rlu_matrix *A, const double *Lhat, int l, double *Wt,
                              double *parts64, int splits_w, void *scratch, hipStream_t st) {
  const int64_t m = A->m, n = A->n;
  if (pp.precision == RLU_PREC_F32) {
    float *Lf = at<float>(scratch, pp.lf);
    hipLaunchKernelGGL(k_to_f32, dim3(ew_blocks(m * l)), dim3(256), 0, st, m, l, Lhat, (int64_t)l, Lf, l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmArgs g{};
    g.compute = RLU_F32;
    g.M = n; g.N = l; g.K = m;
    g.A = A->values; g.lda = A->ld; g.a_dtype = A->dtype; g.trans_a = true;
    g.B = Lf; g.ldb = l;
    g.C = Wt; g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    return gemm_f64_splitk(g, splits_w, parts64, st);
  }
  if (pp.precision != RLU_PREC_BF16_REFINED) return hipErrorInvalidValue;
  uint16_t *Lh = at<uint16_t>(scratch, pp.lhi), *Ll = at<uint16_t>(scratch, pp.llo);
  uint16_t *LhT = at<uint16_t>(scratch, pp.lht);
  hipLaunchKernelGGL(k_split_bf16, dim3(ew_blocks(m * pp.lp)), dim3(256), 0, st, m, l, Lhat, (int64_t)l, Lh, Ll, pp.lp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)(pp.mp / 64), (unsigned)(pp.np_rows / 64)), dim3(256), 0, st, m,
                     pp.lp, (const uint16_t *)Lh, (int64_t)pp.lp, LhT, pp.mp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return bf16_tn(n, l, m, A->values, A->dtype, false, A->ld, LhT, pp.mp, pp.np_rows, Wt, l, pp.wm, pp.wn, pp.splits,
                 pp.Kc, at<float>(scratch, pp.parts), st);
}

hipError_t precision_refine(const PrecPlan &pp, const rlu_matrix *A, int l, double *Wt, const double *Ginv,
                            double *Bt, void *scratch, hipStream_t st) {
  if (pp.precision != RLU_PREC_BF16_REFINED) return hipErrorInvalidValue;
  const int64_t m = A->m, n = A->n;
  hipError_t e;
  {  // X0^T = W0^T G^{-1}, kept in Bt
    GemmArgs g{};
    g.M = n; g.N = l; g.K = l;
    g.A = Wt; g.lda = l; g.a_dtype = RLU_F64;
    g.B = Ginv; g.ldb = l;
    g.C = Bt; g.ldc = l; g.alpha = 1.0; g.beta = 0.0;
    if ((e = gemm_f64(g, st)) != hipSuccess) return e;
  }
  uint16_t *Xh = at<uint16_t>(scratch, pp.xhi), *Xl = at<uint16_t>(scratch, pp.xlo);
  hipLaunchKernelGGL(k_split_bf16, dim3(ew_blocks(n * pp.lp)), dim3(256), 0, st, n, l, (const double *)Bt, (int64_t)l,
                     Xh, Xl, pp.lp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint16_t *RT = at<uint16_t>(scratch, pp.r);
  const uint16_t *Lh = at<uint16_t>(scratch, pp.lhi), *Ll = at<uint16_t>(scratch, pp.llo);
  const uint16_t *LhT = at<uint16_t>(scratch, pp.lht);
  if ((e = bf16_resid(m, n, pp.mp, pp.lp, A->values, A->dtype, A->ld, Lh, Ll, Xh, Xl, RT, pp.mp, st)) != hipSuccess)
    return e;
  // dW^T = bf16(R)^T bf16(Lhat), over W0^T
  if ((e = bf16_tn(n, l, m, RT, 0, true, pp.mp, LhT, pp.mp, pp.np_rows, Wt, l, pp.wm, pp.wn, pp.splits, pp.Kc,
                   at<float>(scratch, pp.parts), st)) != hipSuccess)
    return e;
  GemmArgs g{};  // B^T = X0^T + dW^T G^{-1}
  g.M = n; g.N = l; g.K = l;
  g.A = Wt; g.lda = l; g.a_dtype = RLU_F64;
  g.B = Ginv; g.ldb = l;
  g.C = Bt; g.ldc = l; g.alpha = 1.0; g.beta = 1.0;
  return gemm_f64(g, st);
}

}  // namespace rlu
