// GEMM on CDNA MFMA for the dense contractions of the least-squares product
// (Corollary 3.2's B = L_y^+ P A):
//   W^T = A^T Lhat  (n x l, the dominant contraction, K = m),
//   G   = Lhat^T Lhat, and the small l x l / n x l / m x l products.
// FP64 (v_mfma_f64_16x16x4_f64) throughout, or, for the FP32 form of the
// contraction, FP32 operands and accumulation (v_mfma_f32_16x16x4_f32).
//
// Block: WGM x 2 waves (WGM = 4 for large outputs: two waves per SIMD, so one
// wave's LDS waits and barrier are covered by the other's MFMAs; 2 for small
// ones), each owning FM x FN 16x16 accumulator tiles, so the block tile is
// (16 FM WGM) x (32 FN).  K advances 16 at a time
// through a double-buffered LDS tile: the global loads of stage s + 1 are
// issued before the MFMAs of stage s and written to the other buffer after
// them, one barrier per stage.  Every global load is issued unconditionally
// from an in-bounds address (out-of-range elements read the tile's first
// row / column and are replaced by zero), so a stage's loads are all in
// flight together.  op(A) is A (M x K, row major, optional row gather) or
// A^T (A stored K x M); A may be FP32 storage (widened exactly for FP64).
// Split-K writes per-split partials that a second kernel sums in a fixed
// order (deterministic).
#include <type_traits>
#include <utility>

#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Accumulator and MFMA of one compute type.  Result layouts (lane l, element
// v): FP64 16x16x4 holds D[l/16 + 4v][l%16], FP32 16x16x4 holds
// D[4(l/16) + v][l%16]; both take A[l%16][l/16] and B[l/16][l%16].
template <typename TC> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

struct GemmK {
  int64_t M, N, K;
  const void *A;
  int64_t lda;
  const int32_t *gather;
  const void *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
  int64_t cstride;  // elements between split partials (partial mode)
  int64_t Kc;       // K extent of one split
  double alpha, beta;
  int partial;
  int b_lower;  // B lower triangular: K starts at the column tile's first column
};

constexpr int kBK = 16;

// LDS row stride congruent to 16 mod 32 elements: the four 16-lane groups of
// an operand read (rows k .. k+3) then fall on two disjoint halves of the banks.
constexpr int pad_stride(int w) { return w + ((16 - (w % 32)) + 32) % 32; }

template <typename TC, typename TAt, bool TRA, bool GATH, int WGM, int FM, int FN>
__global__ __launch_bounds__(128 * WGM, 1) void k_gemm(GemmK p) {
  typedef Mfma<TC> MF;
  constexpr int NT = 128 * WGM;  // threads: WGM x 2 waves
  constexpr int BM = 16 * FM * WGM, BN = 32 * FN;
  constexpr int AS = pad_stride(BM), BS = pad_stride(BN);
  constexpr int AR = (kBK * BM) / NT;  // A elements per thread per stage
  constexpr int BR = (kBK * BN) / NT;  // B elements per thread per stage
  static_assert((kBK * BM) % NT == 0 && (kBK * BN) % NT == 0, "stage not divisible among threads");
  __shared__ TC As[2][kBK * AS];
  __shared__ TC Bs[2][kBK * BS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t ks = (int64_t)blockIdx.z * p.Kc;
  const int64_t ke = min(p.K, ks + p.Kc);
  // rows k < n0 of a lower-triangular B are zero in this tile's columns (n0
  // is a multiple of kBK, so the stages stay aligned)
  const int64_t kb = p.b_lower ? max(ks, n0) : ks;
  const TAt *A = reinterpret_cast<const TAt *>(p.A);
  const TC *B = reinterpret_cast<const TC *>(p.B);

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};

  // Out-of-range elements are read from the tile's first row / column (in
  // bounds) and zeroed only when the stage is written to LDS, after the
  // MFMAs, so no instruction consumes a load before the MFMAs have run.
  TAt ra[AR];
  TC rb[BR];
  auto a_ok = [&](int r, int64_t k0) {
    const int e = tid + NT * r;
    int k, m;
    if (TRA) { k = e / BM; m = e % BM; } else { m = e / kBK; k = e % kBK; }
    return k0 + k < ke && m0 + m < p.M;
  };
  auto b_ok = [&](int r, int64_t k0) {
    const int e = tid + NT * r;
    return k0 + e / BN < ke && n0 + e % BN < p.N;
  };
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int e = tid + NT * r;
      int k, m;
      if (TRA) { k = e / BM; m = e % BM; } else { m = e / kBK; k = e % kBK; }
      const bool ok = a_ok(r, k0);
      const int64_t ck = ok ? k0 + k : kb, cm = ok ? m0 + m : m0;
      if (TRA) ra[r] = A[ck * p.lda + cm];
      else ra[r] = A[(GATH ? (int64_t)p.gather[cm] : cm) * p.lda + ck];
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int e = tid + NT * r;
      const bool ok = b_ok(r, k0);
      rb[r] = B[(ok ? k0 + e / BN : kb) * p.ldb + (ok ? n0 + e % BN : n0)];
    }
  };
  auto store = [&](int buf, int64_t k0) {
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int e = tid + NT * r;
      int k, m;
      if (TRA) { k = e / BM; m = e % BM; } else { m = e / kBK; k = e % kBK; }
      As[buf][k * AS + m] = a_ok(r, k0) ? (TC)ra[r] : (TC)0;
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int e = tid + NT * r;
      Bs[buf][(e / BN) * BS + e % BN] = b_ok(r, k0) ? rb[r] : (TC)0;
    }
  };

  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0, kb);
    __syncthreads();
  }
  for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
    const bool more = k0 + kBK < ke;
    if (more) load(k0 + kBK);  // in flight during the MFMAs below
    const TC *as = As[buf] + wm * 16 * FM + (lane & 15);
    const TC *bs = Bs[buf] + wn * 16 * FN + (lane & 15);
#pragma unroll
    for (int kk = 0; kk < kBK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      TC a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = as[kr * AS + i * 16];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = bs[kr * BS + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = MF::step(a[i], b[j], acc[i][j]);
    }
    if (more) {
      store(buf ^ 1, k0 + kBK);
      __syncthreads();
      buf ^= 1;
    }
  }

  // beta != 0: the old C values are loaded first (clamped, unconditional)
  double cold[FM][FN][4];
  const bool use_old = !p.partial && p.beta != 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cold[i][j][v] = 0.0;
        if (use_old) {
          const int64_t m = m0 + wm * 16 * FM + i * 16 + MF::row(lane, v);
          const int64_t n = n0 + wn * 16 * FN + j * 16 + (lane & 15);
          const bool ok = m < p.M && n < p.N;
          const double c = p.C[(ok ? m : m0) * p.ldc + (ok ? n : n0)];
          cold[i][j][v] = ok ? c : 0.0;
        }
      }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 16 * FM + i * 16 + MF::row(lane, v);
        const int64_t n = n0 + wn * 16 * FN + j * 16 + (lane & 15);
        if (m < p.M && n < p.N) {
          const double x = (double)acc[i][j][v];
          if (p.partial) {
            p.C[(int64_t)blockIdx.z * p.cstride + m * p.ldc + n] = x;
          } else {
            double r = p.alpha * x;
            if (use_old) r += p.beta * cold[i][j][v];
            p.C[m * p.ldc + n] = r;
          }
        }
      }
}

// Direct global-to-LDS form for FP64 op(A) = A^T with full 128-row tiles
// (M a multiple of 128, every K extent a multiple of 16, N even, A and B rows
// 16-byte aligned).  Each K row of a stage's A tile (128 doubles, or 128
// FP32 values of FP32-stored A, widened exactly when read from LDS) and B
// tile (BN doubles) is copied by global_load_lds_dwordx4 instructions of one
// wave straight into LDS (16 bytes per lane, lanes contiguous; an FP32 row
// takes the first 32 lanes).  Three buffers per
// operand hold stages s (being multiplied), s + 1 (landed) and s + 2 (in
// flight), so the loads get two stages to land without holding registers;
// the waits on them are the explicit ones before each barrier.  B columns at
// or past N receive copies of the row's first columns: they reach only
// output columns that are not stored.
// 16 bytes per lane from global memory straight into LDS (lane i's bytes at
// lds + 16 i).  A plain device function: the builtin exists only for the
// device, and the kernel template must also instantiate in the host pass.
__device__ inline void lds_copy16(const double *g, double *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0); }
__device__ inline void lds_copy16(const float *g, float *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 0); }
// the same with the nontemporal hint (cache policy bit 1), for an operand
// that every element of is read once per launch
__device__ inline void lds_copy16_nt(const double *g, double *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 2); }
__device__ inline void lds_copy16_nt(const float *g, float *lds) { __builtin_amdgcn_global_load_lds(g, lds, 16, 0, 2); }

template <int FN, typename TA, typename TC>
__global__ __launch_bounds__(512, 1) void k_gemm_dma(GemmK p) {
  typedef Mfma<TC> MF;  // TC: the compute type, which B is stored in
  constexpr int WGM = 4, FM = 2;
  constexpr int BM = 16 * FM * WGM, BN = 32 * FN;
  constexpr int PI = 64 * 16 / (int)sizeof(TC);  // B elements per copy instruction
  constexpr int H = (BN + PI - 1) / PI;          // copy instructions per B row
  // a copy instruction writes PI elements (64 lanes x 16 bytes) whatever BN
  // is: B rows are PI H elements apart (plus the bank padding), so the lanes
  // past BN write padding rather than the next row
  // A rows 144 elements apart: the four k rows of a fragment read start 16
  // doubles (FP32: 64 bytes of 576) apart in the bank order
  constexpr int AS = pad_stride(BM), BS = pad_stride(PI * H);
  static_assert(BM == 128 && kBK == 16, "one 1 KB A row per wave instruction, two rows per wave");
  // separate LDS objects, each named statically below: the compiler then
  // knows a read of one buffer does not wait for copies into another
  __shared__ __align__(16) TA As0[kBK * AS], As1[kBK * AS], As2[kBK * AS];
  __shared__ __align__(16) TC Bs0[kBK * BS], Bs1[kBK * BS], Bs2[kBK * BS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WGM, wn = wave / WGM;
  const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t kb = (int64_t)blockIdx.z * p.Kc;
  const int64_t ke = min(p.K, kb + p.Kc);
  const TA *A = reinterpret_cast<const TA *>(p.A);
  const TC *B = reinterpret_cast<const TC *>(p.B);

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = typename MF::acc_t{0, 0, 0, 0};

  auto uniform_ptr = [](auto *q) {
    const uint64_t u = reinterpret_cast<uint64_t>(q);
    return reinterpret_cast<decltype(q)>(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
  };
  // rows 2 wave and 2 wave + 1 of stage k0's tiles into (as, bs)
  auto copy_stage = [&](TA *as, TC *bs, int64_t k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int kr = 2 * wave + q;
      if constexpr (sizeof(TA) == 8) {
        lds_copy16_nt(uniform_ptr(A + (k0 + kr) * p.lda + m0) + 2 * lane, as + kr * AS);
      } else if (lane < 32) {  // 128 FP32 values: the first 32 lanes
        lds_copy16_nt(uniform_ptr(A + (k0 + kr) * p.lda + m0) + 4 * lane, as + kr * AS);
      }
      const TC *brow = uniform_ptr(B + (k0 + kr) * p.ldb + n0);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        // every lane issues (a fixed count of copies per stage); lanes past
        // N or the tile re-read the row's start into columns not stored
        const int c = PI * h + (16 / (int)sizeof(TC)) * lane;
        const int cc = (c < BN && n0 + c < p.N) ? c : 0;
        lds_copy16(brow + cc, bs + kr * BS + PI * h);
      }
    }
  };
  auto wait_copies = [&](bool newer) {  // all but the newest stage's 2 + 2 H copies landed
    static_assert(H == 1 || H == 2, "");
    if (!newer) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    else if (H == 2) asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  };
  // operand fragments of the four k steps of a stage, in registers; k step
  // kk + 1 is read while k step kk is multiplied
  TC fa[kBK / 4][FM], fb[kBK / 4][FN];
  auto load_kk = [&](const TA *asb, const TC *bsb, int kk) __attribute__((always_inline)) {
    const TA *as = asb + wm * 16 * FM + (lane & 15);
    const TC *bs = bsb + wn * 16 * FN + (lane & 15);
    const int kr = kk * 4 + (lane >> 4);
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[kk][i] = (TC)as[kr * AS + i * 16];
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[kk][j] = bs[kr * BS + j * 16];
  };
  auto mfma_kk = [&](int kk) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = MF::step(fa[kk][i], fb[kk][j], acc[i][j]);
  };

  if (kb < ke) {
    copy_stage(As0, Bs0, kb);
    const bool m1 = kb + kBK < ke;
    if (m1) copy_stage(As1, Bs1, kb + kBK);
    wait_copies(m1);  // stage 0 landed
    __builtin_amdgcn_s_barrier();
  }
  // Stage s is in buffer s mod 3; its copies are issued while stage s - 2 is
  // multiplied (into the buffer stage s - 3 used), right after the first k
  // step's fragments of stage s - 2 have been read: a wait the compiler puts
  // before those LDS reads then covers only copies issued a stage earlier,
  // never the ones just issued (the later reads get no wait).  They are issued every
  // stage (a fixed count, so the compiler's own waits before the LDS reads
  // stay exact): without a stage s + 2 the free buffer receives a copy of
  // stage s, which nothing reads.  After the MFMAs: the wait for stage
  // s + 1 and a bare barrier (the workgroup fence of __syncthreads would
  // also wait for the copies still in flight; every wave's LDS reads of
  // stage s precede its barrier).
#define RLU_DMA_STEP(ASC, BSC, ASN, BSN, K0)                                         \
  {                                                                                  \
    const int64_t k0_ = (K0);                                                        \
    const bool more1 = k0_ + kBK < ke, more2 = k0_ + 2 * kBK < ke;                   \
    load_kk(ASC, BSC, 0);                                                            \
    copy_stage(ASN, BSN, more2 ? k0_ + 2 * kBK : k0_);                               \
    load_kk(ASC, BSC, 1);                                                            \
    mfma_kk(0);                                                                      \
    load_kk(ASC, BSC, 2);                                                            \
    mfma_kk(1);                                                                      \
    load_kk(ASC, BSC, 3);                                                            \
    mfma_kk(2);                                                                      \
    mfma_kk(3);                                                                      \
    if (more1) {                                                                     \
      wait_copies(true);                                                             \
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");                             \
      __builtin_amdgcn_s_barrier();                                                  \
    }                                                                                \
    __builtin_amdgcn_sched_barrier(0);                                               \
  }
  // K extents are multiples of 16 here: whole groups of three stages, then
  // the zero to two stages left (which start again at buffer 0)
  const int64_t ns = (ke - kb) / kBK;
  int64_t k0 = kb;
  for (int64_t g3 = 0; g3 + 3 <= ns; g3 += 3, k0 += 3 * kBK) {
    RLU_DMA_STEP(As0, Bs0, As2, Bs2, k0)
    RLU_DMA_STEP(As1, Bs1, As0, Bs0, k0 + kBK)
    RLU_DMA_STEP(As2, Bs2, As1, Bs1, k0 + 2 * kBK)
  }
  if (k0 < ke) RLU_DMA_STEP(As0, Bs0, As2, Bs2, k0)
  if (k0 + kBK < ke) RLU_DMA_STEP(As1, Bs1, As0, Bs0, k0 + kBK)
#undef RLU_DMA_STEP

  // epilogue: plain (beta = 0) or partial stores
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 16 * FM + i * 16 + MF::row(lane, v);
        const int64_t n = n0 + wn * 16 * FN + j * 16 + (lane & 15);
        if (m < p.M && n < p.N) {
          const double x = (double)acc[i][j][v];
          if (p.partial) p.C[(int64_t)blockIdx.z * p.cstride + m * p.ldc + n] = x;
          else p.C[m * p.ldc + n] = p.alpha * x;
        }
      }
}

__global__ void k_splitk_reduce(int64_t M, int64_t N, int splits, const double *__restrict__ parts,
                                double *__restrict__ C, int64_t ldc, double alpha, double beta) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    // partials in order 0, 1, 2, ... (a fixed summation order); eight loads
    // in flight at a time
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = parts[(int64_t)(z + u) * total + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < splits; ++z) s += parts[(int64_t)z * total + e];
    const int64_t m = e / N, n = e - m * N;
    double r = alpha * s;
    if (beta != 0.0) r += beta * C[m * ldc + n];
    C[m * ldc + n] = r;
  }
}

// Tile shape for an M x N output with inner dimension K.  FN (N tile =
// 32 FN) from 7, 6, 4, 2, 1 minimises padded width x (1 + 1/FN): the second
// factor charges narrow tiles for their extra operand reads per MFMA and
// extra passes over op(A) (one per N tile); at most 2 for K <= 128.  FM = 2; the 8-wave block (M
// tile 128) when M and K are large (deep products fill the device through
// K splits), else the 4-wave block (M tile 64, twice the blocks).
struct Shape {
  int wgm, fm, fn;
  int bm() const { return 16 * fm * wgm; }
  int bn() const { return 32 * fn; }
};
static Shape pick_shape(int64_t M, int64_t N, int64_t K) {
  static const int fns[] = {7, 6, 4, 2, 1};
  int best = 1;
  double best_cost = 1e300;
  for (int fn : fns) {
    const double cost = (double)(ceil_div(N, 32 * fn) * 32 * fn) * (1.0 + 1.0 / fn);
    if (cost < best_cost) { best_cost = cost; best = fn; }
  }
  // shallow products (the LU's trailing updates) are bound by load latency
  // rather than by operand traffic: narrow tiles, several blocks per CU
  if (K <= 128 && best > 2) best = 2;
  return Shape{(M >= 1024 && K >= 1024) ? 4 : 2, 2, best};
}

template <typename TC, typename TAt, bool TRA, bool GATH, int WGM>
static hipError_t dispatch_fn(const Shape &sh, dim3 grid, GemmK k, hipStream_t st) {
  switch (sh.fn) {
#define RLU_FN(F)                                                                                \
  case F:                                                                                        \
    hipLaunchKernelGGL((k_gemm<TC, TAt, TRA, GATH, WGM, 2, F>), grid, dim3(128 * WGM), 0, st, k); \
    break;
    RLU_FN(1) RLU_FN(2) RLU_FN(4) RLU_FN(6) RLU_FN(7)
#undef RLU_FN
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TC, typename TAt, bool TRA, bool GATH>
static hipError_t dispatch_shape(const Shape &sh, dim3 grid, GemmK k, hipStream_t st) {
  if (sh.fm != 2) return hipErrorInvalidValue;
  if (sh.wgm == 4) return dispatch_fn<TC, TAt, TRA, GATH, 4>(sh, grid, k, st);
  if (sh.wgm == 2) return dispatch_fn<TC, TAt, TRA, GATH, 2>(sh, grid, k, st);
  return hipErrorInvalidValue;
}

// wide: 128-row tiles of eight waves whatever M (see gemm_f64_splitk)
static hipError_t launch(const GemmArgs &g, int splits, int64_t Kc, double *parts, hipStream_t st,
                         bool wide = false) {
  if (g.trans_b) return hipErrorInvalidValue;
  Shape sh = pick_shape(g.M, g.N, g.K);
  if (wide) sh.wgm = 4;
  if (g.b_lower) sh.fn = std::min(sh.fn, 2);  // 64-column tiles: each skips its zero rows of B
  GemmK k;
  k.M = g.M; k.N = g.N; k.K = g.K;
  k.b_lower = g.b_lower ? 1 : 0;
  k.A = g.A; k.lda = g.lda; k.gather = g.gather;
  k.B = g.B; k.ldb = g.ldb;
  k.alpha = g.alpha; k.beta = g.beta;
  k.Kc = Kc;
  if (parts) {
    k.C = parts; k.ldc = g.N; k.cstride = g.M * g.N; k.partial = 1;
  } else {
    k.C = g.C; k.ldc = g.ldc; k.cstride = 0; k.partial = 0;
  }
  const dim3 grid((unsigned)ceil_div(g.M, sh.bm()), (unsigned)ceil_div(g.N, sh.bn()), (unsigned)splits);
  if (g.compute == RLU_F32) {
    if (!g.trans_a || g.gather) return hipErrorInvalidValue;
    const bool f32a = g.a_dtype == RLU_F32;
    // the direct-to-LDS form: B (FP32) rows copied four values per lane
    const bool full = sh.wgm == 4 && sh.fm == 2 && g.M % 128 == 0 && g.K % kBK == 0 && Kc % kBK == 0 &&
                      g.N % 4 == 0 && g.lda % (f32a ? 4 : 2) == 0 && g.ldb % 4 == 0 &&
                      ((reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B)) & 15) == 0 &&
                      (k.partial || g.beta == 0.0) && !g.b_lower;
    if (full) {
      switch (sh.fn) {
#define RLU_FN(F)                                                                            \
  case F:                                                                                    \
    if (f32a) hipLaunchKernelGGL((k_gemm_dma<F, float, float>), grid, dim3(512), 0, st, k);   \
    else hipLaunchKernelGGL((k_gemm_dma<F, double, float>), grid, dim3(512), 0, st, k);       \
    return hipGetLastError();
        RLU_FN(4) RLU_FN(6) RLU_FN(7)
#undef RLU_FN
        default: break;
      }
    }
    if (f32a) return dispatch_shape<float, float, true, false>(sh, grid, k, st);
    return dispatch_shape<float, double, true, false>(sh, grid, k, st);
  }
  if (g.compute != RLU_F64) return hipErrorInvalidValue;
  if (g.trans_a) {
    if (g.gather) return hipErrorInvalidValue;
    const bool f32a = g.a_dtype == RLU_F32;
    const bool full = sh.wgm == 4 && sh.fm == 2 && g.M % 128 == 0 && g.K % kBK == 0 && Kc % kBK == 0 &&
                      g.N % 2 == 0 && g.lda % (f32a ? 4 : 2) == 0 && g.ldb % 2 == 0 &&
                      ((reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B)) & 15) == 0 &&
                      (k.partial || g.beta == 0.0) && !g.b_lower;
    if (full) {
      switch (sh.fn) {
#define RLU_FN(F)                                                                     \
  case F:                                                                             \
    if (f32a) hipLaunchKernelGGL((k_gemm_dma<F, float, double>), grid, dim3(512), 0, st, k);   \
    else hipLaunchKernelGGL((k_gemm_dma<F, double, double>), grid, dim3(512), 0, st, k);       \
    return hipGetLastError();
        RLU_FN(4) RLU_FN(6) RLU_FN(7)
#undef RLU_FN
        default: break;
      }
    }
    if (f32a) return dispatch_shape<double, float, true, false>(sh, grid, k, st);
    return dispatch_shape<double, double, true, false>(sh, grid, k, st);
  }
  if (g.a_dtype == RLU_F32) {  // FP32 storage, widened exactly (the explicit projection's A)
    if (g.gather) return hipErrorInvalidValue;
    return dispatch_shape<double, float, false, false>(sh, grid, k, st);
  }
  if (g.a_dtype != RLU_F64) return hipErrorInvalidValue;
  if (g.gather) return dispatch_shape<double, double, false, true>(sh, grid, k, st);
  return dispatch_shape<double, double, false, false>(sh, grid, k, st);
}

hipError_t gemm_f64(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return launch(g, 1, std::max<int64_t>(g.K, 1), nullptr, st);
}

// K splits: the count (1 .. 64, each split at least 256 deep, or 32 deep for
// products with fewer tiles than CUs) that minimises rounds of co-resident
// blocks (one per CU) per unit of work; ties go to fewer splits.
int choose_splits(int64_t M, int64_t N, int64_t K, int num_cu) {
  const Shape sh = pick_shape(M, N, K);
  const int64_t tiles = ceil_div(M, sh.bm()) * ceil_div(N, sh.bn());
  // splits at least 256 deep, or 32 deep when the tiles alone leave CUs idle
  const int64_t depth = tiles < num_cu ? 32 : 256;
  const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(64, K / depth));
  int64_t best = 1;
  double best_cost = 1e300;
  for (int64_t s = 1; s <= smax; ++s) {
    const double cost = (double)ceil_div(tiles * s, (int64_t)num_cu) / (double)s;
    if (cost < best_cost - 1e-12) { best_cost = cost; best = s; }
  }
  return (int)best;
}

size_t gemm_f64_splitk_scratch(int64_t M, int64_t N, int splits) {
  return splits > 1 ? align_up((size_t)splits * M * N * sizeof(double), 256) : 0;
}

static hipError_t splitk_run(const GemmArgs &g, int splits, double *parts, hipStream_t st, bool wide) {
  int64_t Kc = ceil_div(g.K, splits);
  Kc = ceil_div(Kc, kBK) * kBK;
  const int used = (int)ceil_div(g.K, Kc);
  hipError_t e = launch(g, used, Kc, parts, st, wide);
  if (e != hipSuccess) return e;
  const int64_t total = g.M * g.N;
  const int blocks = (int)std::min<int64_t>(4096, ceil_div(total, 256));
  hipLaunchKernelGGL(k_splitk_reduce, dim3(std::max(1, blocks)), dim3(256), 0, st, g.M, g.N, used,
                     parts, g.C, g.ldc, g.alpha, g.beta);
  return hipGetLastError();
}

hipError_t gemm_f64_splitk(const GemmArgs &g, int splits, double *parts, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (splits <= 1 || parts == nullptr) return gemm_f64(g, st);
  // A^T B with at least 512 rows that are not whole 128-row tiles (the Gram
  // matrix of l = 520, for one): the whole tiles on the direct-to-LDS kernel
  // with 128-row tiles, then the rows left on the general one, through the
  // same partials one after the other (the stream orders them).  As one
  // product on 64-row tiles the 520 x 520 x 32768 Gram matrix ran at
  // 26 TF/s.
  if (g.trans_a && g.compute == RLU_F64 && !g.gather && g.M >= 512 && g.M % 128 != 0 && g.K >= 1024) {
    const int64_t Mf = g.M / 128 * 128;
    const size_t esz = g.a_dtype == RLU_F32 ? 4 : 8;
    GemmArgs a = g, b = g;
    a.M = Mf;
    b.M = g.M - Mf;
    b.A = static_cast<const char *>(g.A) + (size_t)Mf * esz;  // A is K x M: columns Mf ..
    b.C = g.C + Mf * g.ldc;
    // K splits for one round of the wide tiles (at most the caller's count,
    // which sized the partials)
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
    const Shape sh = pick_shape(Mf, g.N, g.K);
    const int64_t tiles = (Mf / 128) * ceil_div(g.N, (int64_t)sh.bn());
    const int sa = (int)std::max<int64_t>(1, std::min<int64_t>(splits, ncu / std::max<int64_t>(1, tiles)));
    hipError_t e = splitk_run(a, sa, parts, st, true);
    if (e != hipSuccess) return e;
    return splitk_run(b, splits, parts, st, false);
  }
  return splitk_run(g, splits, parts, st, false);
}

}  // namespace rlu
