// FP64 GEMM on CDNA MFMA (v_mfma_f64_16x16x4_f64) for the dense
// contractions of the least-squares product (Corollary 3.2's B = L_y^+ P A):
//   W^T = A^T Lhat  (n x l, the dominant contraction, K = m),
//   G   = Lhat^T Lhat, and the small l x l / n x l / m x l products.
//
// Block tile 64 (M) x 16*TN (N), K staged through LDS 32 at a time with
// the next tile's global loads in flight (in registers) during the MFMAs of
// the current one; the four waves of a block each own 16 rows of the tile
// and TN 16x16 accumulators.  op(A) is A (M x K, row major, optional row gather) or A^T
// (A stored K x M).  A may be FP32 storage, widened exactly to FP64 on load.
// Split-K writes per-split partials that a second kernel sums in a fixed
// order (deterministic).
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

typedef double v4d __attribute__((ext_vector_type(4)));

struct GemmK {
  int64_t M, N, K;
  const void *A;
  int64_t lda;
  const int32_t *gather;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
  int64_t cstride;  // elements between split partials (partial mode)
  int64_t Kc;       // K extent of one split
  double alpha, beta;
  int partial;
};

constexpr int kBM = 64, kBK = 32;

// LDS row strides (doubles) congruent to 16 mod 32, i.e. 128 bytes mod 256:
// the four 16-lane groups of an MFMA operand read (rows k..k+3) then fall on
// two disjoint halves of the banks, the minimum of two passes per read.
constexpr int pad_stride(int w) { return w + ((16 - (w % 32)) + 32) % 32; }

template <typename TAt, bool TRA, bool GATH, int TN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmK p) {
  constexpr int BN = 16 * TN;
  constexpr int AS = pad_stride(kBM);
  constexpr int BS = pad_stride(BN);
  constexpr int AR = (kBK * kBM) / 256;  // A elements per thread per tile
  constexpr int BR = (kBK * BN) / 256;   // B elements per thread per tile
  __shared__ double As[kBK * AS];
  __shared__ double Bs[kBK * BS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kBM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t kb = (int64_t)blockIdx.z * p.Kc;
  const int64_t ke = min(p.K, kb + p.Kc);
  const TAt *A = reinterpret_cast<const TAt *>(p.A);
  v4d acc[TN];
#pragma unroll
  for (int t = 0; t < TN; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};

  TAt ra[AR];
  double rb[BR];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int e = tid + 256 * r;
      int k, m;
      if (TRA) { k = e >> 6; m = e & 63; } else { m = e >> 5; k = e & 31; }
      const int64_t gk = k0 + k, gm = m0 + m;
      TAt v = (TAt)0;
      if (gk < ke && gm < p.M) {
        if (TRA) v = A[gk * p.lda + gm];
        else v = A[(GATH ? (int64_t)p.gather[gm] : gm) * p.lda + gk];
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int e = tid + 256 * r;
      const int k = e / BN, n = e - k * BN;
      const int64_t gk = k0 + k, gn = n0 + n;
      rb[r] = (gk < ke && gn < p.N) ? p.B[gk * p.ldb + gn] : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int e = tid + 256 * r;
      int k, m;
      if (TRA) { k = e >> 6; m = e & 63; } else { m = e >> 5; k = e & 31; }
      As[k * AS + m] = (double)ra[r];
    }
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int e = tid + 256 * r;
      const int k = e / BN, n = e - k * BN;
      Bs[k * BS + n] = rb[r];
    }
  };

  if (kb < ke) {
    load(kb);
    store();
    __syncthreads();
  }
  for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
    const bool more = k0 + kBK < ke;
    if (more) load(k0 + kBK);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < kBK / 4; ++kk) {
      const double a = As[(kk * 4 + (lane >> 4)) * AS + wave * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < TN; ++t) {
        const double b = Bs[(kk * 4 + (lane >> 4)) * BS + t * 16 + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }

#pragma unroll
  for (int t = 0; t < TN; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = m0 + wave * 16 + (lane >> 4) + 4 * v;  // D row = lane/16 + 4 v
      const int64_t n = n0 + t * 16 + (lane & 15);
      if (m < p.M && n < p.N) {
        if (p.partial) {
          p.C[(int64_t)blockIdx.z * p.cstride + m * p.ldc + n] = acc[t][v];
        } else {
          double r = p.alpha * acc[t][v];
          if (p.beta != 0.0) r += p.beta * p.C[m * p.ldc + n];
          p.C[m * p.ldc + n] = r;
        }
      }
    }
  }
}

__global__ void k_splitk_reduce(int64_t M, int64_t N, int splits, const double *__restrict__ parts,
                                double *__restrict__ C, int64_t ldc, double alpha, double beta) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += parts[(int64_t)z * total + e];
    const int64_t m = e / N, n = e - m * N;
    double r = alpha * s;
    if (beta != 0.0) r += beta * C[m * ldc + n];
    C[m * ldc + n] = r;
  }
}

static int pick_tn(int64_t N) {
  const int64_t t = ceil_div(N, 16);
  if (t <= 1) return 1;
  if (t <= 2) return 2;
  if (t <= 4) return 4;
  if (t <= 7) return 7;
  if (t <= 8) return 8;
  if (t <= 14) return 14;
  return 16;
}

template <typename TAt, bool TRA, bool GATH>
static hipError_t dispatch_tn(int tn, dim3 grid, GemmK k, hipStream_t st) {
  switch (tn) {
#define RLU_TN(T)                                                                            \
  case T:                                                                                    \
    hipLaunchKernelGGL((k_gemm_f64<TAt, TRA, GATH, T>), grid, dim3(256), 0, st, k); break;
    RLU_TN(1) RLU_TN(2) RLU_TN(4) RLU_TN(7) RLU_TN(8) RLU_TN(14) RLU_TN(16)
#undef RLU_TN
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch(const GemmArgs &g, int splits, int64_t Kc, double *parts, hipStream_t st) {
  if (g.trans_b) return hipErrorInvalidValue;
  const int tn = pick_tn(g.N);
  GemmK k;
  k.M = g.M; k.N = g.N; k.K = g.K;
  k.A = g.A; k.lda = g.lda; k.gather = g.gather;
  k.B = g.B; k.ldb = g.ldb;
  k.alpha = g.alpha; k.beta = g.beta;
  k.Kc = Kc;
  if (parts) {
    k.C = parts; k.ldc = g.N; k.cstride = g.M * g.N; k.partial = 1;
  } else {
    k.C = g.C; k.ldc = g.ldc; k.cstride = 0; k.partial = 0;
  }
  const dim3 grid((unsigned)ceil_div(g.M, kBM), (unsigned)ceil_div(g.N, 16 * tn), (unsigned)splits);
  if (g.trans_a) {
    if (g.gather) return hipErrorInvalidValue;
    if (g.a_dtype == RLU_F32) return dispatch_tn<float, true, false>(tn, grid, k, st);
    return dispatch_tn<double, true, false>(tn, grid, k, st);
  }
  if (g.a_dtype != RLU_F64) return hipErrorInvalidValue;
  if (g.gather) return dispatch_tn<double, false, true>(tn, grid, k, st);
  return dispatch_tn<double, false, false>(tn, grid, k, st);
}

hipError_t gemm_f64(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return launch(g, 1, std::max<int64_t>(g.K, 1), nullptr, st);
}

int choose_splits(int64_t M, int64_t N, int64_t K, int num_cu) {
  const int tn = pick_tn(N);
  const int64_t tiles = ceil_div(M, kBM) * ceil_div(N, 16 * tn);
  int64_t s = ceil_div((int64_t)num_cu, tiles);  // one block per CU (register bound)
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / 256));
  s = std::min<int64_t>(s, 64);
  return (int)std::max<int64_t>(1, s);
}

size_t gemm_f64_splitk_scratch(int64_t M, int64_t N, int splits) {
  return splits > 1 ? align_up((size_t)splits * M * N * sizeof(double), 256) : 0;
}

hipError_t gemm_f64_splitk(const GemmArgs &g, int splits, double *parts, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (splits <= 1 || parts == nullptr) return gemm_f64(g, st);
  int64_t Kc = ceil_div(g.K, splits);
  Kc = ceil_div(Kc, kBK) * kBK;
  const int used = (int)ceil_div(g.K, Kc);
  hipError_t e = launch(g, used, Kc, parts, st);
  if (e != hipSuccess) return e;
  const int64_t total = g.M * g.N;
  const int blocks = (int)std::min<int64_t>(4096, ceil_div(total, 256));
  hipLaunchKernelGGL(k_splitk_reduce, dim3(std::max(1, blocks)), dim3(256), 0, st, g.M, g.N, used,
                     parts, g.C, g.ldc, g.alpha, g.beta);
  return hipGetLastError();
}

}  // namespace rlu
