// Fused sketch of a dense row-major A (Algorithm 1 step 2):
//   Y[i, :] = ((A[i, :] S^T) diag(d)) T R        (Sections 2.1 and 2.2)
// One block owns one row at a time: the SEM pass accumulates the row into s
// LDS buckets with native LDS FP64 atomics (bucket and folded sign come from
// the column code table), the length-s real transform runs in LDS, and only
// the l selected coordinates are evaluated and written.  Y0 never leaves LDS.
//
// The first PF x 256 entries of the block's next row (and their codes) are
// loaded into registers before the current row's transform, so the row
// stream overlaps the transform; the twiddles and the selection live in LDS
// for that reason (a global load inside the transform would wait for the
// prefetch).  Longer rows stream their remainder 16 loads per thread deep.
#include "fft_lds.h"
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

template <typename T>
__device__ inline double to_f64(T v) { return (double)v; }

// LDS: the transform's two N-complex buffers, four twiddle tables, selection.
static inline int tw_bits(int log2N) { return log2N >> 1; }
static size_t sketch_lds_bytes(int s, int l) {
  const int N = s >> 1, log2N = ilog2_exact(N), b = tw_bits(log2N);
  const int nlo = 1 << b, nhi = N >> b;
  return (size_t)(2 * N + 2 * (nlo + nhi)) * sizeof(double2) + (size_t)l * sizeof(int32_t);
}

template <typename T, int PF>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_dense(
    int64_t m, int64_t n, const T *__restrict__ A, int64_t lda, int s, int log2N, int l,
    const uint32_t *__restrict__ code, const int32_t *__restrict__ sel,
    const double2 *__restrict__ twf, const double2 *__restrict__ twp, double *__restrict__ Y,
    int64_t ldy) {
  extern __shared__ double2 lds2[];
  constexpr int TH = kSketchThreads;
  constexpr int U = 16;
  const int N = s >> 1;
  const int tid = threadIdx.x;
  const double rs = 1.0 / sqrt((double)s);
  const double r2s = sqrt(2.0) * rs;
  double2 *buf = lds2;
  double2 *tab = lds2 + 2 * N;
  const int b = log2N >> 1, nlo = 1 << b, nhi = N >> b;
  int32_t *sel_s = reinterpret_cast<int32_t *>(tab + 2 * (nlo + nhi));
  for (int i = tid; i < nlo; i += TH) {
    tab[i] = twf[i];
    tab[nlo + nhi + i] = twp[i];
  }
  for (int i = tid; i < nhi; i += TH) {
    tab[nlo + i] = twf[i << b];
    tab[2 * nlo + nhi + i] = twp[i << b];
  }
  for (int q = tid; q < l; q += TH) sel_s[q] = sel[q];
  const TwSplit tf{tab, tab + nlo, b, nlo - 1};
  const TwSplit tp{tab + nlo + nhi, tab + 2 * nlo + nhi, b, nlo - 1};

  T pv[PF];
  uint32_t pc[PF];
  auto prefetch = [&](int64_t row) {  // clamped: column 0 stands in past the row's end
    const T *a = A + row * lda;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int64_t j = tid + (int64_t)u * TH;
      const int64_t jj = j < n ? j : 0;
      pv[u] = a[jj];
      pc[u] = code[jj];
    }
  };

  int64_t row = blockIdx.x;
  if (row < m) prefetch(row);
  for (; row < m; row += gridDim.x) {
    double *y0 = reinterpret_cast<double *>(buf);
    for (int i = tid; i < s; i += TH) y0[i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u)
      if (tid + (int64_t)u * TH < n) atomicAdd(&y0[code_bucket(pc[u])], code_apply(pc[u], to_f64(pv[u])));
    const T *a = A + row * lda;
    int64_t j = (int64_t)PF * TH + tid;
    for (; j + (U - 1) * TH < n; j += U * TH) {
      T v[U];
      uint32_t c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) { v[u] = a[j + u * TH]; c[u] = code[j + u * TH]; }
#pragma unroll
      for (int u = 0; u < U; ++u) atomicAdd(&y0[code_bucket(c[u])], code_apply(c[u], to_f64(v[u])));
    }
    for (; j < n; j += TH) {
      const uint32_t c = code[j];
      atomicAdd(&y0[code_bucket(c)], code_apply(c, to_f64(a[j])));
    }
    __syncthreads();
    if (row + gridDim.x < m) prefetch(row + gridDim.x);  // in flight during the transform

    const double2 *Z = fft_lds<TH>(buf, buf + N, N, log2N, tf);
    double *yrow = Y + row * ldy;
    for (int q = tid; q < l; q += TH) yrow[q] = real_coord(Z, s, sel_s[q], tp, rs, r2s);
    __syncthreads();
  }
}

template <typename T>
static void launch_pf(int pf, dim3 grid, size_t lds, hipStream_t st, int64_t m, int64_t n, const T *A,
                      int64_t lda, int s, int log2N, int l, const uint32_t *code, const int32_t *sel,
                      const double2 *twf, const double2 *twp, double *Y, int64_t ldy) {
  switch (pf) {
#define RLU_PF(P)                                                                                           \
  case P:                                                                                                   \
    hipLaunchKernelGGL((k_sketch_dense<T, P>), grid, dim3(kSketchThreads), lds, st, m, n, A, lda, s, log2N, \
                       l, code, sel, twf, twp, Y, ldy);                                                     \
    break;
    RLU_PF(4) RLU_PF(8) RLU_PF(16)
#undef RLU_PF
    default: break;
  }
}

hipError_t launch_sketch_dense(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s,
                               int l, const uint32_t *code, const int32_t *sel,
                               const double2 *twf, const double2 *twp, double *Y, int64_t ldy,
                               int num_cu, hipStream_t st) {
  const size_t lds = sketch_lds_bytes(s, l);
  const int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (160 * 1024) / lds));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)num_cu * per_cu));
  const int log2N = ilog2_exact(s / 2);
  // registers of the next-row prefetch: up to 16 values per thread (the rest
  // streams); 32 would halve the blocks a CU holds
  int pf = 4;
  while (pf < 16 && (int64_t)pf * kSketchThreads < n) pf *= 2;
  if (dtype == RLU_F64)
    launch_pf<double>(pf, dim3(grid), lds, st, m, n, (const double *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy);
  else
    launch_pf<float>(pf, dim3(grid), lds, st, m, n, (const float *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy);
  return hipGetLastError();
}

void sketch_dense_set_attrs() {
  const int bytes = (int)sketch_lds_bytes(kMaxS, 1024);  // l <= 1024 (validated far below)
#define RLU_ATTR(T, P) \
  hipFuncSetAttribute((const void *)k_sketch_dense<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  RLU_ATTR(double, 4) RLU_ATTR(double, 8) RLU_ATTR(double, 16)
  RLU_ATTR(float, 4) RLU_ATTR(float, 8) RLU_ATTR(float, 16)
#undef RLU_ATTR
}

}  // namespace rlu
