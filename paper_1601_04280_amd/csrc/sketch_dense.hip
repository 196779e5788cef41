// Fused sketch of a dense row-major A (Algorithm 1 step 2):
//   Y[i, :] = ((A[i, :] S^T) diag(d)) T R        (Sections 2.1 and 2.2)
// One block owns one row at a time: the SEM pass streams the row from HBM
// once and accumulates into s LDS buckets with native LDS FP64 atomics
// (bucket and folded sign come from the column code table), the length-s
// real transform runs in LDS, and only the l selected coordinates are
// evaluated and written.  Y0 never leaves LDS.
#include "fft_lds.h"
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

template <typename T>
__device__ inline double to_f64(T v) { return (double)v; }

template <typename T>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_dense(
    int64_t m, int64_t n, const T *__restrict__ A, int64_t lda, int s, int log2N, int l,
    const uint32_t *__restrict__ code, const int32_t *__restrict__ sel,
    const double2 *__restrict__ twf, const double2 *__restrict__ twp, double *__restrict__ Y,
    int64_t ldy) {
  extern __shared__ double2 lds2[];
  double *y0 = reinterpret_cast<double *>(lds2);
  const int N = s >> 1;
  const int tid = threadIdx.x;
  const double rs = 1.0 / sqrt((double)s);
  const double r2s = sqrt(2.0) * rs;
  constexpr int TH = kSketchThreads;
  constexpr int U = 4;

  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    for (int i = tid; i < s; i += TH) y0[i] = 0.0;
    __syncthreads();

    const T *a = A + row * lda;
    int64_t j = tid;
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

    const double2 *Z = fft_lds<TH>(lds2, lds2 + N, N, log2N, twf);
    double *yrow = Y + row * ldy;
    for (int q = tid; q < l; q += TH) yrow[q] = real_coord(Z, s, sel[q], twp, rs, r2s);
    __syncthreads();
  }
}

hipError_t launch_sketch_dense(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s,
                               int l, const uint32_t *code, const int32_t *sel,
                               const double2 *twf, const double2 *twp, double *Y, int64_t ldy,
                               int num_cu, hipStream_t st) {
  const size_t lds = (size_t)s * 2 * sizeof(double);
  const int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (160 * 1024) / lds));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)num_cu * per_cu));
  const int log2N = ilog2_exact(s / 2);
  if (dtype == RLU_F64) {
    hipLaunchKernelGGL(k_sketch_dense<double>, dim3(grid), dim3(kSketchThreads), lds, st, m, n,
                       (const double *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy);
  } else {
    hipLaunchKernelGGL(k_sketch_dense<float>, dim3(grid), dim3(kSketchThreads), lds, st, m, n,
                       (const float *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy);
  }
  return hipGetLastError();
}

void sketch_dense_set_attrs() {
  hipFuncSetAttribute((const void *)k_sketch_dense<double>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, kMaxS * 2 * sizeof(double));
  hipFuncSetAttribute((const void *)k_sketch_dense<float>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, kMaxS * 2 * sizeof(double));
}

}  // namespace rlu
