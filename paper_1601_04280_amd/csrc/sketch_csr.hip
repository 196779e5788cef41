// Sparse (CSR) input: the sketch of Algorithm 1 step 2 and the contraction
// W^T = A^T Lhat of the least-squares product, with cost proportional to
// nnz(A) (the sparse complexity of Section 3.1; Theorem 2.9).
//
// Sketch.  A row with a handful of nonzeros touches a handful of the s SEM
// buckets, so instead of an s-point transform per row, each selected real
// Fourier coordinate is evaluated directly from the row's nonzeros:
//   Y[i, q] = w_q * sum_j sgn'(j) A[i, j] cos(2 pi (a_q h(j) + o_q) / s)
// with (a_q, o_q, w_q) from f = sel[q] (N = s/2):
//   f = 0: (0, 0, 1/sqrt s);  f = N: (N, 0, 1/sqrt s);
//   0 < f < N: (f, 0, sqrt(2/s));  f > N: (s - f, 3s/4, -sqrt(2/s))
// (sin x = cos(x - pi/2), and the -s/4 shift is 3s/4 mod s).  sgn'(j) is the
// SEM sign folded with the transform's diagonal, as in the dense kernel.
// Cost 2 nnz l flops; one wavefront per row, each lane a few outputs, the
// row's nonzeros broadcast lane by lane, cos(2 pi k / s) from an LDS table.
// With the Walsh-Hadamard transform (HAD) the kernel is the sign
// (-1)^popcount(b & sel[q]) and the weight 1/sqrt s.
//
// Contraction.  A^T is built once per call as CSC (column counts, scan,
// scatter with atomic cursors); one wavefront per column then gathers rows of
// Lhat.  The order of a column's entries follows the scatter, so W is
// reproducible to rounding, not bit for bit.
//
// Column indices outside [0, n) and inconsistent row pointers are not
// trusted: such entries are skipped and counted in rlu_info.bad_index.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

__device__ inline int64_t clamp_ptr(int32_t p, int64_t nnz) {
  return p < 0 ? 0 : (p > nnz ? nnz : (int64_t)p);
}

template <int QPL, bool HAD>
__global__ __launch_bounds__(256) void k_sketch_csr(int64_t m, int64_t n, int64_t nnz,
                                                    const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int s, int l,
                                                    const uint32_t *__restrict__ code,
                                                    const int32_t *__restrict__ sel,
                                                    const double2 *__restrict__ twp, double *__restrict__ Y,
                                                    int64_t ldy, int32_t *bad_index) {
  extern __shared__ double ctab[];  // cos(2 pi k / s), k < s
  const int tid = threadIdx.x, lane = tid & 63;
  const int N = s >> 1;
  for (int k = tid; k < s; k += 256) ctab[k] = (k < N) ? twp[k].x : -twp[k - N].x;
  __syncthreads();
  const double rs = 1.0 / sqrt((double)s);
  const double r2s = sqrt(2.0) * rs;
  const uint32_t mask = (uint32_t)s - 1u;
  uint32_t qa[QPL], qo[QPL];
  double qw[QPL];
#pragma unroll
  for (int t = 0; t < QPL; ++t) {
    const int q = lane + 64 * t;
    const int f = q < l ? sel[q] : 0;
    if (HAD) { qa[t] = (uint32_t)f; qo[t] = 0; qw[t] = rs; }
    else if (f == 0) { qa[t] = 0; qo[t] = 0; qw[t] = rs; }
    else if (f == N) { qa[t] = (uint32_t)N; qo[t] = 0; qw[t] = rs; }
    else if (f < N) { qa[t] = (uint32_t)f; qo[t] = 0; qw[t] = r2s; }
    else { qa[t] = (uint32_t)(s - f); qo[t] = (uint32_t)(3 * (s / 4)); qw[t] = -r2s; }
  }
  int bad = 0;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (tid >> 6); i < m; i += waves) {
    const int64_t lo = clamp_ptr(row_ptr[i], nnz);
    const int64_t hi = max(lo, clamp_ptr(row_ptr[i + 1], nnz));
    double acc[QPL];
#pragma unroll
    for (int t = 0; t < QPL; ++t) acc[t] = 0.0;
    for (int64_t base = lo; base < hi; base += 64) {
      const int64_t k = base + lane;
      uint32_t b = 0;
      double sv = 0.0;
      if (k < hi) {
        const int32_t j = col[k];
        if (j >= 0 && j < n) {
          const uint32_t c = code[j];
          b = code_bucket(c);
          sv = code_apply(c, val[k]);
        } else {
          ++bad;
        }
      }
      const int cnt = (int)min((int64_t)64, hi - base);
      for (int e = 0; e < cnt; ++e) {
        const uint32_t be = (uint32_t)__builtin_amdgcn_readlane((int)b, e);
        const int64_t bits = __double_as_longlong(sv);
        const int lo32 = __builtin_amdgcn_readlane((int)(uint32_t)bits, e);
        const int hi32 = __builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), e);
        const double ve = __longlong_as_double(((int64_t)(uint32_t)hi32 << 32) | (uint32_t)lo32);
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
          if (HAD) acc[t] += (__popc(qa[t] & be) & 1) ? -ve : ve;
          else acc[t] += ve * ctab[(qa[t] * be + qo[t]) & mask];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < QPL; ++t) {
      const int q = lane + 64 * t;
      if (q < l) Y[i * ldy + q] = qw[t] * acc[t];
    }
  }
  if (bad) atomicAdd(bad_index, bad);
}

hipError_t launch_sketch_csr(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col,
                             const double *val, int64_t nnz, int s, int l, const uint32_t *code,
                             const int32_t *sel, const double2 *twf, const double2 *twp, double *Y,
                             int64_t ldy, int32_t *bad_index, int num_cu, bool hadamard, hipStream_t st) {
  (void)twf;
  const int qpl = (int)ceil_div(l, 64);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 4), (int64_t)num_cu * 8));
  const size_t lds = (size_t)s * sizeof(double);
#define RLU_CSR_Q(Q)                                                                                    \
  case Q:                                                                                               \
    if (hadamard)                                                                                       \
      hipLaunchKernelGGL((k_sketch_csr<Q, true>), dim3(blocks), dim3(256), lds, st, m, n, nnz, row_ptr,  \
                         col, val, s, l, code, sel, twp, Y, ldy, bad_index);                            \
    else                                                                                                \
      hipLaunchKernelGGL((k_sketch_csr<Q, false>), dim3(blocks), dim3(256), lds, st, m, n, nnz, row_ptr, \
                         col, val, s, l, code, sel, twp, Y, ldy, bad_index);                            \
    break;
  switch (qpl) {
    RLU_CSR_Q(1) RLU_CSR_Q(2) RLU_CSR_Q(3) RLU_CSR_Q(4) RLU_CSR_Q(5) RLU_CSR_Q(6) RLU_CSR_Q(7)
    RLU_CSR_Q(8) RLU_CSR_Q(9)
    default: return hipErrorInvalidValue;
  }
#undef RLU_CSR_Q
  return hipGetLastError();
}

void sketch_csr_set_attrs() {
#define RLU_CSR_A(Q)                                                                                            \
  (void)hipFuncSetAttribute((const void *)k_sketch_csr<Q, false>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                            kMaxS * 8);                                                                          \
  (void)hipFuncSetAttribute((const void *)k_sketch_csr<Q, true>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxS * 8);
  RLU_CSR_A(1) RLU_CSR_A(2) RLU_CSR_A(3) RLU_CSR_A(4) RLU_CSR_A(5) RLU_CSR_A(6) RLU_CSR_A(7) RLU_CSR_A(8)
  RLU_CSR_A(9)
#undef RLU_CSR_A
}

// ---- row pointer check ------------------------------------------------------------

__global__ void k_csr_check(int64_t m, int64_t nnz, const int32_t *__restrict__ row_ptr, int validate,
                            rlu_info *info) {
  int bad = 0;
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i0 == 0) bad += (row_ptr[0] != 0) + ((int64_t)row_ptr[m] != nnz);
  if (validate)
    for (int64_t i = i0; i < m; i += (int64_t)gridDim.x * blockDim.x) bad += (row_ptr[i + 1] < row_ptr[i]);
  if (bad) atomicAdd(&info->bad_index, bad);
}

hipError_t launch_csr_check(const rlu_matrix *A, int validate_cols, rlu_info *info, hipStream_t st) {
  const int blocks = validate_cols ? (int)std::min<int64_t>(1024, ceil_div(A->m, 256)) : 1;
  hipLaunchKernelGGL(k_csr_check, dim3(std::max(1, blocks)), dim3(256), 0, st, A->m, A->nnz, A->row_ptr,
                     validate_cols, info);
  return hipGetLastError();
}

// ---- CSC (A^T) build and the sparse contraction -------------------------------------

__global__ void k_col_count(int64_t m, int64_t n, int64_t nnz, const int32_t *__restrict__ row_ptr,
                            const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += waves) {
    const int64_t lo = clamp_ptr(row_ptr[i], nnz), hi = max(lo, clamp_ptr(row_ptr[i + 1], nnz));
    for (int64_t k = lo + lane; k < hi; k += 64) {
      const int32_t j = col[k];
      if (j >= 0 && j < n) atomicAdd(&cnt[j], 1);
    }
  }
}

// exclusive scan of n counts (one block): colptr[0..n]
__global__ __launch_bounds__(1024) void k_scan(int64_t n, const int32_t *__restrict__ cnt, int32_t *__restrict__ colptr) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int64_t per = ceil_div(n, 1024);
  const int64_t a = tid * per, b = min(n, a + per);
  int32_t s = 0;
  for (int64_t i = a; i < b; ++i) s += cnt[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid ? part[tid - 1] : 0;
  for (int64_t i = a; i < b; ++i) {
    colptr[i] = run;
    run += cnt[i];
  }
  if (tid == 1023) colptr[n] = part[1023];
}

__global__ void k_col_scatter(int64_t m, int64_t n, int64_t nnz, const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ col, const double *__restrict__ val,
                              const int32_t *__restrict__ colptr, int32_t *__restrict__ cursor,
                              int32_t *__restrict__ crow, double *__restrict__ cval) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += waves) {
    const int64_t lo = clamp_ptr(row_ptr[i], nnz), hi = max(lo, clamp_ptr(row_ptr[i + 1], nnz));
    for (int64_t k = lo + lane; k < hi; k += 64) {
      const int32_t j = col[k];
      if (j >= 0 && j < n) {
        const int32_t p = colptr[j] + atomicAdd(&cursor[j], 1);
        crow[p] = (int32_t)i;
        cval[p] = val[k];
      }
    }
  }
}

// W^T[j][:] = sum over column j of A: v * Lhat[row][:]   (one wavefront per column)
template <int QPL>
__global__ __launch_bounds__(256) void k_spmm_t(int64_t n, int l, const int32_t *__restrict__ colptr,
                                                const int32_t *__restrict__ crow, const double *__restrict__ cval,
                                                const double *__restrict__ Lhat, double *__restrict__ Wt) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < n; j += waves) {
    double acc[QPL];
#pragma unroll
    for (int t = 0; t < QPL; ++t) acc[t] = 0.0;
    const int32_t a = colptr[j], b = colptr[j + 1];
    for (int32_t base = a; base < b; base += 64) {
      const int32_t p = base + lane;
      const int32_t r = p < b ? crow[p] : 0;
      const double v = p < b ? cval[p] : 0.0;
      const int cnt = min(64, b - base);
      for (int e = 0; e < cnt; ++e) {
        const int re = __builtin_amdgcn_readlane(r, e);
        const int64_t bits = __double_as_longlong(v);
        const int lo32 = __builtin_amdgcn_readlane((int)(uint32_t)bits, e);
        const int hi32 = __builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), e);
        const double ve = __longlong_as_double(((int64_t)(uint32_t)hi32 << 32) | (uint32_t)lo32);
        const double *lr = Lhat + (int64_t)re * l;
#pragma unroll
        for (int t = 0; t < QPL; ++t) {
          const int q = lane + 64 * t;
          if (q < l) acc[t] += ve * lr[q];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < QPL; ++t) {
      const int q = lane + 64 * t;
      if (q < l) Wt[j * l + q] = acc[t];
    }
  }
}

size_t csc_scratch_bytes(int64_t n, int64_t nnz) {
  return align_up((size_t)(n + 1) * 4, 256) * 3 + align_up((size_t)nnz * 4, 256) + align_up((size_t)nnz * 8, 256);
}

hipError_t build_csc(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                     int64_t nnz, void *scratch, int num_cu, hipStream_t st, CscView *out) {
  char *w = reinterpret_cast<char *>(scratch);
  const size_t nb4 = align_up((size_t)(n + 1) * 4, 256);
  int32_t *cnt = reinterpret_cast<int32_t *>(w);
  int32_t *colptr = reinterpret_cast<int32_t *>(w + nb4);
  int32_t *cursor = reinterpret_cast<int32_t *>(w + 2 * nb4);
  int32_t *crow = reinterpret_cast<int32_t *>(w + 3 * nb4);
  double *cval = reinterpret_cast<double *>(w + 3 * nb4 + align_up((size_t)nnz * 4, 256));
  hipError_t e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(cnt), 0u, n + 1, st)) != hipSuccess) return e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(cursor), 0u, n + 1, st)) != hipSuccess) return e;
  const int rblocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 4), (int64_t)num_cu * 16));
  hipLaunchKernelGGL(k_col_count, dim3(rblocks), dim3(256), 0, st, m, n, nnz, row_ptr, col, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, n, cnt, colptr);
  hipLaunchKernelGGL(k_col_scatter, dim3(rblocks), dim3(256), 0, st, m, n, nnz, row_ptr, col, val, colptr,
                     cursor, crow, cval);
  out->colptr = colptr;
  out->crow = crow;
  out->cval = cval;
  return hipGetLastError();
}

hipError_t contraction_csr(int64_t m, int64_t n, int l, const int32_t *row_ptr, const int32_t *col,
                           const double *val, int64_t nnz, const double *Lhat, double *Wt, void *scratch,
                           int num_cu, hipStream_t st) {
  CscView cs;
  hipError_t e = build_csc(m, n, row_ptr, col, val, nnz, scratch, num_cu, st, &cs);
  if (e != hipSuccess) return e;
  const int32_t *colptr = cs.colptr, *crow = cs.crow;
  const double *cval = cs.cval;
  const int qpl = (int)ceil_div(l, 64);
  const int cblocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4), (int64_t)num_cu * 16));
#define RLU_SPMM_Q(Q)                                                                                  \
  case Q:                                                                                              \
    hipLaunchKernelGGL(k_spmm_t<Q>, dim3(cblocks), dim3(256), 0, st, n, l, colptr, crow, cval, Lhat, Wt); \
    break;
  switch (qpl) {
    RLU_SPMM_Q(1) RLU_SPMM_Q(2) RLU_SPMM_Q(3) RLU_SPMM_Q(4) RLU_SPMM_Q(5) RLU_SPMM_Q(6) RLU_SPMM_Q(7)
    RLU_SPMM_Q(8) RLU_SPMM_Q(9)
    default: return hipErrorInvalidValue;
  }
#undef RLU_SPMM_Q
  return hipGetLastError();
}

}  // namespace rlu
