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
// reproducible to rounding, not bit for bit, unless the columns are sorted by
// row after the scatter (RLU_FLAG_DETERMINISTIC).
//
// Column indices outside [0, n) and inconsistent row pointers are not
// trusted: such entries are skipped and counted in rlu_info.bad_index.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

__device__ inline int64_t clamp_ptr(int32_t p, int64_t nnz) {
  return p < 0 ? 0 : (p > nnz ? nnz : (int64_t)p);
}

// GT: the cos table is read from global memory (s > kLdsMaxS) instead of LDS.
template <int QPL, bool HAD, bool GT>
__global__ __launch_bounds__(256) void k_sketch_csr(int64_t m, int64_t n, int64_t nnz,
                                                    const int32_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int s, int l,
                                                    const uint32_t *__restrict__ code,
                                                    const int32_t *__restrict__ sel,
                                                    const double2 *__restrict__ twp,
                                                    const double *__restrict__ gctab, double *__restrict__ Y,
                                                    int64_t ldy, int32_t *bad_index) {
  extern __shared__ double lctab[];  // cos(2 pi k / s), k < s
  const int tid = threadIdx.x, lane = tid & 63;
  const int N = s >> 1;
  if (!GT && !HAD) {
    for (int k = tid; k < s; k += 256) lctab[k] = (k < N) ? twp[k].x : -twp[k - N].x;
    __syncthreads();
  }
  const double *ctab = GT ? gctab : lctab;
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

// outputs per lane of the CSR kernels: l <= 64 QPL, QPL in {1..9, 12, 16}
static int csr_qpl(int l) {
  const int q = (int)ceil_div(l, 64);
  return q <= 9 ? q : (q <= 12 ? 12 : (q <= 16 ? 16 : 0));
}

hipError_t launch_sketch_csr(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col,
                             const double *val, int64_t nnz, int s, int l, const uint32_t *code,
                             const int32_t *sel, const double2 *twp, const double *gctab, double *Y,
                             int64_t ldy, int32_t *bad_index, int num_cu, bool hadamard, hipStream_t st) {
  const int qpl = csr_qpl(l);
  const bool gt = !hadamard && s > kLdsMaxS;
  if (gt && !gctab) return hipErrorInvalidValue;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, 4), (int64_t)num_cu * 8));
  const size_t lds = hadamard || gt ? 0 : (size_t)s * sizeof(double);
#define RLU_CSR_Q(Q)                                                                                       \
  case Q:                                                                                                  \
    if (hadamard)                                                                                          \
      hipLaunchKernelGGL((k_sketch_csr<Q, true, false>), dim3(blocks), dim3(256), lds, st, m, n, nnz,      \
                         row_ptr, col, val, s, l, code, sel, twp, gctab, Y, ldy, bad_index);               \
    else if (gt)                                                                                           \
      hipLaunchKernelGGL((k_sketch_csr<Q, false, true>), dim3(blocks), dim3(256), lds, st, m, n, nnz,      \
                         row_ptr, col, val, s, l, code, sel, twp, gctab, Y, ldy, bad_index);               \
    else                                                                                                   \
      hipLaunchKernelGGL((k_sketch_csr<Q, false, false>), dim3(blocks), dim3(256), lds, st, m, n, nnz,     \
                         row_ptr, col, val, s, l, code, sel, twp, gctab, Y, ldy, bad_index);               \
    break;
  switch (qpl) {
    RLU_CSR_Q(1) RLU_CSR_Q(2) RLU_CSR_Q(3) RLU_CSR_Q(4) RLU_CSR_Q(5) RLU_CSR_Q(6) RLU_CSR_Q(7)
    RLU_CSR_Q(8) RLU_CSR_Q(9) RLU_CSR_Q(12) RLU_CSR_Q(16)
    default: return hipErrorInvalidValue;
  }
#undef RLU_CSR_Q
  return hipGetLastError();
}

void sketch_csr_set_attrs() {
#define RLU_CSR_A(Q)                                                                                      \
  (void)hipFuncSetAttribute((const void *)k_sketch_csr<Q, false, false>,                                 \
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMaxS * 8);
  RLU_CSR_A(1) RLU_CSR_A(2) RLU_CSR_A(3) RLU_CSR_A(4) RLU_CSR_A(5) RLU_CSR_A(6) RLU_CSR_A(7) RLU_CSR_A(8)
  RLU_CSR_A(9) RLU_CSR_A(12) RLU_CSR_A(16)
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

// CSC copy of A by a two-pass bucket sort with no device-wide atomics (a
// device-scope atomic on this chip is performed beyond the per-die L2
// caches, so one per nonzero into n shared counters is slow), laid out so
// that the scattered writes of each pass stay within a region that the L2
// caches can gather into whole lines.  Columns are grouped into Q buckets of
// R consecutive columns (R = 512, or a larger power of two when n needs it,
// so that Q <= kMaxBuckets); the nonzeros [0, nnz) are cut into kBktChunks
// equal chunks.
//   0. k_csr_rows: the row of every entry (one pass over the row pointers);
//   1. k_bkt_count: per chunk, LDS counts of its entries per bucket, stored
//      bucket-major (cnt[q][b]), so that their exclusive scan gives every
//      (bucket, chunk) pair its run in a bucket-ordered staging array;
//   2. k_bkt_scatter: each chunk writes its entries (column, row, value) to
//      its runs, from LDS cursors;
//   3. k_bkt_place: one block per bucket counts its entries per column in
//      LDS, scans them into the column pointers and writes every entry to its
//      column's place, all within the bucket's part of the CSC arrays.
// A column's entries come chunk by chunk, so in increasing row order across
// chunks; within one chunk they follow the LDS cursor increments (sorted
// afterwards in deterministic mode).  Entries with a column outside [0, n)
// are left out (the sketch counts them in rlu_info.bad_index).
constexpr int kBktChunks = 256;
constexpr int kMaxBuckets = 16384;
constexpr int kMinBucketCols = 512;
constexpr int kMaxBucketCols = 32768;
constexpr int kScanTile = 4096;
constexpr int kBktUnroll = 8;  // entries per lane per pass, their loads issued together

static int bucket_cols(int64_t n) {
  int64_t r = kMinBucketCols;
  while (ceil_div(n, r) > kMaxBuckets) r *= 2;
  return (int)r;
}

__global__ __launch_bounds__(256) void k_bkt_count(int64_t n, int64_t nnz, int R, int Q,
                                                   const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
  extern __shared__ int32_t h[];  // Q counters
  const int tid = threadIdx.x, B = gridDim.x, b = blockIdx.x;
  for (int q = tid; q < Q; q += 256) h[q] = 0;
  __syncthreads();
  const int64_t k0 = nnz * b / B, k1 = nnz * (b + 1) / B;
  for (int64_t kb = k0 + tid; kb < k1; kb += 256 * kBktUnroll) {  // kBktUnroll loads in flight per lane
    int32_t c[kBktUnroll];
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) c[u] = kb + 256 * u < k1 ? col[kb + 256 * u] : -1;
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u)
      if (c[u] >= 0 && c[u] < n) atomicAdd(&h[c[u] / R], 1);
  }
  __syncthreads();
  for (int q = tid; q < Q; q += 256) cnt[(int64_t)q * B + b] = h[q];
}

struct BktEntry {
  int32_t col, row;
  double val;
};

__global__ __launch_bounds__(256) void k_bkt_scatter(int64_t n, int64_t nnz, int R, int Q,
                                                     const int32_t *__restrict__ col, const double *__restrict__ val,
                                                     const int32_t *__restrict__ rowidx,
                                                     const int32_t *__restrict__ off, BktEntry *__restrict__ stage) {
  extern __shared__ int32_t cur[];  // Q cursors
  const int tid = threadIdx.x, B = gridDim.x, b = blockIdx.x;
  for (int q = tid; q < Q; q += 256) cur[q] = off[(int64_t)q * B + b];
  __syncthreads();
  const int64_t k0 = nnz * b / B, k1 = nnz * (b + 1) / B;
  for (int64_t kb = k0 + tid; kb < k1; kb += 256 * kBktUnroll) {
    BktEntry e[kBktUnroll];
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) {
      const int64_t k = kb + 256 * u;
      const bool in = k < k1;
      e[u].col = in ? col[k] : -1;
      e[u].row = in ? rowidx[k] : 0;
      e[u].val = in ? val[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) {
      if (e[u].col < 0 || e[u].col >= n) continue;
      const int32_t pos = atomicAdd(&cur[e[u].col / R], 1);
      stage[pos] = e[u];
    }
  }
}

// One block (1024 threads) per bucket q: its entries are stage[off[q B] ..
// off[(q + 1) B]), its columns q R .. q R + R - 1.
__global__ __launch_bounds__(1024) void k_bkt_place(int64_t n, int R, int Q, int B, const int32_t *__restrict__ off,
                                                    const BktEntry *__restrict__ stage, int32_t *__restrict__ colptr,
                                                    int32_t *__restrict__ crow, double *__restrict__ cval) {
  extern __shared__ int32_t cc[];  // R counters, then cursors
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = blockIdx.x;
  const int64_t c0 = (int64_t)q * R;
  const int cw = (int)min<int64_t>(R, n - c0);
  const int32_t e0 = off[(int64_t)q * B], e1 = off[(int64_t)(q + 1) * B];
  for (int i = tid; i < cw; i += 1024) cc[i] = 0;
  __syncthreads();
  for (int32_t eb = e0 + tid; eb < e1; eb += 1024 * kBktUnroll) {
    int32_t c[kBktUnroll];
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) c[u] = eb + 1024 * u < e1 ? stage[eb + 1024 * u].col - (int32_t)c0 : -1;
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u)
      if (c[u] >= 0) atomicAdd(&cc[c[u]], 1);
  }
  __syncthreads();
  // exclusive scan of the cw counts, 1024 at a time, from e0
  int32_t base = e0;
  for (int i0 = 0; i0 < cw; i0 += 1024) {
    const int i = i0 + tid;
    const int32_t x = i < cw ? cc[i] : 0;
    int32_t incl = x;
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int32_t before = base, round = 0;
    for (int w = 0; w < 16; ++w) {
      before += w < wv ? wsum[w] : 0;
      round += wsum[w];
    }
    if (i < cw) {
      const int32_t ex = before + incl - x;
      colptr[c0 + i] = ex;
      cc[i] = ex;
    }
    __syncthreads();
    base += round;
  }
  if (q == Q - 1 && tid == 0) colptr[n] = e1;
  __syncthreads();
  for (int32_t eb = e0 + tid; eb < e1; eb += 1024 * kBktUnroll) {
    BktEntry en[kBktUnroll];
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) {
      const int32_t e = eb + 1024 * u < e1 ? eb + 1024 * u : e0;  // past the end: a repeat, not placed
      en[u] = stage[e];
    }
#pragma unroll
    for (int u = 0; u < kBktUnroll; ++u) {
      if (eb + 1024 * u >= e1) continue;
      const int32_t pos = atomicAdd(&cc[en[u].col - (int32_t)c0], 1);
      crow[pos] = en[u].row;
      cval[pos] = en[u].val;
    }
  }
}

// scan, phase 1: the sum of each tile of kScanTile counts
__global__ __launch_bounds__(256) void k_scan_tiles(int64_t total, const int32_t *__restrict__ v,
                                                    int32_t *__restrict__ tile_sum) {
  __shared__ int32_t ws[4];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  int32_t acc = 0;
  for (int64_t i = t0 + threadIdx.x; i < min(total, t0 + kScanTile); i += 256) acc += v[i];
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// scan, phase 2 (one block): exclusive scan of the tile sums in place
__global__ __launch_bounds__(1024) void k_scan_tile_sums(int ntiles, int32_t *__restrict__ tile_sum) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (ntiles + 1023) / 1024;
  const int a = min(ntiles, tid * per), e = min(ntiles, a + per);
  int32_t run = 0;
  for (int i = a; i < e; ++i) run += tile_sum[i];
  part[tid] = run;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t x = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  int32_t base = tid ? part[tid - 1] : 0;
  for (int i = a; i < e; ++i) {
    const int32_t x = tile_sum[i];
    tile_sum[i] = base;
    base += x;
  }
}

// scan, phase 3: out[i] = exclusive prefix of v (each tile from its base);
// out[total] = the sum
__global__ __launch_bounds__(256) void k_scan_apply(int64_t total, const int32_t *__restrict__ v,
                                                    const int32_t *__restrict__ tile_sum, int32_t *__restrict__ out) {
  __shared__ int32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  int32_t base = tile_sum[blockIdx.x];
  for (int64_t c0 = t0; c0 < min(total, t0 + kScanTile); c0 += 256) {
    const int64_t i = c0 + tid;
    const int32_t x = i < total ? v[i] : 0;
    int32_t incl = x;
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int32_t before = base;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    if (i < total) out[i] = before + incl - x;
    const int32_t round = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    base += round;
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 0) out[total] = base;
}

// The row of every entry, written row by row (one wavefront per row):
// rowidx[k] = i for k in [row_ptr[i], row_ptr[i+1]).  Consistent row
// pointers cover every entry exactly once; with inconsistent ones (flagged
// by the row pointer check) an entry keeps row 0 or takes one of the rows
// that claim it, always a valid row.
__global__ __launch_bounds__(256) void k_csr_rows(int64_t m, int64_t nnz, const int32_t *__restrict__ row_ptr,
                                                  int32_t *__restrict__ rowidx) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = w0; i < m; i += nw) {
    const int64_t a = clamp_ptr(row_ptr[i], nnz), b = clamp_ptr(row_ptr[i + 1], nnz);
    for (int64_t k = a + lane; k < b; k += 64) rowidx[k] = (int32_t)i;
  }
}

// Sorts every column's entries of the CSC copy by row (RLU_FLAG_DETERMINISTIC):
// the scatter leaves them in arrival order, which changes run to run.  The
// rows of a column are distinct, so the sorted order is unique.  One block per
// column; a bitonic sort in its ascending-only form (at the first step of each
// merge the partner is i ^ (k - 1), then i ^ j), so positions past the
// column's end act as +infinity and never move.  Columns of up to kSortLds
// entries are sorted in LDS, longer ones in place in global memory.
constexpr int kSortLds = 2048;
__global__ __launch_bounds__(256) void k_csc_sort(int64_t n, const int32_t *__restrict__ colptr,
                                                  int32_t *__restrict__ crow, double *__restrict__ cval) {
  __shared__ int32_t sr[kSortLds];
  __shared__ double sv[kSortLds];
  const int tid = threadIdx.x;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int32_t a = colptr[j], len = colptr[j + 1] - a;
    if (len < 2) continue;  // uniform over the block
    const bool in_lds = len <= kSortLds;
    int32_t *r = in_lds ? sr : crow + a;
    double *v = in_lds ? sv : cval + a;
    if (in_lds) {
      for (int i = tid; i < len; i += 256) {
        sr[i] = crow[a + i];
        sv[i] = cval[a + i];
      }
    }
    __syncthreads();
    int P = 1;
    while (P < len) P <<= 1;
    for (int k = 2; k <= P; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int i = tid; i < P; i += 256) {
          const int q = jj == (k >> 1) ? (i ^ (k - 1)) : (i ^ jj);
          if (q > i && q < len && r[i] > r[q]) {
            const int32_t tr = r[i];
            r[i] = r[q];
            r[q] = tr;
            const double tv = v[i];
            v[i] = v[q];
            v[q] = tv;
          }
        }
        __syncthreads();
      }
    }
    if (in_lds) {
      for (int i = tid; i < len; i += 256) {
        crow[a + i] = sr[i];
        cval[a + i] = sv[i];
      }
    }
    __syncthreads();
  }
}

// W^T[j][:] = sum over column j of A: v * Lhat[row][:]   (one wavefront per column;
// Lhat's rows ldh apart)
// The column's entries are taken UNR at a time: the UNR rows of Lhat are all
// loaded before any is used (UNR x QPL loads in flight per lane), then added
// in entry order, so the sums are the same as one entry at a time.
template <int QPL>
__global__ __launch_bounds__(256) void k_spmm_t(int64_t n, int l, const int32_t *__restrict__ colptr,
                                                const int32_t *__restrict__ crow, const double *__restrict__ cval,
                                                const double *__restrict__ Lhat, int64_t ldh, double *__restrict__ Wt) {
  constexpr int UNR = QPL <= 2 ? 8 : (QPL <= 4 ? 4 : 2);
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
      const int64_t bits = __double_as_longlong(v);
      const int cnt = min(64, b - base);
      for (int e0 = 0; e0 < cnt; e0 += UNR) {
        double lv[UNR][QPL], ve[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int eu = min(e0 + u, cnt - 1);  // uniform; past the end: a repeat, weighted 0
          const int re = __builtin_amdgcn_readlane(r, eu);
          const int lo32 = __builtin_amdgcn_readlane((int)(uint32_t)bits, eu);
          const int hi32 = __builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), eu);
          ve[u] = e0 + u < cnt ? __longlong_as_double(((int64_t)(uint32_t)hi32 << 32) | (uint32_t)lo32) : 0.0;
          const double *lr = Lhat + (int64_t)re * ldh;
#pragma unroll
          for (int t = 0; t < QPL; ++t) {
            const int q = lane + 64 * t;
            lv[u][t] = q < l ? lr[q] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          if (e0 + u < cnt) {
#pragma unroll
            for (int t = 0; t < QPL; ++t) acc[t] += ve[u] * lv[u][t];
          }
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

static int padded_ld(int l) { return (int)ceil_div(l, 16) * 16; }  // 16 doubles: one 128-byte line

size_t csc_scratch_bytes(int64_t n, int64_t nnz, int64_t m, int l) {
  const int64_t Q = ceil_div(std::max<int64_t>(n, 1), bucket_cols(n));
  const int64_t cells = Q * kBktChunks;
  size_t b = align_up((size_t)cells * 4, 256) + align_up((size_t)(cells + 1) * 4, 256) +
             align_up((size_t)ceil_div(cells, kScanTile) * 4, 256) +
             align_up((size_t)(n + 1) * 4, 256) + align_up((size_t)nnz * 4, 256) + align_up((size_t)nnz * 8, 256) +
             align_up((size_t)nnz * 4, 256) + align_up((size_t)nnz * sizeof(BktEntry), 256);
  if (l > 0 && padded_ld(l) != l) b += align_up((size_t)m * padded_ld(l) * 8, 256);
  return b;
}

hipError_t build_csc(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                     int64_t nnz, void *scratch, int num_cu, bool sorted, hipStream_t st, CscView *out) {
  const int R = bucket_cols(n);
  if (R > kMaxBucketCols) return hipErrorInvalidValue;
  const int Q = (int)ceil_div(std::max<int64_t>(n, 1), R);
  const int64_t cells = (int64_t)Q * kBktChunks;
  const int64_t ntiles = ceil_div(cells, kScanTile);
  if (ntiles > 1024 * 1024) return hipErrorInvalidValue;
  char *w = reinterpret_cast<char *>(scratch);
  int32_t *cnt = reinterpret_cast<int32_t *>(w);  // entries per (bucket, chunk), bucket-major
  w += align_up((size_t)cells * 4, 256);
  int32_t *off = reinterpret_cast<int32_t *>(w);  // their exclusive scan, off[cells] = the total
  w += align_up((size_t)(cells + 1) * 4, 256);
  int32_t *tsum = reinterpret_cast<int32_t *>(w);
  w += align_up((size_t)ntiles * 4, 256);
  int32_t *colptr = reinterpret_cast<int32_t *>(w);
  w += align_up((size_t)(n + 1) * 4, 256);
  int32_t *crow = reinterpret_cast<int32_t *>(w);
  w += align_up((size_t)nnz * 4, 256);
  double *cval = reinterpret_cast<double *>(w);
  w += align_up((size_t)nnz * 8, 256);
  int32_t *rowidx = reinterpret_cast<int32_t *>(w);
  w += align_up((size_t)nnz * 4, 256);
  BktEntry *stage = reinterpret_cast<BktEntry *>(w);
  hipError_t e;
  if (nnz > 0) {
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t *>(rowidx), 0u, nnz, st)) != hipSuccess) return e;
    const unsigned rb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)num_cu * 16, ceil_div(m, 4)));
    hipLaunchKernelGGL(k_csr_rows, dim3(rb), dim3(256), 0, st, m, nnz, row_ptr, rowidx);
  }
  const size_t qlds = (size_t)Q * 4;
  if ((e = hipFuncSetAttribute((const void *)k_bkt_count, hipFuncAttributeMaxDynamicSharedMemorySize, (int)qlds)) !=
          hipSuccess ||
      (e = hipFuncSetAttribute((const void *)k_bkt_scatter, hipFuncAttributeMaxDynamicSharedMemorySize, (int)qlds)) !=
          hipSuccess ||
      (e = hipFuncSetAttribute((const void *)k_bkt_place, hipFuncAttributeMaxDynamicSharedMemorySize, R * 4)) !=
          hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bkt_count, dim3(kBktChunks), dim3(256), qlds, st, n, nnz, R, Q, col, cnt);
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(256), 0, st, cells, cnt, tsum);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(1024), 0, st, (int)ntiles, tsum);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(256), 0, st, cells, cnt, tsum, off);
  if (nnz > 0)
    hipLaunchKernelGGL(k_bkt_scatter, dim3(kBktChunks), dim3(256), qlds, st, n, nnz, R, Q, col, val, rowidx, off,
                       stage);
  hipLaunchKernelGGL(k_bkt_place, dim3(Q), dim3(1024), (size_t)R * 4, st, n, R, Q, (int)kBktChunks, off, stage, colptr,
                     crow, cval);
  if (sorted) {
    const int sblocks = (int)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)num_cu * 8));
    hipLaunchKernelGGL(k_csc_sort, dim3(sblocks), dim3(256), 0, st, n, colptr, crow, cval);
  }
  out->colptr = colptr;
  out->crow = crow;
  out->cval = cval;
  return hipGetLastError();
}

hipError_t contraction_csr(int64_t m, int64_t n, int l, const int32_t *row_ptr, const int32_t *col,
                           const double *val, int64_t nnz, const double *Lhat, double *Wt, void *scratch,
                           int num_cu, bool sorted, hipStream_t st) {
  CscView cs;
  hipError_t e = build_csc(m, n, row_ptr, col, val, nnz, scratch, num_cu, sorted, st, &cs);
  if (e != hipSuccess) return e;
  const int32_t *colptr = cs.colptr, *crow = cs.crow;
  const double *cval = cs.cval;
  // The gathers read one row of Lhat per nonzero: with rows padded to whole
  // 128-byte lines (and line-aligned) each row takes ceil(l / 16) lines
  // instead of one more for most rows, so Lhat is copied first when l is not
  // a multiple of 16 (its copy moves 2 m l 8 bytes; the gathers nnz l 8).
  const double *Lg = Lhat;
  int64_t ldg = l;
  if (padded_ld(l) != l) {
    double *Lp = reinterpret_cast<double *>(reinterpret_cast<char *>(scratch) + csc_scratch_bytes(n, nnz));
    if ((e = launch_copy_rows(m, l, Lhat, l, Lp, padded_ld(l), st)) != hipSuccess) return e;
    Lg = Lp;
    ldg = padded_ld(l);
  }
  const int qpl = csr_qpl(l);
  const int cblocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4), (int64_t)num_cu * 16));
#define RLU_SPMM_Q(Q)                                                                                  \
  case Q:                                                                                              \
    hipLaunchKernelGGL(k_spmm_t<Q>, dim3(cblocks), dim3(256), 0, st, n, l, colptr, crow, cval, Lg, ldg, Wt); \
    break;
  switch (qpl) {
    RLU_SPMM_Q(1) RLU_SPMM_Q(2) RLU_SPMM_Q(3) RLU_SPMM_Q(4) RLU_SPMM_Q(5) RLU_SPMM_Q(6) RLU_SPMM_Q(7)
    RLU_SPMM_Q(8) RLU_SPMM_Q(9) RLU_SPMM_Q(12) RLU_SPMM_Q(16)
    default: return hipErrorInvalidValue;
  }
#undef RLU_SPMM_Q
  return hipGetLastError();
}

}  // namespace rlu
