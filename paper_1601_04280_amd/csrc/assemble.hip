// Assembly of the outputs of Algorithm 1 steps 6-7 and small utilities.
//
// The column-pivoted LU of B (l x n) runs as the row-pivoted LU of B^T:
// Q^T B^T = L' U' gives B Q = U'^T L'^T = (U'^T D^{-1}) (D L'^T) with
// D = diag(U'), so
//   L~[i][j] = U'[j][i] / U'[j][j]   (i > j; unit diagonal),
//   U[j][q]  = U'[j][j] L'[q][j]     (q >= j),
// and a zero pivot (U'[j][j] = 0) leaves column j of L~ as e_j and row j of
// U zero, the same rule as for the row-pivoted LU.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_ltilde(int l, const double *__restrict__ Up, double *__restrict__ Lt) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < l * l; e += gridDim.x * blockDim.x) {
    const int i = e / l, j = e - i * l;
    double v = 0.0;
    if (i == j) v = 1.0;
    else if (i > j) {
      const double d = Up[(int64_t)j * l + j];
      v = (d != 0.0) ? Up[(int64_t)j * l + i] / d : 0.0;
    }
    Lt[e] = v;
  }
}

// U (l x n, row major): rows j, columns q.  Tile 32 rows of U x 64 columns:
// the gathered rows of L' (contiguous in j) are staged through LDS so both
// the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void k_assemble_u(int l, int64_t n, const double *__restrict__ Up,
                                                    const double *__restrict__ Lphat,
                                                    const int32_t *__restrict__ perm_c,
                                                    double *__restrict__ U, int64_t ldu) {
  __shared__ double T[64][33];
  const int j0 = blockIdx.y * 32;
  const int64_t q0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 32; e += 256) {
    const int qq = e / 32, jj = e - qq * 32;
    const int64_t q = q0 + qq;
    const int j = j0 + jj;
    T[qq][jj] = (q < n && j < l) ? Lphat[(int64_t)perm_c[q] * l + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 32; e += 256) {
    const int jj = e / 64, qq = e - jj * 64;
    const int64_t q = q0 + qq;
    const int j = j0 + jj;
    if (q < n && j < l) U[(int64_t)j * ldu + q] = (q < j) ? 0.0 : Up[(int64_t)j * l + j] * T[qq][jj];
  }
}

__global__ __launch_bounds__(256) void k_transpose(int64_t rows, int64_t cols, const double *__restrict__ in,
                                                   int64_t ldin, double *__restrict__ out, int64_t ldout) {
  __shared__ double T[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    T[k][tx] = (r < rows && c < cols) ? in[r * ldin + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[c * ldout + r] = T[tx][k];
  }
}

__global__ void k_copy_rows(int64_t rows, int64_t cols, const double *__restrict__ in, int64_t ldin,
                            double *__restrict__ out, int64_t ldout) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    out[r * ldout + c] = in[r * ldin + c];
  }
}

__global__ void k_finalize(rlu_info *info, const int32_t *abort_flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*abort_flag) {
    info->timeouts += 1;
    info->status = RLU_ERR_DEVICE;
  } else if (info->status == RLU_OK && info->nonfinite) {
    info->status = RLU_ERR_NUMERIC;
  } else if (info->status == RLU_OK && info->bad_index) {
    info->status = RLU_ERR_INVALID_ARG;
  }
}

// Pivot screening (rlu_info.min_gap_*).  At step j of the tall LU the
// candidates' magnitudes are |x_i| = |L[i][j]| |U[j][j]|, the winner's being
// |U[j][j]| itself, so the step's top-two gap (|x_1| - |x_2|) / |x_1| is
// 1 - max |L[i][j]| over the rows that lost.  Lhat holds L in X's row order;
// rows pivoted earlier hold 0 in column j and the step's own pivot row
// (perm[j]) holds 1, so that row is skipped.  maxbits[j] receives the
// column's maximum as the bit pattern of a non-negative double, whose order
// as an unsigned integer is that of the value (zeroed beforehand).
// Block: 64 columns (blockIdx.y) x rows_per_block rows; lane = column,
// wave w takes rows w, w + 4, ...; eight loads in flight per lane, then a
// reduction over the four waves in LDS and one atomic per column and block.
__global__ __launch_bounds__(256) void k_gap_colmax(int64_t rows, int l, const double *__restrict__ Lhat,
                                                    const int32_t *__restrict__ perm, int64_t rows_per_block,
                                                    unsigned long long *__restrict__ maxbits) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  const bool live = c < l;
  const int64_t skip = live ? perm[c] : -1;
  const int cc = live ? c : 0;
  double mx = 0.0;
  for (int64_t rb = r0 + w; rb < r1; rb += 4 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = rb + 4 * u;
      v[u] = (r < r1) ? Lhat[r * l + cc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = rb + 4 * u;
      const double a = fabs(v[u]);
      if (r < r1 && r != skip && a > mx) mx = a;
    }
  }
  red[w][lane] = mx;
  __syncthreads();
  if (w == 0 && live) {
    mx = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
    if (mx > 0.0) atomicMax(&maxbits[c], (unsigned long long)__double_as_longlong(mx));
  }
}

// min over the counted steps of 1 - maxbits[j]; a step counts when it had
// another candidate (rows - j > 1) and a nonzero pivot.  One block.
__global__ __launch_bounds__(256) void k_gap_min(int64_t rows, int l, const double *__restrict__ U,
                                                 const unsigned long long *__restrict__ maxbits,
                                                 double *__restrict__ out) {
  __shared__ double red[256];
  double g = __longlong_as_double(0x7ff0000000000000ll);  // +inf
  for (int j = threadIdx.x; j < l; j += blockDim.x) {
    if (rows - j > 1 && U[(int64_t)j * l + j] != 0.0) {
      const double v = 1.0 - __longlong_as_double((long long)maxbits[j]);
      g = v < g ? v : g;
    }
  }
  red[threadIdx.x] = g;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_store_f64(double *p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

hipError_t launch_pivot_gap(int64_t rows, int l, const double *Lhat, const int32_t *perm, const double *U,
                            unsigned long long *maxbits, double *out, hipStream_t st) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(maxbits), 0u, (int64_t)l * 2, st);
  if (e != hipSuccess) return e;
  // 128 rows per block (32 loads per lane), more for tall matrices so that
  // at most about 1024 blocks meet at each column's atomic
  const int64_t rpb = align_up(std::max<int64_t>(128, ceil_div(rows, 1024)), 32);
  const dim3 grid((unsigned)ceil_div(rows, rpb), (unsigned)ceil_div(l, 64));
  hipLaunchKernelGGL(k_gap_colmax, grid, dim3(256), 0, st, rows, l, Lhat, perm, rpb, maxbits);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_gap_min, dim3(1), dim3(256), 0, st, rows, l, U, maxbits, out);
  return hipGetLastError();
}

hipError_t launch_store_f64(double *p, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_store_f64, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(count, 256)));
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

hipError_t launch_ltilde(int l, const double *Up, double *Lt, hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div((int64_t)l * l, 256)));
  hipLaunchKernelGGL(k_ltilde, dim3(blocks), dim3(256), 0, st, l, Up, Lt);
  return hipGetLastError();
}

hipError_t launch_assemble_u(int l, int64_t n, const double *Up, const double *Lphat,
                             const int32_t *perm_c, double *U, int64_t ldu, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(l, 32));
  hipLaunchKernelGGL(k_assemble_u, grid, dim3(256), 0, st, l, n, Up, Lphat, perm_c, U, ldu);
  return hipGetLastError();
}

hipError_t launch_transpose(int64_t rows, int64_t cols, const double *in, int64_t ldin, double *out,
                            int64_t ldout, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, rows, cols, in, ldin, out, ldout);
  return hipGetLastError();
}

hipError_t launch_copy_rows(int64_t rows, int64_t cols, const double *in, int64_t ldin,
                            double *out, int64_t ldout, hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(rows * cols, 256)));
  hipLaunchKernelGGL(k_copy_rows, dim3(blocks), dim3(256), 0, st, rows, cols, in, ldin, out, ldout);
  return hipGetLastError();
}

hipError_t launch_finalize(rlu_info *info, const int32_t *abort_flag, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, info, abort_flag);
  return hipGetLastError();
}

}  // namespace rlu
