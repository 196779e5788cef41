// Column selection of the rank-k (truncated) output: the first k pivots of
// the column-pivoted QR of the sketch Y (Businger & Golub 1965; Golub & Van
// Loan, Alg. 5.4.1), taken as pivoted Cholesky of G = Y^T Y, which the FP64
// GEMM forms beforehand.  The problem statement of Section 1 asks for
// factors of rank k (L m x k, U k x n); choosing k columns of the l-column
// sketch by this greedy rule, rather than sketching with k columns, keeps the
// oversampling.
//
// k_colsel: one block; thread i owns column i of Y (l <= 1024): its
// remaining squared norm d_i in a register and column i of the triangular
// factor R (R[t][i], t < k) in global memory, stored Rt[i k + t] so that a
// thread reads its own entries contiguously.  Step j:
//   1. block arg-max of d over the columns not yet chosen: larger d wins,
//      ties go to the smaller current position, and the winner p exchanges
//      positions with the column at position j (LAPACK ipiv semantics);
//   2. r_jj = sqrt(d_p); the winner's r_tp (t < j) are staged in LDS;
//   3. every remaining column i forms r_ji = (G[p][i] - sum_{t<j} r_tp r_ti)
//      / r_jj (t ascending) and d_i -= r_ji^2.
// A step whose best d is not positive (the remaining columns lie in the span
// of the chosen ones) takes its winner by the same rule, sets r_jj = 0,
// updates nothing and is counted in rlu_info.zero_pivots_sel.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void k_colsel(int l, int k, const double *__restrict__ G,
                                                        double *__restrict__ Rt, int32_t *__restrict__ ysel,
                                                        rlu_info *info) {
  __shared__ double s_rp[kMaxL];           // the winner's r_tp, t < j
  __shared__ int32_t s_col_at[kMaxL];      // column at each position
  __shared__ Cand s_wave[kSelThreads / 64];
  __shared__ Cand s_win;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool own = tid < l;
  double d = own ? G[(int64_t)tid * l + tid] : 0.0;
  int pos = tid;  // current position of column tid
  bool chosen = false;
  int zero_steps = 0;
  for (int i = tid; i < l; i += kSelThreads) s_col_at[i] = i;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    Cand c;
    c.v = (own && !chosen) ? (d == d ? d : -__builtin_inf()) : -__builtin_inf();
    c.pos = (own && !chosen) ? pos : 0x7fffffff;
    c.idx = tid;
    c = wave_argmax(c);
    if (lane == 0) s_wave[wave] = c;
    __syncthreads();
    if (wave == 0) {
      Cand w;
      if (lane < kSelThreads / 64) w = s_wave[lane];
      else { w.v = -__builtin_inf(); w.pos = 0x7fffffff; w.idx = 0; }
      w = wave_argmax(w);
      if (lane == 0) s_win = w;
    }
    __syncthreads();
    const Cand w = s_win;
    const int p = w.idx, ppos = w.pos;
    const int displaced = s_col_at[j];  // the column now at position j moves to ppos
    const bool positive = w.v > 0.0;
    const double rjj = positive ? sqrt(w.v) : 0.0;
    if (!positive) ++zero_steps;
    for (int t = tid; t < j; t += kSelThreads) s_rp[t] = Rt[(int64_t)p * k + t];
    __syncthreads();  // s_rp staged; s_col_at[j] read by every thread
    if (tid == 0) {
      s_col_at[ppos] = displaced;
      s_col_at[j] = p;
      ysel[j] = p;
    }
    if (own) {
      if (tid == p) {
        chosen = true;
        pos = j;
        Rt[(int64_t)tid * k + j] = rjj;
      } else {
        if (tid == displaced) pos = ppos;
        if (!chosen) {
          double r = 0.0;
          if (positive) {
            double dot = 0.0;
            const double *ri = Rt + (int64_t)tid * k;
            for (int t = 0; t < j; ++t) dot = fma(s_rp[t], ri[t], dot);
            r = (G[(int64_t)p * l + tid] - dot) / rjj;
            d -= r * r;
          }
          Rt[(int64_t)tid * k + j] = r;
        }
      }
    }
    __syncthreads();  // every Rt entry of step j written before the next step reads it
  }
  if (tid == 0 && zero_steps) atomicAdd(&info->zero_pivots_sel, zero_steps);
}

// Yk[i][q] = Y[i][ysel[q]]  (m x k, ld k)
__global__ void k_gather_cols(int64_t m, int k, const double *__restrict__ Y, int64_t ldy,
                              const int32_t *__restrict__ ysel, double *__restrict__ Yk) {
  const int64_t total = m * (int64_t)k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    const int q = (int)(e - i * k);
    Yk[e] = Y[i * ldy + ysel[q]];
  }
}

hipError_t launch_colsel(int l, int k, const double *G, double *Rt, int32_t *ysel, rlu_info *info, hipStream_t st) {
  if (l < 1 || l > kMaxL || k < 1 || k > l) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colsel, dim3(1), dim3(kSelThreads), 0, st, l, k, G, Rt, ysel, info);
  return hipGetLastError();
}

hipError_t launch_gather_cols(int64_t m, int k, const double *Y, int64_t ldy, const int32_t *ysel, double *Yk,
                              hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(8192, ceil_div(m * (int64_t)k, 256)));
  hipLaunchKernelGGL(k_gather_cols, dim3(blocks), dim3(256), 0, st, m, k, Y, ldy, ysel, Yk);
  return hipGetLastError();
}

}  // namespace rlu
