// Inverse Cholesky factor of the Gram matrix of the least-squares product.
//
// B = L_y^+ P A = (Lhat^T Lhat)^{-1} Lhat^T A with Lhat = P^T L_y
// (Corollary 3.2's product through the normal equations).  With
// G = Lhat^T Lhat = L L^T, G^{-1} = L^{-T} L^{-1}.
//
// k_chol: one block; right-looking Cholesky over 32-column panels held in
//   LDS.  Inside a panel each column is finished Crout-style (its update by
//   the panel's previous columns is a dot product per row, one row per
//   thread), then scaled; the trailing matrix is updated in global memory
//   with 4x4 register tiles.  The inverse of each 32x32 diagonal block is
//   kept for the next kernel.
// k_trinv: one block per column c of L^{-1}; blocked forward substitution
//   x[I] = inv(L[I][I]) (e_c[I] - L[I][0:i0] x[0:i0]) over 32-row blocks.
// A non-positive pivot (G numerically singular) sets RLU_ERR_NUMERIC.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kCT = 256;
constexpr int kCNB = 32;

__global__ __launch_bounds__(kCT) void k_chol(int l, double *__restrict__ G, double *__restrict__ Dinv,
                                              rlu_info *info) {
  extern __shared__ double P[];  // (l) x (kCNB + 1): rows j0.. of the current panel, then l for tcol
  __shared__ double D[kCNB][kCNB + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  constexpr int PS = kCNB + 1;
  double *tcol = P + (size_t)l * PS;
  if (tid == 0) s_bad = 0;

  for (int j0 = 0; j0 < l; j0 += kCNB) {
    const int nbp = min(kCNB, l - j0), rows = l - j0;
    __syncthreads();
    for (int e = tid; e < rows * nbp; e += kCT) {
      const int r = e / nbp, c = e - r * nbp;
      P[r * PS + c] = G[(int64_t)(j0 + r) * l + j0 + c];
    }
    __syncthreads();
    for (int c = 0; c < nbp; ++c) {
      // column c minus its update by the panel's columns 0..c-1 (rows >= c)
      for (int r = c + tid; r < rows; r += kCT) {
        double acc = P[r * PS + c];
        for (int u = 0; u < c; ++u) acc -= P[r * PS + u] * P[c * PS + u];
        tcol[r] = acc;
      }
      __syncthreads();
      double d = tcol[c];
      if (!(d > 0.0)) {
        if (tid == 0) s_bad = 1;
        d = 1.0;
      }
      const double sd = sqrt(d);
      for (int r = c + tid; r < rows; r += kCT) P[r * PS + c] = (r == c) ? sd : tcol[r] / sd;
      __syncthreads();
    }
    // L panel -> G (lower part), zeros above the diagonal of the block
    for (int e = tid; e < rows * nbp; e += kCT) {
      const int r = e / nbp, c = e - r * nbp;
      G[(int64_t)(j0 + r) * l + j0 + c] = (r >= c) ? P[r * PS + c] : 0.0;
    }
    // inverse of the diagonal block (lower): column per thread
    if (tid < nbp) {
      const int c = tid;
      for (int r = 0; r < kCNB; ++r) D[r][c] = 0.0;
      for (int r = c; r < nbp; ++r) {
        double acc = (r == c) ? 1.0 : 0.0;
        for (int u = c; u < r; ++u) acc -= P[r * PS + u] * D[u][c];
        D[r][c] = acc / P[r * PS + r];
      }
    }
    __syncthreads();
    double *dblk = Dinv + (size_t)(j0 / kCNB) * kCNB * kCNB;
    for (int e = tid; e < kCNB * kCNB; e += kCT) dblk[e] = D[e / kCNB][e % kCNB];

    // trailing update of the lower triangle of G[j1:, j1:] with 4x4 tiles
    const int j1 = j0 + nbp, t = l - j1;
    const int tb = (t + 3) / 4;
    const int ntiles = tb * (tb + 1) / 2;
    for (int q = tid; q < ntiles; q += kCT) {
      // q -> (bi, bj) with bj <= bi
      int bi = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
      while (bi * (bi + 1) / 2 > q) --bi;
      const int bj = q - bi * (bi + 1) / 2;
      const int i0 = bi * 4, jb0 = bj * 4;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, jj = jb0 + b;
          acc[a][b] = (i < t && jj <= i) ? G[(int64_t)(j1 + i) * l + j1 + jj] : 0.0;
        }
      for (int c = 0; c < nbp; ++c) {
        double pi[4], pj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          pi[a] = (i0 + a < t) ? P[(nbp + i0 + a) * PS + c] : 0.0;
          pj[a] = (jb0 + a < t) ? P[(nbp + jb0 + a) * PS + c] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] -= pi[a] * pj[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, jj = jb0 + b;
          if (i < t && jj <= i) G[(int64_t)(j1 + i) * l + j1 + jj] = acc[a][b];
        }
    }
  }
  if (tid == 0 && s_bad) atomicExch(&info->status, (int)RLU_ERR_NUMERIC);
}

__global__ __launch_bounds__(256) void k_trinv(int l, const double *__restrict__ L,
                                               const double *__restrict__ Dinv, double *__restrict__ Linv) {
  __shared__ double x[1024];
  __shared__ double tv[kCNB];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int r = tid >> 3, q = tid & 7;
  for (int t = tid; t < l; t += 256) x[t] = 0.0;
  __syncthreads();
  for (int i0 = (c / kCNB) * kCNB; i0 < l; i0 += kCNB) {
    const int nbp = min(kCNB, l - i0);
    double acc = 0.0;
    if (r < nbp)
      for (int u = c + q; u < i0; u += 8) acc += L[(int64_t)(i0 + r) * l + u] * x[u];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    if (q == 0 && r < kCNB) tv[r] = (r < nbp) ? (((i0 + r == c) ? 1.0 : 0.0) - acc) : 0.0;
    __syncthreads();
    if (tid < nbp) {
      const double *dblk = Dinv + (size_t)(i0 / kCNB) * kCNB * kCNB + (size_t)tid * kCNB;
      double s = 0.0;
      for (int rp = 0; rp <= tid; ++rp) s += dblk[rp] * tv[rp];
      x[i0 + tid] = s;
    }
    __syncthreads();
  }
  for (int t = tid; t < l; t += 256) Linv[(int64_t)t * l + c] = (t >= c) ? x[t] : 0.0;
}

size_t chol_scratch_bytes(int l) { return align_up((size_t)ceil_div(l, kCNB) * kCNB * kCNB * 8, 256); }

hipError_t launch_chol_inv(int l, double *G, double *Linv, double *dinv_scratch, rlu_info *info,
                           hipStream_t st) {
  if (l > 1024) return hipErrorInvalidValue;
  const size_t lds = (size_t)l * (kCNB + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCT), lds, st, l, G, dinv_scratch, info);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_trinv, dim3(l), dim3(256), 0, st, l, G, dinv_scratch, Linv);
  return hipGetLastError();
}

}  // namespace rlu
