// Inverse Cholesky factor of the Gram matrix of the least-squares product.
//
// B = L_y^+ P A = (Lhat^T Lhat)^{-1} Lhat^T A with Lhat = P^T L_y
// (Corollary 3.2's product through the normal equations).  With
// G = Lhat^T Lhat = L L^T, G^{-1} = L^{-T} L^{-1}; this kernel produces
// L^{-1} (l x l lower).  One block of 1024 threads: a right-looking
// Cholesky with 32-wide panels held in LDS and the trailing update in
// global memory, then the inverse row block by row block:
//   Linv[I][I] = inv(L[I][I]),  Linv[I][0:i0] = -Linv[I][I] (L[I][0:i0] Linv[0:i0][0:i0]).
// A non-positive pivot (G numerically singular) sets RLU_ERR_NUMERIC.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kCT = 1024;
constexpr int kCNB = 32;

__global__ __launch_bounds__(kCT) void k_chol_inv(int l, double *__restrict__ G,
                                                  double *__restrict__ Linv, rlu_info *info) {
  extern __shared__ double P[];  // l x (kCNB + 1)
  __shared__ double D[kCNB][kCNB + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  constexpr int PS = kCNB + 1;
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
      if (tid == 0) {
        double d = P[c * PS + c];
        if (!(d > 0.0)) { s_bad = 1; d = 1.0; }
        P[c * PS + c] = sqrt(d);
      }
      __syncthreads();
      const double piv = P[c * PS + c];
      for (int r = c + 1 + tid; r < rows; r += kCT) P[r * PS + c] /= piv;
      __syncthreads();
      const int w = nbp - c - 1;
      if (w > 0) {
        for (int e = tid; e < (rows - c - 1) * w; e += kCT) {
          const int r = c + 1 + e / w, cc = c + 1 + e % w;
          if (r >= cc) P[r * PS + cc] -= P[r * PS + c] * P[cc * PS + c];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * nbp; e += kCT) {
      const int r = e / nbp, c = e - r * nbp;
      G[(int64_t)(j0 + r) * l + j0 + c] = (r >= c) ? P[r * PS + c] : 0.0;
    }
    const int j1 = j0 + nbp, t = l - j1;
    for (int e = tid; e < t * t; e += kCT) {
      const int i = e / t, k = e - i * t;
      if (k <= i) {
        double acc = G[(int64_t)(j1 + i) * l + j1 + k];
        for (int c = 0; c < nbp; ++c) acc -= P[(i + nbp) * PS + c] * P[(k + nbp) * PS + c];
        G[(int64_t)(j1 + i) * l + j1 + k] = acc;
      }
    }
    __syncthreads();
  }

  // Linv, row block by row block.  G now holds L in its lower triangle.
  for (int i0 = 0; i0 < l; i0 += kCNB) {
    const int nbp = min(kCNB, l - i0);
    if (tid < nbp) {  // column tid of inv(L[I][I])
      const int c = tid;
      for (int r = 0; r < kCNB; ++r) D[r][c] = 0.0;
      for (int r = c; r < nbp; ++r) {
        double acc = (r == c) ? 1.0 : 0.0;
        for (int u = c; u < r; ++u) acc -= G[(int64_t)(i0 + r) * l + i0 + u] * D[u][c];
        D[r][c] = acc / G[(int64_t)(i0 + r) * l + i0 + r];
      }
    }
    __syncthreads();
    for (int col = tid; col < l; col += kCT) {
      if (col >= i0 + nbp) {
        for (int r = 0; r < nbp; ++r) Linv[(int64_t)(i0 + r) * l + col] = 0.0;
      } else if (col >= i0) {
        for (int r = 0; r < nbp; ++r) Linv[(int64_t)(i0 + r) * l + col] = D[r][col - i0];
      } else {
        double tv[kCNB];
#pragma unroll
        for (int r = 0; r < kCNB; ++r) tv[r] = 0.0;
        for (int k = col; k < i0; ++k) {
          const double lk = Linv[(int64_t)k * l + col];
#pragma unroll
          for (int r = 0; r < kCNB; ++r)
            if (r < nbp) tv[r] += G[(int64_t)(i0 + r) * l + k] * lk;
        }
#pragma unroll
        for (int r = 0; r < kCNB; ++r) {
          if (r < nbp) {
            double acc = 0.0;
#pragma unroll
            for (int rp = 0; rp < kCNB; ++rp)
              if (rp <= r) acc += D[r][rp] * tv[rp];
            Linv[(int64_t)(i0 + r) * l + col] = -acc;
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) atomicExch(&info->status, (int)RLU_ERR_NUMERIC);
}

hipError_t launch_chol_inv(int l, double *G, double *Linv, rlu_info *info, hipStream_t st) {
  const size_t lds = (size_t)l * (kCNB + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_chol_inv,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kCT), lds, st, l, G, Linv, info);
  return hipGetLastError();
}

}  // namespace rlu
