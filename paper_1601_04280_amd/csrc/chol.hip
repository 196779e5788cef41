// Inverse Cholesky factor of the Gram matrix of the least-squares product.
//
// B = L_y^+ P A = (Lhat^T Lhat)^{-1} Lhat^T A with Lhat = P^T L_y
// (Corollary 3.2's product through the normal equations).  With
// G = Lhat^T Lhat = L L^T, G^{-1} = L^{-T} L^{-1}.
//
// k_chol: one block of 8 waves, G (l x l, lower part) in global memory
//   (L2-resident), right-looking over 16-column panels j0:
//   1. wave 0 factors the 16 x 16 diagonal block, one row per lane, and
//      inverts it through LDS (D = L11^{-1}, kept for k_trinv);
//   2. every thread solves rows of the panel below it, L21 = G21 L11^{-T}
//      (row r: L21[r][c] = sum_{c' <= c} G21[r][c'] D[c][c']), into G and LDS;
//   3. the waves update the lower 16 x 16 tiles of the trailing matrix,
//      G22 -= L21 L21^T, with v_mfma_f64_16x16x4_f64 (K = 16: four steps),
//      eight tiles per wave per round trip to L2.
//   Four barriers per panel.
// k_trinv: one block per column c of L^{-1}; blocked forward substitution
//   x[I] = D_I (e_c[I] - L[I][0:i0] x[0:i0]) over the 16-row blocks I.
// A non-positive pivot (G numerically singular) sets RLU_ERR_NUMERIC.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

typedef double v4d_c __attribute__((ext_vector_type(4)));

constexpr int kCT = 512;  // threads of k_chol
constexpr int kCNB = 16;   // panel width
constexpr int kPS = kCNB + 1;
constexpr int kTG = 8;     // trailing tiles per wave per round trip

__global__ __launch_bounds__(kCT) void k_chol(int l, double *__restrict__ G, double *__restrict__ Dinv,
                                              rlu_info *info) {
  extern __shared__ double P[];  // rows below the diagonal block x 16 (stride kPS): the panel's L21
  __shared__ double D[kCNB][kCNB];
  __shared__ double L11s[kCNB][kCNB + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bad = 0;

  for (int j0 = 0; j0 < l; j0 += kCNB) {
    const int nb = min(kCNB, l - j0);
    const int j1 = j0 + nb, t = l - j1;
    // 1. diagonal block: lane r holds row r of G[j0:j1, j0:j1] (lower part);
    //    the factor goes to G and to L11s (identity rows / columns past nb)
    if (wave == 0) {
      double a[kCNB];
      const int r = lane;
#pragma unroll
      for (int c = 0; c < kCNB; ++c) a[c] = (r < nb && c <= r && c < nb) ? G[(int64_t)(j0 + r) * l + j0 + c] : 0.0;
      int bad = 0;
#pragma unroll
      for (int c = 0; c < kCNB; ++c) {
        if (c < nb) {
          double d = __shfl(a[c], c, 64);  // pivot: row c, column c
          if (!(d > 0.0)) {
            bad = 1;
            d = 1.0;
          }
          const double sq = sqrt(d);
          if (r == c) a[c] = sq;
          else if (r > c) a[c] /= sq;
          // update of the columns right of c: a[r][c'] -= a[r][c] * a[c'][c]
#pragma unroll
          for (int cp = c + 1; cp < kCNB; ++cp) {
            const double lc = __shfl(a[c], cp, 64);  // row cp, column c
            if (r >= cp) a[cp] -= a[c] * lc;
          }
        }
      }
      if (bad && lane == 0) s_bad = 1;
      if (r < kCNB) {
#pragma unroll
        for (int c = 0; c < kCNB; ++c) {
          const double v = (c <= r) ? a[c] : 0.0;
          L11s[r][c] = (r < nb) ? v : (r == c ? 1.0 : 0.0);
          if (r < nb && c < nb) G[(int64_t)(j0 + r) * l + j0 + c] = v;
        }
      }
    }
    __syncthreads();
    if (wave == 0 && lane < kCNB) {  // column `lane` of L11^{-1} by forward substitution
      const int r = lane;
      double x[kCNB];
#pragma unroll
      for (int i = 0; i < kCNB; ++i) {
        double sum = (i == r) ? 1.0 : 0.0;
#pragma unroll
        for (int u = 0; u < i; ++u) sum -= L11s[i][u] * x[u];
        x[i] = (i >= r) ? sum / L11s[i][i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < kCNB; ++i) D[i][r] = (i < nb && r < nb) ? x[i] : 0.0;
    }
    __syncthreads();
    double *dblk = Dinv + (size_t)(j0 / kCNB) * kCNB * kCNB;
    if (tid < kCNB * kCNB) dblk[tid] = D[tid / kCNB][tid % kCNB];

    // 2. L21 = G21 L11^{-T}
    for (int rr = tid; rr < t; rr += kCT) {
      const int64_t row = j1 + rr;
      double g[kCNB];
#pragma unroll
      for (int c = 0; c < kCNB; ++c) g[c] = c < nb ? G[row * l + j0 + c] : 0.0;
#pragma unroll
      for (int c = 0; c < kCNB; ++c) {
        double s = 0.0;
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) s += g[cp] * D[c][cp];
        P[rr * kPS + c] = s;
        if (c < nb) G[row * l + j0 + c] = s;
        __builtin_amdgcn_sched_barrier(0);  // keep D's reads per column: no hoisting of all 136
      }
    }
    __syncthreads();

    // 3. trailing update of the lower tiles: G22 -= L21 L21^T.  Each wave takes
    //    groups of kTG tiles: all their loads first, then the MFMAs, then the
    //    stores, so one L2 round trip is paid per group rather than per tile.
    const int tb = (t + 15) / 16;
    const int ntiles = tb * (tb + 1) / 2;
    for (int q0 = wave * kTG; q0 < ntiles; q0 += (kCT / 64) * kTG) {
      v4d_c acc[kTG];
      int bis[kTG], bjs[kTG];
#pragma unroll
      for (int g = 0; g < kTG; ++g) {
        const int q = min(q0 + g, ntiles - 1);  // past the end: a copy of the last tile, not stored
        int bi = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
        while (bi * (bi + 1) / 2 > q) --bi;
        bis[g] = bi;
        bjs[g] = q - bi * (bi + 1) / 2;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = bis[g] * 16 + (lane >> 4) + 4 * v, j = bjs[g] * 16 + (lane & 15);
          const bool ok = i < t && j < t;
          const double c = G[(int64_t)(j1 + (ok ? i : 0)) * l + j1 + (ok ? j : 0)];
          acc[g][v] = ok ? c : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < kTG; ++g) {
#pragma unroll
        for (int kk = 0; kk < kCNB / 4; ++kk) {
          const int k = kk * 4 + (lane >> 4);
          const int ia = bis[g] * 16 + (lane & 15), jb = bjs[g] * 16 + (lane & 15);
          const double av = ia < t ? -P[ia * kPS + k] : 0.0;
          const double bv = jb < t ? P[jb * kPS + k] : 0.0;
          acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[g], 0, 0, 0);
        }
      }
#pragma unroll
      for (int g = 0; g < kTG; ++g) {
        if (q0 + g < ntiles) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = bis[g] * 16 + (lane >> 4) + 4 * v, j = bjs[g] * 16 + (lane & 15);
            if (i < t && j < t) G[(int64_t)(j1 + i) * l + j1 + j] = acc[g][v];
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) atomicExch(&info->status, (int)RLU_ERR_NUMERIC);
}

// One block per column c of L^{-1}: 16 rows per block step, 16 threads per row.
__global__ __launch_bounds__(256) void k_trinv(int l, const double *__restrict__ L,
                                               const double *__restrict__ Dinv, double *__restrict__ Linv) {
  __shared__ double x[1024];
  __shared__ double tv[kCNB];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int r = tid >> 4, q = tid & 15;
  for (int t = tid; t < l; t += 256) x[t] = 0.0;
  __syncthreads();
  for (int i0 = (c / kCNB) * kCNB; i0 < l; i0 += kCNB) {
    const int nbp = min(kCNB, l - i0);
    double acc = 0.0;
    if (r < nbp)
      for (int u = c + q; u < i0; u += 16) acc += L[(int64_t)(i0 + r) * l + u] * x[u];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 8, 64);
    if (q == 0) tv[r] = (r < nbp) ? (((i0 + r == c) ? 1.0 : 0.0) - acc) : 0.0;
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
  const size_t lds = (size_t)std::max(1, l - 1) * kPS * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCT), lds, st, l, G, dinv_scratch, info);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_trinv, dim3(l), dim3(256), 0, st, l, G, dinv_scratch, Linv);
  return hipGetLastError();
}

}  // namespace rlu
