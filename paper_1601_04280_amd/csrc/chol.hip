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

__device__ inline double readlane_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// 1 / sqrt(d) for d > 0: the hardware estimate and two Newton steps
// (y <- y + y (1 - d y^2) / 2), which take it to full double precision.
__device__ inline double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// k_chol_reg: the same right-looking factorization for l <= 256 with the
// whole lower tile triangle held in registers: tile q of the packed lower
// triangle (column-major over 16 x 16 tiles) lives in wave q % 8, slot q / 8,
// in the MFMA accumulator layout (lane: row lane/16 + 4v, column lane%16).
// Per panel p, with no global-memory round trip:
//   A. the owners copy column p's tiles to LDS (diagonal tile to Dg, the
//      rest to P, double-buffered by panel parity);
//   B. wave 0 factors the diagonal block (lane r holds row r; pivots and
//      column entries are broadcast with readlane; reciprocal square roots
//      by refined estimate) and inverts it (D = L11^{-1});
//   C. one thread per row below solves L21 = G21 L11^{-T} into P and G;
//   D. each wave updates its trailing tiles, G22 -= L21 L21^T, by MFMA with
//      operands read from P.
// Three barriers per panel.  L (lower part) and the D blocks are written out
// as in k_chol.
template <int TPW>
__global__ __launch_bounds__(kCT) void k_chol_reg(int l, double *__restrict__ G, double *__restrict__ Dinv,
                                                  rlu_info *info) {
  extern __shared__ double P2[];  // 2 buffers x (l - 16) rows x kPS
  __shared__ double Dg[kCNB][kCNB + 1];
  __shared__ double L11s[kCNB][kCNB + 1];
  __shared__ double D[kCNB][kCNB];
  __shared__ double rinv[kCNB];
  __shared__ int s_bad;
  constexpr int NWv = kCT / 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tb = (l + kCNB - 1) / kCNB;
  const int ntiles = tb * (tb + 1) / 2;
  const int prow = max(1, l - kCNB);  // rows of one P buffer
  if (tid == 0) s_bad = 0;

  int bis[TPW], bjs[TPW];
  v4d_c acc[TPW];
#pragma unroll
  for (int sl = 0; sl < TPW; ++sl) {
    const int q = sl * NWv + wave;
    int bj = -1, bi = -1;
    if (q < ntiles) {  // column-major packed lower triangle: column bj holds tb - bj tiles
      int rest = q;
      bj = 0;
      while (rest >= tb - bj) { rest -= tb - bj; ++bj; }
      bi = bj + rest;
    }
    bis[sl] = bi;
    bjs[sl] = bj;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bi * kCNB + (lane >> 4) + 4 * v, j = bj * kCNB + (lane & 15);
      const bool ok = q < ntiles && i < l && j < l;
      const double c = G[(ok ? i : 0) * l + (ok ? j : 0)];  // l <= 256: 32-bit offsets
      acc[sl][v] = ok ? c : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  for (int p = 0; p < tb; ++p) {
    const int j0 = p * kCNB, nb = min(kCNB, l - j0), j1 = j0 + nb, t = l - j1;
    double *P = P2 + (size_t)(p & 1) * prow * kPS;
    int ln = lane;  // lane, recomputed per panel rather than per-slot values hoisted
    asm volatile("" : "+v"(ln));
    // A. column p's tiles to LDS
#pragma unroll
    for (int sl = 0; sl < TPW; ++sl) {
      if (bjs[sl] == p) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = (ln >> 4) + 4 * v, c = ln & 15;
          if (bis[sl] == p) Dg[r][c] = (r < nb && c < nb) ? acc[sl][v] : (r == c ? 1.0 : 0.0);  // identity padding
          else {
            const int pr = bis[sl] * kCNB + r - j1;
            if (pr < t) P[pr * kPS + c] = acc[sl][v];
          }
        }
      }
    }
    __syncthreads();
    // B. factor and invert the diagonal block (rows past nb: identity),
    //    straight-line: every lane updates all its entries; those right of
    //    the diagonal are never read (pivots and broadcasts read row cp,
    //    column c < cp), and lanes 16..63 repeat rows 0..15 without storing
    if (wave == 0) {
      // opaque to loop-invariant code motion: otherwise every lane mask of
      // the unrolled factorization is hoisted out of the panel loop
      int r = lane;
      asm volatile("" : "+v"(r));
      const int rr = r & (kCNB - 1);
      double a[kCNB];
#pragma unroll
      for (int c = 0; c < kCNB; ++c) a[c] = Dg[rr][c];
      bool bad = false;
      double myrs = 1.0;
#pragma unroll
      for (int c = 0; c < kCNB; ++c) {
        double d = readlane_f64(a[c], c);
        bad |= !(d > 0.0);
        d = (d > 0.0) ? d : 1.0;
        const double rs = rsqrt_f64(d);
        a[c] = (rr == c) ? d * rs : a[c] * rs;
        myrs = (rr == c) ? rs : myrs;
#pragma unroll
        for (int cp = c + 1; cp < kCNB; ++cp) a[cp] = fma(-a[c], readlane_f64(a[c], cp), a[cp]);
      }
      if (bad && lane == 0) s_bad = 1;
      if (r < kCNB) {
        rinv[r] = myrs;
#pragma unroll
        for (int c = 0; c < kCNB; ++c) L11s[r][c] = (c <= r) ? a[c] : 0.0;
        if (r < nb) {
          double *grow = G + (int64_t)(j0 + r) * l + j0;
#pragma unroll
          for (int c = 0; c < kCNB; ++c)
            if (c < nb) grow[c] = (c <= r) ? a[c] : 0.0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (r < kCNB) {  // column r of L11^{-1}; entries above row r come out zero
        double x[kCNB];
#pragma unroll
        for (int i = 0; i < kCNB; ++i) {
          double sum = (i == r) ? 1.0 : 0.0;
#pragma unroll
          for (int u = 0; u < i; ++u) sum = fma(-L11s[i][u], x[u], sum);
          x[i] = sum * rinv[i];
          __builtin_amdgcn_sched_barrier(0);
        }
        double *dblk = Dinv + (size_t)p * kCNB * kCNB;
#pragma unroll
        for (int i = 0; i < kCNB; ++i) {
          D[i][r] = x[i];
          dblk[i * kCNB + r] = x[i];
        }
      }
    }
    __syncthreads();
    // C. L21 = G21 L11^{-T}, one row per thread
    if (tid < t) {
      double g[kCNB];
#pragma unroll
      for (int c = 0; c < kCNB; ++c) g[c] = P[tid * kPS + c];
      double *grow = G + (int64_t)(j1 + tid) * l + j0;
#pragma unroll
      for (int c = 0; c < kCNB; ++c) {
        double s = 0.0;
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) s = fma(g[cp], D[c][cp], s);
        P[tid * kPS + c] = s;
        if (c < nb) grow[c] = s;
        if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // D's reads four columns at a time
      }
    }
    __syncthreads();
    // D. trailing tiles
#pragma unroll
    for (int sl = 0; sl < TPW; ++sl) {
      if (bjs[sl] > p) {
#pragma unroll
        for (int kk = 0; kk < kCNB / 4; ++kk) {
          const int k = kk * 4 + (ln >> 4);
          const int ia = bis[sl] * kCNB + (ln & 15) - j1, jb = bjs[sl] * kCNB + (ln & 15) - j1;
          const double av = ia < t ? -P[ia * kPS + k] : 0.0;
          const double bv = jb < t ? P[jb * kPS + k] : 0.0;
          acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[sl], 0, 0, 0);
        }
      }
      if (sl & 1) __builtin_amdgcn_sched_barrier(0);  // operands two tiles at a time
    }
  }
  __syncthreads();
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

typedef void (*CholRegKernel)(int, double *, double *, rlu_info *);

// tiles per wave for a lower tile triangle of tb x tb tiles (tb <= 16)
static CholRegKernel chol_reg_kernel(int tb) {
  const int per_wave = (tb * (tb + 1) / 2 + 7) / 8;
  if (per_wave <= 4) return k_chol_reg<4>;
  if (per_wave <= 8) return k_chol_reg<8>;
  if (per_wave <= 12) return k_chol_reg<12>;
  if (per_wave <= 14) return k_chol_reg<14>;
  if (per_wave <= 17) return k_chol_reg<17>;
  return nullptr;
}

hipError_t launch_chol_inv(int l, double *G, double *Linv, double *dinv_scratch, rlu_info *info,
                           hipStream_t st) {
  if (l > 1024) return hipErrorInvalidValue;
  hipError_t e;
  const int tb = (l + kCNB - 1) / kCNB;
  if (CholRegKernel k = tb <= 16 ? chol_reg_kernel(tb) : nullptr) {
    const size_t lds = (size_t)2 * std::max(1, l - kCNB) * kPS * sizeof(double);
    if ((e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k, dim3(1), dim3(kCT), lds, st, l, G, dinv_scratch, info);
  } else {
    const size_t lds = (size_t)std::max(1, l - 1) * kPS * sizeof(double);
    if ((e = hipFuncSetAttribute((const void *)k_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCT), lds, st, l, G, dinv_scratch, info);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_trinv, dim3(l), dim3(256), 0, st, l, G, dinv_scratch, Linv);
  return hipGetLastError();
}

}  // namespace rlu
