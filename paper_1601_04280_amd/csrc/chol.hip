// Inverse Cholesky factor of the Gram matrix of the least-squares product.
//
// B = L_y^+ P A = (Lhat^T Lhat)^{-1} Lhat^T A with Lhat = P^T L_y
// (Corollary 3.2's product through the normal equations).  With
// G = Lhat^T Lhat = L L^T, G^{-1} = L^{-T} L^{-1}.
//
// k_chol_reg (l <= 256, or one diagonal panel of a larger G): one block of
//   8 waves with the lower tile triangle in registers, right-looking over
//   16-column panels (details at the kernel).  Larger l: panels of at most
//   256 columns chained through the FP64 GEMM (launch_chol_inv).
// k_trinv: one block per column c of L^{-1}; blocked forward substitution
//   x[I] = D_I (e_c[I] - L[I][0:i0] x[0:i0]) over the 16-row blocks I.
// A non-positive pivot (G numerically singular) sets RLU_ERR_NUMERIC.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

typedef double v4d_c __attribute__((ext_vector_type(4)));

constexpr int kCT = 512;  // threads of k_chol_reg
constexpr int kCNB = 16;   // panel width
constexpr int kPS = kCNB + 1;

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

// k_chol_reg: right-looking factorization of an l x l block (l <= 256, row
// stride ld) with the whole lower tile triangle held in registers: tile q of the packed lower
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
// Three barriers per panel.  L (lower part) goes back to G and the 16 x 16
// diagonal inverses D to Dinv, in panel order, for k_trinv.
template <int TPW>
__global__ __launch_bounds__(kCT) void k_chol_reg(int l, int ld, double *__restrict__ G, double *__restrict__ Dinv,
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
      const double c = G[(ok ? i : 0) * ld + (ok ? j : 0)];  // l <= 256, ld <= 1024: 32-bit offsets
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
          double *grow = G + (int64_t)(j0 + r) * ld + j0;
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
      double *grow = G + (int64_t)(j1 + tid) * ld + j0;
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

// One block per column c of L^{-1} (L: l x l lower, row stride ld; the
// result goes to Linv with the same stride): 16 rows per block step, 16
// threads per row.
__global__ __launch_bounds__(256) void k_trinv(int l, int ld, const double *__restrict__ L,
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
      for (int u = c + q; u < i0; u += 16) acc += L[(int64_t)(i0 + r) * ld + u] * x[u];
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
  for (int t = tid; t < l; t += 256) Linv[(int64_t)t * ld + c] = (t >= c) ? x[t] : 0.0;
}

// Blocked form for l > 256: panels of nb <= 256 columns (equal widths,
// multiples of 16), each factored by k_chol_reg and inverted by k_trinv in
// place, with the panel products on the FP64 GEMM.  G is the full symmetric
// Gram matrix; the trailing updates are applied to whole squares, so the
// block right of a diagonal block stays the transpose of the one below it.
// For panel p (rows and columns J = j0 .. j1 - 1, T = j1 .. l - 1):
//   1. L_JJ = chol(G_JJ) (k_chol_reg), X_JJ = L_JJ^{-1} (k_trinv) into Linv;
//   2. L_TJ^T = X_JJ G_JT, kept in Linv's upper part (free until the end);
//   3. G_TT -= L_TJ L_TJ^T.
// Then the blocks of L^{-1} below the diagonal, row panel by row panel:
//   X_IK = -X_II (sum over panels P < I of L_IP X_PK) for the columns K < I,
// i.e. X_I,<I = -X_II (L^T_<I,I)^T X_<I,<I, and Linv's upper part is cleared.
static int chol_panels(int l) { return l <= 256 ? 1 : (l + 255) / 256; }
static int chol_panel_width(int l) {
  const int P = chol_panels(l);
  return (int)ceil_div(ceil_div(l, P), kCNB) * kCNB;
}

size_t chol_scratch_bytes(int l) {
  size_t b = align_up((size_t)ceil_div(l, kCNB) * kCNB * kCNB * 8, 256);
  if (l > 256) b += align_up((size_t)chol_panel_width(l) * l * 8, 256);  // X_I,<I products
  return b;
}

typedef void (*CholRegKernel)(int, int, double *, double *, rlu_info *);

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

// zeros of Linv right of the diagonal blocks (panels of nb), in columns c0 .. c1 - 1
__global__ void k_clear_upper(int l, int nb, int c0, int c1, double *__restrict__ Linv) {
  const int w = c1 - c0;
  const int64_t total = (int64_t)c0 * w;  // rows above column c0's panel end at most c0
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / w), c = c0 + (int)(e - (int64_t)r * w);
    if (c >= (r / nb + 1) * nb) Linv[(int64_t)r * l + c] = 0.0;
  }
}

static hipError_t chol_reg_launch(int n, int ld, double *G, double *Dinv, rlu_info *info, hipStream_t st) {
  const int tb = (n + kCNB - 1) / kCNB;
  CholRegKernel k = chol_reg_kernel(tb);
  if (!k) return hipErrorInvalidValue;
  const size_t lds = (size_t)2 * std::max(1, n - kCNB) * kPS * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(1), dim3(kCT), lds, st, n, ld, G, Dinv, info);
  return hipGetLastError();
}

hipError_t launch_chol_inv(int l, double *G, double *Linv, double *dinv_scratch, rlu_info *info,
                           hipStream_t st) {
  if (l > 1024) return hipErrorInvalidValue;
  hipError_t e;
  if (l <= 256) {
    if ((e = chol_reg_launch(l, l, G, dinv_scratch, info, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_trinv, dim3(l), dim3(256), 0, st, l, l, G, dinv_scratch, Linv);
    return hipGetLastError();
  }
  const int nbw = chol_panel_width(l);
  double *Tx = dinv_scratch + align_up((size_t)ceil_div(l, kCNB) * kCNB * kCNB * 8, 256) / 8;
  auto gemm = [&](int64_t M, int64_t N, int64_t K, const double *A, bool ta, const double *B, double *C,
                  double alpha, double beta) {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = l; g.a_dtype = RLU_F64; g.trans_a = ta;
    g.B = B; g.ldb = l;
    g.C = C; g.ldc = l; g.alpha = alpha; g.beta = beta;
    g.compute = RLU_F64;
    return gemm_f64(g, st);
  };
  for (int j0 = 0; j0 < l; j0 += nbw) {
    const int nb = std::min(nbw, l - j0), j1 = j0 + nb, t = l - j1;
    double *Gjj = G + (int64_t)j0 * l + j0;
    double *Xjj = Linv + (int64_t)j0 * l + j0;
    double *dblk = dinv_scratch + (size_t)(j0 / kCNB) * kCNB * kCNB;
    if ((e = chol_reg_launch(nb, l, Gjj, dblk, info, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_trinv, dim3(nb), dim3(256), 0, st, nb, l, Gjj, dblk, Xjj);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (t == 0) break;
    double *LTjt = Linv + (int64_t)j0 * l + j1;  // L_TJ^T, in Linv's upper part
    if ((e = gemm(nb, t, nb, Xjj, false, G + (int64_t)j0 * l + j1, LTjt, 1.0, 0.0)) != hipSuccess) return e;
    if ((e = gemm(t, t, nb, LTjt, true, LTjt, G + (int64_t)j1 * l + j1, -1.0, 1.0)) != hipSuccess) return e;
  }
  auto clear = [&](int c0, int c1) {
    hipLaunchKernelGGL(k_clear_upper, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div((int64_t)c0 * (c1 - c0), 256)))),
                       dim3(256), 0, st, l, nbw, c0, c1, Linv);
    return hipGetLastError();
  };
  int i0 = nbw;
  for (; i0 < l; i0 += nbw) {
    const int nb = std::min(nbw, l - i0);
    // the previous column panel's L^T blocks are spent: X_<I,<I is lower triangular
    if ((e = clear(i0 - nbw, i0)) != hipSuccess) return e;
    // Tx (nb x i0) = (L^T_<I,I)^T X_<I,<I, then X_I,<I = -X_II Tx
    if ((e = gemm(nb, i0, i0, Linv + i0, true, Linv, Tx, 1.0, 0.0)) != hipSuccess) return e;
    if ((e = gemm(nb, i0, nb, Linv + (int64_t)i0 * l + i0, false, Tx, Linv + (int64_t)i0 * l, -1.0, 0.0)) !=
        hipSuccess)
      return e;
  }
  return clear(i0 - nbw, l);
}

}  // namespace rlu
