// LU with partial (row) pivoting of a tall matrix, P X = L U
// (Algorithm 1 step 3; the column-pivoted LU of step 6 runs through this
// code on B^T).
//
// Blocked right-looking, one panel of NB columns at a time:
//   1. k_gepp_panel (cooperative launch) eliminates the panel's columns.
//      Block g owns rows [g R, (g+1) R), RPT rows per thread, and each thread
//      keeps its rows' panel in registers.  Rows never move: positions are
//      tracked (in registers, saved in global memory between panels), and a
//      pivot step exchanges positions (LAPACK ipiv semantics).  Per step the
//      blocks talk once, through tagged 64-bit words (data + step tag in one
//      word, see rlu_device.h), in a double-buffered slot per block:
//        * every block publishes its best candidate (largest magnitude, ties
//          to the smallest position) and that row's remaining panel values;
//        * every block polls all headers until they carry the step's tag,
//          reduces them to the same winner, and reads the winner's row;
//        * every thread scales its rows and updates their remaining panel in
//          registers, and the block publishes the next step's candidate.
//      No read-modify-write atomics and no cache-wide fences sit on this
//      path.  Each row's panel is kept shifted (the current pivot column is
//      always x[0]), so a step is a straight-line x[k] = x[k+1] - m * p[k+1]
//      with static register indices, and the multiplier goes straight to L.
//   2. k_u12: U12 = L11^{-1} X[pivot rows, panel end:], a small triangular
//      solve, four lanes of a wave per column (also the U output rows of the
//      panel).
//   3. the trailing update X[:, panel end:] -= L[:, panel] U12 on the FP64
//      MFMA GEMM.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kGeppThreads = 256;
constexpr int kTrailW = 64;
constexpr int kHdrWords = 4;  // |v| lo, |v| hi, position, row

struct GeppKArgs {
  int64_t M;
  int l, R, SSW;
  int j0, nbp;       // this panel: columns [j0, j0 + nbp)
  const double *X;   // source of the panel columns (row major, ldx)
  int64_t ldx;
  double *Lhat;      // M x l, row major
  double *U;         // l x l
  int32_t *perm;     // written after the last panel
  int32_t *ipiv;
  int32_t *posg;     // positions between panel launches (M)
  int32_t *rowAt;    // pivot row of every step (l)
  uint64_t *slots;   // [2][G][SSW] tagged words, zeroed before the first panel
  int32_t *abort_flag;
  uint64_t timeout_ticks;
  rlu_info *info;
  int which;
};

__device__ inline Cand block_argmax(Cand c, Cand *s_red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  c = wave_argmax(c);
  if (lane == 0) s_red[wave] = c;
  __syncthreads();
  Cand b = s_red[0];
#pragma unroll
  for (int w = 1; w < kGeppThreads / 64; ++w)
    if (cand_better(s_red[w].v, s_red[w].pos, b.v, b.pos)) b = s_red[w];
  __syncthreads();
  return b;
}

__device__ inline double pivot_mag(double v) {
  const double a = fabs(v);
  return (a == a && a <= 1.7976931348623157e308) ? a : -1.0;  // non-finite -> -1
}

// Publish a candidate held in LDS (vals): values and header, all tagged.
__device__ inline void publish(uint64_t *sl, const Cand &c, int row, const double *vals, int nbp,
                               uint32_t tag) {
  for (int cc = threadIdx.x; cc < nbp; cc += kGeppThreads) tw_put_f64(sl + kHdrWords + 2 * cc, vals[cc], tag);
  if (threadIdx.x == 0) {
    const uint64_t b = (uint64_t)__double_as_longlong(c.v);
    tw_put(sl + 0, (uint32_t)b, tag);
    tw_put(sl + 1, (uint32_t)(b >> 32), tag);
    tw_put(sl + 2, (uint32_t)c.pos, tag);
    tw_put(sl + 3, (uint32_t)row, tag);
  }
}

// Block-wide copy of `total` values into LDS: load(e) -> dst(e), with eight
// global loads in flight per thread before any LDS store (a plain strided
// loop would wait for every load in turn).
template <typename LoadF, typename StoreF>
__device__ inline void block_copy(int total, LoadF load, StoreF store) {
  constexpr int B = 8;
  for (int e0 = threadIdx.x; e0 < total; e0 += kGeppThreads * B) {
    double v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + kGeppThreads * u;
      v[u] = (e < total) ? load(e) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + kGeppThreads * u;
      if (e < total) store(e, v[u]);
    }
  }
}

template <int RPT, int NB>
__global__ __launch_bounds__(kGeppThreads) void k_gepp_panel(GeppKArgs a) {
  __shared__ Cand s_red[kGeppThreads / 64];
  __shared__ Cand s_win;
  __shared__ int s_wrow, s_zero, s_nonfinite, s_ok;
  __shared__ double pvs[2 * NB];   // winner's row, shifted: pvs[k] = column j + k (zero padded)
  __shared__ double cvals[NB];     // this block's candidate row, shifted the same way

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l = a.l, j0 = a.j0, nbp = a.nbp, j1 = j0 + nbp;
  const int64_t M = a.M;
  const int64_t r0 = (int64_t)g * a.R;
  const uint64_t tmo = a.timeout_ticks;

  // x[q][k]: column (current step + k) of this thread's row q, updated
  // through the previous step; shifting by one column per step keeps every
  // register index static.
  double x[RPT][NB];
  int pos[RPT];
  int64_t row[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int li = tid + kGeppThreads * q;
    const bool owned = li < a.R && r0 + li < M;
    row[q] = owned ? r0 + li : -1;  // -1 never matches a winner's row
    pos[q] = owned ? (j0 == 0 ? (int)row[q] : a.posg[row[q]]) : -1;  // -1: no row
  }
  if (tid == 0) { s_zero = 0; s_nonfinite = 0; }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const bool live = pos[q] >= j0;
#pragma unroll
    for (int k = 0; k < NB; ++k) x[q][k] = (live && k < nbp) ? a.X[row[q] * a.ldx + j0 + k] : 0.0;
  }
  {  // candidate for the panel's first column
    Cand cand{-2.0, 0x7fffffff, -1};
    int owner_q = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (pos[q] >= j0) {
        const double av = pivot_mag(x[q][0]);
        if (cand_better(av, pos[q], cand.v, cand.pos)) { cand = Cand{av, pos[q], tid + kGeppThreads * q}; owner_q = q; }
      }
    }
    const Cand best = block_argmax(cand, s_red);
    if (best.idx >= 0 && best.idx == cand.idx) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == owner_q)
#pragma unroll
          for (int k = 0; k < NB; ++k) cvals[k] = x[q][k];
    }
    __syncthreads();
    uint64_t *sl = a.slots + ((size_t)(j0 & 1) * G + g) * a.SSW;
    publish(sl, best, best.idx >= 0 ? (int)(r0 + best.idx) : -1, cvals, nbp, (uint32_t)(j0 + 1));
  }

  for (int c = 0; c < nbp; ++c) {
    const int j = j0 + c;
    const int rem = nbp - c;  // columns j .. j1-1 still in the panel
    const uint32_t tag = (uint32_t)(j + 1);
    const uint64_t *slp = a.slots + (size_t)(j & 1) * G * a.SSW;
    if (wave == 0) {  // all headers of step j -> winner (G <= 256: <= 4 slots per lane)
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      uint64_t h0[4], h1[4], h2[4];
      int ok = 1;
      for (uint32_t it = 1;; ++it) {
        int ready = 1;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int s = lane + 64 * qq;
          if (s < G) {
            const uint64_t *sl = slp + (size_t)s * a.SSW;
            h0[qq] = tw_get(sl);
            h1[qq] = tw_get(sl + 1);
            h2[qq] = tw_get(sl + 2);
            ready &= (tw_tag(h0[qq]) == tag) & (tw_tag(h1[qq]) == tag) & (tw_tag(h2[qq]) == tag);
          }
        }
        if (__all(ready)) break;
        if ((it & 255) == 0 && !poll_ok(t0, tmo, a.abort_flag)) { ok = 0; break; }
      }
      Cand best{-3.0, 0x7fffffff, -1};
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int s = lane + 64 * qq;
        if (s < G) {
          const double v = tw_f64(h0[qq], h1[qq]);
          const int p = (int)tw_data(h2[qq]);
          if (cand_better(v, p, best.v, best.pos)) best = Cand{v, p, s};
        }
      }
      best = wave_argmax(best);
      ok = __all(ok);
      // the winner's (shifted) panel row and row index, read by the same wave
      if (ok) {
        const uint64_t *wsl = slp + (size_t)best.idx * a.SSW;
        for (int k = lane; k < 2 * NB; k += 64) {
          double v = 0.0;
          if (k < rem) {
            uint64_t lo, hi;
            for (uint32_t it = 1;; ++it) {
              lo = tw_get(wsl + kHdrWords + 2 * k);
              hi = tw_get(wsl + kHdrWords + 2 * k + 1);
              if (tw_tag(lo) == tag && tw_tag(hi) == tag) break;
              if ((it & 255) == 0 && !poll_ok(t0, tmo, a.abort_flag)) { ok = 0; break; }
            }
            v = tw_f64(lo, hi);
          }
          pvs[k] = v;
        }
        if (lane == 0) {
          uint64_t w3;
          for (uint32_t it = 1;; ++it) {
            w3 = tw_get(wsl + 3);
            if (tw_tag(w3) == tag) break;
            if ((it & 255) == 0 && !poll_ok(t0, tmo, a.abort_flag)) { ok = 0; break; }
          }
          s_wrow = (int)tw_data(w3);
        }
        ok = __all(ok);
      }
      if (lane == 0) { s_win = best; s_ok = ok; }
    }
    __syncthreads();
    if (!s_ok) return;
    const Cand win = s_win;
    const int wrow = s_wrow, wpos = win.pos;
    const bool zero = !(win.v > 0.0);
    const double piv = pvs[0];
    if (g == 0) {
      if (tid == 0) {
        if (a.ipiv) a.ipiv[j] = wpos;
        a.rowAt[j] = wrow;
        if (zero) ++s_zero;
      }
      double *urow = a.U + (size_t)j * l;
      for (int cc = tid; cc < j1; cc += kGeppThreads) urow[cc] = (cc < j) ? 0.0 : pvs[cc - j];
    }

    // positions, multipliers, and the shifted update of the whole panel
    const bool next = (c + 1 < nbp);
    Cand cand{-2.0, 0x7fffffff, -1};
    int owner_q = 0, nonfinite = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (row[q] == wrow) pos[q] = j;
      else if (pos[q] == j) pos[q] = wpos;
      if (pos[q] > j) {
        const double mlt = zero ? 0.0 : x[q][0] / piv;
        a.Lhat[row[q] * l + j] = mlt;
#pragma clang loop unroll(full)
        for (int k = 0; k + 1 < NB; ++k) x[q][k] = x[q][k + 1] - mlt * pvs[k + 1];
        x[q][NB - 1] = 0.0;
        if (next) {
          const double av = pivot_mag(x[q][0]);
          nonfinite += (av < 0.0);
          if (cand_better(av, pos[q], cand.v, cand.pos)) { cand = Cand{av, pos[q], tid + kGeppThreads * q}; owner_q = q; }
        }
      }
    }
    if (nonfinite) atomicAdd(&s_nonfinite, nonfinite);
    if (next) {
      const Cand best = block_argmax(cand, s_red);
      if (best.idx >= 0 && best.idx == cand.idx) {
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == owner_q)
#pragma unroll
            for (int k = 0; k < NB; ++k) cvals[k] = x[q][k];
      }
      __syncthreads();
      uint64_t *sl = a.slots + ((size_t)((j + 1) & 1) * G + g) * a.SSW;
      publish(sl, best, best.idx >= 0 ? (int)(r0 + best.idx) : -1, cvals, rem - 1, tag + 1);
    }
    __syncthreads();
  }

  // L entries of rows pivoted in this panel or before: 1 on the pivot, 0
  // after; positions saved for the next panel, the permutation after the last
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int p = pos[q];
    if (p < 0) continue;
    if (p < j1)
      for (int jj = max(j0, p); jj < j1; ++jj) a.Lhat[row[q] * l + jj] = (jj == p) ? 1.0 : 0.0;
    if (j1 < l) a.posg[row[q]] = p;
    else a.perm[p] = (int32_t)row[q];
  }
  __syncthreads();
  if (tid == 0) {
    if (g == 0 && s_zero) atomicAdd(a.which ? &a.info->zero_pivots_b : &a.info->zero_pivots_y, s_zero);
    if (s_nonfinite) atomicAdd(&a.info->nonfinite, s_nonfinite);
  }
}

// U12 = L11^{-1} X[pivot rows, j1:] for 64 columns per block, four lanes of
// one wave per column: L11 (unit lower, the panel's multipliers on its own
// pivot rows) sits in LDS; lane `part` holds the column's entries 4q + part
// in registers.  Row i's correction is summed in four interleaved partial
// sums, combined with two shuffles, and applied by the lane that owns row i:
// no block barrier inside the substitution.  Also the U output rows
// [j0, j1), columns j1:.
template <int NB>
__global__ __launch_bounds__(256) void k_u12(int l, int j0, int nbp, const double *__restrict__ Lhat,
                                             const int32_t *__restrict__ rowAt, const double *__restrict__ X,
                                             int64_t ldx, double *__restrict__ U) {
  constexpr int Q = NB / 4;
  __shared__ double L11[NB][NB + 1];
  const int tid = threadIdx.x;
  const int j1 = j0 + nbp;
  for (int e = tid; e < NB * NB; e += 256) {
    const int t = e / NB, tp = e - t * NB;
    L11[t][tp] = (t < nbp && tp < t) ? Lhat[(int64_t)rowAt[j0 + t] * l + j0 + tp] : 0.0;
  }
  __syncthreads();
  const int col = tid >> 2, part = tid & 3;
  const int c = j1 + blockIdx.x * 64 + col;
  const bool active = c < l;
  double xs[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = 4 * q + part;
    xs[q] = (active && i < nbp) ? X[(int64_t)rowAt[j0 + i] * ldx + c] : 0.0;
  }
#pragma unroll
  for (int i = 1; i < NB; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q <= (i - 1) / 4; ++q) {
      const int u = 4 * q + part;
      if (u < i) acc += L11[i][u] * xs[q];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (part == (i & 3)) xs[i >> 2] -= acc;
  }
  if (active) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = 4 * q + part;
      if (i < nbp) U[(int64_t)(j0 + i) * l + c] = xs[q];
    }
  }
}

typedef void (*GeppKernel)(GeppKArgs);

static GeppKernel gepp_kernel(int rpt) {
  switch (rpt) {
    case 1: return k_gepp_panel<1, 64>;
    case 2: return k_gepp_panel<2, 32>;
    case 4: return k_gepp_panel<4, 16>;
    case 8: return k_gepp_panel<8, 8>;
    default: return nullptr;
  }
}

bool plan_gepp(int64_t rows, int cols, const DevCaps &caps, GeppPlan *plan, std::string *why) {
  if (rows < cols || cols < 1) { *why = "tall LU needs rows >= cols >= 1"; return false; }
  const int gmax = std::min(256, std::max(1, caps.num_cu));
  // ~256 rows per block (one per thread), and few enough blocks that the
  // all-to-all header exchange stays cheap.
  int64_t G = std::min<int64_t>(gmax, std::max<int64_t>(1, ceil_div(rows, kGeppThreads)));
  int64_t R = ceil_div(rows, G);
  G = ceil_div(rows, R);
  int rpt = 1;
  while (rpt < 8 && (int64_t)rpt * kGeppThreads < R) rpt *= 2;
  if ((int64_t)rpt * kGeppThreads < R) { *why = "matrix too tall for the register-resident panel"; return false; }
  const int nb = 64 / rpt;
  plan->G = (int)G;
  plan->R = (int)R;
  plan->nb = nb;
  plan->multi = cols > nb;
  plan->slot_stride = (int)align_up(kHdrWords + 2 * nb, 16);  // words
  plan->lds = 0;
  return true;
}

// slots (2 x G x slot_stride words), positions (rows ints), pivot rows (cols
// ints), and the row-major working copy of the trailing columns when the
// factorization has more than one panel
size_t gepp_workspace_bytes(int64_t rows, int cols, const GeppPlan &plan) {
  size_t b = align_up((size_t)2 * plan.G * plan.slot_stride * 8, 256);
  b += align_up((size_t)rows * 4, 256) + align_up((size_t)cols * 4, 256);
  if (plan.multi) b += align_up((size_t)rows * cols * 8, 256);
  return b;
}

hipError_t launch_gepp(int64_t rows, int cols, const double *X, int64_t ldx, double *Lhat, double *U,
                       int32_t *perm, int32_t *ipiv, void *ws, int32_t *abort_flag, rlu_info *info,
                       int which, const GeppPlan &plan, hipStream_t st) {
  GeppKernel k = gepp_kernel(64 / plan.nb);
  if (!k) return hipErrorInvalidValue;
  char *w = reinterpret_cast<char *>(ws);
  const size_t slot_bytes = align_up((size_t)2 * plan.G * plan.slot_stride * 8, 256);
  uint64_t *slots = reinterpret_cast<uint64_t *>(w);
  int32_t *posg = reinterpret_cast<int32_t *>(w + slot_bytes);
  int32_t *rowAt = reinterpret_cast<int32_t *>(w + slot_bytes + align_up((size_t)rows * 4, 256));
  double *Wk = reinterpret_cast<double *>(w + slot_bytes + align_up((size_t)rows * 4, 256) +
                                          align_up((size_t)cols * 4, 256));
  // the tagged words must start from zero for this factorization
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(slots), 0u, (int64_t)(slot_bytes / 4), st);
  if (e != hipSuccess) return e;
  const double *src = X;
  int64_t ldsrc = ldx;
  if (plan.multi) {  // trailing columns are updated in place in a working copy
    if ((e = launch_copy_rows(rows, cols, X, ldx, Wk, cols, st)) != hipSuccess) return e;
    src = Wk;
    ldsrc = cols;
  }
  GeppKArgs a;
  a.M = rows;
  a.l = cols;
  a.R = plan.R;
  a.SSW = plan.slot_stride;
  a.ldx = ldsrc;
  a.X = src;
  a.Lhat = Lhat;
  a.U = U;
  a.perm = perm;
  a.ipiv = ipiv;
  a.posg = posg;
  a.rowAt = rowAt;
  a.slots = slots;
  a.abort_flag = abort_flag;
  a.timeout_ticks = 200000000ull;  // 2 s of the 100 MHz counter
  a.info = info;
  a.which = which;
  for (int j0 = 0; j0 < cols; j0 += plan.nb) {
    const int nbp = std::min(plan.nb, cols - j0), j1 = j0 + nbp;
    a.j0 = j0;
    a.nbp = nbp;
    void *args[] = {&a};
    e = hipLaunchCooperativeKernel((const void *)k, dim3(plan.G), dim3(kGeppThreads), args, 0, st);
    if (e != hipSuccess) return e;
    if (j1 >= cols) break;
    const int J2 = cols - j1;
    const dim3 ug((unsigned)ceil_div(J2, 64));
    switch (plan.nb) {
      case 64: hipLaunchKernelGGL(k_u12<64>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 32: hipLaunchKernelGGL(k_u12<32>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 16: hipLaunchKernelGGL(k_u12<16>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 8: hipLaunchKernelGGL(k_u12<8>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // trailing update: Wk[:, j1:] -= Lhat[:, j0:j1] U[j0:j1, j1:]
    GemmArgs gm{};
    gm.M = rows; gm.N = J2; gm.K = nbp;
    gm.A = Lhat + j0; gm.lda = cols; gm.a_dtype = RLU_F64; gm.trans_a = false;
    gm.B = U + (size_t)j0 * cols + j1; gm.ldb = cols;
    gm.C = Wk + j1; gm.ldc = cols;
    gm.alpha = -1.0; gm.beta = 1.0;
    if ((e = gemm_f64(gm, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rlu
