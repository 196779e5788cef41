// LU with partial (row) pivoting of a tall matrix, P X = L U
// (Algorithm 1 step 3; the column-pivoted LU of step 6 runs through this
// kernel on B^T).
//
// One cooperative launch; block g owns rows [g R, (g+1) R) of X and keeps
// them in LDS for the current panel of nb columns.  Rows never move: each
// block tracks the current position of its rows, and a pivot step exchanges
// positions (LAPACK ipiv semantics).  Per elimination step there is exactly
// one device-wide barrier:
//   * every block publishes its best candidate for the step (largest
//     magnitude, ties to the smallest position) together with that row's
//     panel values, in a double-buffered slot;
//   * after the barrier every block reduces the slots to the same winner,
//     scales its rows, updates the next column first, publishes the next
//     step's candidate and arrives, and only then updates the rest of the
//     panel (the update overlaps the barrier).
// Panels narrower than the matrix use a blocked right-looking update:
// U12 = L11^{-1} X12 (L11^{-1} is built row by row during the panel from the
// winners' multipliers) computed cooperatively, one barrier, then each block
// updates its own rows' trailing columns.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kGeppThreads = 256;
constexpr int kTrailW = 64;

struct GeppKArgs {
  int64_t M;
  int l, R, nb, SS, multi;
  const double *X;
  int64_t ldx;
  double *Wk;
  double *Lhat;
  double *U;
  int32_t *perm;
  int32_t *ipiv;
  double *slots;
  GridSync gs;
  rlu_info *info;
  int which;
};

__device__ inline void slot_put_header(double *sl, double v, int pos, int row) {
  sl[0] = v;
  int32_t *ip = reinterpret_cast<int32_t *>(sl + 1);
  ip[0] = pos;
  ip[1] = row;
}
__device__ inline int slot_pos(const double *sl) { return reinterpret_cast<const int32_t *>(sl + 1)[0]; }
__device__ inline int slot_row(const double *sl) { return reinterpret_cast<const int32_t *>(sl + 1)[1]; }

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

__global__ __launch_bounds__(kGeppThreads) void k_gepp(GeppKArgs a) {
  extern __shared__ double lds[];
  __shared__ Cand s_red[kGeppThreads / 64];
  __shared__ Cand s_win;
  __shared__ int s_flag, s_wrow, s_zero, s_nonfinite;

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int l = a.l, nb = a.nb, R = a.R, SS = a.SS, PS = nb + 1;
  const int64_t r0 = (int64_t)g * R;
  const int nr = (int)max((int64_t)0, min((int64_t)R, a.M - r0));
  const bool multi = a.multi != 0;

  double *panel = lds;
  double *Linv = panel + (size_t)R * PS;
  double *Uc = Linv + (multi ? nb * nb : 0);
  double *pivrow = Uc + (multi ? nb * kTrailW : 0);
  double *multL = pivrow + nb;
  int *pos = reinterpret_cast<int *>(multL + R);
  int *rowAt = pos + R;

  for (int i = tid; i < nr; i += kGeppThreads) pos[i] = (int)(r0 + i);
  if (tid == 0) { s_zero = 0; s_nonfinite = 0; }
  uint32_t bar_no = 0;

  for (int j0 = 0; j0 < l; j0 += nb) {
    const int nbp = min(nb, l - j0), j1 = j0 + nbp;
    const double *src = (j0 == 0) ? a.X : a.Wk;
    const int64_t lds_src = (j0 == 0) ? a.ldx : (int64_t)l;
    __syncthreads();
    for (int e = tid; e < nr * nbp; e += kGeppThreads) {
      const int i = e / nbp, c = e - i * nbp;
      if (pos[i] >= j0) panel[i * PS + c] = src[(r0 + i) * lds_src + j0 + c];
    }
    __syncthreads();
    {  // candidate for the panel's first column
      Cand cand{-2.0, 0x7fffffff, -1};
      for (int i = tid; i < nr; i += kGeppThreads) {
        if (pos[i] >= j0) {
          const double av = pivot_mag(panel[i * PS]);
          if (cand_better(av, pos[i], cand.v, cand.pos)) cand = Cand{av, pos[i], i};
        }
      }
      cand = block_argmax(cand, s_red);
      double *sl = a.slots + ((size_t)(j0 & 1) * G + g) * SS;
      if (tid == 0) slot_put_header(sl, cand.v, cand.pos, cand.idx >= 0 ? (int)(r0 + cand.idx) : -1);
      if (cand.idx >= 0)
        for (int c = tid; c < nbp; c += kGeppThreads) sl[4 + c] = panel[cand.idx * PS + c];
      grid_arrive(a.gs);
      ++bar_no;
    }

    for (int c = 0; c < nbp; ++c) {
      const int j = j0 + c;
      if (!grid_wait(a.gs, bar_no, &s_flag)) return;
      const int par = j & 1;
      if (wave == 0) {
        Cand best{-3.0, 0x7fffffff, -1};
        for (int s = lane; s < G; s += 64) {
          const double *sl = a.slots + ((size_t)par * G + s) * SS;
          const double v = sl[0];
          const int p = slot_pos(sl);
          if (cand_better(v, p, best.v, best.pos)) best = Cand{v, p, s};
        }
        best = wave_argmax(best);
        if (lane == 0) s_win = best;
      }
      __syncthreads();
      const Cand win = s_win;
      const double *wsl = a.slots + ((size_t)par * G + win.idx) * SS;
      for (int cc = tid; cc < nbp; cc += kGeppThreads) pivrow[cc] = wsl[4 + cc];
      if (tid == 0) s_wrow = slot_row(wsl);
      __syncthreads();
      const int wrow = s_wrow, wpos = win.pos;
      const bool zero = !(win.v > 0.0);
      const double piv = pivrow[c];
      if (g == 0) {
        if (tid == 0) {
          if (a.ipiv) a.ipiv[j] = wpos;
          if (zero) ++s_zero;
        }
        double *urow = a.U + (size_t)j * l;
        for (int cc = tid; cc < j1; cc += kGeppThreads) urow[cc] = (cc < j) ? 0.0 : pivrow[cc - j0];
      }
      if (tid == 0) rowAt[c] = wrow;
      for (int i = tid; i < nr; i += kGeppThreads) {
        const int p = pos[i];
        if (r0 + i == wrow) pos[i] = j;
        else if (p == j) pos[i] = wpos;
      }
      if (multi) {  // row c of L11^{-1}: Linv[c][t] = -sum_{u=t}^{c-1} L11[c][u] Linv[u][t]
        for (int t = tid; t < nb; t += kGeppThreads) {
          double v;
          if (t < c) {
            double acc = 0.0;
            for (int u = t; u < c; ++u) acc += pivrow[u] * Linv[u * nb + t];
            v = -acc;
          } else {
            v = (t == c) ? 1.0 : 0.0;
          }
          Linv[c * nb + t] = v;
        }
      }
      __syncthreads();

      const bool next = (c + 1 < nbp);
      Cand cand{-2.0, 0x7fffffff, -1};
      int nonfinite = 0;
      for (int i = tid; i < nr; i += kGeppThreads) {
        if (pos[i] > j) {
          const double mlt = zero ? 0.0 : panel[i * PS + c] / piv;
          panel[i * PS + c] = mlt;
          multL[i] = mlt;
          if (next) {
            const double v = panel[i * PS + c + 1] - mlt * pivrow[c + 1];
            panel[i * PS + c + 1] = v;
            const double av = pivot_mag(v);
            nonfinite += (av < 0.0);
            if (cand_better(av, pos[i], cand.v, cand.pos)) cand = Cand{av, pos[i], i};
          }
        } else {
          multL[i] = 0.0;
        }
      }
      if (nonfinite) atomicAdd(&s_nonfinite, nonfinite);
      if (next) {
        cand = block_argmax(cand, s_red);
        double *sl = a.slots + ((size_t)((j + 1) & 1) * G + g) * SS;
        const int ci = cand.idx;
        if (tid == 0) slot_put_header(sl, cand.v, cand.pos, ci >= 0 ? (int)(r0 + ci) : -1);
        if (ci >= 0) {
          const double mc = multL[ci];
          for (int cc = tid; cc < nbp; cc += kGeppThreads) {
            double v = panel[ci * PS + cc];
            if (cc > c + 1) v -= mc * pivrow[cc];
            sl[4 + cc] = v;
          }
        }
        grid_arrive(a.gs);
        ++bar_no;
      } else {
        __syncthreads();
      }
      const int w = nbp - c - 2;
      if (w > 0) {
        for (int e = tid; e < nr * w; e += kGeppThreads) {
          const int i = e / w, cc = c + 2 + (e - i * w);
          if (pos[i] > j) panel[i * PS + cc] -= multL[i] * pivrow[cc];
        }
      }
      __syncthreads();
    }

    // L columns [j0, j1) of every row this block owns
    for (int e = tid; e < nr * nbp; e += kGeppThreads) {
      const int i = e / nbp, c = e - i * nbp, jj = j0 + c, p = pos[i];
      double v;
      if (p < j0) v = 0.0;
      else if (p >= j1) v = panel[i * PS + c];
      else v = (jj < p) ? panel[i * PS + c] : (jj == p ? 1.0 : 0.0);
      a.Lhat[(r0 + i) * l + jj] = v;
    }
    if (!multi || j1 >= l) continue;

    // U12 = L11^{-1} X[pivot rows, j1:], spread over the whole grid
    const int J2 = l - j1;
    for (int64_t e = (int64_t)g * kGeppThreads + tid; e < (int64_t)nbp * J2;
         e += (int64_t)G * kGeppThreads) {
      const int t = (int)(e / J2), cc = j1 + (int)(e - (int64_t)t * J2);
      double acc = 0.0;
      for (int tp = 0; tp <= t; ++tp) acc += Linv[t * nb + tp] * src[(int64_t)rowAt[tp] * lds_src + cc];
      a.U[(size_t)(j0 + t) * l + cc] = acc;
    }
    grid_arrive(a.gs);
    ++bar_no;
    if (!grid_wait(a.gs, bar_no, &s_flag)) return;

    // trailing update of this block's rows that are still unpivoted
    for (int cb = j1; cb < l; cb += kTrailW) {
      const int cw = min(kTrailW, l - cb);
      for (int e = tid; e < nbp * kTrailW; e += kGeppThreads) {
        const int t = e / kTrailW, k = e - t * kTrailW;
        Uc[e] = (k < cw) ? a.U[(size_t)(j0 + t) * l + cb + k] : 0.0;
      }
      __syncthreads();
      const int k = tid & 63;
      if (k < cw) {
        for (int i = tid >> 6; i < nr; i += kGeppThreads / 64) {
          if (pos[i] >= j1) {
            double acc = src[(r0 + i) * lds_src + cb + k];
            for (int t = 0; t < nbp; ++t) acc -= panel[i * PS + t] * Uc[t * kTrailW + k];
            a.Wk[(r0 + i) * l + cb + k] = acc;
          }
        }
      }
      __syncthreads();
    }
  }

  __syncthreads();
  for (int i = tid; i < nr; i += kGeppThreads) a.perm[pos[i]] = (int32_t)(r0 + i);
  if (tid == 0) {
    if (g == 0 && s_zero) atomicAdd(a.which ? &a.info->zero_pivots_b : &a.info->zero_pivots_y, s_zero);
    if (s_nonfinite) atomicAdd(&a.info->nonfinite, s_nonfinite);
  }
}

static size_t gepp_lds_bytes(int R, int nb, bool multi) {
  size_t b = (size_t)R * (nb + 1) * 8;
  if (multi) b += (size_t)nb * nb * 8 + (size_t)nb * kTrailW * 8;
  b += (size_t)nb * 8 + (size_t)R * 8 + (size_t)R * 4 + (size_t)nb * 4;
  return align_up(b, 16);
}

bool plan_gepp(int64_t rows, int cols, const DevCaps &caps, GeppPlan *plan, std::string *why) {
  if (rows < cols || cols < 1) { *why = "tall LU needs rows >= cols >= 1"; return false; }
  const int gmax = std::max(1, caps.num_cu);
  const int64_t rmin = 64;
  int64_t G = std::min<int64_t>(gmax, std::max<int64_t>(1, ceil_div(rows, rmin)));
  int64_t R = ceil_div(rows, G);
  G = ceil_div(rows, R);
  const size_t budget = std::min<size_t>(caps.max_lds, 160 * 1024) - 1024;
  int nb = cols;
  bool multi = false;
  if (gepp_lds_bytes((int)R, cols, false) > budget) {
    multi = true;
    nb = 0;
    for (int cand = std::min(64, cols - 1); cand >= 1; --cand)
      if (gepp_lds_bytes((int)R, cand, true) <= budget) { nb = cand; break; }
    if (nb < 1) { *why = "matrix too tall for the LDS-resident panel"; return false; }
  }
  plan->G = (int)G;
  plan->R = (int)R;
  plan->nb = nb;
  plan->multi = multi;
  plan->slot_stride = (int)align_up(4 + nb, 8);
  plan->lds = gepp_lds_bytes((int)R, nb, multi);
  return true;
}

size_t gepp_workspace_bytes(int64_t rows, int cols, const GeppPlan &plan) {
  (void)rows; (void)cols;
  return align_up((size_t)2 * plan.G * plan.slot_stride * sizeof(double), 256);
}

hipError_t launch_gepp(int64_t rows, int cols, const double *X, int64_t ldx, double *work,
                       double *Lhat, double *U, int32_t *perm, int32_t *ipiv, void *ws,
                       uint32_t *bar_counter, int32_t *abort_flag, rlu_info *info, int which,
                       const GeppPlan &plan, hipStream_t st) {
  GeppKArgs a;
  a.M = rows;
  a.l = cols;
  a.R = plan.R;
  a.nb = plan.nb;
  a.SS = plan.slot_stride;
  a.multi = plan.multi ? 1 : 0;
  a.X = X;
  a.ldx = ldx;
  a.Wk = work;
  a.Lhat = Lhat;
  a.U = U;
  a.perm = perm;
  a.ipiv = ipiv;
  a.slots = reinterpret_cast<double *>(ws);
  a.gs.counter = bar_counter;
  a.gs.abort_flag = abort_flag;
  a.gs.nblocks = (uint32_t)plan.G;
  a.gs.timeout_ticks = 200000000ull;  // 2 s of the 100 MHz counter
  a.info = info;
  a.which = which;
  void *args[] = {&a};
  hipError_t e = hipFuncSetAttribute((const void *)k_gepp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)plan.lds);
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel((const void *)k_gepp, dim3(plan.G), dim3(kGeppThreads), args,
                                    (unsigned)plan.lds, st);
}

int gepp_max_blocks_per_cu(size_t lds) {
  int nblk = 0;
  hipFuncSetAttribute((const void *)k_gepp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, (const void *)k_gepp, kGeppThreads, lds) !=
      hipSuccess)
    return 0;
  return nblk;
}

}  // namespace rlu
