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
// Widest panel whose trailing update streams through k_trail_update; 64-wide
// panels (rows held one per thread) keep the MFMA GEMM, which measured faster
// there (2.87 against 2.91 ms per 16384 x 8192 decomposition).
constexpr int kTrailMaxK = 32;

struct GeppKArgs {
  int64_t M;
  int l, R, SSW, HS;  // SSW: words per candidate row; HS: words per header row (>= blocks)
  int j0, nbp;       // this panel: columns [j0, j0 + nbp)
  const double *X;   // source of the panel columns (row major, ldx)
  int64_t ldx;
  double *Lhat;      // M x l, row major
  double *U;         // l x l
  int32_t *perm;     // written after the last panel
  int32_t *ipiv;
  int32_t *posg;     // positions between panel launches (M)
  int32_t *rowAt;    // pivot row of every step (l)
  uint64_t *slots;   // [2][G][SSW] tagged words: each block's candidate row
  uint64_t *hdr;     // [2][kHdrWords][HS] tagged words: the candidates' headers
                     // (both zeroed before the first panel)
  int32_t *abort_flag;
  uint64_t timeout_ticks;
  rlu_info *info;
  int which;
};

// ---- arg-max across a wave --------------------------------------------------
// Candidate order: larger |value|, then smaller position.  Positions of real
// candidates are distinct, so the winner is unique.
template <int CTRL>
__device__ inline int dpp_mov(int v) { return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false); }

template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_mov<CTRL>((int)b), hi = dpp_mov<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ inline double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src), hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Winner of the wave's 64 candidates, in every lane.  The largest value by a
// max reduction (DPP inside 16-lane rows: quad_perm [1,0,3,2], [2,3,0,1],
// row_half_mirror, row_mirror; readlane across the four rows), its lane by
// ballot; only when several lanes hold that value does a min reduction of
// their positions decide.  Values are never NaN (non-finite ones arrive as
// -1).  Must be called with all lanes active.
__device__ inline Cand wave_argmax_dpp(const Cand &c) {
  double m = c.v;
  m = fmax(m, dpp_f64<0xB1>(m));
  m = fmax(m, dpp_f64<0x4E>(m));
  m = fmax(m, dpp_f64<0x141>(m));
  m = fmax(m, dpp_f64<0x140>(m));
  m = fmax(fmax(readlane_d(m, 0), readlane_d(m, 16)), fmax(readlane_d(m, 32), readlane_d(m, 48)));
  const bool top = (c.v == m);
  uint64_t bal = __ballot(top);
  if (__popcll(bal) > 1) {
    int p = top ? c.pos : 0x7fffffff;
    p = min(p, dpp_mov<0xB1>(p));
    p = min(p, dpp_mov<0x4E>(p));
    p = min(p, dpp_mov<0x141>(p));
    p = min(p, dpp_mov<0x140>(p));
    p = min(min(__builtin_amdgcn_readlane(p, 0), __builtin_amdgcn_readlane(p, 16)),
            min(__builtin_amdgcn_readlane(p, 32), __builtin_amdgcn_readlane(p, 48)));
    bal = __ballot(top && c.pos == p);
  }
  const int L = __builtin_ctzll(bal);  // m is some lane's value: bal != 0
  Cand r;
  r.v = m;
  r.pos = __builtin_amdgcn_readlane(c.pos, L);
  r.idx = __builtin_amdgcn_readlane(c.idx, L);
  return r;
}

__device__ inline double pivot_mag(double v) {
  const double a = fabs(v);
  return (a == a && a <= 1.7976931348623157e308) ? a : -1.0;  // non-finite -> -1
}

// Header of a published candidate: |value| (two words), position, row.
// Word w of every block's header sits in row w of a [4][hs] array, so the
// poll's loads (one block per lane) read consecutive words.  Lane w writes
// word w: one store instruction for the header.
__device__ inline void put_header_word(uint64_t *hp, int64_t hs, const Cand &c, int row, uint32_t tag, int w) {
  const uint64_t b = (uint64_t)__double_as_longlong(c.v);
  const uint32_t d = w == 0 ? (uint32_t)b : w == 1 ? (uint32_t)(b >> 32) : w == 2 ? (uint32_t)c.pos : (uint32_t)row;
  tw_put(hp + w * hs, d, tag);
}

template <int RPT, int NB>
__global__ __launch_bounds__(kGeppThreads) void k_gepp_panel(GeppKArgs a) {
  constexpr int NW = kGeppThreads / 64;
  constexpr int kKG = NB < 8 ? NB : 8;  // column group of the uniform skips
  // per-step state, double-buffered by step parity so that two block
  // barriers per step suffice (see the step loop); cvals and cmlt are written
  // and read by one wave between the barriers of a step
  __shared__ Cand s_red[2][NW];
  __shared__ Cand s_win[2];
  __shared__ int s_wrow[2], s_ok[2];
  __shared__ int s_zero, s_nonfinite;
  __shared__ double pvs[2][2 * NB];  // winner's row, shifted: pvs[p][k] = column j + k (zero padded)
  __shared__ __align__(16) double cvals[NB];  // the block winner's row (before this step's update), staged
  __shared__ double cmlt;                     // and its multiplier of this step

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
    const int li = tid + kGeppThreads * q;  // row of the block; candidates carry it as their idx
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

  // Block arg-max of the threads' candidates with one barrier (fence-free:
  // only LDS is exchanged): each wave's winner goes to s_red; after the
  // barrier every wave picks the block's winner from the NW entries, wave 0
  // publishes its header at once, and only the winning wave stages the
  // winner's row in LDS (its owning lane writes it; LDS operations of one wave
  // complete in order) and publishes the values, tagged, one per lane.
  // Other blocks read the values only after they have seen every header, so
  // the staging stays off the exchange's critical path.
  // The staged row is the candidate's row before this step's update, with
  // its multiplier; with pv != nullptr the publishing lanes apply the update
  // (x[k + 1] - mlt pv[k + 1]), which the block's other rows get afterwards.
  auto propose = [&](const Cand &cand, int owner_q, int par, uint64_t *sl, uint64_t *hp, int nvals, uint32_t tag,
                     const double *pv, const double *mltq) __attribute__((always_inline)) {
    const Cand wb = wave_argmax_dpp(cand);
    if (lane == 0) s_red[par][wave] = wb;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    Cand best = s_red[par][0];
    int bw = 0;
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const Cand r = s_red[par][w];
      const bool t = cand_better(r.v, r.pos, best.v, best.pos);
      best.v = t ? r.v : best.v;
      best.pos = t ? r.pos : best.pos;
      best.idx = t ? r.idx : best.idx;
      bw = t ? w : bw;
    }
    if (wave == 0 && lane < kHdrWords) put_header_word(hp, a.HS, best, best.idx >= 0 ? (int)(r0 + best.idx) : -1, tag, lane);
    if (wave == bw && best.idx >= 0) {
      if (tid == best.idx % kGeppThreads) {  // the winning lane stages row owner_q
        double rv[NB];
        double mo = mltq ? mltq[0] : 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) rv[k] = x[0][k];
#pragma unroll
        for (int q = 1; q < RPT; ++q) {
          const bool take = (q == owner_q);
          if (mltq) mo = take ? mltq[q] : mo;
#pragma unroll
          for (int k = 0; k < NB; ++k) rv[k] = take ? x[q][k] : rv[k];
        }
        // only the values the publication reads (indices up to nvals), in
        // groups of kKG under a uniform branch
#pragma unroll
        for (int g0 = 0; g0 < NB; g0 += kKG)
          if (g0 <= nvals) {
#pragma unroll
            for (int k = g0; k < g0 + kKG; k += 2)  // 16-byte stores (NB and kKG are even)
              *reinterpret_cast<double2 *>(&cvals[k]) = make_double2(rv[k], rv[k + 1]);
          }
        cmlt = mo;
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (lane < nvals) {  // nvals <= NB <= 64: one value per lane
        const int ci = min(lane + (pv ? 1 : 0), NB - 1);
        const double cv = cvals[ci];
        tw_put_f64(sl + 2 * lane, pv ? cv - cmlt * pv[ci] : cv, tag);
      }
    }
  };

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
    propose(cand, owner_q, 1, a.slots + ((size_t)(j0 & 1) * G + g) * a.SSW,
            a.hdr + (size_t)(j0 & 1) * kHdrWords * a.HS + g, nbp, (uint32_t)(j0 + 1), nullptr, nullptr);
  }

  // Step c uses buffers [c & 1]: wave 0 fills them before barrier S1(c); the
  // other waves read them after S1(c); the next writes to the same buffers
  // come at step c + 2, after every wave has passed S1(c + 1), hence done
  // with step c.  S2(c) is the barrier inside propose (s_red[c & 1] too);
  // cvals is rewritten at step c + 1 only after S2(c + 1), which every wave
  // reaches after its part of step c's publication.
  for (int c = 0; c < nbp; ++c) {
    const int j = j0 + c, par = c & 1;
    const int rem = nbp - c;  // columns j .. j1-1 still in the panel
    const uint32_t tag = (uint32_t)(j + 1);
    const uint64_t *slp = a.slots + (size_t)(j & 1) * G * a.SSW;
    const uint64_t *hpp = a.hdr + (size_t)(j & 1) * kHdrWords * a.HS;
    if (wave == 0) {  // all headers of step j -> winner (G <= 256: <= 4 slots per lane)
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      uint64_t h0[4] = {0, 0, 0, 0}, h1[4] = {0, 0, 0, 0}, h2[4] = {0, 0, 0, 0}, h3[4] = {0, 0, 0, 0};
      const int ng = (G + 63) >> 6;  // slot groups (uniform)
      int ok = 1;
      for (uint32_t it = 1;; ++it) {
        // every group's loads first (lanes past G load nothing), then the
        // tag checks: a round is one memory round trip at any G
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          if (qq < ng && lane + 64 * qq < G) {
            const uint64_t *hq = hpp + lane + 64 * qq;
            h0[qq] = tw_get(hq);
            h1[qq] = tw_get(hq + a.HS);
            h2[qq] = tw_get(hq + 2 * a.HS);
            h3[qq] = tw_get(hq + 3 * a.HS);
          }
        }
        int ready = 1;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          if (qq < ng)
            ready &= (lane + 64 * qq >= G) | ((tw_tag(h0[qq]) == tag) & (tw_tag(h1[qq]) == tag) &
                                              (tw_tag(h2[qq]) == tag) & (tw_tag(h3[qq]) == tag));
        }
        if (__all(ready)) break;
        if ((it & 255) == 0 && !poll_ok(t0, tmo, a.abort_flag)) { ok = 0; break; }
      }
      Cand best{-3.0, 0x7fffffff, -1};
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int sidx = lane + 64 * qq;
        if (sidx < G) {
          const double v = tw_f64(h0[qq], h1[qq]);
          const int p = (int)tw_data(h2[qq]);
          if (cand_better(v, p, best.v, best.pos)) best = Cand{v, p, sidx};
        }
      }
      best = wave_argmax_dpp(best);
      ok = __all(ok);
      // the winner's row index (header word 3, already read by the lane that
      // polled its slot) and its shifted panel row, one value per lane
      // (rem <= NB <= 64), in a single round of loads
      if (ok) {
        const int wq = best.idx >> 6;
        uint64_t hw = h3[0];
#pragma unroll
        for (int qq = 1; qq < 4; ++qq) hw = (qq == wq) ? h3[qq] : hw;
        const int wrow_read = __builtin_amdgcn_readlane((int)tw_data(hw), best.idx & 63);
        const uint64_t *wsl = slp + (size_t)best.idx * a.SSW;
        double v = 0.0;
        if (lane < rem) {
          uint64_t lo, hi;
          for (uint32_t it = 1;; ++it) {
            lo = tw_get(wsl + 2 * lane);
            hi = tw_get(wsl + 2 * lane + 1);
            if (tw_tag(lo) == tag && tw_tag(hi) == tag) break;
            if ((it & 255) == 0 && !poll_ok(t0, tmo, a.abort_flag)) { ok = 0; break; }
          }
          v = tw_f64(lo, hi);
        }
#pragma unroll
        for (int k = lane; k < 2 * NB; k += 64) pvs[par][k] = (k == lane) ? v : 0.0;
        if (lane == 0) s_wrow[par] = wrow_read;
        ok = __all(ok);
      }
      if (lane == 0) { s_win[par] = best; s_ok[par] = ok; }
    }
    // S1(c), fence-free: wave 0 hands over LDS values only
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (!s_ok[par]) return;
    const Cand win = s_win[par];
    const int wrow = s_wrow[par], wpos = win.pos;
    const bool zero = !(win.v > 0.0);
    const double *pv = pvs[par];
    const double piv = pv[0];

    // positions and multipliers; column j + 1 of every live row first (the
    // next step's candidates), the rest of the shifted update after this
    // block's candidate is published
    const bool next = (c + 1 < nbp);
    Cand cand{-2.0, 0x7fffffff, -1};
    int owner_q = 0, nonfinite = 0;
    double mltq[RPT], x1[RPT];
    bool live[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (row[q] == wrow) pos[q] = j;
      else if (pos[q] == j) pos[q] = wpos;
      live[q] = pos[q] > j;
      mltq[q] = (live[q] && !zero) ? x[q][0] / piv : 0.0;
      x1[q] = x[q][1] - mltq[q] * pv[1];
      if (live[q]) {
        if (next) {
          const double av = pivot_mag(x1[q]);
          nonfinite += (av < 0.0);
          if (cand_better(av, pos[q], cand.v, cand.pos)) { cand = Cand{av, pos[q], tid + kGeppThreads * q}; owner_q = q; }
        }
      }
    }
    if (next)
      propose(cand, owner_q, par, a.slots + ((size_t)((j + 1) & 1) * G + g) * a.SSW,
              a.hdr + (size_t)((j + 1) & 1) * kHdrWords * a.HS + g, rem - 1, tag + 1, pv, mltq);
    if (nonfinite) atomicAdd(&s_nonfinite, nonfinite);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (live[q]) {
        a.Lhat[row[q] * l + j] = mltq[q];
        x[q][0] = x1[q];
        // columns from rem on are zero and stay zero (pv is zero padded):
        // whole groups of kKG columns past rem are skipped (uniform branch)
#pragma unroll
        for (int g0 = 0; g0 < NB; g0 += kKG) {
          if (g0 < rem) {
#pragma unroll
            for (int k = (g0 ? g0 : 1); k < g0 + kKG; ++k) x[q][k] = (k + 1 < NB) ? x[q][k + 1] - mltq[q] * pv[k + 1] : 0.0;
          }
        }
      }
    }
    if (g == 0) {
      if (tid == 0) {
        if (a.ipiv) a.ipiv[j] = wpos;
        a.rowAt[j] = wrow;
        if (zero) ++s_zero;
      }
      double *urow = a.U + (size_t)j * l;
      for (int cc = tid; cc < j1; cc += kGeppThreads) urow[cc] = (cc < j) ? 0.0 : pv[cc - j];
    }
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

// U12 for 64-column panels by blocked substitution on MFMA: with L11 split
// into 16 x 16 blocks L_IJ and D_I = L_II^{-1} (each diagonal block inverted
// once per block by forward substitution, 16 steps), for I = 0 .. 3
//   X_I <- D_I (X_I - sum_{J < I} L_IJ X_J)
// on v_mfma_f64_16x16x4.  Each wave owns 16 of the block's 64 columns, so
// the four phases need no block barrier (a wave reads back only its own
// columns; its LDS operations complete in order).  Rows past the panel's
// nbp carry an identity L11 row and zero data.
typedef double v4d_u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_u12_mfma(int l, int j0, int nbp, const double *__restrict__ Lhat,
                                                  const int32_t *__restrict__ rowAt, const double *__restrict__ X,
                                                  int64_t ldx, double *__restrict__ U) {
  constexpr int NB = 64, P = NB + 4;  // row stride of the LDS tiles
  __shared__ double Ls[NB * P];        // L11 (unit lower; identity past nbp)
  __shared__ double Xs[NB * P];        // the block's 64 columns of X, then of U12
  __shared__ double Ds[4][16][17];     // inverses of the diagonal blocks
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j1 = j0 + nbp, cb = j1 + blockIdx.x * NB;
  // Tile row t = wave + 4 u, column = lane: the row is uniform in the wave,
  // so its pivot row comes from the one rowAt load per lane by readlane and
  // all 32 tile loads of a thread are in flight together (unconditional,
  // from clamped in-range addresses, the out-of-range values zeroed after).
  const int prow = lane < nbp ? rowAt[j0 + lane] : 0;
  const int lc = min(j0 + lane, l - 1), xc = min(cb + lane, l - 1);
  double lv[16], xv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u)
    lv[u] = Lhat[(int64_t)__builtin_amdgcn_readlane(prow, wave + 4 * u) * l + lc];
#pragma unroll
  for (int u = 0; u < 16; ++u)
    xv[u] = X[(int64_t)__builtin_amdgcn_readlane(prow, wave + 4 * u) * ldx + xc];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = wave + 4 * u;
    Ls[t * P + lane] = (t < nbp && lane < t) ? lv[u] : 0.0;
  }
  // the unit diagonal, by the lane that zeroed it (row lane is this wave's)
  if ((lane & 3) == wave) Ls[lane * P + lane] = 1.0;
  __syncthreads();
  if (tid < 64) {  // column c of D_I, I = tid / 16
    const int I = tid >> 4, c = tid & 15;
    double x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double sum = (r == c) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < r; ++u) sum = fma(-Ls[(16 * I + r) * P + 16 * I + u], x[u], sum);
      x[r] = sum;
      Ds[I][r][c] = sum;
    }
  }
  // X's loads were in flight during the inversions
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = wave + 4 * u;
    Xs[t * P + lane] = (t < nbp && cb + lane < l) ? xv[u] : 0.0;
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  const int col = 16 * wave + lr;
#pragma unroll
  for (int I = 0; I < 4; ++I) {
    v4d_u acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = Xs[(16 * I + lk + 4 * v) * P + col];
#pragma unroll
    for (int J = 0; J < I; ++J)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = -Ls[(16 * I + lr) * P + 16 * J + 4 * kk + lk];
        const double b = Xs[(16 * J + 4 * kk + lk) * P + col];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) Xs[(16 * I + lk + 4 * v) * P + col] = acc[v];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the wave's other lanes read these
    v4d_u r = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double a = Ds[I][lr][4 * kk + lk];
      const double b = Xs[(16 * I + 4 * kk + lk) * P + col];
      r = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, r, 0, 0, 0);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int v = 0; v < 4; ++v) Xs[(16 * I + lk + 4 * v) * P + col] = r[v];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
  // U rows j0 .. j1-1, the wave's own columns
  if (cb + col < l) {
    for (int i = lk; i < nbp; i += 4) U[(int64_t)(j0 + i) * l + cb + col] = Xs[i * P + col];
  }
}

// Trailing update of a tall panel, C[M x N] -= L[M x KB] U[KB x N] (the
// product in the same row-major layout as the GEMM's): a rank-KB update is
// a streaming read-modify-write of C with KB flops per byte at most, so
// instead of MFMA tiles, lane j of a wave keeps column j's KB entries of U
// in registers and the wave walks a run of rows, eight at a time; each row's
// KB multipliers are uniform across the wave (scalar loads).
template <int KB>
__global__ __launch_bounds__(256) void k_trail_update(int64_t M, int N, const double *__restrict__ L, int64_t ldl,
                                                      const double *__restrict__ U, int64_t ldu,
                                                      double *__restrict__ C, int64_t ldc, int64_t rows_per_wave) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = blockIdx.y * 64 + lane;
  const bool live = c < N;
  const int cc = live ? c : 0;
  double u[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) u[k] = U[(int64_t)k * ldu + cc];
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * rows_per_wave;
  const int64_t r1 = r0 + rows_per_wave < M ? r0 + rows_per_wave : M;
  constexpr int RB = 8;  // rows per batch: their loads are in flight together
  for (int64_t r = r0; r < r1; r += RB) {
    double cv[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) cv[i] = (r + i < r1) ? C[(r + i) * ldc + cc] : 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      if (r + i < r1) {
        const double *lr = L + (r + i) * ldl;
        // two interleaved partial sums halve the dependent chain
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < KB; k += 2) {
          s0 = __builtin_fma(lr[k], u[k], s0);
          s1 = __builtin_fma(lr[k + 1], u[k + 1], s1);
        }
        cv[i] -= s0 + s1;
      }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if (r + i < r1 && live) C[(r + i) * ldc + c] = cv[i];
  }
}

static hipError_t launch_trail_update(int64_t M, int N, int K, const double *L, int64_t ldl, const double *U,
                                      int64_t ldu, double *C, int64_t ldc, hipStream_t st) {
  // enough waves for about eight per SIMD, runs of whole row batches
  const int64_t rpw = align_up(std::max<int64_t>(8, ceil_div(M, (int64_t)256 * 4 * 8)), 8);
  const dim3 grid((unsigned)ceil_div(M, 4 * rpw), (unsigned)ceil_div(N, 64));
  switch (K) {
    case 8: hipLaunchKernelGGL(k_trail_update<8>, grid, dim3(256), 0, st, M, N, L, ldl, U, ldu, C, ldc, rpw); break;
    case 16: hipLaunchKernelGGL(k_trail_update<16>, grid, dim3(256), 0, st, M, N, L, ldl, U, ldu, C, ldc, rpw); break;
    case 32: hipLaunchKernelGGL(k_trail_update<32>, grid, dim3(256), 0, st, M, N, L, ldl, U, ldu, C, ldc, rpw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
  // about one row per thread where possible, and few enough blocks that the
  // all-to-all exchange stays cheap
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
  plan->slot_stride = (int)align_up(2 * nb, 16);  // words
  plan->lds = 0;
  return true;
}

// header rows: a multiple of 64 words, at least one per block
static int64_t header_stride(const GeppPlan &plan) { return align_up((int64_t)plan.G, 64); }

// exchange words (candidate rows 2 x G x slot_stride, headers 2 x 4 x
// header_stride), positions (rows ints), pivot rows (cols ints), and the
// row-major working copy of the trailing columns when the factorization has
// more than one panel
static size_t exchange_bytes(const GeppPlan &plan) {
  return align_up(((size_t)2 * plan.G * plan.slot_stride + (size_t)2 * kHdrWords * header_stride(plan)) * 8, 256);
}

size_t gepp_workspace_bytes(int64_t rows, int cols, const GeppPlan &plan) {
  size_t b = exchange_bytes(plan);
  b += align_up((size_t)rows * 4, 256) + align_up((size_t)cols * 4, 256);
  if (plan.multi) b += align_up((size_t)rows * cols * 8, 256);
  return b;
}

hipError_t launch_gepp(int64_t rows, int cols, const double *X, int64_t ldx, double *Lhat, double *U,
                       int32_t *perm, int32_t *ipiv, void *ws, int32_t *abort_flag, rlu_info *info,
                       int which, const GeppPlan &plan, bool exclusive, bool x_scratch, hipStream_t st) {
  GeppKernel k = gepp_kernel(64 / plan.nb);
  if (!k) return hipErrorInvalidValue;
  char *w = reinterpret_cast<char *>(ws);
  const size_t slot_bytes = exchange_bytes(plan);
  uint64_t *slots = reinterpret_cast<uint64_t *>(w);
  uint64_t *hdr = slots + (size_t)2 * plan.G * plan.slot_stride;
  int32_t *posg = reinterpret_cast<int32_t *>(w + slot_bytes);
  int32_t *rowAt = reinterpret_cast<int32_t *>(w + slot_bytes + align_up((size_t)rows * 4, 256));
  double *Wk = reinterpret_cast<double *>(w + slot_bytes + align_up((size_t)rows * 4, 256) +
                                          align_up((size_t)cols * 4, 256));
  // the tagged words must start from zero for this factorization
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(slots), 0u, (int64_t)(slot_bytes / 4), st);
  if (e != hipSuccess) return e;
  // the matrix whose trailing columns the updates rewrite: X itself when it
  // is the library's scratch, else a working copy
  double *work = nullptr;
  const double *src = X;
  int64_t ldsrc = ldx;
  if (plan.multi && x_scratch) {
    work = const_cast<double *>(X);
  } else if (plan.multi) {
    if ((e = launch_copy_rows(rows, cols, X, ldx, Wk, cols, st)) != hipSuccess) return e;
    work = Wk;
    src = Wk;
    ldsrc = cols;
  }
  GeppKArgs a;
  a.M = rows;
  a.l = cols;
  a.R = plan.R;
  a.SSW = plan.slot_stride;
  a.HS = (int)header_stride(plan);
  a.ldx = ldsrc;
  a.X = src;
  a.Lhat = Lhat;
  a.U = U;
  a.perm = perm;
  a.ipiv = ipiv;
  a.posg = posg;
  a.rowAt = rowAt;
  a.slots = slots;
  a.hdr = hdr;
  a.abort_flag = abort_flag;
  a.timeout_ticks = 200000000ull;  // 2 s of the 100 MHz counter
  a.info = info;
  a.which = which;
  for (int j0 = 0; j0 < cols; j0 += plan.nb) {
    const int nbp = std::min(plan.nb, cols - j0), j1 = j0 + nbp;
    a.j0 = j0;
    a.nbp = nbp;
    void *args[] = {&a};
    // the blocks wait for each other: co-resident by a cooperative launch, or
    // by the caller's guarantee that nothing else occupies the device
    e = exclusive ? hipLaunchKernel((const void *)k, dim3(plan.G), dim3(kGeppThreads), args, 0, st)
                  : hipLaunchCooperativeKernel((const void *)k, dim3(plan.G), dim3(kGeppThreads), args, 0, st);
    if (e != hipSuccess) return e;
    if (j1 >= cols) break;
    const int J2 = cols - j1;
    const dim3 ug((unsigned)ceil_div(J2, 64));
    switch (plan.nb) {
      case 64: hipLaunchKernelGGL(k_u12_mfma, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 32: hipLaunchKernelGGL(k_u12<32>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 16: hipLaunchKernelGGL(k_u12<16>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      case 8: hipLaunchKernelGGL(k_u12<8>, ug, dim3(256), 0, st, cols, j0, nbp, Lhat, rowAt, src, ldsrc, U); break;
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // trailing update: work[:, j1:] -= Lhat[:, j0:j1] U[j0:j1, j1:]
    if (nbp <= kTrailMaxK) {
      if ((e = launch_trail_update(rows, J2, nbp, Lhat + j0, cols, U + (size_t)j0 * cols + j1, cols, work + j1, ldsrc,
                                   st)) != hipSuccess)
        return e;
      continue;
    }
    GemmArgs gm{};
    gm.M = rows; gm.N = J2; gm.K = nbp;
    gm.A = Lhat + j0; gm.lda = cols; gm.a_dtype = RLU_F64; gm.trans_a = false;
    gm.B = U + (size_t)j0 * cols + j1; gm.ldb = cols;
    gm.C = work + j1; gm.ldc = ldsrc;
    gm.alpha = -1.0; gm.beta = 1.0;
    if ((e = gemm_f64(gm, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rlu
