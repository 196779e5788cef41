// The second projection of Algorithm 1 (steps 4-5): Omega_2 = Pi_2 S_2,
// k_2 x m, applied to P A and to L_y along their m rows.
//
// S_2 (an l_2 x m SEM, Section 2.2) sends row i of P A, with sign sgn_2(i),
// into bucket h_2(i).  On the device that is a gather rather than a scatter:
// the rows of each bucket are listed once (k_omega2_lists), and one block per
// (64 buckets x 64 columns) tile sums the listed rows of A, in pivoted order,
// reading every element of A exactly once, then writes its tile transposed:
// Z0^T (cols x l_2), so that each column of S_2 P A is one contiguous row.
// Pi_2 (the SRFT of Section 2.1 down those columns) is then the row sketch
// kernel run on Z0^T with the identity as its SEM and d_2 folded into the
// codes.  For CSR A, Omega_2 P A is instead the CSR sketch kernel run on a
// CSC copy of A (the CSR form of A^T) with Omega_2's codes by row of A.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

constexpr int kListThreads = 1024;
constexpr int kTile = 64;  // buckets and columns of one gather tile

// Bucket lists of S_2 over the m pivoted positions: start[b] .. start[b+1]
// index `list`, whose entries are a position i with bit 31 set when
// sgn_2(i) = -1.  Also the codes of the transform step: code2[j] = j with
// bit 31 set when d_2(j) = -1.  One block; counts, then offsets, then
// placement (in any order within a bucket), all in LDS; with `ordered`, each
// list is then sorted by position (insertion sort, one thread per bucket).
__global__ void __launch_bounds__(kListThreads) k_omega2_lists(int64_t m, int l2, int log2l2, uint64_t key_sem,
                                                               uint64_t key_signs, int32_t *__restrict__ start,
                                                               uint32_t *__restrict__ list,
                                                               uint32_t *__restrict__ code2, int ordered) {
  extern __shared__ uint32_t cnt[];  // l2 counters, then kListThreads / 64 wave totals
  uint32_t *wsum = cnt + l2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = tid; b < l2; b += kListThreads) {
    cnt[b] = 0;
    code2[b] = (uint32_t)b | ((uint32_t)(draw(key_signs, (uint64_t)b) >> 63) << 31);
  }
  __syncthreads();
  for (int64_t i = tid; i < m; i += kListThreads) {
    const uint64_t r = draw(key_sem, (uint64_t)i);
    atomicAdd(&cnt[(uint32_t)(r >> (64 - log2l2))], 1u);
  }
  __syncthreads();
  // exclusive scan of the counts: each thread a run of `per` buckets
  const int per = (l2 + kListThreads - 1) / kListThreads;
  const int b0 = tid * per, b1 = min(l2, b0 + per);
  uint32_t run = 0;
  for (int b = b0; b < b1; ++b) run += cnt[b];
  uint32_t incl = run;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wv; ++w) base += wsum[w];
  uint32_t off = base + incl - run;
  __syncthreads();  // every total read before the counts turn into cursors
  for (int b = b0; b < b1; ++b) {
    const uint32_t c = cnt[b];
    start[b] = (int32_t)off;
    cnt[b] = off;
    off += c;
  }
  if (tid == 0) start[l2] = (int32_t)m;
  __syncthreads();
  for (int64_t i = tid; i < m; i += kListThreads) {
    const uint64_t r = draw(key_sem, (uint64_t)i);
    const uint32_t slot = atomicAdd(&cnt[(uint32_t)(r >> (64 - log2l2))], 1u);
    list[slot] = (uint32_t)i | ((uint32_t)(r & 1u) << 31);
  }
  if (!ordered) return;
  __syncthreads();  // every entry placed (and visible to the block) before the sort
  for (int b = tid; b < l2; b += kListThreads) {
    const int32_t a = start[b], e = start[b + 1];
    for (int32_t p = a + 1; p < e; ++p) {
      const uint32_t x = list[p];
      int32_t q = p - 1;
      while (q >= a && (list[q] & 0x7FFFFFFFu) > (x & 0x7FFFFFFFu)) {
        list[q + 1] = list[q];
        --q;
      }
      list[q + 1] = x;
    }
  }
}

template <typename T>
__device__ inline double load_nt(const T *p) {
  return (double)__builtin_nontemporal_load(p);
}

// Z0^T[c, b] = sum over the list of bucket b of sgn_2(i) X[perm[i], c]:
// S_2 P X, transposed.  Block (bx, by): columns 64 bx .., buckets 64 by ..,
// whose list entries are one contiguous range (the list is grouped by
// bucket).  The block stages that range, kGatherChunk entries at a time, in
// LDS as (row of X, bucket, sign); each wave then takes a contiguous quarter
// of the chunk, lane = column, eight independent row reads in flight, and
// adds each into the tile with an LDS atomic (two waves meet only at a
// bucket their quarters share).  Every element of X is read once overall.
constexpr int kGatherChunk = 1024;
constexpr int kGatherUnroll = 8;

// ORD (RLU_FLAG_DETERMINISTIC, with ordered lists): wave w instead takes the
// tile's buckets 16 w .. 16 w + 15, whose entries are one contiguous range,
// staged 256 at a time in the wave's own quarter of the staging arrays; each
// tile cell is then summed by one lane in list order, with plain LDS adds.
template <typename T, bool ORD>
__global__ void __launch_bounds__(256) k_omega2_gather(int64_t ncols, const T *__restrict__ X, int64_t ldx,
                                                        const int32_t *__restrict__ perm,
                                                        const int32_t *__restrict__ start,
                                                        const uint32_t *__restrict__ list, int l2,
                                                        double *__restrict__ Z0T, int64_t ldz) {
  __shared__ double tile[kTile][kTile + 1];
  __shared__ int32_t ent_row[kGatherChunk];
  __shared__ uint8_t ent_meta[kGatherChunk];  // bucket within the tile | sign << 7
  __shared__ int32_t st_s[kTile + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kTile, b0 = (int64_t)blockIdx.y * kTile;
  const int nb = (int)min<int64_t>(kTile, l2 - b0);
  const int64_t col = c0 + lane;
  const bool cok = col < ncols;
  const T *xc = X + (cok ? col : 0);
  for (int i = tid; i < kTile * (kTile + 1); i += 256) (&tile[0][0])[i] = 0.0;
  if (tid <= nb) st_s[tid] = start[b0 + tid];
  __syncthreads();
  if (ORD) {
    const int bw0 = min(nb, 16 * wv), bw1 = min(nb, 16 * wv + 16);
    const int Ea = st_s[bw0], Eb = st_s[bw1];
    int32_t *er = ent_row + wv * (kGatherChunk / 4);
    uint8_t *em = ent_meta + wv * (kGatherChunk / 4);
    for (int cb = Ea; cb < Eb; cb += kGatherChunk / 4) {
      const int ce = min(kGatherChunk / 4, Eb - cb);
      for (int t = lane; t < ce; t += 64) {
        const uint32_t c = list[cb + t];
        er[t] = perm[c & 0x7FFFFFFFu];
        int lo = bw0, hi = bw1 - 1;  // the last bb with st_s[bb] <= cb + t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (st_s[mid] <= cb + t) lo = mid; else hi = mid - 1;
        }
        em[t] = (uint8_t)(lo | ((c >> 31) << 7));
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the wave's LDS operations complete in order
      for (int e = 0; e < ce; e += kGatherUnroll) {
        double v[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
          const int eu = min(e + u, ce - 1);
          v[u] = cok ? load_nt(xc + (int64_t)er[eu] * ldx) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
          if (e + u < ce) {
            const uint8_t mt = em[e + u];
            tile[mt & 0x7F][lane] += (mt >> 7) ? -v[u] : v[u];
          }
        }
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // read before the next staging overwrites
    }
    __syncthreads();
    const int64_t bo = b0 + lane;
    if (lane < nb) {
      for (int c = wv; c < kTile; c += 4)
        if (c0 + c < ncols) Z0T[(c0 + c) * ldz + bo] = tile[lane][c];
    }
    return;
  }
  const int E0 = st_s[0], E1 = st_s[nb];
  for (int cb = E0; cb < E1; cb += kGatherChunk) {
    const int ce = min(kGatherChunk, E1 - cb);
    for (int t = tid; t < ce; t += 256) {
      const uint32_t c = list[cb + t];
      ent_row[t] = perm[c & 0x7FFFFFFFu];
      // bucket of entry cb + t: the last bb with st_s[bb] <= cb + t
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st_s[mid] <= cb + t) lo = mid; else hi = mid - 1;
      }
      ent_meta[t] = (uint8_t)(lo | ((c >> 31) << 7));
    }
    __syncthreads();
    const int per = (ce + 3) >> 2;
    const int ea = min(ce, wv * per), eb = min(ce, ea + per);
    for (int e = ea; e < eb; e += kGatherUnroll) {
      double v[kGatherUnroll];
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        const int eu = min(e + u, eb - 1);
        v[u] = cok ? load_nt(xc + (int64_t)ent_row[eu] * ldx) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        if (e + u < eb) {
          const uint8_t mt = ent_meta[e + u];
          atomicAdd(&tile[mt & 0x7F][lane], (mt >> 7) ? -v[u] : v[u]);
        }
      }
    }
    __syncthreads();  // the chunk's entries are read before the next chunk is staged
  }
  const int64_t bo = b0 + lane;
  if (lane < nb) {
    for (int c = wv; c < kTile; c += 4)
      if (c0 + c < ncols) Z0T[(c0 + c) * ldz + bo] = tile[lane][c];
  }
}

__global__ void k_omega2_rowcodes(int64_t m, int log2l2, uint64_t key_sem, uint64_t key_signs,
                                  const int32_t *__restrict__ perm, uint32_t *__restrict__ code_row) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r = draw(key_sem, (uint64_t)p);
    const uint32_t b = (uint32_t)(r >> (64 - log2l2));
    const uint32_t neg = (uint32_t)(r & 1u) ^ (uint32_t)(draw(key_signs, b) >> 63);
    code_row[perm[p]] = b | (neg << 31);
  }
}

hipError_t launch_omega2_rowcodes(int64_t m, int l2, uint64_t seed, const int32_t *perm, uint32_t *code_row,
                                  hipStream_t st) {
  if (m < 1 || l2 < 2 || l2 > kMaxS || (l2 & (l2 - 1))) return hipErrorInvalidValue;
  const int blocks = (int)std::min<int64_t>(1024, ceil_div(m, 256));
  hipLaunchKernelGGL(k_omega2_rowcodes, dim3(blocks), dim3(256), 0, st, m, ilog2_exact(l2),
                     stream_key(seed, kStreamSem2), stream_key(seed, kStreamSigns2), perm, code_row);
  return hipGetLastError();
}

hipError_t launch_omega2_lists(int64_t m, int l2, uint64_t seed, int32_t *start, uint32_t *list,
                               uint32_t *code2, bool ordered, hipStream_t st) {
  if (m < 1 || m > INT32_MAX || l2 < 2 || l2 > kMaxS || (l2 & (l2 - 1))) return hipErrorInvalidValue;
  const size_t lds = ((size_t)l2 + kListThreads / 64) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_omega2_lists, dim3(1), dim3(kListThreads), lds, st, m, l2, ilog2_exact(l2),
                     stream_key(seed, kStreamSem2), stream_key(seed, kStreamSigns2), start, list, code2,
                     ordered ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_omega2_gather(int64_t ncols, const void *X, int dtype, int64_t ldx, const int32_t *perm,
                                const int32_t *start, const uint32_t *list, int l2, double *Z0T, int64_t ldz,
                                bool ordered, hipStream_t st) {
  if (ncols < 1 || l2 < 1 || ldz < l2 || ldx < ncols) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ceil_div(ncols, kTile), (unsigned)ceil_div(l2, kTile));
#define RLU_GATHER(T, O)                                                                                      \
  hipLaunchKernelGGL((k_omega2_gather<T, O>), grid, dim3(256), 0, st, ncols, (const T *)X, ldx, perm, start, \
                     list, l2, Z0T, ldz)
  if (dtype == RLU_F64) {
    if (ordered) RLU_GATHER(double, true); else RLU_GATHER(double, false);
  } else {
    if (ordered) RLU_GATHER(float, true); else RLU_GATHER(float, false);
  }
#undef RLU_GATHER
  return hipGetLastError();
}

}  // namespace rlu
