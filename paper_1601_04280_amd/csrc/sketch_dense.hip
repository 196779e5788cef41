// Fused sketch of a dense row-major A (Algorithm 1 step 2):
//   Y[i, :] = ((A[i, :] S^T) diag(d)) T R        (Sections 2.1 and 2.2)
// One block owns one row at a time: the SEM pass accumulates the row into s
// LDS buckets with native LDS FP64 atomics (bucket and folded sign come from
// the column code table), the length-s real transform runs in LDS, and only
// the l selected coordinates are evaluated and written.  Y0 never leaves LDS.
//
// The first PF x 256 entries of the block's next row (and their codes) are
// loaded into registers before the current row's transform, so the row
// stream overlaps the transform; the twiddles and the selection live in LDS
// for that reason (a global load inside the transform would wait for the
// prefetch).  Longer rows stream their remainder 16 loads per thread deep.
#include <type_traits>

#include "fft_lds.h"
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

template <typename T>
__device__ inline double to_f64(T v) { return (double)v; }

// LDS: the transform's two N-complex buffers, four twiddle tables, selection.
static inline int tw_bits(int log2N) { return log2N >> 1; }
static size_t sketch_lds_bytes(int s, int l) {
  const int N = s >> 1, log2N = ilog2_exact(N), b = tw_bits(log2N);
  const int nlo = 1 << b, nhi = N >> b;
  return (size_t)(2 * N + 2 * (nlo + nhi)) * sizeof(double2) + (size_t)l * sizeof(int32_t);
}

// ---- Walsh-Hadamard form of the transform ------------------------------------
// T = H_s / sqrt(s) with H in Sylvester order, H[b][c] = (-1)^popcount(b & c)
// (the subsampled randomized Hadamard transform of the paper's experiments,
// Section 4).  The unnormalised transform in place, in passes of up to four
// butterfly stages held in registers: pass p pairs indices that differ in
// bits 4p .. 4p + 3; a group is the 2^ns indices sharing every other bit.
// The output stays in natural order, so coordinate c is read at position c.
template <typename Idx>
__device__ inline void fwht_group(double *z, int base, int stride, int ns, Idx idx) {
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < (1 << ns)) v[k] = z[idx(base + k * stride)];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t < ns) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (!(k & (1 << t))) {
          const double a = v[k], b = v[k | (1 << t)];
          v[k] = a + b;
          v[k | (1 << t)] = a - b;
        }
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < (1 << ns)) z[idx(base + k * stride)] = v[k];
}

// by one wave over a row buffer of the wave-specialised sketch, value b at
// b + (b >> 4) in this form: the first pass's lanes read 17 doubles apart,
// about two-way LDS bank conflicts (the FFT's layout, b + 2 (b >> 5), puts
// them 16 apart); the wave's LDS operations complete in order, so a pass
// reads what the previous one wrote
__device__ inline int hpad(int b) { return b + (b >> 4); }
__device__ inline void fwht_wave(double *z, int log2s, int ln) {
  const int s = 1 << log2s;
  for (int st0 = 0; st0 < log2s; st0 += 4) {
    const int ns = min(4, log2s - st0);
    for (int gi = ln; gi < (s >> ns); gi += 64) {
      const int base = ((gi >> st0) << (st0 + ns)) + (gi & ((1 << st0) - 1));
      fwht_group(z, base, 1 << st0, ns, [](int b) { return hpad(b); });
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
}

// by a block of TH threads over an unpadded buffer, a barrier after each pass
template <int TH>
__device__ inline void fwht_block(double *z, int log2s, int tid) {
  const int s = 1 << log2s;
  for (int st0 = 0; st0 < log2s; st0 += 4) {
    const int ns = min(4, log2s - st0);
    for (int gi = tid; gi < (s >> ns); gi += TH) {
      const int base = ((gi >> st0) << (st0 + ns)) + (gi & ((1 << st0) - 1));
      fwht_group(z, base, 1 << st0, ns, [](int b) { return b; });
    }
    __syncthreads();
  }
}

template <typename T, int PF>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_dense(
    int64_t m, int64_t n, const T *__restrict__ A, int64_t lda, int s, int log2N, int l,
    const uint32_t *__restrict__ code, const int32_t *__restrict__ sel,
    const double2 *__restrict__ twf, const double2 *__restrict__ twp, double *__restrict__ Y,
    int64_t ldy, int hadamard) {
  extern __shared__ double2 lds2[];
  constexpr int TH = kSketchThreads;
  constexpr int U = 16;
  const int N = s >> 1;
  const int tid = threadIdx.x;
  const double rs = 1.0 / sqrt((double)s);
  const double r2s = sqrt(2.0) * rs;
  double2 *buf = lds2;
  double2 *tab = lds2 + 2 * N;
  const int b = log2N >> 1, nlo = 1 << b, nhi = N >> b;
  int32_t *sel_s = reinterpret_cast<int32_t *>(tab + 2 * (nlo + nhi));
  for (int i = tid; i < nlo; i += TH) {
    tab[i] = twf[i];
    tab[nlo + nhi + i] = twp[i];
  }
  for (int i = tid; i < nhi; i += TH) {
    tab[nlo + i] = twf[i << b];
    tab[2 * nlo + nhi + i] = twp[i << b];
  }
  for (int q = tid; q < l; q += TH) sel_s[q] = sel[q];
  const TwSplit tf{tab, tab + nlo, b, nlo - 1};
  const TwSplit tp{tab + nlo + nhi, tab + 2 * nlo + nhi, b, nlo - 1};

  T pv[PF];
  uint32_t pc[PF];
  auto prefetch = [&](int64_t row) {  // clamped: column 0 stands in past the row's end
    const T *a = A + row * lda;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int64_t j = tid + (int64_t)u * TH;
      const int64_t jj = j < n ? j : 0;
      pv[u] = __builtin_nontemporal_load(a + jj);  // A: read once
      pc[u] = code[jj];
    }
  };

  int64_t row = blockIdx.x;
  if (row < m) prefetch(row);
  for (; row < m; row += gridDim.x) {
    double *y0 = reinterpret_cast<double *>(buf);
    for (int i = tid; i < s; i += TH) y0[i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u)
      if (tid + (int64_t)u * TH < n) atomicAdd(&y0[code_bucket(pc[u])], code_apply(pc[u], to_f64(pv[u])));
    const T *a = A + row * lda;
    int64_t j = (int64_t)PF * TH + tid;
    for (; j + (U - 1) * TH < n; j += U * TH) {
      T v[U];
      uint32_t c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) { v[u] = __builtin_nontemporal_load(a + j + u * TH); c[u] = code[j + u * TH]; }
#pragma unroll
      for (int u = 0; u < U; ++u) atomicAdd(&y0[code_bucket(c[u])], code_apply(c[u], to_f64(v[u])));
    }
    for (; j < n; j += TH) {
      const uint32_t c = code[j];
      atomicAdd(&y0[code_bucket(c)], code_apply(c, to_f64(__builtin_nontemporal_load(a + j))));
    }
    __syncthreads();
    if (row + gridDim.x < m) prefetch(row + gridDim.x);  // in flight during the transform

    double *yrow = Y + row * ldy;
    if (hadamard) {  // in place on the bucket sums, natural order
      fwht_block<TH>(y0, log2N + 1, tid);
      for (int q = tid; q < l; q += TH) yrow[q] = y0[sel_s[q]] * rs;
    } else {
      const double2 *Z = fft_lds<TH>(buf, buf + N, N, log2N, tf);
      for (int q = tid; q < l; q += TH) yrow[q] = real_coord(Z, s, sel_s[q], tp, rs, r2s);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Bucket-ordered form (RLU_FLAG_DETERMINISTIC).  The atomic forms above add a
// row's values into its buckets in whatever order the waves reach LDS, so the
// bucket sums are reproducible only to rounding.  Here every bucket sum is
// formed in ascending column order, as the definition of Section 2.2 lists
// the columns: y0[b] = ((c_j1 A[i, j1] + c_j2 A[i, j2]) + ...), j1 < j2 < ...,
// c_j the folded sign, so the result is the same on every run.
//
// Tables (k_ordered_tables, once per call): the columns are cut into chunks
// of C (a power of two, C <= min(s, 8192)); inside chunk c they are listed by
// bucket, ascending column within a bucket:
//   blist[c C + p] = column - c C, bit 31 set for a negative folded sign;
//   boff[c (s + 1) + b] = start of bucket b's run in blist (absolute index),
//   boff[c (s + 1) + s] = end of the chunk's entries.
// One block per chunk sorts the keys (bucket, column) in LDS (bitonic; the
// keys are distinct, so the order is unique) and finds each bucket's start by
// binary search.
// Kernel: one block per row at a time.  Thread t owns buckets b = t mod TH.
// Per chunk the row's C values are staged in LDS (in the second half of the
// transform's buffer, idle until the transform) and each thread adds its
// buckets' entries in list order; then the transform as in k_sketch_dense.
// ---------------------------------------------------------------------------
constexpr int kOrdThreads = 256;
constexpr int kOrdMaxChunk = 8192;  // 13 bits of column within a chunk
constexpr int kOrdColBits = 13;

int ordered_chunk(int s) { return std::min(s, kOrdMaxChunk); }

__global__ __launch_bounds__(kOrdThreads) void k_ordered_tables(int64_t n, int s, int C,
                                                                const uint32_t *__restrict__ code,
                                                                uint32_t *__restrict__ blist,
                                                                int32_t *__restrict__ boff) {
  extern __shared__ uint32_t key[];  // C keys: bucket << 13 | column within the chunk
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x, j0 = c * (int64_t)C;
  const int len = (int)min<int64_t>(C, n - j0);
  for (int e = tid; e < C; e += kOrdThreads)
    key[e] = e < len ? (code_bucket(code[j0 + e]) << kOrdColBits) | (uint32_t)e : 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= C; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < C; i += kOrdThreads) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = key[i], b = key[ixj];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < len; p += kOrdThreads) {
    const uint32_t e = key[p] & ((1u << kOrdColBits) - 1u);
    blist[j0 + p] = e | (code[j0 + e] & 0x80000000u);
  }
  int32_t *off = boff + c * (int64_t)(s + 1);
  for (int b = tid; b <= s; b += kOrdThreads) {
    int lo = 0, hi = len;  // first p with bucket(key[p]) >= b
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((key[mid] >> kOrdColBits) < (uint32_t)b) lo = mid + 1; else hi = mid;
    }
    off[b] = (int32_t)(j0 + lo);
  }
}

template <typename T>
__global__ __launch_bounds__(kOrdThreads) void k_sketch_ordered(
    int64_t m, int64_t n, const T *__restrict__ A, int64_t lda, int s, int log2N, int l, int C,
    const uint32_t *__restrict__ blist, const int32_t *__restrict__ boff, const int32_t *__restrict__ sel,
    const double2 *__restrict__ twf, const double2 *__restrict__ twp, double *__restrict__ Y, int64_t ldy,
    int hadamard) {
  extern __shared__ double2 lds2[];
  constexpr int TH = kOrdThreads;
  const int N = s >> 1;
  const int tid = threadIdx.x;
  const double rs = 1.0 / sqrt((double)s);
  const double r2s = sqrt(2.0) * rs;
  double2 *buf = lds2;
  double2 *tab = lds2 + 2 * N;
  const int b = log2N >> 1, nlo = 1 << b, nhi = N >> b;
  int32_t *sel_s = reinterpret_cast<int32_t *>(tab + 2 * (nlo + nhi));
  for (int i = tid; i < nlo; i += TH) {
    tab[i] = twf[i];
    tab[nlo + nhi + i] = twp[i];
  }
  for (int i = tid; i < nhi; i += TH) {
    tab[nlo + i] = twf[i << b];
    tab[2 * nlo + nhi + i] = twp[i << b];
  }
  for (int q = tid; q < l; q += TH) sel_s[q] = sel[q];
  const TwSplit tf{tab, tab + nlo, b, nlo - 1};
  const TwSplit tp{tab + nlo + nhi, tab + 2 * nlo + nhi, b, nlo - 1};
  double *y0 = reinterpret_cast<double *>(buf);
  double *chunk = reinterpret_cast<double *>(buf + N);  // C <= s values
  const int64_t nch = (n + C - 1) / C;
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const T *a = A + row * lda;
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t j0 = c * C;
      const int len = (int)min<int64_t>(C, n - j0);
      for (int e = tid; e < len; e += TH) chunk[e] = to_f64(__builtin_nontemporal_load(a + j0 + e));
      __syncthreads();
      const int32_t *off = boff + c * (int64_t)(s + 1);
      for (int bk = tid; bk < s; bk += TH) {
        const int p0 = off[bk], p1 = off[bk + 1];
        double acc = c == 0 ? 0.0 : y0[bk];
        for (int p = p0; p < p1; ++p) {
          const uint32_t e = blist[p];
          const double v = chunk[e & 0x7FFFFFFFu];
          acc += (e >> 31) ? -v : v;
        }
        y0[bk] = acc;
      }
      __syncthreads();  // the chunk is read before the next one lands
    }
    double *yrow = Y + row * ldy;
    if (hadamard) {
      fwht_block<TH>(y0, log2N + 1, tid);
      for (int q = tid; q < l; q += TH) yrow[q] = y0[sel_s[q]] * rs;
    } else {
      const double2 *Z = fft_lds<TH>(buf, buf + N, N, log2N, tf);
      for (int q = tid; q < l; q += TH) yrow[q] = real_coord(Z, s, sel_s[q], tp, rs, r2s);
    }
    __syncthreads();
  }
}

size_t ordered_tables_bytes(int64_t n, int s) {
  const int C = ordered_chunk(s);
  const int64_t nch = (n + C - 1) / C;
  return align_up((size_t)n * 4, 256) + (size_t)nch * (size_t)(s + 1) * 4;
}

hipError_t launch_sketch_ordered(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s, int l,
                                 const uint32_t *code, const int32_t *sel, const double2 *twf, const double2 *twp,
                                 void *tables, double *Y, int64_t ldy, int num_cu, bool hadamard, hipStream_t st) {
  const int C = ordered_chunk(s);
  const int64_t nch = (n + C - 1) / C;
  if (nch > INT32_MAX || n > INT32_MAX) return hipErrorInvalidValue;
  uint32_t *blist = reinterpret_cast<uint32_t *>(tables);
  int32_t *boff = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(tables) + align_up((size_t)n * 4, 256));
  hipLaunchKernelGGL(k_ordered_tables, dim3((unsigned)nch), dim3(kOrdThreads), (size_t)C * 4, st, n, s, C, code,
                     blist, boff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sketch_lds_bytes(s, l);
  const int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (160 * 1024) / lds));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)num_cu * per_cu));
  const int log2N = ilog2_exact(s / 2);
  const int had = hadamard ? 1 : 0;
  if (dtype == RLU_F64)
    hipLaunchKernelGGL(k_sketch_ordered<double>, dim3(grid), dim3(kOrdThreads), lds, st, m, n, (const double *)A,
                       lda, s, log2N, l, C, blist, boff, sel, twf, twp, Y, ldy, had);
  else
    hipLaunchKernelGGL(k_sketch_ordered<float>, dim3(grid), dim3(kOrdThreads), lds, st, m, n, (const float *)A, lda,
                       s, log2N, l, C, blist, boff, sel, twf, twp, Y, ldy, had);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wave-specialised form (s <= 4096, aligned rows whose length is a multiple of
// the vector width): blocks of four waves, four blocks per CU (two at
// s = 4096, whose two row buffers take 70 KB of LDS).  Three waves
// stream row r with 16-byte loads, a chunk of the row in flight per thread,
// and scatter it into LDS buffer r & 1; the fourth meanwhile transforms row
// r - 1 in the other buffer, writes its l coordinates and clears the
// buffer.  One block barrier per row, and the transform (by one wave, in
// place, decimation in frequency, with the split twiddle tables in LDS) is
// off the row stream's critical path.  Where the transform would outlast a
// row's stream, the streaming waves take over the read-out and clearing
// (SPLIT, three barriers per row; see the kernel).
// Complex index i is stored at i + i / 16 (one pad per 16) so that the
// passes' strided accesses spread over the LDS banks.
constexpr int kWsSem = 192;                 // streaming threads (three waves)
constexpr int kWsThreads = kWsSem + 64;     // plus the transform wave: one wave per SIMD
constexpr int kWsMaxN = 2048;               // complex length (s <= 4096; two blocks per CU at s = 4096)

__host__ __device__ inline int padc(int i) { return i + (i >> 4); }

// In-place decimation-in-frequency transform of N <= 2048 complex values by
// one wave (kernel e^{-2 pi i / N}).  Passes of radix 16 while the block size
// M is at least 16, then one pass of radix 8, 4 or 2 for what is left
// (1024 = 16 16 4, 2048 = 16 16 8).  A pass of radix R over blocks of size M = R S computes,
// for each block start g and 0 <= j < S, from a_r = z[g + j + r S]:
//   y_m = (sum_r a_r e^{-2 pi i r m / R}) w^{j m},  w = e^{-2 pi i / M},
// and stores y_m back at z[g + j + m S].  A butterfly reads and writes the
// same positions, so one buffer suffices, and the spectrum comes out in
// digit-reversed order (dif_pos).  A radix-16 pass has N/16 <= 128 butterflies:
// one or two per lane, 16 values in registers each, one LDS round trip per
// pass.
__device__ inline void dft4(double2 &x0, double2 &x1, double2 &x2, double2 &x3) {
  const double2 s02 = cadd(x0, x2), d02 = csub(x0, x2), s13 = cadd(x1, x3), d13 = csub(x1, x3);
  const double2 md13 = make_double2(d13.y, -d13.x);  // -i (x1 - x3)
  x0 = cadd(s02, s13);
  x1 = cadd(d02, md13);
  x2 = csub(s02, s13);
  x3 = csub(d02, md13);
}

// 16-point DFT as 4 x 4: a[r0 + 4 r1] -> DFTs over r1, twiddles
// e^{-2 pi i r0 m1 / 16}, DFTs over r0.  Output m = m1 + 4 m0 lands in
// a[4 m1 + m0].
__device__ inline void dft16(double2 (&a)[16]) {
  constexpr double C8 = 0.92387953251128674, S8 = 0.38268343236508977, R2 = 0.70710678118654752;
#pragma unroll
  for (int r0 = 0; r0 < 4; ++r0) dft4(a[r0], a[r0 + 4], a[r0 + 8], a[r0 + 12]);
  a[1 + 4] = cmul(a[1 + 4], make_double2(C8, -S8));    // w^1
  a[1 + 8] = cmul(a[1 + 8], make_double2(R2, -R2));    // w^2
  a[1 + 12] = cmul(a[1 + 12], make_double2(S8, -C8));  // w^3
  a[2 + 4] = cmul(a[2 + 4], make_double2(R2, -R2));    // w^2
  a[2 + 8] = make_double2(a[2 + 8].y, -a[2 + 8].x);    // w^4 = -i
  a[2 + 12] = cmul(a[2 + 12], make_double2(-R2, -R2)); // w^6
  a[3 + 4] = cmul(a[3 + 4], make_double2(S8, -C8));    // w^3
  a[3 + 8] = cmul(a[3 + 8], make_double2(-R2, -R2));   // w^6
  a[3 + 12] = cmul(a[3 + 12], make_double2(-C8, S8));  // w^9
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) dft4(a[4 * m1], a[4 * m1 + 1], a[4 * m1 + 2], a[4 * m1 + 3]);
}

__device__ inline void fft_wave(double2 *z, int N, const TwSplit &twf, int lane) {
  int M = N;
  for (; M >= 16; M >>= 4) {
    const int S = M >> 4, lS = __builtin_ctz(S);
    for (int bf = lane; bf < (N >> 4); bf += 64) {  // one butterfly per lane (two at N = 2048)
      const int jj = bf & (S - 1), g = (bf >> lS) * M;
      double2 a[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) a[r] = z[padc(g + jj + r * S)];
      const double2 w = twf(jj * (N / M));
      dft16(a);
      double2 pw = w;  // w^m by repeated products: within a few ulp of the table's
#pragma unroll
      for (int m = 1; m < 16; ++m) {
        const int idx = 4 * (m & 3) + (m >> 2);
        a[idx] = cmul(a[idx], pw);
        if (m < 15) pw = cmul(pw, w);
      }
#pragma unroll
      for (int m = 0; m < 16; ++m) z[padc(g + jj + m * S)] = a[4 * (m & 3) + (m >> 2)];
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the next pass reads other lanes' writes
  }
  if (M == 8) {  // radix 8 over blocks of 8 (S = 1: no twiddles), as even and odd 4-point DFTs
    constexpr double R2 = 0.70710678118654752;
    for (int b = lane; b < (N >> 3); b += 64) {
      double2 a[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) a[r] = z[padc(8 * b + r)];
      dft4(a[0], a[2], a[4], a[6]);
      dft4(a[1], a[3], a[5], a[7]);
      const double2 o1 = cmul(a[3], make_double2(R2, -R2));   // w8^1
      const double2 o2 = make_double2(a[5].y, -a[5].x);       // w8^2 = -i
      const double2 o3 = cmul(a[7], make_double2(-R2, -R2));  // w8^3
      z[padc(8 * b)] = cadd(a[0], a[1]);
      z[padc(8 * b + 4)] = csub(a[0], a[1]);
      z[padc(8 * b + 1)] = cadd(a[2], o1);
      z[padc(8 * b + 5)] = csub(a[2], o1);
      z[padc(8 * b + 2)] = cadd(a[4], o2);
      z[padc(8 * b + 6)] = csub(a[4], o2);
      z[padc(8 * b + 3)] = cadd(a[6], o3);
      z[padc(8 * b + 7)] = csub(a[6], o3);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    return;
  }
  if (M == 4) {  // radix 4 over blocks of 4 (S = 1: no twiddles)
    for (int b = lane; b < (N >> 2); b += 64) {
      double2 a0 = z[padc(4 * b)], a1 = z[padc(4 * b + 1)], a2 = z[padc(4 * b + 2)], a3 = z[padc(4 * b + 3)];
      dft4(a0, a1, a2, a3);
      z[padc(4 * b)] = a0;
      z[padc(4 * b + 1)] = a1;
      z[padc(4 * b + 2)] = a2;
      z[padc(4 * b + 3)] = a3;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  } else if (M == 2) {
    for (int b = lane; b < (N >> 1); b += 64) {
      const double2 a0 = z[padc(2 * b)], a1 = z[padc(2 * b + 1)];
      z[padc(2 * b)] = cadd(a0, a1);
      z[padc(2 * b + 1)] = csub(a0, a1);
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
}

// Position of frequency k in the digit-reversed output of fft_wave: k's
// digits, least significant first, in the radices of the passes, weight the
// strides N/16, N/256, ... of those passes.
__host__ __device__ inline int dif_pos(int k, int N) {
  int p = 0, M = N;
  for (; M >= 16; M >>= 4) {
    p += (k & 15) * (M >> 4);
    k >>= 4;
  }
  if (M == 8) return p + (k & 7);
  if (M == 4) p += k & 3;
  else if (M == 2) p += k & 1;
  return p;
}

// Where coordinate f of the real transform reads the digit-reversed padded
// spectrum: positions of Z_g and Z_{N-g}, g, and which formula applies
// (0: f = 0, 1: f = N, 2: f < N, 3: f > N); packed in two ints.
__device__ inline int2 coord_code(int f, int s) {
  const int N = s >> 1;
  const int g = (f == 0 || f == N) ? 0 : (f < N ? f : s - f);
  const int mode = f == 0 ? 0 : (f == N ? 1 : (f < N ? 2 : 3));
  const int p1 = g ? padc(dif_pos(g, N)) : 0, p2 = g ? padc(dif_pos(N - g, N)) : 0;
  return make_int2(p1 | (p2 << 16), g | (mode << 16));
}

__device__ inline double coord_value(const double2 *Z, int2 cd, const TwSplit &twp, double rs, double r2s) {
  const int mode = cd.y >> 16, g = cd.y & 0xFFFF;
  const double2 zg = Z[cd.x & 0xFFFF], zn = Z[cd.x >> 16];
  if (mode < 2) return (mode == 0 ? zg.x + zg.y : zg.x - zg.y) * rs;
  const double er = 0.5 * (zg.x + zn.x), ei = 0.5 * (zg.y - zn.y);
  const double orr = 0.5 * (zg.y + zn.y), oi = -0.5 * (zg.x - zn.x);
  const double2 w = twp(g);
  if (mode == 2) return (er + (w.x * orr - w.y * oi)) * r2s;
  return (ei + (w.x * oi + w.y * orr)) * r2s;
}

template <typename T> struct WsVec;
template <> struct WsVec<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  typedef uint32_t C __attribute__((ext_vector_type(2)));
  static constexpr int kW = 2, kU = 8;
};
template <> struct WsVec<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  typedef uint32_t C __attribute__((ext_vector_type(4)));
  static constexpr int kW = 4, kU = 4;
};

// SPLIT (read-out by the streaming waves): registers for two blocks per CU,
// which is what the LDS of the long transforms that take it allows anyway
template <typename T, int SPLIT>
__global__ __launch_bounds__(kWsThreads, SPLIT ? 2 : 4) void k_sketch_ws(int64_t m, int64_t n, const T *__restrict__ A, int64_t lda,
                                                          int s, int log2N, int l, const uint32_t *__restrict__ code,
                                                          const int32_t *__restrict__ sel,
                                                          const double2 *__restrict__ twf,
                                                          const double2 *__restrict__ twp, double *__restrict__ Y,
                                                          int64_t ldy, uint32_t *__restrict__ next_row, int hadamard) {
  constexpr bool split_out = SPLIT != 0;
  typedef typename WsVec<T>::V VT;
  typedef typename WsVec<T>::C CT;
  constexpr int W = WsVec<T>::kW, U = WsVec<T>::kU;
  constexpr int64_t kChunk = (int64_t)kWsSem * U * W;  // elements per chunk of a row
  extern __shared__ double2 lds2[];
  const int N = s >> 1, NP = padc(N);
  const int tb = log2N >> 1, nlo = 1 << tb, nhi = N >> tb;
  double2 *tab = lds2 + 2 * NP;  // split twiddle tables of twf and twp
  int2 *code_s = reinterpret_cast<int2 *>(tab + 2 * (nlo + nhi));  // per coordinate: coord_code
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < 2 * NP; i += kWsThreads) lds2[i] = make_double2(0.0, 0.0);
  for (int i = tid; i < nlo; i += kWsThreads) {
    tab[i] = twf[i];
    tab[nlo + nhi + i] = twp[i];
  }
  for (int i = tid; i < nhi; i += kWsThreads) {
    tab[nlo + i] = twf[i << tb];
    tab[2 * nlo + nhi + i] = twp[i << tb];
  }
  // per coordinate: its read-out code (the Hadamard form reads position sel[q])
  for (int q = tid; q < l; q += kWsThreads) code_s[q] = hadamard ? make_int2(sel[q], 0) : coord_code(sel[q], s);
  const TwSplit tf{tab, tab + nlo, tb, nlo - 1};
  const TwSplit tp{tab + nlo + nhi, tab + 2 * nlo + nhi, tb, nlo - 1};
  // Rows: the block's first K rows strided by the grid (K G <= 3m/4), then
  // rows from a global counter as blocks go (blocks sharing a CU progress at
  // different rates; one counter for all rows would serialise on its
  // address).  Fetched two ahead into a ring of eight LDS slots: slot
  // (it + 2) & 7 is written in iteration it and read from iteration it + 1
  // on; iteration it reads slots it - 2 .. it + 1.  A block's rows
  // increase, so once a slot holds m or more, all later ones do.
  __shared__ int64_t s_row[8];
  const int64_t G = gridDim.x, K = (m / G) * 3 / 4;
  auto fetch = [&](int64_t j) -> int64_t {
    if (j < K) return (int64_t)blockIdx.x + j * G;
    const int64_t r = K * G + (int64_t)atomicAdd(next_row, 1u);
    return r < m ? r : m;
  };
  if (tid == 0) {
    s_row[0] = fetch(0);
    s_row[1] = s_row[0] < m ? fetch(1) : m;
  }
  __syncthreads();
  const double rs = 1.0 / sqrt((double)s), r2s = sqrt(2.0) * rs;

  // streaming waves: chunks of U vector loads per thread, two register sets
  // (chunk k + 1 is loaded while chunk k is scattered; the next row's first
  // chunk before the row barrier)
  VT va[U], vb[U];
  CT ca[U], cb[U];
  const int64_t nch = (n + kChunk - 1) / kChunk;
  auto load = [&](VT(&v)[U], CT(&c)[U], int64_t row, int64_t k, int tx) __attribute__((always_inline)) {
    const T *aj = A + row * lda + k * kChunk;
    const uint32_t *cj = code + k * kChunk;
    const uint32_t nj = (uint32_t)min<int64_t>(n - k * kChunk, kChunk);
#pragma unroll
    for (int u = 0; u < U; ++u) {  // 32-bit offsets from uniform bases; clamped, masked when scattered
      const uint32_t e = (uint32_t)(u * kWsSem + tx) * W;
      const uint32_t ee = e < nj ? e : 0;
      v[u] = __builtin_nontemporal_load(reinterpret_cast<const VT *>(aj + ee));  // A: read once
      c[u] = *reinterpret_cast<const CT *>(cj + ee);
    }
  };
  auto scatter = [&](const VT(&v)[U], const CT(&c)[U], double *y0, int64_t k, int tx) __attribute__((always_inline)) {
    const uint32_t nj = (uint32_t)min<int64_t>(n - k * kChunk, kChunk);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = (uint32_t)(u * kWsSem + tx) * W;
      if (e < nj) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
          const uint32_t b = code_bucket(c[u][q]);
          atomicAdd(&y0[hadamard ? b + (b >> 4) : b + 2 * (b >> 5)], code_apply(c[u][q], (double)v[u][q]));
        }
      }
    }
  };
  // A row's l coordinates from its transformed buffer z, by nt threads
  // (index t0), UR coordinates per thread at a time with their loads first;
  // then (clear) the buffer zeroed for the next row.
  auto readout = [&](auto ur, double2 *z, int64_t row, int t0, int nt) __attribute__((always_inline)) {
    constexpr int UR = decltype(ur)::value;
    double *yrow = Y + row * ldy;
    if (hadamard) {
      const double *zr = reinterpret_cast<const double *>(z);
      for (int q = t0; q < l; q += nt) yrow[q] = zr[hpad(code_s[q].x)] * rs;
    } else {
      for (int q0 = 0; q0 < l; q0 += UR * nt) {
        int2 cd[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) cd[u] = code_s[min(q0 + t0 + nt * u, l - 1)];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int q = q0 + t0 + nt * u;
          const double v = coord_value(z, cd[u], tp, rs, r2s);
          if (q < l) yrow[q] = v;
        }
      }
    }
  };
  auto clear = [&](double2 *z, int t0, int nt) __attribute__((always_inline)) {
    for (int i = t0; i < NP; i += nt) z[i] = make_double2(0.0, 0.0);
  };
  // The two roles run separate row loops with the same number of block
  // barriers (they read the same slots), one per row, or two with
  // split_out: the roles' registers are never live
  // at the same time.  Thread indices are made opaque to loop-invariant code
  // motion, which would otherwise hoist every lane mask and offset of the
  // unrolled loops out of the row loop (and spill them).
  // Iteration it streams row cur into buffer it & 1 and transforms row prev
  // in buffer (it - 1) & 1.  The transform wave also reads prev's
  // coordinates out and clears its buffer, unless split_out (a transform
  // longer than a row's stream): then the streaming waves do that for row
  // prev2 at the start of the next iteration but one, before they stream
  // into the same buffer, with a barrier after the read-out (the three waves
  // read what the others clear) and one after the clearing: three barriers
  // per row.
  // the transform role rotates with the block index, so that the transform
  // waves of the blocks sharing a CU sit on different SIMDs
  const int fw = (int)(blockIdx.x & 3);
  const int srank = (wave - fw + 3) & 3;  // 0..2 for the streaming waves
  const int sid = srank * 64 + (tid & 63);
  if (wave != fw) {
    if (s_row[0] < m) load(va, ca, s_row[0], 0, sid);
    for (int it = 0;; ++it) {
      const int64_t cur = s_row[it & 7], prev = it ? s_row[(it - 1) & 7] : m;
      const int64_t prev2 = (split_out && it >= 2) ? s_row[(it - 2) & 7] : m;
      if (cur >= m && prev >= m && prev2 >= m) break;
      int tx = sid;
      asm volatile("" : "+v"(tx));
      if (tx == 0) s_row[(it + 2) & 7] = s_row[(it + 1) & 7] < m ? fetch(it + 2) : m;
      if (split_out) {
        double2 *zb = (it & 1) ? lds2 + NP : lds2;
        if (prev2 < m) readout(std::integral_constant<int, 1>(), zb, prev2, tx, kWsSem);
        __syncthreads();
        if (prev2 < m) clear(zb, tx, kWsSem);
        __syncthreads();
      }
      if (cur < m) {  // stream row cur into buffer it & 1
        double *y0 = reinterpret_cast<double *>((it & 1) ? lds2 + NP : lds2);
        for (int64_t k = 0; k < nch; k += 2) {
          if (k + 1 < nch) load(vb, cb, cur, k + 1, tx);
          scatter(va, ca, y0, k, tx);
          if (k + 1 < nch) {
            if (k + 2 < nch) load(va, ca, cur, k + 2, tx);
            scatter(vb, cb, y0, k + 1, tx);
          }
        }
        const int64_t nxt = s_row[(it + 1) & 7];
        if (nxt < m) load(va, ca, nxt, 0, tx);
      }
      __syncthreads();
    }
  } else {
    for (int it = 0;; ++it) {
      const int64_t cur = s_row[it & 7], prev = it ? s_row[(it - 1) & 7] : m;
      const int64_t prev2 = (split_out && it >= 2) ? s_row[(it - 2) & 7] : m;
      if (cur >= m && prev >= m && prev2 >= m) break;
      int tx = tid;
      asm volatile("" : "+v"(tx));
      if (split_out) {
        __syncthreads();
        __syncthreads();
      }
      if (prev < m) {  // transform row prev (buffer (it - 1) & 1)
        double2 *z = ((it - 1) & 1) ? lds2 + NP : lds2;
        const int ln = tx & 63;
        if (hadamard) fwht_wave(reinterpret_cast<double *>(z), log2N + 1, ln);  // in place, natural order
        else fft_wave(z, N, tf, ln);
        if (!split_out) {
          readout(std::integral_constant<int, 4>(), z, prev, ln, 64);
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // one wave: its reads before its clearing
          clear(z, ln, 64);
        }
      }
      __syncthreads();
    }
  }
}

static size_t sketch_ws_lds_bytes(int s, int l) {
  const int N = s >> 1, log2N = ilog2_exact(N), b = tw_bits(log2N);
  return (size_t)(2 * padc(N) + 2 * ((1 << b) + (N >> b))) * sizeof(double2) + (size_t)l * sizeof(int2);
}

template <typename T>
static void launch_pf(int pf, dim3 grid, size_t lds, hipStream_t st, int64_t m, int64_t n, const T *A,
                      int64_t lda, int s, int log2N, int l, const uint32_t *code, const int32_t *sel,
                      const double2 *twf, const double2 *twp, double *Y, int64_t ldy, int hadamard) {
  switch (pf) {
#define RLU_PF(P)                                                                                           \
  case P:                                                                                                   \
    hipLaunchKernelGGL((k_sketch_dense<T, P>), grid, dim3(kSketchThreads), lds, st, m, n, A, lda, s, log2N, \
                       l, code, sel, twf, twp, Y, ldy, hadamard);                                           \
    break;
    RLU_PF(4) RLU_PF(8) RLU_PF(16)
#undef RLU_PF
    default: break;
  }
}

hipError_t launch_sketch_dense(int64_t m, int64_t n, const void *A, int dtype, int64_t lda, int s,
                               int l, const uint32_t *code, const int32_t *sel,
                               const double2 *twf, const double2 *twp, double *Y, int64_t ldy,
                               uint32_t *row_counter, int num_cu, bool hadamard, hipStream_t st) {
  const int W = dtype == RLU_F64 ? 2 : 4;
  const int had = hadamard ? 1 : 0;
  if (s >= 8 && s <= 2 * kWsMaxN && n % W == 0 && lda % W == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
      l <= 1024) {
    const size_t lds = sketch_ws_lds_bytes(s, l);
    // blocks per CU as the runtime resolves them (registers, LDS and its
    // allocation granularity): a grid of resident blocks, each taking every
    // grid-th row, with no second round of blocks
    // the read-out goes to the streaming waves when the transform outlasts a
    // row's stream: s / 2 complex points against the row's bytes, as measured
    // (N = 2048 took 13 us per row against 7 us for a 64 KB row; N = 1024
    // took 6 us against 8 us)
    const bool split = (int64_t)(s / 2) * 32 >= n * (dtype == RLU_F64 ? 8 : 4);
    const void *kfn = dtype == RLU_F64 ? (split ? (const void *)k_sketch_ws<double, 1> : (const void *)k_sketch_ws<double, 0>)
                                       : (split ? (const void *)k_sketch_ws<float, 1> : (const void *)k_sketch_ws<float, 0>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kWsThreads, lds) != hipSuccess || per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 1;
    }
    per_cu = std::min(per_cu, 4);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)num_cu * per_cu));
    const int log2N = ilog2_exact(s / 2);
#define RLU_WS(TT, SP)                                                                                         \
  hipLaunchKernelGGL((k_sketch_ws<TT, SP>), dim3(grid), dim3(kWsThreads), lds, st, m, n, (const TT *)A, lda, s, \
                     log2N, l, code, sel, twf, twp, Y, ldy, row_counter, had)
    if (dtype == RLU_F64) {
      if (split) RLU_WS(double, 1);
      else RLU_WS(double, 0);
    } else {
      if (split) RLU_WS(float, 1);
      else RLU_WS(float, 0);
    }
#undef RLU_WS
    return hipGetLastError();
  }
  const size_t lds = sketch_lds_bytes(s, l);
  const int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (160 * 1024) / lds));
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)num_cu * per_cu));
  const int log2N = ilog2_exact(s / 2);
  // registers of the next-row prefetch: up to 16 values per thread (the rest
  // streams); 32 would halve the blocks a CU holds
  int pf = 4;
  while (pf < 16 && (int64_t)pf * kSketchThreads < n) pf *= 2;
  if (dtype == RLU_F64)
    launch_pf<double>(pf, dim3(grid), lds, st, m, n, (const double *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy,
                      had);
  else
    launch_pf<float>(pf, dim3(grid), lds, st, m, n, (const float *)A, lda, s, log2N, l, code, sel, twf, twp, Y, ldy,
                     had);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Explicit projection (s > kLdsMaxS: the row's s buckets no longer fit in LDS).
// Y = A Omega^T with Omega^T = S^T diag(d) T R formed as an n x l matrix:
// column j of A reaches coordinate q through its one bucket, so
//   Omega^T[j, q] = sgn'(j) T[h(j), sel[q]],
// sgn'(j) the SEM sign folded with d (the column code), and T's entry from
// the real Fourier basis (f = sel[q], N = s/2, k = (a h + o) mod s):
//   f = 0: 1/sqrt s;  f = N: cos(pi h)/sqrt s;
//   0 < f < N: sqrt(2/s) cos(2 pi f h / s);
//   f > N: -sqrt(2/s) sin(2 pi (s - f) h / s) = -sqrt(2/s) cos(2 pi ((s - f) h + 3s/4) / s),
// or (-1)^popcount(h & f) / sqrt s for the Walsh-Hadamard form.  The product
// is the same linear map as the transform route, summed in another order.
// ---------------------------------------------------------------------------
__global__ void k_cos_table(int s, const double2 *__restrict__ twp, double *__restrict__ ctab) {
  const int N = s >> 1;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < s; k += gridDim.x * blockDim.x)
    ctab[k] = k < N ? twp[k].x : -twp[k - N].x;
}

hipError_t launch_cos_table(int s, const double2 *twp, double *ctab, hipStream_t st) {
  const int blocks = std::max(1, std::min(1024, (s + 255) / 256));
  hipLaunchKernelGGL(k_cos_table, dim3(blocks), dim3(256), 0, st, s, twp, ctab);
  return hipGetLastError();
}

__global__ void k_explicit_projection(int64_t n, int s, int l, const uint32_t *__restrict__ code,
                                      const int32_t *__restrict__ sel, const double *__restrict__ ctab,
                                      int hadamard, double *__restrict__ OmT) {
  const int N = s >> 1;
  const double rs = 1.0 / sqrt((double)s), r2s = sqrt(2.0) * rs;
  const uint32_t mask = (uint32_t)s - 1u;
  const int64_t total = n * (int64_t)l;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / l;
    const int q = (int)(e - j * l);
    const uint32_t c = code[j], h = code_bucket(c);
    const uint32_t f = (uint32_t)sel[q];
    double v;
    if (hadamard) {
      v = (__popc(h & f) & 1) ? -rs : rs;
    } else if (f == 0) {
      v = rs;
    } else if (f == (uint32_t)N) {
      v = (h & 1) ? -rs : rs;
    } else if (f < (uint32_t)N) {
      v = r2s * ctab[(f * h) & mask];
    } else {
      v = -r2s * ctab[(((uint32_t)s - f) * h + 3u * ((uint32_t)s >> 2)) & mask];
    }
    OmT[e] = code_apply(c, v);
  }
}

hipError_t launch_explicit_projection(int64_t n, int s, int l, const uint32_t *code, const int32_t *sel,
                                      const double *ctab, bool hadamard, double *OmT, hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(8192, ceil_div(n * (int64_t)l, 256)));
  hipLaunchKernelGGL(k_explicit_projection, dim3(blocks), dim3(256), 0, st, n, s, l, code, sel, ctab,
                     hadamard ? 1 : 0, OmT);
  return hipGetLastError();
}

void sketch_dense_set_attrs() {
  const int bytes = (int)sketch_lds_bytes(kLdsMaxS, 1024);  // l <= 1024 (validated far below)
  hipFuncSetAttribute((const void *)k_sketch_ordered<double>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  hipFuncSetAttribute((const void *)k_sketch_ordered<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  hipFuncSetAttribute((const void *)k_ordered_tables, hipFuncAttributeMaxDynamicSharedMemorySize, kOrdMaxChunk * 4);
  const int ws_bytes = (int)sketch_ws_lds_bytes(2 * kWsMaxN, 1024);
  hipFuncSetAttribute((const void *)k_sketch_ws<double, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, ws_bytes);
  hipFuncSetAttribute((const void *)k_sketch_ws<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, ws_bytes);
  hipFuncSetAttribute((const void *)k_sketch_ws<float, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, ws_bytes);
  hipFuncSetAttribute((const void *)k_sketch_ws<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, ws_bytes);
#define RLU_ATTR(T, P) \
  hipFuncSetAttribute((const void *)k_sketch_dense<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  RLU_ATTR(double, 4) RLU_ATTR(double, 8) RLU_ATTR(double, 16)
  RLU_ATTR(float, 4) RLU_ATTR(float, 8) RLU_ATTR(float, 16)
#undef RLU_ATTR
}

}  // namespace rlu
