// Random parameters of Algorithm 1 step 1 (SEM of Section 2.2, SRFT of
// Section 2.1), drawn on the device by the counter-based rule of rlu.h.
#include "rlu_device.h"
#include "rlu_internal.h"

namespace rlu {

// Column codes of the fused sketch (bucket | folded sign), and optionally
// the raw SEM parameters h(j), sgn(j) for bit-exact checks.
__global__ void k_sem_codes(int64_t n, int log2s, uint64_t key_sem, uint64_t key_signs,
                            uint32_t *__restrict__ code, int32_t *__restrict__ h_out,
                            int8_t *__restrict__ sgn_out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r = draw(key_sem, (uint64_t)j);
    const uint32_t b = (uint32_t)(r >> (64 - log2s));
    const int neg_sem = (int)(r & 1u);
    if (code) {
      const int neg_d = (int)(draw(key_signs, b) >> 63);
      code[j] = b | ((uint32_t)(neg_sem ^ neg_d) << 31);
    }
    if (h_out) h_out[j] = (int32_t)b;
    if (sgn_out) sgn_out[j] = neg_sem ? (int8_t)-1 : (int8_t)1;
  }
}

// SRFT diagonal d, Fourier twiddles, and the selected coordinates.
//   twf[k] = exp(-2 pi i k / N), N = s/2 (complex FFT of the packed row)
//   twp[f] = exp(-2 pi i f / s), f < N   (split of the real-input spectrum)
// The selection is a partial Fisher-Yates shuffle over 0 .. s-1 with
// counter-based draws; block 0 resolves each selected coordinate
// independently (see below).
__global__ void k_srft_params(int s, int l, uint64_t key_signs, uint64_t key_sel,
                              int8_t *__restrict__ d_out, int32_t *__restrict__ sel,
                              double2 *__restrict__ twf, double2 *__restrict__ twp) {
  extern __shared__ int32_t idx[];
  const int N = s >> 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s; i += gridDim.x * blockDim.x) {
    if (d_out) d_out[i] = (draw(key_signs, (uint64_t)i) >> 63) ? (int8_t)-1 : (int8_t)1;
    if (i < N) {
      double sn, cs;
      if (twf) {
        sincospi(-2.0 * (double)i / (double)N, &sn, &cs);
        twf[i] = make_double2(cs, sn);
      }
      if (twp) {
        sincospi(-2.0 * (double)i / (double)s, &sn, &cs);
        twp[i] = make_double2(cs, sn);
      }
    }
  }
  if (sel == nullptr || blockIdx.x != 0) return;
  // Swap i exchanges positions i and j_i (i <= j_i < s); all j_i first.
  int32_t *jsw = idx;
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    const uint64_t r = draw(key_sel, (uint64_t)i);
    jsw[i] = i + (int)__umul64hi(r, (uint64_t)(s - i));
  }
  __syncthreads();
  // sel[i] is what position j_i holds just before swap i: its initial value
  // j_i unless an earlier swap k wrote it (the latest k < i with j_k = j_i),
  // in which case it is what position k held just before swap k, and so on
  // back (each step moves to an earlier swap).  Same result as running the
  // swaps in order, one thread per coordinate.
  // (The search reads every earlier j_k rather than stopping at the first
  // match from the end: independent LDS reads instead of a dependent chain.)
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    int p = jsw[i], t = i;
    for (;;) {
      int last = -1;
#pragma unroll 8
      for (int k = 0; k < t; ++k) last = (jsw[k] == p) ? k : last;
      if (last < 0) break;
      p = last;
      t = last;
    }
    sel[i] = p;
  }
}

void launch_sem_codes(int64_t n, int s, uint64_t seed, uint32_t *code, int32_t *h, int8_t *sgn,
                      hipStream_t st) {
  const int log2s = ilog2_exact(s);
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_sem_codes, dim3(std::max(1, blocks)), dim3(256), 0, st, n, log2s,
                     stream_key(seed, kStreamSem), stream_key(seed, kStreamSigns), code, h, sgn);
}

void launch_srft_params(int s, int l, uint64_t seed, int8_t *d, int32_t *sel, double2 *twf,
                        double2 *twp, hipStream_t st, bool second) {
  const int blocks = std::max(1, std::min(64, (s + 255) / 256));
  const size_t lds = sel ? (size_t)std::max(1, l) * sizeof(int32_t) : 0;  // the l swap targets
  hipLaunchKernelGGL(k_srft_params, dim3(blocks), dim3(256), lds, st, s, l,
                     stream_key(seed, second ? kStreamSigns2 : kStreamSigns),
                     stream_key(seed, second ? kStreamSelect2 : kStreamSelect), d, sel, twf, twp);
}

}  // namespace rlu
