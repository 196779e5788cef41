// Block-wide in-LDS transform for the SRFT stage (Section 2.1), and the
// evaluation of selected real coordinates.
//
// A real row z of length s is packed as N = s/2 complex values
// z'[k] = z[2k] + i z[2k+1] (this is just z's memory viewed as double2),
// transformed by an N-point Stockham FFT (radix 4, one leading radix-2 stage
// when log2 N is odd, kernel e^{-2 pi i / N}), and the requested coordinates
// of the length-s real spectrum are then split out of Z = FFT(z'):
//   E_g = (Z_g + conj Z_{N-g}) / 2,  O_g = (Z_g - conj Z_{N-g}) / (2i),
//   X_g = E_g + e^{-2 pi i g / s} O_g    (0 < g < N),
//   X_0 = Re Z_0 + Im Z_0,  X_{s/2} = Re Z_0 - Im Z_0.
// Coordinates are taken on the orthonormal real basis
//   c_0 = X_0 / sqrt s, c_{s/2} = X_{s/2} / sqrt s,
//   c_f = sqrt 2 Re X_f / sqrt s, c_{s-f} = sqrt 2 Im X_f / sqrt s.
#pragma once

#include <hip/hip_runtime.h>

namespace rlu {

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 w) {
  return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// Powers w^e (0 <= e < N) of a root of unity from two small LDS tables:
// w^e = lo[e mod 2^b] * hi[e >> b], with lo[i] = w^i and hi[i] = w^(i 2^b).
// The product of two correctly rounded unit values is within a few ulp of
// w^e.  Keeps the transform free of global loads, so loads issued before it
// (the next row's prefetch) are not waited for inside it.
struct TwSplit {
  const double2 *lo, *hi;
  int b, mask;
  __device__ inline double2 operator()(int e) const { return cmul(lo[e & mask], hi[e >> b]); }
};

// In: x (N complex, LDS).  Uses y (N complex, LDS) as the other ping-pong
// buffer.  Returns the buffer that holds the spectrum.  Must be called by
// every thread of the block; ends with a block barrier.
template <int THREADS, typename TW>
__device__ inline double2 *fft_lds(double2 *x, double2 *y, int N, int log2N, const TW &twf) {
  const int tid = threadIdx.x;
  int Ns = 1;
  if (log2N & 1) {
    const int h = N >> 1;
    for (int j = tid; j < h; j += THREADS) {
      const double2 a = x[j], b = x[j + h];
      y[2 * j] = cadd(a, b);
      y[2 * j + 1] = csub(a, b);
    }
    __syncthreads();
    double2 *t = x; x = y; y = t;
    Ns = 2;
  }
  const int N4 = N >> 2;
  while (Ns < N) {
    const int tstep = N / (4 * Ns);
    for (int j = tid; j < N4; j += THREADS) {
      const int k = j & (Ns - 1);
      double2 v0 = x[j], v1 = x[j + N4], v2 = x[j + 2 * N4], v3 = x[j + 3 * N4];
      if (Ns > 1) {
        const int e = k * tstep;
        v1 = cmul(v1, twf(e));
        v2 = cmul(v2, twf(2 * e));
        v3 = cmul(v3, twf(3 * e));
      }
      const double2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3);
      const double2 d3 = csub(v1, v3);
      const double2 a3 = make_double2(d3.y, -d3.x);  // (v1 - v3) * (-i)
      const int base = (j - k) * 4 + k;
      y[base] = cadd(a0, a2);
      y[base + Ns] = cadd(a1, a3);
      y[base + 2 * Ns] = csub(a0, a2);
      y[base + 3 * Ns] = csub(a1, a3);
    }
    __syncthreads();
    double2 *t = x; x = y; y = t;
    Ns <<= 2;
  }
  return x;
}

// Coordinate f (0 <= f < s) of the orthonormal real transform, from the
// packed spectrum Z (N = s/2 complex values); twp(g) = exp(-2 pi i g / s).
template <typename TW>
__device__ inline double real_coord(const double2 *Z, int s, int f, const TW &twp, double rs, double r2s) {
  const int N = s >> 1;
  if (f == 0) { const double2 z0 = Z[0]; return (z0.x + z0.y) * rs; }
  if (f == N) { const double2 z0 = Z[0]; return (z0.x - z0.y) * rs; }
  const int g = f < N ? f : s - f;
  const double2 zg = Z[g], zn = Z[N - g];
  const double er = 0.5 * (zg.x + zn.x), ei = 0.5 * (zg.y - zn.y);
  const double orr = 0.5 * (zg.y + zn.y), oi = -0.5 * (zg.x - zn.x);
  const double2 w = twp(g);
  if (f < N) return (er + (w.x * orr - w.y * oi)) * r2s;
  return (ei + (w.x * oi + w.y * orr)) * r2s;
}

}  // namespace rlu
