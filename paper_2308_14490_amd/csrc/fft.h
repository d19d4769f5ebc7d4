// FP64 complex FFT building blocks for gfx950.
//
// A line of n = 2^q complex values is transformed by a group of n/16 threads,
// each holding 16 values in registers.  Thread t holds elements t + m*(n/16),
// m = 0..15, both before and after the transform (Stockham autosort with a
// leftover radix 2/4/8 first): the forward transform of one line can feed an
// inverse transform (or a pointwise product) without a trip through LDS.
// Passes in between exchange through LDS.
//
// Sign convention: forward = sum_m x[m] exp(-2 pi i k m / n) (unnormalised),
// inverse = the same with +i; callers fold 1/n into their spectra.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace az {

constexpr int RADIX = 16;
// Twiddle table: for every n = 2^l <= TW_FULL the n roots w_n^i =
// exp(-2 pi i i / n) are stored contiguously at offset n, so the roots one
// transform length uses share few cache lines.  Longer lengths n <= TW_SIZE
// only ever need their first 256 roots (the four-step twiddle takes w_n^e as
// w_n^(e mod 256) w_(n/256)^(e div 256)), which sit at offset n as well.
constexpr int TW_LOG = 20;
constexpr int TW_SIZE = 1 << TW_LOG;
constexpr int TW_FULL = 1 << 13;
constexpr int TW_ENTRIES = 2 * TW_SIZE;

// v unchanged, but opaque to the optimiser: addresses derived from it inside
// a loop are recomputed in each iteration instead of being hoisted out and
// kept live in registers for the whole loop.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
// The same, available only once dep has been computed: loads addressed from
// the result wait for dep instead of being issued ahead of it.
__device__ __forceinline__ int opaque_after(int v, double dep) {
  asm volatile("" : "+v"(v) : "v"(dep));
  return v;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// cos(2 pi m / 16), sin(2 pi m / 16) from cos(pi/8) = sqrt(2 + sqrt 2)/2,
// sin(pi/8) = sqrt(2 - sqrt 2)/2 and sqrt(1/2).
#define AZ_C1 0.92387953251128675613
#define AZ_S1 0.38268343236508977173
#define AZ_R2 0.70710678118654752440

// Multiply by exp(-+ 2 pi i m/16) (minus sign for the forward transform).
// After unrolling m is a constant and the switch folds away.
template <bool INV>
__device__ __forceinline__ double2 rot16(double2 a, int m) {
  m &= 15;
  double c, s;
  switch (m) {
    case 0: return a;
    case 4: return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
    case 8: return make_double2(-a.x, -a.y);
    case 12: return INV ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
    case 1: c = AZ_C1; s = AZ_S1; break;
    case 2: c = AZ_R2; s = AZ_R2; break;
    case 3: c = AZ_S1; s = AZ_C1; break;
    case 5: c = -AZ_S1; s = AZ_C1; break;
    case 6: c = -AZ_R2; s = AZ_R2; break;
    case 7: c = -AZ_C1; s = AZ_S1; break;
    case 9: c = -AZ_C1; s = -AZ_S1; break;
    case 10: c = -AZ_R2; s = -AZ_R2; break;
    case 11: c = -AZ_S1; s = -AZ_C1; break;
    case 13: c = AZ_S1; s = -AZ_C1; break;
    case 14: c = AZ_R2; s = -AZ_R2; break;
    default: c = AZ_C1; s = -AZ_S1; break;   // 15
  }
  // exp(-i theta) = c - i s (forward), exp(+i theta) = c + i s (inverse)
  const double ss = INV ? s : -s;
  return make_double2(fma(a.x, c, -a.y * ss), fma(a.x, ss, a.y * c));
}

// In-register DFT of size R (1, 2, 4, 8, 16), natural order in and out.
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(double2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(double2* a) {
    const double2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(double2* a) {
    const double2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const double2 t2 = cadd(a[1], a[3]), t3 = rot16<INV>(csub(a[1], a[3]), 4);
    a[0] = cadd(t0, t2);
    a[1] = cadd(t1, t3);
    a[2] = csub(t0, t2);
    a[3] = csub(t1, t3);
  }
};

// R = R1 * R2 split: n = n1 + R1 n2, k = R2 k1 + k2.
template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_split(double2* a) {
  constexpr int R = R1 * R2;
  double2 y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    double2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n1 + R1 * n2];
    Dft<R2, INV>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 + R1 * k2] = rot16<INV>(t[k2], n1 * k2 * (16 / R));
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    double2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 + R1 * k2];
    Dft<R1, INV>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) a[R2 * k1 + k2] = t[k1];
  }
}

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(double2* a) { dft_split<2, 4, INV>(a); }
};

template <bool INV>
struct Dft<16, INV> {
  __device__ __forceinline__ static void run(double2* a) { dft_split<4, 4, INV>(a); }
};

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Leftover radix of n = R0 * 16^q (R0 in {1, 2, 4, 8}).
template <int N>
struct Sched {
  static constexpr int LOG = ilog2(N);
  static constexpr int Q = LOG / 4;
  static constexpr int R0 = 1 << (LOG % 4);
  static constexpr int T = N / RADIX;    // threads per line
  static_assert((1 << LOG) == N && N >= RADIX, "line length must be a power of two >= 16");
};

// LDS addressing.  Row layout: line-major with one pad slot per 16 elements
// (keeps the stride-16 writes of the first pass on distinct banks).  Column
// layout: element-major, lines interleaved (C lines, line index fastest).
struct RowLds {
  double2* base;
  int line_stride;
  __device__ __forceinline__ double2& at(int line, int e) const {
    return base[line * line_stride + e + (e >> 4)];
  }
  __host__ __device__ static constexpr int stride(int n) { return n + n / 16; }
};
struct ColLds {
  double2* base;
  int C;
  __device__ __forceinline__ double2& at(int line, int e) const { return base[e * C + line]; }
};

// One Stockham pass with radix RP at span p; data in registers a[16]
// (thread t holds elements t + m*T).  Writes the pass output to LDS.
template <int N, int RP, bool INV, class Lds>
__device__ __forceinline__ void stockham_pass(double2* a, const Lds& lds, int line, int t, int p,
                                              const double2* __restrict__ tw) {
  constexpr int T = N / RADIX;
  constexpr int C = RADIX / RP;        // butterflies per thread
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int b = t + i * T;
    const int k = b & (p - 1);
    double2 v[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) v[j] = a[i + j * C];
    if (p > 1) {
#pragma unroll
      for (int j = 1; j < RP; ++j) {
        double2 w = tw[p * RP + j * k];
        if (INV) w.y = -w.y;
        v[j] = cmul(v[j], w);
      }
    }
    Dft<RP, INV>::run(v);
    const int base = (b - k) * RP + k;
#pragma unroll
    for (int j = 0; j < RP; ++j) lds.at(line, base + j * p) = v[j];
  }
}

// Last pass (radix 16, span N/16): result stays in registers.
template <int N, bool INV>
__device__ __forceinline__ void stockham_last(double2* a, int t, const double2* __restrict__ tw) {
  constexpr int P = N / RADIX;
  if (P > 1) {
#pragma unroll
    for (int j = 1; j < RADIX; ++j) {
      double2 w = tw[N + j * t];
      if (INV) w.y = -w.y;
      a[j] = cmul(a[j], w);
    }
  }
  Dft<RADIX, INV>::run(a);
}

template <int N, class Lds>
__device__ __forceinline__ void lds_gather(double2* a, const Lds& lds, int line, int t) {
  constexpr int T = N / RADIX;
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = lds.at(line, t + m * T);
}

// Full transform of one line held in registers (element t + m*N/16 in a[m]).
// Every thread of the block must call it (it contains barriers) with the
// same N.  LDS is free for reuse when it returns.
template <int N, bool INV, class Lds>
__device__ __forceinline__ void fft_line(double2* a, const Lds& lds, int line, int t,
                                         const double2* __restrict__ tw) {
  using S = Sched<N>;
  int p = 1;
  if (S::R0 > 1) {
    stockham_pass<N, S::R0, INV>(a, lds, line, t, p, tw);
    __syncthreads();
    lds_gather<N>(a, lds, line, t);
    __syncthreads();
    p *= S::R0;
  }
#pragma unroll
  for (int q = 0; q < S::Q - 1; ++q) {
    stockham_pass<N, RADIX, INV>(a, lds, line, t, p, tw);
    __syncthreads();
    lds_gather<N>(a, lds, line, t);
    __syncthreads();
    p *= RADIX;
  }
  stockham_last<N, INV>(a, t, tw);
}

}  // namespace az
