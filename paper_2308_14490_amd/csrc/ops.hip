// Structured operators of the AZ method on gfx950: A (collocation matrix)
// and Z* (regularised periodic inverse), both applied to blocks of real
// vectors through FFTs, plus the spectra they use (step 0 of section 3.2.3).
//
// A = R Pi^T P* B F* and Z* = F B^+ P E (section 3.2.2).  With the shifted
// grids written out (Pi groups the fine grid into s^dim phases), phase r of
// A^c x is IDFT(d_r .* DFT(x)) and Z* y = IDFT(w .* sum_r conj(d_r) .* DFT(y_r))
// with d_r the DFT of the kernel on shifted grid r (Lemma 4.2) and
// w = 1 / sum_r |d_r|^2 (eq. B_pinv), regularised.  Both maps are complex
// linear and map real vectors to real vectors, so two real vectors travel
// as the real and imaginary parts of one complex vector: every transform
// does useful work on both halves.
//
// Paths:
//   fused  (1D, N <= 8192): one kernel per operator, the whole transform of
//          a vector pair in one workgroup.
//   engine (1D, N > 8192, and 2D): three passes over an N1 x N2 array
//          (column FFT; row FFT + spectral product + row IFFT; column IFFT),
//          the 1D case being the four-step factorisation with twiddles.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "fft.h"
#include "geo.h"
#include "internal.h"

namespace az {

// ------------------------------------------------------------------ twiddles

static const double2* g_tw[64] = {};
static std::mutex g_tw_mu;

int ops_init_twiddles(int device, const double2** tw) {
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if (device < 0 || device >= 64) return AZRBF_EINVAL;
  if (!g_tw[device]) {
    std::vector<double2> h(TW_ENTRIES, make_double2(0.0, 0.0));
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int n = 1; n <= TW_SIZE; n *= 2) {
      const int used = n <= TW_FULL ? n : 256;
      for (int i = 0; i < used; ++i) {
        const long double a = -2.0L * pi * (long double)i / (long double)n;
        h[n + i] = make_double2((double)cosl(a), (double)sinl(a));
      }
    }
    double2* d = nullptr;
    if (hipMalloc(&d, sizeof(double2) * TW_ENTRIES) != hipSuccess) return AZRBF_ENOMEM;
    if (hipMemcpy(d, h.data(), sizeof(double2) * TW_ENTRIES, hipMemcpyHostToDevice) != hipSuccess)
      return AZRBF_EHIP;
    g_tw[device] = d;
  }
  *tw = g_tw[device];
  return AZRBF_OK;
}


// Y[row, v0..v0+1] = alpha * val + beta * Yin[row, v0..v0+1] (Yin unread if beta == 0;
// Yin may equal Y).
__device__ __forceinline__ void store_pair(double* Y, int64_t ldy, const double* Yin, int64_t ldyi, int64_t row,
                                           int64_t v0, int64_t nvec, double2 val, double alpha, double beta) {
  double* p0 = Y + row + ldy * v0;
  const double* q0 = Yin + row + ldyi * v0;
  *p0 = beta == 0.0 ? alpha * val.x : fma(alpha, val.x, beta * *q0);
  if (v0 + 1 < nvec) {
    double* p1 = p0 + ldy;
    *p1 = beta == 0.0 ? alpha * val.y : fma(alpha, val.y, beta * q0[ldyi]);
  }
}

__device__ __forceinline__ double2 load_pair(const double* X, int64_t ldx, int64_t row, int64_t v0,
                                             int64_t nvec) {
  if (v0 >= nvec) return make_double2(0.0, 0.0);
  const double* p0 = X + row + ldx * v0;
  return make_double2(*p0, v0 + 1 < nvec ? p0[ldx] : 0.0);
}

template <int N>
struct Fused {
  static constexpr int T = N / RADIX;
  static constexpr int LINES = T >= 256 ? 1 : 256 / T;
  static constexpr int BLOCK = LINES * T;
  static constexpr int LDS = LINES * RowLds::stride(N) * (int)sizeof(double2);
};

// ------------------------------------------------------------------ fused 1D

// The s phases are transformed one at a time, each written (A) or
// accumulated (Z*) at once, with the thread's indices opaque in each, so that
// no address is computed ahead and held across the transforms.  Holding all
// phases in registers to store the s rows of a coefficient index together
// (contiguous rows per store) needed up to 512 registers per lane (occupancy
// 1, scratch spills for s = 4 and for N = 8192, whose 512-thread blocks cap a
// wave at 256) and was slower: the phases' rows meet again in L2 before they
// go to HBM.
// Phases r0 .. r1 - 1 of the block's vector pair (all of them: 0 .. S).
template <int N, int S>
__device__ __forceinline__ void fused_A_block(const Geo& g, const double2* __restrict__ tw,
                                              const double* __restrict__ X, int64_t ldx, int64_t nvec, double alpha,
                                              double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy,
                                              int64_t blk, int r0 = 0, int r1 = S) {
  using F = Fused<N>;
  extern __shared__ double2 smem[];
  const RowLds lds{smem, RowLds::stride(N)};
  const int t = threadIdx.x % F::T, line = threadIdx.x / F::T;
  const int64_t v0 = 2 * (blk * F::LINES + line);
  double2 a[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = load_pair(X, ldx, t + m * F::T, v0, nvec);
  fft_line<N, false>(a, lds, line, t, tw);
#pragma unroll 1
  for (int r = r0; r < r1; ++r) {
    const int tt = opaque(t), ll = opaque(line);
    double2 res[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) res[m] = cmul(a[m], g.spA[(int64_t)r * N + tt + m * F::T]);
    fft_line<N, true>(res, lds, ll, tt, tw);
    if (v0 < nvec) {
#pragma unroll
      for (int m = 0; m < RADIX; ++m) {
        const int64_t row = (int64_t)S * (tt + m * F::T) + r - g.i0;
        if (row >= 0 && row < g.M) store_pair(Y, ldy, Yin, ldyi, row, v0, nvec, res[m], alpha, beta);
      }
    }
  }
}

template <int N, int S>
__global__ void __launch_bounds__(Fused<N>::BLOCK)
k_fused_A(Geo g, const double2* __restrict__ tw, const double* __restrict__ X, int64_t ldx,
          int64_t nvec, double alpha, double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy) {
  fused_A_block<N, S>(g, tw, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, blockIdx.x);
}

template <int N, int S>
__device__ __forceinline__ void fused_Z_block(const Geo& g, const double2* __restrict__ tw,
                                              const double* __restrict__ R, int64_t ldr, int64_t nvec, double alpha,
                                              double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz,
                                              int64_t blk) {
  using F = Fused<N>;
  extern __shared__ double2 smem[];
  const RowLds lds{smem, RowLds::stride(N)};
  const int t = threadIdx.x % F::T, line = threadIdx.x / F::T;
  const int64_t v0 = 2 * (blk * F::LINES + line);
  double2 acc[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) acc[m] = make_double2(0.0, 0.0);
#pragma unroll 1
  for (int q = 0; q < S; ++q) {
    const int tt = opaque(t), ll = opaque(line);
    double2 in[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      const int64_t row = (int64_t)S * (tt + m * F::T) + q - g.i0;
      in[m] = (row >= 0 && row < g.M) ? load_pair(R, ldr, row, v0, nvec) : make_double2(0.0, 0.0);
    }
    fft_line<N, false>(in, lds, ll, tt, tw);
#pragma unroll
    for (int m = 0; m < RADIX; ++m) acc[m] = cadd(acc[m], cmul(in[m], g.spZ[(int64_t)q * N + tt + m * F::T]));
  }
  fft_line<N, true>(acc, lds, line, t, tw);
  if (v0 < nvec) {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) store_pair(Z, ldz, Zin, ldzi, t + m * F::T, v0, nvec, acc[m], alpha, beta);
  }
}

template <int N, int S>
__global__ void __launch_bounds__(Fused<N>::BLOCK)
k_fused_Z(Geo g, const double2* __restrict__ tw, const double* __restrict__ R, int64_t ldr,
          int64_t nvec, double alpha, double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz) {
  fused_Z_block<N, S>(g, tw, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, blockIdx.x);
}

// Grouped launches over many plans of one size class (N, S): entry blockIdx.y
// of the operand list, its line block blockIdx.x.  Blocks past an entry's
// vectors leave at once (the whole block: the transform synchronises it).
// One phase per block (blockIdx.z): a grouped launch has few blocks per
// entry, so the s phases run side by side, each block transforming the
// vector pair forward itself (the same values in every block).
template <int N, int S>
__global__ void __launch_bounds__(Fused<N>::BLOCK) k_bat_A(const BatOp* __restrict__ ops) {
  const BatOp o = ops[blockIdx.y];
  if (2 * (int64_t)blockIdx.x * Fused<N>::LINES >= o.nvec) return;
  fused_A_block<N, S>(o.g, o.tw, o.in, o.ldin, o.nvec, o.alpha, o.beta, o.yin, o.ldyi, o.out, o.ldo, blockIdx.x,
                      (int)blockIdx.z, (int)blockIdx.z + 1);
}

template <int N, int S>
__global__ void __launch_bounds__(Fused<N>::BLOCK) k_bat_Z(const BatOp* __restrict__ ops) {
  const BatOp o = ops[blockIdx.y];
  if (2 * (int64_t)blockIdx.x * Fused<N>::LINES >= o.nvec) return;
  fused_Z_block<N, S>(o.g, o.tw, o.in, o.ldin, o.nvec, o.alpha, o.beta, o.yin, o.ldyi, o.out, o.ldo, blockIdx.x);
}

// Forward FFT of complex lines (spectra set-up), natural order, length N <= 8192.
template <int N>
__global__ void __launch_bounds__(Fused<N>::BLOCK)
k_fused_fwd(const double2* __restrict__ tw, const double2* __restrict__ in, double2* __restrict__ out,
            int64_t lines) {
  using F = Fused<N>;
  extern __shared__ double2 smem[];
  const RowLds lds{smem, RowLds::stride(N)};
  const int t = threadIdx.x % F::T, line = threadIdx.x / F::T;
  const int64_t li = (int64_t)blockIdx.x * F::LINES + line;
  double2 a[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m)
    a[m] = li < lines ? in[li * N + t + m * F::T] : make_double2(0.0, 0.0);
  fft_line<N, false>(a, lds, line, t, tw);
  if (li < lines) {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) out[li * N + t + m * F::T] = a[m];
  }
}

// ------------------------------------------------------------------ engine

// Store of one workspace element.  (Non-temporal stores were measured: they
// help the first pass and hurt the next one, which then misses the last-level
// cache; net no gain.)
__device__ __forceinline__ void ws_store(double2* p, double2 v) { *p = v; }


// Column passes: C adjacent columns per block, T = N1/16 threads per column,
// column index fastest (coalesced runs of C elements).
template <int N1>
struct Col {
  static constexpr int T = N1 / RADIX;
  static constexpr int CMAX = T >= 256 ? 1 : 256 / T;
};
// Row passes: LINES rows per block, T = N2/16 threads per row.
template <int N2>
struct Row {
  static constexpr int T = N2 / RADIX;
  static constexpr int LMAX = T >= 256 ? 1 : 256 / T;
};

// w_N^e for the four-step twiddles (N = N1 N2 <= TW_SIZE): for N > 256 the
// product w_N^(e mod 256) w_(N/256)^(e div 256) of two roots from the short
// tables at offsets N and N/256, which stay resident in the vector cache.
__device__ __forceinline__ double2 tw_fwd(const double2* tw, int64_t e, int64_t N) {
  const int64_t r = e & (N - 1);
  if (N <= 256) return tw[N + r];
  return cmul(tw[N + (r & 255)], tw[(N >> 8) + (r >> 8)]);
}

// P1 of A: column DFT of the coefficient pair array, four-step twiddle.
template <int N1, bool TWID>
__global__ void __launch_bounds__(256)
k_col_fwd_A(Geo g, const double2* __restrict__ tw, const double* __restrict__ X, int64_t ldx,
            int64_t nvec, int64_t pair0, double2* __restrict__ ws1, int C) {
  constexpr int T = Col<N1>::T;
  extern __shared__ double2 smem[];
  const ColLds lds{smem, C};
  const int l = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t b = (int64_t)blockIdx.x * C + l;
  const int64_t pair = blockIdx.y;
  const int64_t v0 = 2 * (pair0 + pair);
  double2 a[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = load_pair(X, ldx, (int64_t)(t + m * T) * g.N2 + b, v0, nvec);
  fft_line<N1, false>(a, lds, l, t, tw);
  double2* out = ws1 + pair * g.N;
#pragma unroll
  for (int m = 0; m < RADIX; ++m) {
    const int64_t k1 = t + m * T;
    double2 v = a[m];
    if (TWID) v = cmul(v, tw_fwd(tw, k1 * b, g.N));
    ws_store(&out[k1 * g.N2 + b], v);
  }
}

// Row passes (P2).  A: row DFT, product with each phase's spectrum d_r,
// row IDFT per phase.  Z*: row DFT of each phase, sum of the products with
// w conj(d_r), one row IDFT.  A Z*: Z*'s sum followed, without leaving the
// spectrum, by A's per-phase products and IDFTs: Z*'s inverse transform and
// A's forward transform in between cancel (DFT IDFT = N I, the 1/N of the
// inverse being folded into the spectra, hence the factor N), so A Z* costs
// three passes instead of six; if zrows is given, Z*'s own row output is
// stored as well (its column IDFT gives the coefficients Z* y; it may alias
// the phase-0 slice of ws1, which each block reads before writing).
//
// The phases of a row are spread over PL lines of the block (PL divides the
// number of phases; line q takes phases q, q + PL, ...), so that a thread
// holds one line of 16 values; the lines of a row combine through LDS (Z*:
// sum of the partial sums; A: line 0's forward transform is shared).
// LINES is the number of lines per block (rows per block times PL); ONE:
// PL equals the number of phases (one phase per line, no loops: nothing but
// the line itself is live across a transform).
constexpr int ROW_A = 0, ROW_Z = 1, ROW_AZ = 2, ROW_AZC = 3;   // AZC: A Z* with zrows

template <int N2, bool TWID, int PL, int MODE, bool ONE>
__global__ void __launch_bounds__(256)
k_row(Geo g, const double2* __restrict__ tw, const double2* ws1, double2* __restrict__ ws2, double2* zrows,
      int LINES) {
  constexpr int T = Row<N2>::T;
  extern __shared__ double2 smem[];
  const RowLds lds{smem, RowLds::stride(N2)};
  const int t = threadIdx.x % T, l = threadIdx.x / T;
  const int q = l % PL;
  const int64_t k1 = (int64_t)blockIdx.x * (LINES / PL) + l / PL;
  const int64_t pair = blockIdx.y;
  const int nph = TWID ? g.s : g.s * g.s;
  double2 acc[RADIX];
  // One phase per line: the spectral values this line multiplies by are
  // fetched before its transforms, so that their latency overlaps them (A Z*
  // prefetches Z*'s spectrum only, and not at all when Z*'s rows are stored as
  // well: no registers to spare at two waves per SIMD).
  constexpr bool PRE = ONE && MODE != ROW_AZC;
  constexpr bool PRE_Z = PRE && MODE != ROW_A, PRE_A = PRE && MODE == ROW_A;
  double2 sz[PRE_Z ? RADIX : 1], sa[PRE_A ? RADIX : 1];
  if constexpr (PRE_Z) {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) sz[m] = specZ_d<TWID>(g, q, (int)k1, t + m * T);
  }
  if constexpr (PRE_A) {
    const double sc = MODE == ROW_A ? 1.0 : (double)g.N;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) sa[m] = cscale(specA_d<TWID>(g, q, (int)k1, t + m * T), sc);
  }
  if (MODE == ROW_A) {
    const double2* in = ws1 + pair * g.N + k1 * N2;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) acc[m] = q == 0 ? in[t + m * T] : make_double2(0.0, 0.0);
    fft_line<N2, false>(acc, lds, l, t, tw);
  } else if (ONE) {
    const double2* in = ws1 + (pair * nph + q) * g.N + k1 * N2;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) acc[m] = in[t + m * T];
    fft_line<N2, false>(acc, lds, l, t, tw);
    if constexpr (PRE_Z) {
#pragma unroll
      for (int m = 0; m < RADIX; ++m) acc[m] = cmul(acc[m], sz[m]);
    } else {
      const int tt = opaque(t);
#pragma unroll
      for (int m = 0; m < RADIX; ++m) acc[m] = cmul(acc[m], specZ_d<TWID>(g, q, (int)k1, tt + m * T));
    }
  } else {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) acc[m] = make_double2(0.0, 0.0);
    for (int ph = q; ph < nph; ph += PL) {
      const int tt = opaque(t), ll = opaque(l);
      const int64_t kk = (int64_t)blockIdx.x * (LINES / PL) + ll / PL;
      double2 a[RADIX];
      const double2* in = ws1 + (pair * nph + ph) * g.N + kk * N2;
#pragma unroll
      for (int m = 0; m < RADIX; ++m) a[m] = in[tt + m * T];
      fft_line<N2, false>(a, lds, ll, tt, tw);
#pragma unroll
      for (int m = 0; m < RADIX; ++m) acc[m] = cadd(acc[m], cmul(a[m], specZ_d<TWID>(g, ph, (int)kk, tt + m * T)));
    }
  }
  if (PL > 1) {   // combine the lines of the row (the transform's last barrier left LDS free)
#pragma unroll
    for (int m = 0; m < RADIX; ++m) lds.at(l, t + m * T) = acc[m];
    __syncthreads();
    // in groups of four values, each group's reads issued after the previous
    // group's sums, so that few LDS reads are in flight at once
    int tq = t;
#pragma unroll
    for (int m0 = 0; m0 < RADIX; m0 += 4) {
#pragma unroll
      for (int m = m0; m < m0 + 4; ++m) {
        if (MODE == ROW_A) {
          acc[m] = lds.at(l - q, tq + m * T);
        } else {   // the same order of summation on every line of the row
          double2 v = lds.at(l - q, tq + m * T);
#pragma unroll
          for (int j = 1; j < PL; ++j) v = cadd(v, lds.at(l - q + j, tq + m * T));
          acc[m] = v;
        }
      }
      tq = opaque_after(tq, acc[m0 + 3].x);
    }
    __syncthreads();
  }
  if (MODE == ROW_Z || MODE == ROW_AZC) {
    double2 b[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) b[m] = acc[m];
    fft_line<N2, true>(b, lds, l, t, tw);
    if (q == 0) {
      double2* out = (MODE == ROW_Z ? ws2 + pair * g.N : zrows + pair * nph * g.N) + k1 * N2;
#pragma unroll
      for (int m = 0; m < RADIX; ++m) {
        double2 v = b[m];
        if (TWID) v = cmulc(v, tw_fwd(tw, k1 * (t + m * T), g.N));
        ws_store(&out[t + m * T], v);
      }
    }
  }
  if (MODE == ROW_Z) return;
  const double scale = MODE == ROW_A ? 1.0 : (double)g.N;
  if (ONE) {
    if constexpr (PRE_A) {
#pragma unroll
      for (int m = 0; m < RADIX; ++m) acc[m] = cmul(acc[m], sa[m]);
    } else {
#pragma unroll
      for (int m = 0; m < RADIX; ++m)
        acc[m] = cmul(acc[m], cscale(specA_d<TWID>(g, q, (int)k1, t + m * T), scale));
    }
    fft_line<N2, true>(acc, lds, l, t, tw);
    double2* out = ws2 + (pair * nph + q) * g.N + k1 * N2;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      double2 v = acc[m];
      if (TWID) v = cmulc(v, tw_fwd(tw, k1 * (t + m * T), g.N));
      ws_store(&out[t + m * T], v);
    }
    return;
  }
  for (int ph = q; ph < nph; ph += PL) {
    const int tt = opaque(t), ll = opaque(l);
    const int64_t kk = (int64_t)blockIdx.x * (LINES / PL) + ll / PL;
    double2 b[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) b[m] = cmul(acc[m], cscale(specA_d<TWID>(g, ph, (int)kk, tt + m * T), scale));
    fft_line<N2, true>(b, lds, ll, tt, tw);
    double2* out = ws2 + (pair * nph + ph) * g.N + kk * N2;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      double2 v = b[m];
      if (TWID) v = cmulc(v, tw_fwd(tw, kk * (tt + m * T), g.N));
      ws_store(&out[tt + m * T], v);
    }
  }
}

// P3 of A: column IDFT of every phase, restriction to collocation rows.
// The S phases whose fine-grid points are adjacent (1D: all s phases; 2D:
// the s values of ry for one rx) are handled by different lines of the same
// block, phase index fastest: thread line = column * S + phase, so the C*S
// lines of a block cover C*S consecutive fine-grid points and every load and
// store instruction of a wave touches contiguous rows, while each thread
// holds one line (16 values) only.  C here is the number of lines per block;
// in 2D the s groups of phases (one per rx) are the grid's z dimension.
template <int N1, int S, bool D1>
__global__ void __launch_bounds__(256)
k_col_inv_A(Geo g, const double2* __restrict__ tw, const double2* __restrict__ ws2, int64_t nvec,
            int64_t pair0, double alpha, double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy,
            int C) {
  constexpr int T = Col<N1>::T;
  extern __shared__ double2 smem[];
  const ColLds lds{smem, C};
  const int line = threadIdx.x % C, t = threadIdx.x / C;
  const int ry = line % S;
  const int64_t b = (int64_t)blockIdx.x * (C / S) + line / S;
  const int64_t pair = blockIdx.y;
  const int64_t v0 = 2 * (pair0 + pair);
  const int nph = g.dim == 1 ? S : S * S;
  const int gx = (int)blockIdx.z * S;     // 2D: one rx (group of S phases) per z index
  {
    double2 a[RADIX];
    const double2* in = ws2 + (pair * nph + gx + ry) * g.N;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) a[m] = in[(int64_t)(t + m * T) * g.N2 + b];
    // rows of the line's outputs, and with beta != 0 the rows of Yin they
    // combine with, fetched before the transform so that their latency
    // overlaps it (Yin may be Y: each element is read before it is written,
    // by the same thread)
    int rows[RADIX];
    double2 yin[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      rows[m] = (int)row_of_d<D1>(g, grid_index_s<S, D1>(g, gx / S, ry, t + m * T, b));
      yin[m] = make_double2(0.0, 0.0);
    }
    if (beta != 0.0) {
#pragma unroll
      for (int m = 0; m < RADIX; ++m)
        if (rows[m] >= 0) yin[m] = load_pair(Yin, ldyi, rows[m], v0, nvec);
    }
    fft_line<N1, true>(a, lds, line, t, tw);
    if (v0 < nvec) {
#pragma unroll
      for (int m = 0; m < RADIX; ++m) {
        if (rows[m] < 0) continue;
        double* p0 = Y + rows[m] + ldy * v0;
        *p0 = beta == 0.0 ? alpha * a[m].x : fma(alpha, a[m].x, beta * yin[m].x);
        if (v0 + 1 < nvec) p0[ldy] = beta == 0.0 ? alpha * a[m].y : fma(alpha, a[m].y, beta * yin[m].y);
      }
    }
  }
}

// P1 of Z*: extension by zero to each phase grid, column DFT, twiddle; lines
// laid out as in k_col_inv_A (phase fastest, one line per thread).
template <int N1, bool TWID, int S>
__global__ void __launch_bounds__(256)
k_col_fwd_Z(Geo g, const double2* __restrict__ tw, const double* __restrict__ R, int64_t ldr,
            int64_t nvec, int64_t pair0, double2* __restrict__ ws1, int C) {
  constexpr int T = Col<N1>::T;
  extern __shared__ double2 smem[];
  const ColLds lds{smem, C};
  const int line = threadIdx.x % C, t = threadIdx.x / C;
  const int ry = line % S;
  const int64_t b = (int64_t)blockIdx.x * (C / S) + line / S;
  const int64_t pair = blockIdx.y;
  const int64_t v0 = 2 * (pair0 + pair);
  const int nph = g.dim == 1 ? S : S * S;
  const int gx = (int)blockIdx.z * S;     // 2D: one rx (group of S phases) per z index
  {
    double2 a[RADIX];
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      const int64_t row = row_of_d<TWID>(g, grid_index_s<S, TWID>(g, gx / S, ry, t + m * T, b));
      a[m] = row >= 0 ? load_pair(R, ldr, row, v0, nvec) : make_double2(0.0, 0.0);
    }
    fft_line<N1, false>(a, lds, line, t, tw);
    double2* out = ws1 + (pair * nph + gx + ry) * g.N;
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      const int64_t k1 = t + m * T;
      double2 v = a[m];
      if (TWID) v = cmul(v, tw_fwd(tw, k1 * b, g.N));
      ws_store(&out[k1 * g.N2 + b], v);
    }
  }
}

// P3 of Z*: column IDFT, coefficients out.
template <int N1>
__global__ void __launch_bounds__(256)
k_col_inv_Z(Geo g, const double2* __restrict__ tw, const double2* __restrict__ ws2, int64_t pstride, int64_t nvec,
            int64_t pair0, double alpha, double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz,
            int C) {
  constexpr int T = Col<N1>::T;
  extern __shared__ double2 smem[];
  const ColLds lds{smem, C};
  const int l = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t b = (int64_t)blockIdx.x * C + l;
  const int64_t pair = blockIdx.y;
  const int64_t v0 = 2 * (pair0 + pair);
  double2 a[RADIX];
  const double2* in = ws2 + pair * pstride;
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = in[(int64_t)(t + m * T) * g.N2 + b];
  // with beta != 0 the coefficients combined with are fetched before the
  // transform, so that their latency overlaps it (Zin may be Z: each element
  // is read before it is written, by the same thread)
  double2 zin[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) zin[m] = make_double2(0.0, 0.0);
  if (beta != 0.0) {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) zin[m] = load_pair(Zin, ldzi, (int64_t)(t + m * T) * g.N2 + b, v0, nvec);
  }
  fft_line<N1, true>(a, lds, l, t, tw);
  if (v0 < nvec) {
#pragma unroll
    for (int m = 0; m < RADIX; ++m) {
      double* p0 = Z + (int64_t)(t + m * T) * g.N2 + b + ldz * v0;
      *p0 = beta == 0.0 ? alpha * a[m].x : fma(alpha, a[m].x, beta * zin[m].x);
      if (v0 + 1 < nvec) p0[ldz] = beta == 0.0 ? alpha * a[m].y : fma(alpha, a[m].y, beta * zin[m].y);
    }
  }
}

// Plain forward FFT of complex N1 x N2 arrays in the engine's layout (spectra set-up):
// column pass (with twiddle) then row pass; output in transposed frequency order.
template <int N1, bool TWID>
__global__ void __launch_bounds__(256)
k_col_fwd_C(Geo g, const double2* __restrict__ tw, const double2* __restrict__ in,
            double2* __restrict__ out, int C) {
  constexpr int T = Col<N1>::T;
  extern __shared__ double2 smem[];
  const ColLds lds{smem, C};
  const int l = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t b = (int64_t)blockIdx.x * C + l;
  const int64_t line = blockIdx.y;
  double2 a[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = in[line * g.N + (int64_t)(t + m * T) * g.N2 + b];
  fft_line<N1, false>(a, lds, l, t, tw);
#pragma unroll
  for (int m = 0; m < RADIX; ++m) {
    const int64_t k1 = t + m * T;
    double2 v = a[m];
    if (TWID) v = cmul(v, tw_fwd(tw, k1 * b, g.N));
    out[line * g.N + k1 * g.N2 + b] = v;
  }
}

template <int N2>
__global__ void __launch_bounds__(256)
k_row_fwd_C(Geo g, const double2* __restrict__ tw, double2* __restrict__ data, int LINES) {
  constexpr int T = Row<N2>::T;
  extern __shared__ double2 smem[];
  const RowLds lds{smem, RowLds::stride(N2)};
  const int t = threadIdx.x % T, l = threadIdx.x / T;
  const int64_t k1 = (int64_t)blockIdx.x * LINES + l;
  double2* p = data + (int64_t)blockIdx.y * g.N + k1 * N2;
  double2 a[RADIX];
#pragma unroll
  for (int m = 0; m < RADIX; ++m) a[m] = p[t + m * T];
  fft_line<N2, false>(a, lds, l, t, tw);
#pragma unroll
  for (int m = 0; m < RADIX; ++m) p[t + m * T] = a[m];
}

// ------------------------------------------------------------------ boundary rows

// Y[M + i] = alpha * bweight * r_i . X + beta * Y[M + i] with the boundary
// row r_i = (phi_j(x_b))_j at a Dirichlet point and (n . grad phi_j(x_b) /
// eps)_j at a Neumann point (section 6.3): direct summation over the centres
// within the Gaussian's numerical support (phi < 1e-20), periodized images
// included.  phi'(d) = -2 eps^2 d exp(-eps^2 d^2).
__device__ __forceinline__ double phi_per_dev(double d, double eps, double T, int mimg, double* dphi) {
  double s = 0.0, ds = 0.0;
  for (int m = -mimg; m <= mimg; ++m) {
    const double dm = d - 2.0 * T * m;
    const double x = eps * dm;
    const double e = exp(-x * x);
    s += e;
    ds = fma(-2.0 * eps * eps * dm, e, ds);
  }
  *dphi = ds;
  return s;
}

// One axis of a boundary point's window: the nw centres from j0 on (taken
// modulo n) and the periodized kernel at their distances.
struct AxisWin {
  int n, mimg, W;
  double T, h;
};

// w: the periodized kernel at the window's centres; dw: its derivative in x.
__device__ __forceinline__ int axis_window(const AxisWin& a, double x, double eps, double* w, double* dw) {
  const int nw = 2 * a.W + 2 < a.n ? 2 * a.W + 2 : a.n;
  const int j0 = (int)floor((x + a.T) / a.h) - a.W;
  for (int o = 0; o < nw; ++o) {
    const int j = ((j0 + o) % a.n + a.n) % a.n;
    double d = x - (-a.T + j * a.h);
    d -= 2.0 * a.T * nearbyint(d / (2.0 * a.T));
    w[o] = phi_per_dev(d, eps, a.T, a.mimg, &dw[o]);
  }
  return j0;
}

__global__ void k_boundary_A(int dim, AxisWin ax, AxisWin ay, double eps, const double* __restrict__ bp,
                             const uint8_t* __restrict__ btype, const double* __restrict__ bnorm, int64_t Mb,
                             double bw, const double* __restrict__ X, int64_t ldx, int64_t nvec, double alpha,
                             double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy, int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (i >= Mb || v >= nvec) return;
  const int nwx = 2 * ax.W + 2 < ax.n ? 2 * ax.W + 2 : ax.n;
  const int nwy = 2 * ay.W + 2 < ay.n ? 2 * ay.W + 2 : ay.n;
  double wx[64], wy[64], dwx[64], dwy[64];
  const int jx0 = axis_window(ax, bp[i * dim], eps, wx, dwx);
  const int jy0 = dim == 2 ? axis_window(ay, bp[i * dim + 1], eps, wy, dwy) : 0;
  // Neumann: n . grad / eps = (nx / eps) d/dx + (ny / eps) d/dy of the product basis
  const bool neu = btype && btype[i];
  const double cx = neu ? bnorm[i * dim] / eps : 0.0;
  const double cy = neu && dim == 2 ? bnorm[i * dim + 1] / eps : 0.0;
  const double* x = X + ldx * v;
  double acc = 0.0;
  if (dim == 1) {
    for (int o = 0; o < nwx; ++o) acc = fma(neu ? cx * dwx[o] : wx[o], x[((jx0 + o) % ax.n + ax.n) % ax.n], acc);
  } else {
    for (int ox = 0; ox < nwx; ++ox) {
      const int jx = ((jx0 + ox) % ax.n + ax.n) % ax.n;
      double r = 0.0, rd = 0.0;
      for (int oy = 0; oy < nwy; ++oy) {
        const double xv = x[(int64_t)jx * ay.n + ((jy0 + oy) % ay.n + ay.n) % ay.n];
        r = fma(wy[oy], xv, r);
        rd = fma(dwy[oy], xv, rd);
      }
      acc = neu ? fma(cx * dwx[ox], r, fma(cy * wx[ox], rd, acc)) : fma(wx[ox], r, acc);
    }
  }
  Y[M + i + ldy * v] = beta == 0.0 ? alpha * bw * acc : fma(alpha * bw, acc, beta * Yin[M + i + ldyi * v]);
}

// ------------------------------------------------------------------ right-hand sides

// B[i, v] = c f[i, v] (collocation rows), B[M + j, v] = bw g[j, v] (boundary
// rows; bw g[j, v] / eps at Neumann points, as their rows).
__global__ void k_assemble_rhs(int64_t M, int64_t Mb, const double* f, int64_t ldf, double c, const double* g,
                               int64_t ldg, double bw, const uint8_t* __restrict__ btype, double eps, double* B,
                               int64_t ldb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (i < M) {
    B[i + ldb * v] = c * f[i + ldf * v];
  } else if (i < M + Mb) {
    const double gv = g[(i - M) + ldg * v];
    B[i + ldb * v] = btype && btype[i - M] ? bw * gv / eps : bw * gv;
  }
}

int ops_rhs(const Plan& P, const double* f, int64_t ldf, const double* g, int64_t ldg, int64_t nrhs, double* B,
            int64_t ldb, hipStream_t st) {
  if (nrhs <= 0 || P.Mt == 0) return AZRBF_OK;
  if (nrhs > 65535) return AZRBF_EINVAL;
  // the collocation rows of a boundary value problem carry the operator's
  // normalisation 1 / (2 dim eps^2) (the factor -2 eps^2 of the section 6.1
  // example, applied to -(Lap + k2) u = f), so that the scaled equations keep
  // the solution u
  const double c = P.prob.op == AZRBF_OP_APPROX ? 1.0 : 1.0 / (2.0 * P.dim * P.eps * P.eps);
  const dim3 grid((unsigned)((P.Mt + 255) / 256), (unsigned)nrhs);
  Prof pr("assemble_rhs", 16.0 * (double)P.Mt * nrhs, st);
  launch_kernel(k_assemble_rhs, grid, 256, 0, st, P.M, P.Mb, f, ldf, c, g, ldg, P.bweight, P.btype, P.eps, B, ldb);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// ------------------------------------------------------------------ spectra set-up

// Kernel phi (which = 0) or phi'' (which = 1) sampled at m * hL, m = 0..L-1,
// split into s phases: out[r * n + j] = k[s j + r].
__global__ void k_sample_phases(double2* out, int n, int s, double hL, double eps, double T, int mimg,
                                int which, double* zero4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (zero4 && i < 4) zero4[i] = 0.0;   // the reductions' accumulators (read by later launches)
  if (i >= (int64_t)n * s) return;
  const int r = (int)(i / n), j = (int)(i % n);
  double x = ((int64_t)s * j + r) * hL;
  if (x >= T) x -= 2.0 * T;
  double v = 0.0;
  const double e2 = eps * eps;
  for (int m = -mimg; m <= mimg; ++m) {
    const double d = x - 2.0 * T * m;
    const double g = exp(-e2 * d * d);
    v += which == 0 ? g : -2.0 * e2 * g * (1.0 - 2.0 * e2 * d * d);
  }
  out[i] = make_double2(v, 0.0);
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

// Block-wide (256 threads) maximum of non-negative v and count of flags,
// then one atomic per block instead of one per thread (all threads of the
// block must call it).
__device__ __forceinline__ void block_max_count(double v, int flag, double* vmax, int* count) {
  __shared__ double rm[4];
  __shared__ int rc[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v = fmax(v, __shfl_xor(v, o, 64));
    flag += __shfl_xor(flag, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    rm[threadIdx.x >> 6] = v;
    rc[threadIdx.x >> 6] = flag;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomic_max_nonneg(vmax, fmax(fmax(rm[0], rm[1]), fmax(rm[2], rm[3])));
    const int c = rc[0] + rc[1] + rc[2] + rc[3];
    if (count && c) atomicAdd(count, c);
  }
}

// 1D: combine kernel spectra into d_r (BVP: opscale (d2 + k2 d0)), D = sum |d_r|^2.
__global__ void __launch_bounds__(256)
k_combine_1d(double2* d, const double2* d2, int64_t N, int s, int op, double k2, double opscale, double* D,
             double* dmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    for (int r = 0; r < s; ++r) {
      double2 v = d[(int64_t)r * N + i];
      if (op != AZRBF_OP_APPROX) {
        v = cscale(cadd(d2[(int64_t)r * N + i], cscale(v, k2)), opscale);
        d[(int64_t)r * N + i] = v;
      }
      acc += v.x * v.x + v.y * v.y;
    }
    D[i] = acc;
  }
  block_max_count(acc, 0, dmax, nullptr);
}

__global__ void __launch_bounds__(256)
k_weights_1d(const double2* d, double2* spA, double2* spZ, const double* D, int64_t N, int s, double tauZ,
             const double* dmax, double* wmax, int* zeroed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  int dropped = 0;
  if (i < N) {
    const double Dv = D[i];
    const bool keep = Dv > tauZ * *dmax;
    w = keep ? 1.0 / Dv : 0.0;
    dropped = keep ? 0 : 1;
    const double inv = 1.0 / (double)N;
    for (int r = 0; r < s; ++r) {
      const double2 v = d[(int64_t)r * N + i];
      spA[(int64_t)r * N + i] = cscale(v, inv);
      spZ[(int64_t)r * N + i] = cscale(cconj(v), w * inv);
    }
  }
  block_max_count(w, dropped, wmax, zeroed);
}

__global__ void __launch_bounds__(256) k_D_2d(Geo g, double* D, double* dmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < g.N) {
    const int ka = (int)(i / g.N2), kb = (int)(i % g.N2);
    for (int ph = 0; ph < g.s * g.s; ++ph) {
      const double2 v = spec2d(g, ph, ka, kb);
      acc += v.x * v.x + v.y * v.y;
    }
    D[i] = acc;
  }
  block_max_count(acc, 0, dmax, nullptr);
}

__global__ void __launch_bounds__(256)
k_weights_2d(double* w2, const double* D, int64_t N, double tauZ, const double* dmax, double* wmax,
             int* zeroed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  int dropped = 0;
  if (i < N) {
    const double Dv = D[i];
    const bool keep = Dv > tauZ * *dmax;
    w = keep ? 1.0 / Dv : 0.0;
    dropped = keep ? 0 : 1;
    w2[i] = w / (double)N;
  }
  block_max_count(w, dropped, wmax, zeroed);
}

// ------------------------------------------------------------------ dispatch

// Kernels that need more than 64 KiB of LDS get the attribute once (the
// largest request seen so far is kept per kernel).
template <class K>
static int set_lds(K kern, int bytes) {
  if (bytes <= 64 * 1024) return AZRBF_OK;
  static std::mutex mu;
  static std::map<const void*, int> done;
  std::lock_guard<std::mutex> lk(mu);
  int& have = done[(const void*)kern];
  if (have >= bytes) return AZRBF_OK;
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    return AZRBF_EHIP;
  have = bytes;
  return AZRBF_OK;
}

#define AZ_SWITCH_N(n, F, ...)                                                     \
  switch (n) {                                                                     \
    case 16: return F<16>(__VA_ARGS__);                                            \
    case 32: return F<32>(__VA_ARGS__);                                            \
    case 64: return F<64>(__VA_ARGS__);                                            \
    case 128: return F<128>(__VA_ARGS__);                                          \
    case 256: return F<256>(__VA_ARGS__);                                          \
    case 512: return F<512>(__VA_ARGS__);                                          \
    case 1024: return F<1024>(__VA_ARGS__);                                        \
    case 2048: return F<2048>(__VA_ARGS__);                                        \
    case 4096: return F<4096>(__VA_ARGS__);                                        \
    case 8192: return F<8192>(__VA_ARGS__);                                        \
    default: return AZRBF_EUNSUPPORTED;                                            \
  }

#define AZ_SWITCH_ENGINE(n, F, ...)                                                \
  switch (n) {                                                                     \
    case 16: return F<16>(__VA_ARGS__);                                            \
    case 32: return F<32>(__VA_ARGS__);                                            \
    case 64: return F<64>(__VA_ARGS__);                                            \
    case 128: return F<128>(__VA_ARGS__);                                          \
    case 256: return F<256>(__VA_ARGS__);                                          \
    case 512: return F<512>(__VA_ARGS__);                                          \
    default: return AZRBF_EUNSUPPORTED;                                            \
  }

// Column passes also take the longer columns of 1D transforms up to 2^20
// (N1 = N / 512).
#define AZ_SWITCH_COL(n, F, ...)                                                   \
  switch (n) {                                                                     \
    case 1024: return F<1024>(__VA_ARGS__);                                        \
    case 2048: return F<2048>(__VA_ARGS__);                                        \
    default: AZ_SWITCH_ENGINE(n, F, __VA_ARGS__)                                   \
  }

template <int N, int S>
static int launch_fused_A_s(const Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha,
                            double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  using F = Fused<N>;
  AZ_TRY(set_lds(k_fused_A<N, S>, F::LDS));
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t blocks = (npairs + F::LINES - 1) / F::LINES;
  static const std::string name = "fused_A n=" + std::to_string(N);
  Prof pr(name.c_str(), 8.0 * nvec * (N + P.M * (beta != 0.0 ? 2.0 : 1.0)) + 16.0 * P.s * N, st);
  launch_kernel(k_fused_A<N, S>, dim3((unsigned)blocks), dim3(F::BLOCK), F::LDS, st, P.geo, P.tw, X, ldx, nvec, alpha,
                beta, Yin, ldyi, Y, ldy);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

template <int N>
static int launch_fused_A(const Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha,
                          double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  switch (P.s) {
    case 1: return launch_fused_A_s<N, 1>(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
    case 2: return launch_fused_A_s<N, 2>(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
    case 3: return launch_fused_A_s<N, 3>(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
    default: return launch_fused_A_s<N, 4>(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
  }
}

template <int N, int S>
static int launch_bat_s(int which, const BatOp* ops, int count, int64_t maxvec, double bytes, hipStream_t st) {
  using F = Fused<N>;
  const int64_t blocks = ((maxvec + 1) / 2 + F::LINES - 1) / F::LINES;
  const dim3 grid((unsigned)blocks, (unsigned)count, which == 0 ? (unsigned)S : 1u);
  if (which == 0) {
    AZ_TRY(set_lds(k_bat_A<N, S>, F::LDS));
    static const std::string name = "bat_A n=" + std::to_string(N);
    Prof pr(name.c_str(), bytes, st);
    launch_kernel(k_bat_A<N, S>, grid, dim3(F::BLOCK), F::LDS, st, ops);
  } else {
    AZ_TRY(set_lds(k_bat_Z<N, S>, F::LDS));
    static const std::string name = "bat_Z n=" + std::to_string(N);
    Prof pr(name.c_str(), bytes, st);
    launch_kernel(k_bat_Z<N, S>, grid, dim3(F::BLOCK), F::LDS, st, ops);
  }
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

template <int N>
static int launch_bat(int which, int s, const BatOp* ops, int count, int64_t maxvec, double bytes, hipStream_t st) {
  switch (s) {
    case 1: return launch_bat_s<N, 1>(which, ops, count, maxvec, bytes, st);
    case 2: return launch_bat_s<N, 2>(which, ops, count, maxvec, bytes, st);
    case 3: return launch_bat_s<N, 3>(which, ops, count, maxvec, bytes, st);
    case 4: return launch_bat_s<N, 4>(which, ops, count, maxvec, bytes, st);
    default: return AZRBF_EUNSUPPORTED;
  }
}

int ops_batched(int which, int n, int s, const BatOp* ops, int count, int64_t maxvec, double bytes, hipStream_t st) {
  if (count <= 0 || maxvec <= 0) return AZRBF_OK;
  if (count > 65535 || (which != 0 && which != 1)) return AZRBF_EINVAL;
  AZ_SWITCH_N(n, launch_bat, which, s, ops, count, maxvec, bytes, st)
}

template <int N, int S>
static int launch_fused_Z_s(const Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha,
                            double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz, hipStream_t st) {
  using F = Fused<N>;
  AZ_TRY(set_lds(k_fused_Z<N, S>, F::LDS));
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t blocks = (npairs + F::LINES - 1) / F::LINES;
  static const std::string name = "fused_Z n=" + std::to_string(N);
  Prof pr(name.c_str(), 8.0 * nvec * (P.M + N * (beta != 0.0 ? 2.0 : 1.0)) + 16.0 * P.s * N, st);
  launch_kernel(k_fused_Z<N, S>, dim3((unsigned)blocks), dim3(F::BLOCK), F::LDS, st, P.geo, P.tw, R, ldr, nvec, alpha,
                beta, Zin, ldzi, Z, ldz);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

template <int N>
static int launch_fused_Z(const Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha,
                          double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz, hipStream_t st) {
  switch (P.s) {
    case 1: return launch_fused_Z_s<N, 1>(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
    case 2: return launch_fused_Z_s<N, 2>(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
    case 3: return launch_fused_Z_s<N, 3>(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
    default: return launch_fused_Z_s<N, 4>(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
  }
}

template <int N>
static int launch_fused_fwd(const double2* tw, const double2* in, double2* out, int64_t lines,
                            hipStream_t st) {
  using F = Fused<N>;
  AZ_TRY(set_lds(k_fused_fwd<N>, F::LDS));
  const int64_t blocks = (lines + F::LINES - 1) / F::LINES;
  launch_kernel(k_fused_fwd<N>, dim3((unsigned)blocks), dim3(F::BLOCK), F::LDS, st, tw, in, out, lines);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

static int col_C(int N1, int N2) {
  const int T = N1 / RADIX;
  int C = T >= 256 ? 1 : 256 / T;
  return C > N2 ? N2 : C;
}
static int row_L(int N1, int N2) {
  const int T = N2 / RADIX;
  int Lr = T >= 256 ? 1 : 256 / T;
  return Lr > N1 ? N1 : Lr;
}

// Tile shapes of the engine passes: the plan's tuned values where valid
// (a power of two, at most 256 threads per block, dividing the other axis),
// else the defaults above.
bool engine_shape_ok(int N1, int N2, int C, int Lr, int chunk) {
  auto p2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (C && (!p2(C) || C * (N1 / RADIX) > 256 || C > N2)) return false;
  if (Lr && (!p2(Lr) || Lr * (N2 / RADIX) > 256 || Lr > N1)) return false;
  if (chunk && (chunk < 1 || chunk > 256)) return false;
  return true;
}
static int plan_C(const Plan& P) { return P.tune_C ? P.tune_C : col_C(P.geo.N1, P.geo.N2); }
static int plan_L(const Plan& P) { return P.tune_L ? P.tune_L : row_L(P.geo.N1, P.geo.N2); }

// Column-pass launchers (template on the column length N1).
struct ColArgs {
  const Plan* P;
  int mode;                 // 0 fwd A, 1 inv A, 2 fwd Z, 3 inv Z, 4 fwd complex
  const double* in;
  int64_t ldi;
  const double2* cin;
  double2* cout;
  int64_t nvec, pair0, npairs;
  double alpha, beta;
  const double* oin;
  int64_t ldoi;
  double* out;
  int64_t ldo;
  hipStream_t st;
  int64_t pstride = 0;      // mode 3: complex elements between pairs of the input (0: N)
};

template <int N1>
static int launch_col(const ColArgs& a) {
  const Plan& P = *a.P;
  const Geo& g = P.geo;
  const int C = plan_C(P);
  const int block = C * Col<N1>::T;
  const int lds = C * N1 * (int)sizeof(double2);
  const dim3 grid((unsigned)(g.N2 / C), (unsigned)a.npairs);
  // modes 1 and 2 spread the s phases of a column over s lines of the block:
  // the block takes the largest power-of-two number of whole columns that
  // fits in C lines (at least one column), s lines each
  const int S = g.s;
  int ncols = 1;
  while (2 * ncols * S <= C) ncols *= 2;
  const int Cp = ncols * S;
  const int block_p = Cp * Col<N1>::T;
  const int lds_p = Cp * N1 * (int)sizeof(double2);
  const dim3 grid_p((unsigned)(g.N2 / (Cp / S)), (unsigned)a.npairs, (unsigned)(g.dim == 1 ? 1 : S));
  const bool tw4 = g.dim == 1;
  // built once per instantiation (thread-safe static initialisation)
  static const std::vector<std::string> full = [] {
    const char* names[5] = {"col_fwd_A", "col_inv_A", "col_fwd_Z", "col_inv_Z", "col_fwd_C"};
    std::vector<std::string> v;
    for (const char* n : names) v.push_back(std::string(n) + " n1=" + std::to_string(N1));
    return v;
  }();
  const double vc = (double)std::min<int64_t>(a.nvec - 2 * a.pair0, 2 * a.npairs);
  const double cN = 16.0 * (double)g.N * (double)a.npairs;   // one complex array per pair
  const double bmul = a.beta != 0.0 ? 2.0 : 1.0;
  double bytes = 0;
  switch (a.mode) {
    case 0: bytes = 8.0 * g.N * vc + cN; break;
    case 1: bytes = cN * P.ph + 8.0 * g.M * vc * bmul; break;
    case 2: bytes = 8.0 * g.M * vc + (g.dim == 2 ? 4.0 * (double)P.Lg : 0.0) + cN * P.ph; break;
    case 3: bytes = cN + 8.0 * g.N * vc * bmul; break;
    default: bytes = 2.0 * cN; break;
  }
  Prof pr(full[a.mode].c_str(), bytes, a.st);
  switch (a.mode) {
    case 0:
      if (tw4) {
        AZ_TRY(set_lds(k_col_fwd_A<N1, true>, lds));
        launch_kernel(k_col_fwd_A<N1, true>, grid, block, lds, a.st, g, P.tw, a.in, a.ldi, a.nvec, a.pair0, a.cout, C);
      } else {
        AZ_TRY(set_lds(k_col_fwd_A<N1, false>, lds));
        launch_kernel(k_col_fwd_A<N1, false>, grid, block, lds, a.st, g, P.tw, a.in, a.ldi, a.nvec, a.pair0, a.cout,
                      C);
      }
      break;
    case 1:
#define AZ_COLINV(S, D1)                                                                                \
  AZ_TRY(set_lds(k_col_inv_A<N1, S, D1>, lds_p));                                                       \
  launch_kernel(k_col_inv_A<N1, S, D1>, grid_p, block_p, lds_p, a.st, g, P.tw, a.cin, a.nvec, a.pair0,       \
                a.alpha, a.beta, a.oin, a.ldoi, a.out, a.ldo, Cp);
      if (tw4) {
        if (g.s == 1) { AZ_COLINV(1, true) } else if (g.s == 2) { AZ_COLINV(2, true) }
        else if (g.s == 3) { AZ_COLINV(3, true) } else { AZ_COLINV(4, true) }
      } else {
        if (g.s == 1) { AZ_COLINV(1, false) } else if (g.s == 2) { AZ_COLINV(2, false) }
        else if (g.s == 3) { AZ_COLINV(3, false) } else { AZ_COLINV(4, false) }
      }
#undef AZ_COLINV
      break;
    case 2:
#define AZ_COLFZ(TW, S)                                                                                 \
  AZ_TRY(set_lds(k_col_fwd_Z<N1, TW, S>, lds_p));                                                       \
  launch_kernel(k_col_fwd_Z<N1, TW, S>, grid_p, block_p, lds_p, a.st, g, P.tw, a.in, a.ldi, a.nvec, a.pair0, \
                a.cout, Cp);
      if (tw4) {
        if (g.s == 1) { AZ_COLFZ(true, 1) } else if (g.s == 2) { AZ_COLFZ(true, 2) }
        else if (g.s == 3) { AZ_COLFZ(true, 3) } else { AZ_COLFZ(true, 4) }
      } else {
        if (g.s == 1) { AZ_COLFZ(false, 1) } else if (g.s == 2) { AZ_COLFZ(false, 2) }
        else if (g.s == 3) { AZ_COLFZ(false, 3) } else { AZ_COLFZ(false, 4) }
      }
#undef AZ_COLFZ
      break;
    case 3:
      AZ_TRY(set_lds(k_col_inv_Z<N1>, lds));
      launch_kernel(k_col_inv_Z<N1>, grid, block, lds, a.st, g, P.tw, a.cin, a.pstride ? a.pstride : g.N, a.nvec,
                    a.pair0, a.alpha, a.beta, a.oin, a.ldoi, a.out, a.ldo, C);
      break;
    case 4:
      if (tw4) {
        AZ_TRY(set_lds(k_col_fwd_C<N1, true>, lds));
        launch_kernel(k_col_fwd_C<N1, true>, grid, block, lds, a.st, g, P.tw, a.cin, a.cout, C);
      } else {
        AZ_TRY(set_lds(k_col_fwd_C<N1, false>, lds));
        launch_kernel(k_col_fwd_C<N1, false>, grid, block, lds, a.st, g, P.tw, a.cin, a.cout, C);
      }
      break;
  }
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

struct RowArgs {
  const Plan* P;
  int mode;                 // 0 A, 1 Z, 2 fwd complex in place, 3 A Z*
  const double2* in;
  double2* out;
  int64_t npairs;
  hipStream_t st;
  double2* zrows = nullptr; // mode 3: Z*'s row output as well
};

template <int N2>
static int launch_row(const RowArgs& a) {
  const Plan& P = *a.P;
  const Geo& g = P.geo;
  const int Lr = plan_L(P);
  const int block = Lr * Row<N2>::T;
  const int lds = Lr * RowLds::stride(N2) * (int)sizeof(double2);
  const dim3 grid((unsigned)(g.N1 / Lr), (unsigned)a.npairs);
  const bool tw4 = g.dim == 1;
  static const std::vector<std::string> full = [] {
    const char* names[4] = {"row_A", "row_Z", "row_fwd_C", "row_AZ"};
    std::vector<std::string> v;
    for (const char* n : names) v.push_back(std::string(n) + " n2=" + std::to_string(N2));
    return v;
  }();
  const double cN = 16.0 * (double)g.N * (double)a.npairs;
  const double spec = g.dim == 1 ? 16.0 * (double)g.N * P.s : 0.0;
  const double bytes = a.mode == 2   ? 2.0 * cN
                       : a.mode == 3 ? cN * (2.0 * P.ph + (a.zrows ? 1.0 : 0.0)) + 2.0 * spec
                                     : cN * (1.0 + P.ph) + spec;
  Prof pr(full[a.mode].c_str(), bytes, a.st);
  if (a.mode == 2) {
    AZ_TRY(set_lds(k_row_fwd_C<N2>, lds));
    launch_kernel(k_row_fwd_C<N2>, grid, block, lds, a.st, g, P.tw, a.out, Lr);
    return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  // phases spread over PL lines per row (PL divides the phase count: 1, 2,
  // 3 or 4; the 9 phases of 2D s = 3 take three lines); the block takes the
  // largest power-of-two number of whole rows that fits in Lr lines
  const int PL = P.ph % 3 == 0 ? 3 : (P.ph < 4 ? P.ph : 4);
  int nrows = 1;
  while (2 * nrows * PL <= Lr) nrows *= 2;
  const int lines = nrows * PL;
  const int block_p = lines * Row<N2>::T;
  const int lds_p = lines * RowLds::stride(N2) * (int)sizeof(double2);
  const dim3 grid_p((unsigned)(g.N1 / (lines / PL)), (unsigned)a.npairs);
  const int mode = a.mode == 0 ? ROW_A : a.mode == 1 ? ROW_Z : a.zrows ? ROW_AZC : ROW_AZ;
  auto go = [&](auto kern) -> int {
    AZ_TRY(set_lds(kern, lds_p));
    launch_kernel(kern, grid_p, block_p, lds_p, a.st, g, P.tw, a.in, a.out, a.zrows, lines);
    return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  };
#define AZ_ROWK(TW, PLV, ONEV)                                                        \
  if (mode == ROW_A) return go(k_row<N2, TW, PLV, ROW_A, ONEV>);                      \
  if (mode == ROW_Z) return go(k_row<N2, TW, PLV, ROW_Z, ONEV>);                      \
  if (mode == ROW_AZ) return go(k_row<N2, TW, PLV, ROW_AZ, ONEV>);                    \
  return go(k_row<N2, TW, PLV, ROW_AZC, ONEV>);
  // 1D: s phases, one per line; 2D: s^2 phases, one per line up to s = 2
  if (tw4) {
    if (PL == 1) { AZ_ROWK(true, 1, true) }
    if (PL == 2) { AZ_ROWK(true, 2, true) }
    if (PL == 3) { AZ_ROWK(true, 3, true) }
    AZ_ROWK(true, 4, true)
  }
  if (PL == 1) { AZ_ROWK(false, 1, true) }
  if (P.ph == 4) { AZ_ROWK(false, 4, true) }
  if (P.ph == 2) { AZ_ROWK(false, 2, true) }
  if (P.ph == 9) { AZ_ROWK(false, 3, false) }
  AZ_ROWK(false, 4, false)
#undef AZ_ROWK
}

static int run_col(const ColArgs& a) { AZ_SWITCH_COL(a.P->geo.N1, launch_col, a) }
static int run_row(const RowArgs& a) { AZ_SWITCH_ENGINE(a.P->geo.N2, launch_row, a) }

// Grows the FFT workspace to `pairs` vector pairs; the replaced buffers go
// back to the pool once the work queued on st before the growth is done.
static int ensure_ws(Plan& P, int64_t pairs, hipStream_t st) {
  if (pairs <= P.ws_pairs) return AZRBF_OK;
  const int64_t per = (int64_t)P.ph * P.N * (int64_t)sizeof(double2);
  void *a = nullptr, *b = nullptr;
  AZ_TRY(P.alloc(&a, per * pairs));
  AZ_TRY(P.alloc(&b, per * pairs));
  P.release_one_after(P.ws1, st);
  P.release_one_after(P.ws2, st);
  P.ws1 = (double2*)a;
  P.ws2 = (double2*)b;
  P.ws_pairs = pairs;
  return AZRBF_OK;
}

// Pairs per engine chunk: at most 64, each workspace buffer at most 256 MiB
// (at N = 65536, s = 2 a pair takes 2 MiB; at N = 2^20, 32 MiB).
static int64_t engine_chunk(const Plan& P, int64_t npairs) {
  const int64_t per = (int64_t)P.ph * P.N * (int64_t)sizeof(double2);
  int64_t c = ((int64_t)256 << 20) / per;
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  if (P.tune_chunk > 0) c = P.tune_chunk;
  return npairs < c ? npairs : c;
}

static int boundary_rows(Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                         const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  if (P.Mb == 0) return AZRBF_OK;
  auto axis = [&](int n, double T, double h) {
    AxisWin a;
    a.n = n;
    a.T = T;
    a.h = h;
    a.mimg = (int)ceil(6.8 / (2.0 * P.eps * T)) + 2;
    a.W = (int)ceil(6.8 / (P.eps * h)) + 1;
    return a;
  };
  const AxisWin ax = axis(P.n, P.T, P.h), ay = P.dim == 2 ? axis(P.ny, P.Ty, P.hy) : ax;
  // window lengths must fit k_boundary_A's arrays
  if (std::min(2 * ax.W + 2, ax.n) > 64 || std::min(2 * ay.W + 2, ay.n) > 64) return AZRBF_EUNSUPPORTED;
  const dim3 grid((unsigned)((P.Mb + 127) / 128), (unsigned)nvec);
  Prof pr("boundary_A", 8.0 * (double)P.Mb * nvec * (beta != 0.0 ? 2.0 : 1.0), st);
  launch_kernel(k_boundary_A, grid, 128, 0, st, P.dim, ax, ay, P.eps, P.bpts, P.btype, P.bnorm, P.Mb, P.bweight, X,
                ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, P.M);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

static int fused_A(const Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                   const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  AZ_SWITCH_N(P.n, launch_fused_A, P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st)
}

int ops_apply_A(Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  if (nvec <= 0) return AZRBF_OK;
  if (!Yin) {
    Yin = Y;
    ldyi = ldy;
  }
  if (P.fused || P.generic) {
    if (P.generic) AZ_TRY(gen_apply_A(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st));
    else AZ_TRY(fused_A(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st));
    return boundary_rows(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
  }
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t chunk = engine_chunk(P, npairs);
  AZ_TRY(ensure_ws(P, chunk, st));
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = npairs - p0 < chunk ? npairs - p0 : chunk;
    ColArgs c1{&P, 0, X, ldx, nullptr, P.ws1, nvec, p0, np, 0, 0, nullptr, 0, nullptr, 0, st};
    AZ_TRY(run_col(c1));
    RowArgs r{&P, 0, P.ws1, P.ws2, np, st};
    AZ_TRY(run_row(r));
    ColArgs c3{&P, 1, nullptr, 0, P.ws2, nullptr, nvec, p0, np, alpha, beta, Yin, ldyi, Y, ldy, st};
    AZ_TRY(run_col(c3));
  }
  return boundary_rows(P, X, ldx, nvec, alpha, beta, Yin, ldyi, Y, ldy, st);
}

static int fused_Z(const Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                   const double* Zin, int64_t ldzi, double* Z, int64_t ldz, hipStream_t st) {
  AZ_SWITCH_N(P.n, launch_fused_Z, P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st)
}

// Boundary rows of R are ignored (Z* has zero columns there).
int ops_apply_Z(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                const double* Zin, int64_t ldzi, double* Z, int64_t ldz, hipStream_t st) {
  if (nvec <= 0) return AZRBF_OK;
  if (!Zin) {
    Zin = Z;
    ldzi = ldz;
  }
  if (P.generic) return gen_apply_Z(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
  if (P.fused) return fused_Z(P, R, ldr, nvec, alpha, beta, Zin, ldzi, Z, ldz, st);
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t chunk = engine_chunk(P, npairs);
  AZ_TRY(ensure_ws(P, chunk, st));
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = npairs - p0 < chunk ? npairs - p0 : chunk;
    ColArgs c1{&P, 2, R, ldr, nullptr, P.ws1, nvec, p0, np, 0, 0, nullptr, 0, nullptr, 0, st};
    AZ_TRY(run_col(c1));
    RowArgs r{&P, 1, P.ws1, P.ws2, np, st};
    AZ_TRY(run_row(r));
    ColArgs c3{&P, 3, nullptr, 0, P.ws2, nullptr, nvec, p0, np, alpha, beta, Zin, ldzi, Z, ldz, st};
    AZ_TRY(run_col(c3));
  }
  return AZRBF_OK;
}

// ------------------------------------------------------------------ spectra

static int fft_lines_fwd(Plan& P, const double2* in, double2* out, int n, int64_t lines, bool engine,
                         hipStream_t st) {
  // mixed radix or Bluestein (the plan's other axis may be a power of two)
  if ((n & (n - 1)) != 0) return gfft_lines_fwd(P, in, out, n, lines, st);
  if (!engine) { AZ_SWITCH_N(n, launch_fused_fwd, P.tw, in, out, lines, st) }
  ColArgs c{&P, 4, nullptr, 0, in, out, 0, 0, lines, 0, 0, nullptr, 0, nullptr, 0, st};
  AZ_TRY(run_col(c));
  RowArgs r{&P, 2, nullptr, out, lines, st};
  return run_row(r);
}

int ops_spectra(Plan& P, hipStream_t st) {
  const int n = P.n, s = P.s;
  const int mimg = (int)ceil(6.8 / (2.0 * P.eps * P.T)) + 2;
  const bool bvp = P.prob.op != AZRBF_OP_APPROX;
  const int nk = bvp ? 2 : 1;
  // samples of phi (and phi'') on the s shifted 1D grids, then their DFTs
  double2 *samp = nullptr, *fac = nullptr;
  AZ_TRY(P.alloc((void**)&samp, (int64_t)nk * s * n * sizeof(double2)));
  AZ_TRY(P.alloc((void**)&fac, (int64_t)nk * s * n * sizeof(double2)));
  double* red = nullptr;   // [dmax, wmax, zeroed(int)]
  AZ_TRY(P.alloc((void**)&red, 4 * sizeof(double)));
  const int64_t ns = (int64_t)n * s;
  if (P.generic) AZ_TRY(gen_tables(P, st));
  for (int which = 0; which < nk; ++which) {
    launch_kernel(k_sample_phases, (unsigned)((ns + 255) / 256), 256, 0, st, samp + which * ns, n, s, P.hL, P.eps,
                  P.T, mimg, which, which == 0 ? red : nullptr);
    AZ_HIP(hipGetLastError());
  }
  const bool engine = P.dim == 1 && !P.fused && !P.generic;
  AZ_TRY(fft_lines_fwd(P, samp, fac, n, (int64_t)nk * s, engine, st));
  double* D = nullptr;
  AZ_TRY(P.alloc((void**)&D, P.N * sizeof(double)));
  int* zeroed = (int*)(red + 2);
  if (P.dim == 1) {
    const double opscale = -1.0 / (2.0 * P.eps * P.eps);
    AZ_TRY(P.alloc((void**)&P.spA, (int64_t)s * P.N * sizeof(double2)));
    AZ_TRY(P.alloc((void**)&P.spZ, (int64_t)s * P.N * sizeof(double2)));
    const unsigned nb = (unsigned)((P.N + 255) / 256);
    launch_kernel(k_combine_1d, nb, 256, 0, st, fac, bvp ? fac + ns : nullptr, P.N, s, P.prob.op, P.prob.k2, opscale,
                  D, red);
    AZ_HIP(hipGetLastError());
    launch_kernel(k_weights_1d, nb, 256, 0, st, fac, P.spA, P.spZ, D, P.N, s, P.tauZ, red, red + 1, zeroed);
    AZ_HIP(hipGetLastError());
    P.geo.spA = P.spA;
    P.geo.spZ = P.spZ;
  } else {
    // the y axis has its own samples and factors unless the box is square
    double2* facy = fac;
    if (P.ny != P.n || P.Ty != P.T) {
      const int ny = P.ny;
      const int mimgy = (int)ceil(6.8 / (2.0 * P.eps * P.Ty)) + 2;
      const int64_t nsy = (int64_t)ny * s;
      double2* sampy = nullptr;
      AZ_TRY(P.alloc((void**)&sampy, nk * nsy * (int64_t)sizeof(double2)));
      AZ_TRY(P.alloc((void**)&facy, nk * nsy * (int64_t)sizeof(double2)));
      for (int which = 0; which < nk; ++which) {
        launch_kernel(k_sample_phases, (unsigned)((nsy + 255) / 256), 256, 0, st, sampy + which * nsy, ny, s, P.hLy,
                      P.eps, P.Ty, mimgy, which, nullptr);
        AZ_HIP(hipGetLastError());
      }
      AZ_TRY(fft_lines_fwd(P, sampy, facy, ny, (int64_t)nk * s, false, st));
    }
    P.fac = fac;
    P.facy = facy;
    P.geo.fac = fac;
    P.geo.facy = facy;
    AZ_TRY(P.alloc((void**)&P.w2, P.N * sizeof(double)));
    const unsigned nb = (unsigned)((P.N + 255) / 256);
    launch_kernel(k_D_2d, nb, 256, 0, st, P.geo, D, red);
    AZ_HIP(hipGetLastError());
    launch_kernel(k_weights_2d, nb, 256, 0, st, P.w2, D, P.N, P.tauZ, red, red + 1, zeroed);
    AZ_HIP(hipGetLastError());
    P.geo.w2 = P.w2;
  }
  // max D, max w and the count of dropped frequencies stay on the device
  // (the factor's threshold reads max D there); the host copies are fetched
  // on demand by ops_norms, so that making a plan does not synchronise
  P.dred = red;
  P.norms_pending = true;
  return AZRBF_OK;
}

int plan_on_stream(Plan& P, hipStream_t st) {
  if (P.ready && st != P.ready_stream) AZ_HIP(hipStreamWaitEvent(st, P.ready, 0));
  return AZRBF_OK;
}

int plan_mark_ready(Plan& P, hipStream_t st) {
  if (!P.ready) AZ_HIP(hipEventCreateWithFlags(&P.ready, hipEventDisableTiming));
  AZ_HIP(hipEventRecord(P.ready, st));
  P.ready_stream = st;
  return AZRBF_OK;
}

int ops_norms(Plan& P, hipStream_t st) {
  if (!P.norms_pending) return AZRBF_OK;
  AZ_TRY(plan_on_stream(P, st));
  double hred[4];
  AZ_HIP(hipMemcpyAsync(hred, P.dred, sizeof(hred), hipMemcpyDeviceToHost, st));
  AZ_HIP(hipStreamSynchronize(st));
  P.normA = sqrt(hred[0]);
  P.normZ = sqrt(hred[1]);
  int z;
  std::memcpy(&z, &hred[2], sizeof(int));
  P.zeroed = z;
  P.norms_pending = false;
  return AZRBF_OK;
}

// Out = alpha A Z* R + beta Yin (Yin defaults to Out).  On the engine the
// product stays in the spectrum between the two operators (k_row_AZ); with
// boundary rows the coefficients Z* R are formed as well (into Zs, N x nvec,
// leading dimension N), since those rows of A are applied to coefficients
// directly.  The fused path applies the two operators in turn through Zs.
int ops_apply_AZ(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                 const double* Yin, int64_t ldyi, double* Out, int64_t ldo, double* Zs, hipStream_t st) {
  if (nvec <= 0) return AZRBF_OK;
  if (!Yin) {
    Yin = Out;
    ldyi = ldo;
  }
  if (P.fused || P.generic) {
    AZ_TRY(ops_apply_Z(P, R, ldr, nvec, 1.0, 0.0, nullptr, 0, Zs, P.N, st));
    return ops_apply_A(P, Zs, P.N, nvec, alpha, beta, Yin, ldyi, Out, ldo, st);
  }
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t chunk = engine_chunk(P, npairs);
  AZ_TRY(ensure_ws(P, chunk, st));
  const bool coef = P.Mb > 0;
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = npairs - p0 < chunk ? npairs - p0 : chunk;
    ColArgs c1{&P, 2, R, ldr, nullptr, P.ws1, nvec, p0, np, 0, 0, nullptr, 0, nullptr, 0, st};
    AZ_TRY(run_col(c1));
    RowArgs r{&P, 3, P.ws1, P.ws2, np, st, coef ? P.ws1 : nullptr};
    AZ_TRY(run_row(r));
    if (coef) {
      ColArgs cz{&P, 3, nullptr, 0, P.ws1, nullptr, nvec, p0, np, 1.0, 0.0, Zs, P.N, Zs, P.N, st,
                 (int64_t)P.ph * P.N};
      AZ_TRY(run_col(cz));
    }
    ColArgs c3{&P, 1, nullptr, 0, P.ws2, nullptr, nvec, p0, np, alpha, beta, Yin, ldyi, Out, ldo, st};
    AZ_TRY(run_col(c3));
  }
  if (!coef) return AZRBF_OK;
  return boundary_rows(P, Zs, P.N, nvec, alpha, beta, Yin, ldyi, Out, ldo, st);
}

}  // namespace az
