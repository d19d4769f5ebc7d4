// Operators for grids whose centre counts are not powers of two (n =
// 2^a 3^b 5^c 7^d per axis): the same A = restriction of the circulant
// convolutions of the s^dim shifted grids (section 3.2.2, Lemma 4.2) and
// Z* = F B^+ P E, with the DFTs done by a mixed-radix self-sorting (Stockham)
// FFT in global memory: one launch per radix pass (radices 4, 2, 3, 5, 7),
// each reading and writing the whole batch.  The power-of-two engine keeps
// its register-resident passes; this path trades their speed for sizes such
// as the paper's 100 x 100 and 100 x 50 grids and N = 10^6.
//
// Two real vectors travel as one complex vector (x_{2p} + i x_{2p+1}): the
// operators are real, so the real and imaginary parts stay separate.
#include <vector>

#include "geo.h"
#include "internal.h"

namespace az {

namespace {

constexpr int GEN_RADICES[] = {4, 2, 3, 5, 7};

// Radices of n, largest power-of-two blocks first; empty if n has another
// prime factor.
std::vector<int> radices_of(int64_t n) {
  std::vector<int> r;
  if (n < 1) return r;
  int64_t m = n;
  for (int R : GEN_RADICES) {
    while (m % R == 0) {
      r.push_back(R);
      m /= R;
    }
  }
  if (m != 1) r.clear();
  return r;
}

// exp(sgn 2 pi i a / b) for integers 0 <= a < b, from sincospi of the exact
// ratio (one rounding in the division).
__device__ __forceinline__ double2 root(int64_t a, int64_t b, bool inv) {
  double s, c;
  sincospi(2.0 * (double)a / (double)b, &s, &c);
  return make_double2(c, inv ? s : -s);
}

__device__ __forceinline__ double2 g_cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// One radix-R pass: the n-point lines hold n/R independent R-point DFTs of
// stride n/R; output index k + (j / Ns) Ns R + q Ns for butterfly j
// (k = j mod Ns) after the twiddle exp(-+ 2 pi i q k / (Ns R)).  Line l's
// element e sits at base(l) + e es, base(l) = (l mod inner) s_in +
// (l / inner) s_out.  With line_fast the line index varies fastest across
// threads (strided lines: neighbouring threads read neighbouring lines).
template <int R, bool INV>
__global__ void __launch_bounds__(256)
k_gfft_pass(const double2* __restrict__ in, double2* __restrict__ out, int n, int Ns, int64_t lines, int64_t inner,
            int64_t s_in, int64_t s_out, int64_t es, int line_fast) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = n / R;
  if (t >= lines * nr) return;
  int64_t l;
  int j;
  if (line_fast) {
    l = t % lines;
    j = (int)(t / lines);
  } else {
    l = t / nr;
    j = (int)(t % nr);
  }
  const int64_t base = (l % inner) * s_in + (l / inner) * s_out;
  const int k = j % Ns;
  double2 v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = in[base + (int64_t)(j + q * nr) * es];
  if (Ns > 1) {
#pragma unroll
    for (int q = 1; q < R; ++q) v[q] = g_cmul(v[q], root((int64_t)q * k, (int64_t)Ns * R, INV));
  }
  // R-point DFT by its definition (R <= 7): y_m = sum_q v_q w^(q m)
  double2 w[R];
#pragma unroll
  for (int m = 0; m < R; ++m) w[m] = root(m, R, INV);
  double2 y[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    double2 acc = v[0];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const double2 p = g_cmul(v[q], w[(q * m) % R]);
      acc.x += p.x;
      acc.y += p.y;
    }
    y[m] = acc;
  }
  const int64_t d = (int64_t)(j / Ns) * Ns * R + k;
#pragma unroll
  for (int m = 0; m < R; ++m) out[base + (d + (int64_t)m * Ns) * es] = y[m];
}

template <int R>
int launch_pass(const double2* in, double2* out, int n, int Ns, int64_t lines, int64_t inner, int64_t s_in,
                int64_t s_out, int64_t es, bool line_fast, bool inv, hipStream_t st) {
  const int64_t work = lines * (n / R);
  const unsigned grid = (unsigned)((work + 255) / 256);
  if (inv)
    launch_kernel(k_gfft_pass<R, true>, grid, 256, 0, st, in, out, n, Ns, lines, inner, s_in, s_out, es,
                  (int)line_fast);
  else
    launch_kernel(k_gfft_pass<R, false>, grid, 256, 0, st, in, out, n, Ns, lines, inner, s_in, s_out, es,
                  (int)line_fast);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// FFT of `lines` lines of n points laid out as in k_gfft_pass, ping-ponging
// between a and b; the result ends in *res (a or b).
int gfft(double2* a, double2* b, int n, int64_t lines, int64_t inner, int64_t s_in, int64_t s_out, int64_t es,
         bool line_fast, bool inv, hipStream_t st, double2** res) {
  const std::vector<int> rs = radices_of(n);
  if (rs.empty()) return AZRBF_EUNSUPPORTED;
  if ((int64_t)lines * n / 2 > ((int64_t)1 << 40)) return AZRBF_EUNSUPPORTED;
  double2* src = a;
  double2* dst = b;
  int Ns = 1;
  for (int R : rs) {
    int rc;
    switch (R) {
      case 4: rc = launch_pass<4>(src, dst, n, Ns, lines, inner, s_in, s_out, es, line_fast, inv, st); break;
      case 2: rc = launch_pass<2>(src, dst, n, Ns, lines, inner, s_in, s_out, es, line_fast, inv, st); break;
      case 3: rc = launch_pass<3>(src, dst, n, Ns, lines, inner, s_in, s_out, es, line_fast, inv, st); break;
      case 5: rc = launch_pass<5>(src, dst, n, Ns, lines, inner, s_in, s_out, es, line_fast, inv, st); break;
      default: rc = launch_pass<7>(src, dst, n, Ns, lines, inner, s_in, s_out, es, line_fast, inv, st); break;
    }
    if (rc) return rc;
    Ns *= R;
    std::swap(src, dst);
  }
  *res = src;
  return AZRBF_OK;
}

// The DFT of the coefficient grid of np vector pairs (np blocks of N = N1 N2
// points, index a N2 + b): along b (contiguous lines), then along a (lines of
// stride N2).  1D plans have N1 = 1.
int gfft_grid(const Geo& g, double2* a, double2* b, int64_t np, bool inv, hipStream_t st, double2** res) {
  double2* r1 = nullptr;
  AZ_TRY(gfft(a, b, g.N2, (int64_t)np * g.N1, 1, g.N2, g.N2, 1, false, inv, st, &r1));
  if (g.N1 == 1) {
    *res = r1;
    return AZRBF_OK;
  }
  double2* o1 = r1 == a ? b : a;
  // lines (pair p, column b): base = b + p N, elements at stride N2
  return gfft(r1, o1, g.N1, (int64_t)np * g.N2, g.N2, 1, g.N, g.N2, true, inv, st, res);
}

// C[p][j] = X[j, 2p] + i X[j, 2p+1] for pairs p0.. (a missing second vector reads 0)
__global__ void k_gpack(const double* __restrict__ X, int64_t ldx, int64_t N, int64_t nvec, int64_t p0, int64_t np,
                        double2* __restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * np) return;
  const int64_t p = i / N, j = i % N;
  const int64_t v = 2 * (p0 + p);
  const double re = X[j + ldx * v];
  const double im = v + 1 < nvec ? X[j + ldx * (v + 1)] : 0.0;
  C[i] = make_double2(re, im);
}

// T = spec_A(ph) * C, pointwise per pair
__global__ void k_gmul_A(Geo g, int ph, const double2* __restrict__ C, double2* __restrict__ T, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N * np) return;
  const int64_t j = i % g.N;
  const int ka = (int)(j / g.N2), kb = (int)(j % g.N2);
  T[i] = g_cmul(specA(g, ph, ka, kb), C[i]);
}

// Y[row, 2p..2p+1] = alpha (Re, Im) y + beta Yin for the collocation rows of
// phase ph: coefficient-grid point (a, b) of phase (rx, ry) is fine point
// (s a + rx) L + s b + ry (1D: s b + ph).
__global__ void k_gscatter_A(Geo g, int ph, const double2* __restrict__ Yc, int64_t nvec, int64_t p0, int64_t np,
                             double alpha, double beta, const double* Yin, int64_t ldyi, double* Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N * np) return;
  const int64_t p = i / g.N, j = i % g.N;
  int64_t gi;
  if (g.dim == 1) {
    gi = (int64_t)g.s * j + ph;
  } else {
    const int rx = ph / g.s, ry = ph % g.s;
    const int64_t a = j / g.N2, b = j % g.N2;
    gi = ((int64_t)g.s * a + rx) * g.L + (int64_t)g.s * b + ry;
  }
  const int64_t row = row_of(g, gi);
  if (row < 0) return;
  const double2 y = Yc[i];
  const int64_t v = 2 * (p0 + p);
  Y[row + ldy * v] = beta == 0.0 ? alpha * y.x : fma(alpha, y.x, beta * Yin[row + ldyi * v]);
  if (v + 1 < nvec)
    Y[row + ldy * (v + 1)] = beta == 0.0 ? alpha * y.y : fma(alpha, y.y, beta * Yin[row + ldyi * (v + 1)]);
}

// E[p][j] = (R[row, 2p], R[row, 2p+1]) at the collocation rows of phase ph, 0 elsewhere
__global__ void k_gextend(Geo g, int ph, const double* __restrict__ R, int64_t ldr, int64_t nvec, int64_t p0,
                          int64_t np, double2* __restrict__ E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N * np) return;
  const int64_t p = i / g.N, j = i % g.N;
  int64_t gi;
  if (g.dim == 1) {
    gi = (int64_t)g.s * j + ph;
  } else {
    const int rx = ph / g.s, ry = ph % g.s;
    const int64_t a = j / g.N2, b = j % g.N2;
    gi = ((int64_t)g.s * a + rx) * g.L + (int64_t)g.s * b + ry;
  }
  const int64_t row = row_of(g, gi);
  double2 e = make_double2(0.0, 0.0);
  if (row >= 0) {
    const int64_t v = 2 * (p0 + p);
    e.x = R[row + ldr * v];
    e.y = v + 1 < nvec ? R[row + ldr * (v + 1)] : 0.0;
  }
  E[i] = e;
}

// S (+)= spec_Z(ph) * E (the first phase assigns)
__global__ void k_gmacc_Z(Geo g, int ph, const double2* __restrict__ E, double2* __restrict__ S, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N * np) return;
  const int64_t j = i % g.N;
  const int ka = (int)(j / g.N2), kb = (int)(j % g.N2);
  const double2 t = g_cmul(specZ(g, ph, ka, kb), E[i]);
  if (ph == 0) {
    S[i] = t;
  } else {
    const double2 s = S[i];
    S[i] = make_double2(s.x + t.x, s.y + t.y);
  }
}

// Z[j, 2p..2p+1] = alpha (Re, Im) z + beta Zin
__global__ void k_gunpack(const double2* __restrict__ Zc, int64_t N, int64_t nvec, int64_t p0, int64_t np,
                          double alpha, double beta, const double* Zin, int64_t ldzi, double* Z, int64_t ldz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * np) return;
  const int64_t p = i / N, j = i % N;
  const double2 z = Zc[i];
  const int64_t v = 2 * (p0 + p);
  Z[j + ldz * v] = beta == 0.0 ? alpha * z.x : fma(alpha, z.x, beta * Zin[j + ldzi * v]);
  if (v + 1 < nvec) Z[j + ldz * (v + 1)] = beta == 0.0 ? alpha * z.y : fma(alpha, z.y, beta * Zin[j + ldzi * (v + 1)]);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Pairs per chunk: three N-point complex buffers per pair within 384 MiB.
int64_t gen_chunk(const Plan& P, int64_t npairs) {
  int64_t c = ((int64_t)384 << 20) / (3 * P.N * (int64_t)sizeof(double2));
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  return npairs < c ? npairs : c;
}

int gen_ws(Plan& P, int64_t pairs, hipStream_t st) {
  if (pairs <= P.gws_pairs) return AZRBF_OK;
  double2* old = P.gws;
  AZ_TRY(P.alloc((void**)&P.gws, 3 * P.N * pairs * (int64_t)sizeof(double2)));
  P.release_one_after(old, st);
  P.gws_pairs = pairs;
  return AZRBF_OK;
}

}  // namespace

bool gfft_supported(int64_t n) { return !radices_of(n).empty(); }

int64_t gen_ws_bytes(int64_t N, int64_t npairs) {
  int64_t c = ((int64_t)384 << 20) / (3 * N * (int64_t)sizeof(double2));
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  if (npairs < c) c = npairs;
  return 3 * N * c * (int64_t)sizeof(double2);
}

int gfft_lines_fwd(const double2* in, double2* out, double2* tmp, int n, int64_t lines, hipStream_t st) {
  // copy-free start: the first pass reads `in`, later passes ping-pong
  // between out and tmp; the result is moved to out if it ends in tmp
  const std::vector<int> rs = radices_of(n);
  if (rs.empty()) return AZRBF_EUNSUPPORTED;
  double2* res = nullptr;
  // first pass: in -> tmp, then the rest on (tmp, out)
  const int R0 = rs[0];
  int rc;
  switch (R0) {
    case 4: rc = launch_pass<4>(in, tmp, n, 1, lines, 1, n, n, 1, false, false, st); break;
    case 2: rc = launch_pass<2>(in, tmp, n, 1, lines, 1, n, n, 1, false, false, st); break;
    case 3: rc = launch_pass<3>(in, tmp, n, 1, lines, 1, n, n, 1, false, false, st); break;
    case 5: rc = launch_pass<5>(in, tmp, n, 1, lines, 1, n, n, 1, false, false, st); break;
    default: rc = launch_pass<7>(in, tmp, n, 1, lines, 1, n, n, 1, false, false, st); break;
  }
  if (rc) return rc;
  double2* src = tmp;
  double2* dst = out;
  int Ns = R0;
  for (size_t i = 1; i < rs.size(); ++i) {
    const int R = rs[i];
    switch (R) {
      case 4: rc = launch_pass<4>(src, dst, n, Ns, lines, 1, n, n, 1, false, false, st); break;
      case 2: rc = launch_pass<2>(src, dst, n, Ns, lines, 1, n, n, 1, false, false, st); break;
      case 3: rc = launch_pass<3>(src, dst, n, Ns, lines, 1, n, n, 1, false, false, st); break;
      case 5: rc = launch_pass<5>(src, dst, n, Ns, lines, 1, n, n, 1, false, false, st); break;
      default: rc = launch_pass<7>(src, dst, n, Ns, lines, 1, n, n, 1, false, false, st); break;
    }
    if (rc) return rc;
    Ns *= R;
    std::swap(src, dst);
  }
  res = src;
  if (res != out) AZ_HIP(hipMemcpyAsync(out, res, (size_t)lines * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
  return AZRBF_OK;
}

int gen_apply_A(Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st) {
  const Geo& g = P.geo;
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t chunk = gen_chunk(P, npairs);
  AZ_TRY(gen_ws(P, chunk, st));
  const int64_t N = P.N;
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = npairs - p0 < chunk ? npairs - p0 : chunk;
    double2* b0 = P.gws;
    double2* b1 = b0 + N * np;
    double2* b2 = b1 + N * np;
    Prof pr("generic_A", 16.0 * N * np * (2.0 + 2.0 * P.ph), st);
    launch_kernel(k_gpack, blocks_for(N * np), 256, 0, st, X, ldx, N, nvec, p0, np, b0);
    AZ_HIP(hipGetLastError());
    double2* Ch = nullptr;
    AZ_TRY(gfft_grid(g, b0, b1, np, false, st, &Ch));
    double2* fa = Ch == b0 ? b1 : b0;   // free pair of buffers beside the spectrum
    for (int ph = 0; ph < P.ph; ++ph) {
      launch_kernel(k_gmul_A, blocks_for(N * np), 256, 0, st, g, ph, Ch, fa, np);
      AZ_HIP(hipGetLastError());
      double2* y = nullptr;
      AZ_TRY(gfft_grid(g, fa, b2, np, true, st, &y));
      launch_kernel(k_gscatter_A, blocks_for(N * np), 256, 0, st, g, ph, y, nvec, p0, np, alpha, beta, Yin, ldyi, Y,
                    ldy);
      AZ_HIP(hipGetLastError());
    }
  }
  return AZRBF_OK;
}

int gen_apply_Z(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta, const double* Zin,
                int64_t ldzi, double* Z, int64_t ldz, hipStream_t st) {
  const Geo& g = P.geo;
  const int64_t npairs = (nvec + 1) / 2;
  const int64_t chunk = gen_chunk(P, npairs);
  AZ_TRY(gen_ws(P, chunk, st));
  const int64_t N = P.N;
  for (int64_t p0 = 0; p0 < npairs; p0 += chunk) {
    const int64_t np = npairs - p0 < chunk ? npairs - p0 : chunk;
    double2* S = P.gws;
    double2* b1 = S + N * np;
    double2* b2 = b1 + N * np;
    Prof pr("generic_Z", 16.0 * N * np * (2.0 + 2.0 * P.ph), st);
    for (int ph = 0; ph < P.ph; ++ph) {
      launch_kernel(k_gextend, blocks_for(N * np), 256, 0, st, g, ph, R, ldr, nvec, p0, np, b1);
      AZ_HIP(hipGetLastError());
      double2* e = nullptr;
      AZ_TRY(gfft_grid(g, b1, b2, np, false, st, &e));
      launch_kernel(k_gmacc_Z, blocks_for(N * np), 256, 0, st, g, ph, e, S, np);
      AZ_HIP(hipGetLastError());
    }
    double2* z = nullptr;
    AZ_TRY(gfft_grid(g, S, b1, np, true, st, &z));
    launch_kernel(k_gunpack, blocks_for(N * np), 256, 0, st, z, N, nvec, p0, np, alpha, beta, Zin, ldzi, Z, ldz);
    AZ_HIP(hipGetLastError());
  }
  return AZRBF_OK;
}

}  // namespace az
