// Operators for grids whose centre counts are not powers of two: the same
// A = restriction of the circulant convolutions of the s^dim shifted grids
// (section 3.2.2, Lemma 4.2) and Z* = F B^+ P E, with the DFTs done by a
// mixed-radix self-sorting (Stockham) FFT in global memory: one launch per
// radix pass (radices 4, 2, 3, 5, 7), each reading and writing the whole
// batch.  An axis whose count has a prime factor above 7 takes Bluestein's
// chirp-z form of the DFT: with c_m = exp(i pi m^2 / n), the forward DFT is
// X_k = conj(c_k) sum_j (x_j conj(c_j)) c_(k-j), a convolution of length
// 2n - 1 done by power-of-two transforms of length M >= 2n - 1 (the inverse
// DFT uses conj(c)).  The power-of-two engine keeps its register-resident
// passes; this path trades their speed for sizes such as the paper's
// 100 x 100 and 100 x 50 grids, N = 10^6, or any other count.
//
// Two real vectors travel as one complex vector (x_{2p} + i x_{2p+1}): the
// operators are real, so the real and imaginary parts stay separate.
#include <algorithm>
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

// c_m (inv: conj(c_m)) with the exponent m^2 reduced mod 2n in integers.
__device__ __forceinline__ double2 chirp(int64_t m, int n, bool conj_) {
  const int64_t e = (m * m) % (2 * (int64_t)n);
  double s, c;
  sincospi((double)e / (double)n, &s, &c);
  return make_double2(c, conj_ ? -s : s);
}

// Filter of the convolution: h_m = c_m (m < n), h_(M-m) = c_m (0 < m < n),
// zero between; conj for the inverse transform.
__global__ void k_blue_filter(double2* __restrict__ h, int n, int M, int inv) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double2 v = make_double2(0.0, 0.0);
  if (m < n) v = chirp(m, n, inv != 0);
  else if (m > M - n) v = chirp(M - m, n, inv != 0);
  h[m] = v;
}

// a_l[m] = x_l[m] conj(c_m) (inv: c_m) for m < n, zero up to M; x in the
// line layout of k_gfft_pass.
__global__ void k_blue_pre(const double2* __restrict__ x, int n, int M, int64_t lines, int64_t inner, int64_t s_in,
                           int64_t s_out, int64_t es, int inv, double2* __restrict__ a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= lines * M) return;
  const int64_t l = t / M;
  const int m = (int)(t % M);
  double2 v = make_double2(0.0, 0.0);
  if (m < n) {
    const int64_t base = (l % inner) * s_in + (l / inner) * s_out;
    v = g_cmul(x[base + (int64_t)m * es], chirp(m, n, inv == 0));
  }
  a[t] = v;
}

__global__ void k_blue_mul(double2* __restrict__ a, const double2* __restrict__ hh, int M, int64_t lines) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= lines * M) return;
  a[t] = g_cmul(a[t], hh[t % M]);
}

// X_l[k] = conj(c_k) (inv: c_k) conv_l[k] / M, into the line layout.
__global__ void k_blue_post(const double2* __restrict__ conv, int n, int M, int64_t lines, int64_t inner,
                            int64_t s_in, int64_t s_out, int64_t es, int inv, double2* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= lines * n) return;
  const int64_t l = t / n;
  const int k = (int)(t % n);
  const int64_t base = (l % inner) * s_in + (l / inner) * s_out;
  const double2 v = g_cmul(conv[l * M + k], chirp(k, n, inv == 0));
  const double sc = 1.0 / (double)M;
  y[base + (int64_t)k * es] = make_double2(v.x * sc, v.y * sc);
}

int pow2_at_least(int64_t v) {
  int m = 1;
  while (m < v) m *= 2;
  return m;
}

// Bluestein's DFT of `lines` lines of n points (layout as k_gfft_pass) from
// x into y (y may not overlap x); scr holds 2 lines M points.
int blue_fft(const Plan::BlueAxis& B, const double2* x, double2* y, int64_t lines, int64_t inner, int64_t s_in,
             int64_t s_out, int64_t es, bool inv, double2* scr, hipStream_t st) {
  const int n = B.n, M = B.M;
  double2* a = scr;
  double2* b = scr + lines * M;
  const unsigned gM = (unsigned)((lines * M + 255) / 256);
  launch_kernel(k_blue_pre, gM, 256, 0, st, x, n, M, lines, inner, s_in, s_out, es, (int)inv, a);
  AZ_HIP(hipGetLastError());
  double2* r = nullptr;
  AZ_TRY(gfft(a, b, M, lines, 1, M, M, 1, false, false, st, &r));
  launch_kernel(k_blue_mul, gM, 256, 0, st, r, inv ? B.hi : B.hf, M, lines);
  AZ_HIP(hipGetLastError());
  double2* o = r == a ? b : a;
  double2* c = nullptr;
  AZ_TRY(gfft(r, o, M, lines, 1, M, M, 1, false, true, st, &c));
  launch_kernel(k_blue_post, (unsigned)((lines * n + 255) / 256), 256, 0, st, c, n, M, lines, inner, s_in, s_out, es,
                (int)inv, y);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// An n-point transform of the grid's lines: mixed radix (result in a or b),
// or Bluestein through scr (a -> b).
int axis_fft(const Plan& P, int axis, double2* a, double2* b, int n, int64_t lines, int64_t inner, int64_t s_in,
             int64_t s_out, int64_t es, bool line_fast, bool inv, double2* scr, hipStream_t st, double2** res) {
  if (!radices_of(n).empty()) return gfft(a, b, n, lines, inner, s_in, s_out, es, line_fast, inv, st, res);
  const Plan::BlueAxis& B = P.blue[axis];
  if (B.n != n || !B.hf) return AZRBF_ESTATE;
  AZ_TRY(blue_fft(B, a, b, lines, inner, s_in, s_out, es, inv, scr, st));
  *res = b;
  return AZRBF_OK;
}

// The DFT of the coefficient grid of np vector pairs (np blocks of N = N1 N2
// points, index a N2 + b): along b (contiguous lines), then along a (lines of
// stride N2).  1D plans have N1 = 1.
int gfft_grid(const Plan& P, double2* a, double2* b, int64_t np, bool inv, double2* scr, hipStream_t st,
              double2** res) {
  const Geo& g = P.geo;
  double2* r1 = nullptr;
  // the y axis (1D: the only one) is axis 1 of the tables in 2D, axis 0 in 1D
  AZ_TRY(axis_fft(P, g.N1 == 1 ? 0 : 1, a, b, g.N2, (int64_t)np * g.N1, 1, g.N2, g.N2, 1, false, inv, scr, st, &r1));
  if (g.N1 == 1) {
    *res = r1;
    return AZRBF_OK;
  }
  double2* o1 = r1 == a ? b : a;
  // lines (pair p, column b): base = b + p N, elements at stride N2
  return axis_fft(P, 0, r1, o1, g.N1, (int64_t)np * g.N2, g.N2, 1, g.N, g.N2, true, inv, scr, st, res);
}

// Bluestein scratch per vector pair (doubles2): 2 lines x M for each axis
// that needs it (the larger of the two).
int64_t blue_per_pair(int64_t N1, int64_t N2) {
  int64_t e = 0;
  if (N1 > 1 && radices_of(N1).empty()) e = std::max<int64_t>(e, 2 * N2 * pow2_at_least(2 * N1 - 1));
  if (radices_of(N2).empty()) e = std::max<int64_t>(e, 2 * N1 * pow2_at_least(2 * N2 - 1));
  return e;
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

// Complex entries of workspace per pair: three N-point buffers and the
// Bluestein share.
int64_t per_pair(int64_t N1, int64_t N2) { return 3 * N1 * N2 + blue_per_pair(N1, N2); }

// Pairs per chunk: the per-pair workspace within 384 MiB.
int64_t chunk_of(int64_t N1, int64_t N2, int64_t npairs) {
  int64_t c = ((int64_t)384 << 20) / (per_pair(N1, N2) * (int64_t)sizeof(double2));
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  return npairs < c ? npairs : c;
}

int64_t gen_chunk(const Plan& P, int64_t npairs) { return chunk_of(P.geo.N1, P.geo.N2, npairs); }

int gen_ws(Plan& P, int64_t pairs, hipStream_t st) {
  if (pairs <= P.gws_pairs) return AZRBF_OK;
  double2* old = P.gws;
  AZ_TRY(P.alloc((void**)&P.gws, per_pair(P.geo.N1, P.geo.N2) * pairs * (int64_t)sizeof(double2)));
  P.release_one_after(old, st);
  P.gws_pairs = pairs;
  return AZRBF_OK;
}

}  // namespace

bool gfft_supported(int64_t n) { return !radices_of(n).empty(); }

int64_t gen_ws_bytes(int64_t N1, int64_t N2, int64_t npairs) {
  const int64_t c = chunk_of(N1, N2, npairs);
  int64_t b = per_pair(N1, N2) * c * (int64_t)sizeof(double2);
  for (int64_t n : {N1, N2})   // Bluestein tables
    if (n > 1 && radices_of(n).empty()) b += 2 * pow2_at_least(2 * n - 1) * (int64_t)sizeof(double2);
  return b;
}

int gen_tables(Plan& P, hipStream_t st) {
  const int ns[2] = {P.geo.N1, P.geo.N2};
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ns[ax];
    const int slot = P.dim == 1 ? 0 : ax;
    if (n <= 1 || !radices_of(n).empty() || P.blue[slot].hf) continue;
    Plan::BlueAxis& B = P.blue[slot];
    B.n = n;
    B.M = pow2_at_least(2 * (int64_t)n - 1);
    AZ_TRY(P.alloc((void**)&B.hf, (int64_t)B.M * sizeof(double2)));
    AZ_TRY(P.alloc((void**)&B.hi, (int64_t)B.M * sizeof(double2)));
    double2* tmp = nullptr;
    AZ_TRY(P.alloc((void**)&tmp, 2 * (int64_t)B.M * sizeof(double2)));
    for (int inv = 0; inv < 2; ++inv) {
      launch_kernel(k_blue_filter, (unsigned)((B.M + 255) / 256), 256, 0, st, tmp, n, B.M, inv);
      AZ_HIP(hipGetLastError());
      double2* r = nullptr;
      AZ_TRY(gfft(tmp, tmp + B.M, B.M, 1, 1, B.M, B.M, 1, false, false, st, &r));
      AZ_HIP(hipMemcpyAsync(inv ? B.hi : B.hf, r, (size_t)B.M * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    P.release_one_after(tmp, st);
  }
  return AZRBF_OK;
}

int gfft_lines_fwd(Plan& P, const double2* in, double2* out, int n, int64_t lines, hipStream_t st) {
  const std::vector<int> rs = radices_of(n);
  if (rs.empty()) {   // Bluestein: the table of this length, scratch for the convolutions
    const Plan::BlueAxis* B = nullptr;
    for (const auto& b : P.blue)
      if (b.n == n && b.hf) B = &b;
    if (!B) return AZRBF_ESTATE;
    double2* scr = nullptr;
    AZ_TRY(P.alloc((void**)&scr, 2 * lines * (int64_t)B->M * sizeof(double2)));
    const int rc = blue_fft(*B, in, out, lines, 1, n, n, 1, false, scr, st);
    P.release_one_after(scr, st);
    return rc;
  }
  // the first pass reads `in`, later passes ping-pong between out and tmp;
  // the result is moved to out if it ends in tmp
  double2* tmp = nullptr;
  AZ_TRY(P.alloc((void**)&tmp, lines * n * (int64_t)sizeof(double2)));
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
  P.release_one_after(tmp, st);
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
    double2* scr = b2 + N * np;
    Prof pr("generic_A", 16.0 * N * np * (2.0 + 2.0 * P.ph), st);
    launch_kernel(k_gpack, blocks_for(N * np), 256, 0, st, X, ldx, N, nvec, p0, np, b0);
    AZ_HIP(hipGetLastError());
    double2* Ch = nullptr;
    AZ_TRY(gfft_grid(P, b0, b1, np, false, scr, st, &Ch));
    double2* fa = Ch == b0 ? b1 : b0;   // free pair of buffers beside the spectrum
    for (int ph = 0; ph < P.ph; ++ph) {
      launch_kernel(k_gmul_A, blocks_for(N * np), 256, 0, st, g, ph, Ch, fa, np);
      AZ_HIP(hipGetLastError());
      double2* y = nullptr;
      AZ_TRY(gfft_grid(P, fa, b2, np, true, scr, st, &y));
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
    double2* scr = b2 + N * np;
    Prof pr("generic_Z", 16.0 * N * np * (2.0 + 2.0 * P.ph), st);
    for (int ph = 0; ph < P.ph; ++ph) {
      launch_kernel(k_gextend, blocks_for(N * np), 256, 0, st, g, ph, R, ldr, nvec, p0, np, b1);
      AZ_HIP(hipGetLastError());
      double2* e = nullptr;
      AZ_TRY(gfft_grid(P, b1, b2, np, false, scr, st, &e));
      launch_kernel(k_gmacc_Z, blocks_for(N * np), 256, 0, st, g, ph, e, S, np);
      AZ_HIP(hipGetLastError());
    }
    double2* z = nullptr;
    AZ_TRY(gfft_grid(P, S, b1, np, true, scr, st, &z));
    launch_kernel(k_gunpack, blocks_for(N * np), 256, 0, st, z, N, nvec, p0, np, alpha, beta, Zin, ldzi, Z, ldz);
    AZ_HIP(hipGetLastError());
  }
  return AZRBF_OK;
}

}  // namespace az
