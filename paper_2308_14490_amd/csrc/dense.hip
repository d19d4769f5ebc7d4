// Low-rank stage of the AZ method on gfx950 (section 3.2.3, "Low-rank solver
// for Ax = b"): a Gaussian sketch Omega, the sketch W = (A - A Z* A) Omega,
// its SVD through a Householder tall-skinny QR and a one-sided Jacobi SVD of
// the small triangular factor, and the per-right-hand-side solve of
// Algorithm 1 with optional refinement passes.
//
// Sketch widths k <= 64: every TSQR block holds RB x k values in LDS, the
// Jacobi SVD of the k x k factor runs in one workgroup.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace az {

constexpr int KMAX = 64;       // largest sketch width of this path
constexpr int TSQR_RB = 256;   // rows per TSQR block (= threads per block)

// ------------------------------------------------------------------ Philox4x32-10

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += W0;
      k.y += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__global__ void k_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* __restrict__ dst, int64_t ld) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (4 * q >= rows || c >= cols) return;
  const uint4 w = philox4x32_10(make_uint4((uint32_t)q, (uint32_t)c, 0u, 0u),
                                make_uint2((uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)));
  const double s = 1.0 / 4294967296.0;
  const double u0 = ((double)w.x + 0.5) * s, u1 = ((double)w.y + 0.5) * s;
  const double u2 = ((double)w.z + 0.5) * s, u3 = ((double)w.w + 0.5) * s;
  const double twopi = 6.283185307179586;
  const double r0 = sqrt(-2.0 * log(u0)), t0 = twopi * u1;
  const double r1 = sqrt(-2.0 * log(u2)), t1 = twopi * u3;
  const double z[4] = {r0 * cos(t0), r0 * sin(t0), r1 * cos(t1), r1 * sin(t1)};
  double* out = dst + c * ld;
  for (int i = 0; i < 4; ++i)
    if (4 * q + i < rows) out[4 * q + i] = z[i];
}

int dense_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* dst, int64_t ld, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return AZRBF_OK;
  const int64_t nq = (rows + 3) / 4;
  Prof pr("gaussian", 8.0 * rows * cols, st);
  k_gaussian<<<dim3((unsigned)((nq + 255) / 256), (unsigned)cols), 256, 0, st>>>(seed, rows, cols, dst, ld);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Column sums of v_t * x_c[t] for columns c in [c0, k) over a 256-thread
// block; result in wv[c].  red holds 4 * KMAX doubles.
__device__ __forceinline__ void block_dots(const double* x, int ldx, double v, int c0, int k, double* red,
                                           double* wv) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int c = c0; c < k; ++c) {
    const double s = wave_sum(v * x[c * ldx + t]);
    if (lane == 0) red[w * KMAX + c] = s;
  }
  __syncthreads();
  if (t >= c0 && t < k) wv[t] = (red[t] + red[KMAX + t]) + (red[2 * KMAX + t] + red[3 * KMAX + t]);
  __syncthreads();
}

// ------------------------------------------------------------------ TSQR

constexpr int TSQR_LDL = TSQR_RB + 1;

static int tsqr_lds_bytes(int k) {
  return (int)(sizeof(double) * ((int64_t)TSQR_LDL * k + 4 * KMAX + 2 * KMAX));
}

// Householder QR of one RB x k block of A (rows >= m read as zero).
// Reflector j is H_j = I - tau_j v_j v_j^T with v_j[j] = 1, zero above.
// Out: R (upper k x k, zeros below) at rows b*k.. of Rout, the reflectors
// over the block's rows of V, and tau at taus[b*k + j].
__global__ void __launch_bounds__(TSQR_RB)
k_tsqr_block(const double* __restrict__ A, int64_t lda, int64_t m, int k, double* __restrict__ Rout,
             int64_t ldr, double* __restrict__ V, int64_t ldv, double* __restrict__ taus) {
  extern __shared__ double sm[];
  double* a = sm;                              // RB x k, column-major, ld TSQR_LDL
  double* red = sm + (int64_t)TSQR_LDL * k;    // 4 * KMAX
  double* wv = red + 4 * KMAX;                 // KMAX
  double* scal = wv + KMAX;                    // [beta, tau]
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * TSQR_RB;
  const int64_t gi = r0 + t;
  for (int c = 0; c < k; ++c) a[c * TSQR_LDL + t] = gi < m ? A[gi + lda * c] : 0.0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    const double x = t > j ? a[j * TSQR_LDL + t] : 0.0;
    const double s = wave_sum(x * x);
    if ((t & 63) == 0) red[t >> 6] = s;
    __syncthreads();
    if (t == 0) {
      const double sig2 = (red[0] + red[1]) + (red[2] + red[3]);
      const double alpha = a[j * TSQR_LDL + j];
      double beta = alpha, tau = 0.0;
      if (sig2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
        tau = (beta - alpha) / beta;
      }
      scal[0] = beta;
      scal[1] = tau;
      scal[2] = sig2 > 0.0 ? 1.0 / (alpha - beta) : 0.0;
    }
    __syncthreads();
    const double tau = scal[1];
    const double v = t == j ? 1.0 : (t > j ? x * scal[2] : 0.0);
    block_dots(a, TSQR_LDL, v, j + 1, k, red, wv);
    for (int c = j + 1; c < k; ++c) a[c * TSQR_LDL + t] -= tau * wv[c] * v;
    if (t > j) a[j * TSQR_LDL + t] = v;
    if (t == j) a[j * TSQR_LDL + j] = scal[0];
    if (t == 0) taus[(int64_t)blockIdx.x * k + j] = tau;
    __syncthreads();
  }
  for (int c = 0; c < k; ++c) {
    if (t < k) Rout[(int64_t)blockIdx.x * k + t + ldr * c] = t <= c ? a[c * TSQR_LDL + t] : 0.0;
    if (gi < m) V[gi + ldv * c] = t > c ? a[c * TSQR_LDL + t] : (t == c ? 1.0 : 0.0);
  }
}

// E_b = H_0 ... H_{k-1} [C_b; 0] for block b: C_b is rows b*k.. of the
// level above's explicit Q (Cup), or the identity at the top (Cup null).
__global__ void __launch_bounds__(TSQR_RB)
k_tsqr_formq(const double* __restrict__ V, int64_t ldv, const double* __restrict__ taus, int64_t m, int k,
             const double* __restrict__ Cup, int64_t ldc, double* __restrict__ E, int64_t lde) {
  extern __shared__ double sm[];
  double* e = sm;
  double* red = sm + (int64_t)TSQR_LDL * k;
  double* wv = red + 4 * KMAX;
  const int t = threadIdx.x;
  const int64_t gi = (int64_t)blockIdx.x * TSQR_RB + t;
  for (int c = 0; c < k; ++c) {
    double val = 0.0;
    if (t < k) val = Cup ? Cup[(int64_t)blockIdx.x * k + t + ldc * c] : (t == c ? 1.0 : 0.0);
    e[c * TSQR_LDL + t] = val;
  }
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double v = (t >= j && gi < m) ? V[gi + ldv * j] : 0.0;
    const double tau = taus[(int64_t)blockIdx.x * k + j];
    block_dots(e, TSQR_LDL, v, 0, k, red, wv);
    for (int c = 0; c < k; ++c) e[c * TSQR_LDL + t] -= tau * wv[c] * v;
    __syncthreads();
  }
  if (gi < m)
    for (int c = 0; c < k; ++c) E[gi + lde * c] = e[c * TSQR_LDL + t];
}

struct TsqrLevel {
  int64_t m, nb;
  double* A;     // level input; overwritten by the level's reflectors
  double* tau;   // nb x k
  double* R;     // stacked R factors (nb*k x k): the next level's input
};

static void tsqr_plan(int64_t m, int k, std::vector<TsqrLevel>& lv, int64_t* scratch_doubles,
                      int64_t* e_doubles) {
  lv.clear();
  int64_t mm = m, tot = 0, emax = 0;
  while (true) {
    TsqrLevel L{};
    L.m = mm;
    L.nb = (mm + TSQR_RB - 1) / TSQR_RB;
    lv.push_back(L);
    tot += L.nb * k + L.nb * k * k;
    if (lv.size() > 1) emax = std::max(emax, mm * k);
    if (L.nb == 1) break;
    mm = L.nb * k;
  }
  *scratch_doubles = tot;
  *e_doubles = emax;
}

static int64_t tsqr_scratch_doubles(int64_t m, int k) {
  std::vector<TsqrLevel> lv;
  int64_t s, e;
  tsqr_plan(m, k, lv, &s, &e);
  return s + 2 * e;
}

// W (m x k, ld m) is destroyed (level-0 reflectors); Q (m x k, ld m) and
// R (k x k, ld k) out.
static int tsqr(double* W, int64_t m, int k, double* scratch, double* Q, double* R, hipStream_t st) {
  std::vector<TsqrLevel> lv;
  int64_t sd, ed;
  tsqr_plan(m, k, lv, &sd, &ed);
  double* p = scratch;
  for (size_t l = 0; l < lv.size(); ++l) {
    lv[l].tau = p;
    p += lv[l].nb * k;
    lv[l].R = p;
    p += lv[l].nb * k * k;
    lv[l].A = l == 0 ? W : lv[l - 1].R;
  }
  double* Ebuf[2] = {p, p + ed};
  const int lds = tsqr_lds_bytes(k);
  if (lds > 64 * 1024) {
    AZ_HIP(hipFuncSetAttribute((const void*)k_tsqr_block, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    AZ_HIP(hipFuncSetAttribute((const void*)k_tsqr_formq, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  }
  for (size_t l = 0; l < lv.size(); ++l) {
    const TsqrLevel& L = lv[l];
    Prof pr(l == 0 ? "tsqr_block" : "tsqr_block (tree)", 16.0 * L.m * k + 8.0 * L.nb * k * (k + 1), st);
    k_tsqr_block<<<(unsigned)L.nb, TSQR_RB, lds, st>>>(L.A, L.m, L.m, k, L.R, L.nb * k, L.A, L.m, L.tau);
    AZ_HIP(hipGetLastError());
  }
  AZ_HIP(hipMemcpyAsync(R, lv.back().R, sizeof(double) * k * k, hipMemcpyDeviceToDevice, st));
  const double* up = nullptr;
  int64_t ldup = 0;
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    const TsqrLevel& L = lv[l];
    double* E = l == 0 ? Q : Ebuf[l & 1];
    Prof pr(l == 0 ? "tsqr_formq" : "tsqr_formq (tree)", 16.0 * L.m * k + 8.0 * L.nb * k * (k + 1), st);
    k_tsqr_formq<<<(unsigned)L.nb, TSQR_RB, lds, st>>>(L.A, L.m, L.tau, L.m, k, up, ldup, E, L.m);
    AZ_HIP(hipGetLastError());
    up = E;
    ldup = L.m;
  }
  return AZRBF_OK;
}

// ------------------------------------------------------------------ Jacobi SVD

// One-sided Jacobi SVD of the k x k matrix R (k even, <= KMAX) in one block:
// columns of A = R are orthogonalised by plane rotations from the right,
// A V = U S.  Pairs follow the round-robin (circle) schedule, k/2 pairs per
// round handled by groups of G = 512/k threads.  On exit: sig (descending),
// Pm = sum_{i < rank} v_i u_i^T / sigma_i with rank = #{sigma_i > thr}.
__global__ void __launch_bounds__(256)
k_jacobi(const double* __restrict__ R, int k, double thr, double tol, int max_sweeps, double* __restrict__ sig,
         double* __restrict__ Pm, int* __restrict__ info) {
  __shared__ double A[KMAX * (KMAX + 1)];
  __shared__ double V[KMAX * (KMAX + 1)];
  __shared__ double sv[KMAX];
  __shared__ int ord[KMAX];
  __shared__ int pos[KMAX];
  __shared__ int off_flag;
  const int lda = KMAX + 1;
  const int t = threadIdx.x;
  for (int i = t; i < k * k; i += blockDim.x) {
    const int r = i % k, c = i / k;
    A[c * lda + r] = R[r + (int64_t)k * c];
    V[c * lda + r] = r == c ? 1.0 : 0.0;
  }
  if (t < k) pos[t] = t;
  __syncthreads();
  const int G = 512 / k;                 // threads per pair (k/2 pairs * G = 256)
  const int pair = t / G, gl = t % G;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (t == 0) off_flag = 0;
    __syncthreads();
    for (int round = 0; round < k - 1; ++round) {
      // circle schedule: positions pos[0..k-1]; pair i = (pos[i], pos[k-1-i])
      const int p = pos[pair], q = pos[k - 1 - pair];
      double al = 0.0, be = 0.0, ga = 0.0;
      for (int r = gl; r < k; r += G) {
        const double x = A[p * lda + r], y = A[q * lda + r];
        al = fma(x, x, al);
        be = fma(y, y, be);
        ga = fma(x, y, ga);
      }
      for (int o = G / 2; o > 0; o >>= 1) {
        al += __shfl_xor(al, o, G);
        be += __shfl_xor(be, o, G);
        ga += __shfl_xor(ga, o, G);
      }
      double c = 1.0, s = 0.0;
      bool rot = false;
      if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = 1.0 / sqrt(1.0 + tt * tt);
        s = c * tt;
        rot = true;
      }
      if (rot) {
        if (gl == 0) off_flag = 1;
        for (int r = gl; r < k; r += G) {
          const double x = A[p * lda + r], y = A[q * lda + r];
          A[p * lda + r] = c * x - s * y;
          A[q * lda + r] = s * x + c * y;
          const double vx = V[p * lda + r], vy = V[q * lda + r];
          V[p * lda + r] = c * vx - s * vy;
          V[q * lda + r] = s * vx + c * vy;
        }
      }
      __syncthreads();
      if (t == 0) {   // rotate positions 1..k-1
        const int last = pos[k - 1];
        for (int i = k - 1; i > 1; --i) pos[i] = pos[i - 1];
        pos[1] = last;
      }
      __syncthreads();
    }
    const int flag = off_flag;
    __syncthreads();
    if (!flag) break;
  }
  // singular values, order, rank
  if (t < k) {
    double s2 = 0.0;
    for (int r = 0; r < k; ++r) s2 = fma(A[t * lda + r], A[t * lda + r], s2);
    sv[t] = sqrt(s2);
  }
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < k; ++i) ord[i] = i;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j)
        if (sv[ord[j]] > sv[ord[i]]) {
          const int tmp = ord[i];
          ord[i] = ord[j];
          ord[j] = tmp;
        }
    int rank = 0;
    for (int i = 0; i < k; ++i)
      if (sv[ord[i]] > thr) ++rank;
    info[0] = rank;
    info[1] = sweep;
  }
  __syncthreads();
  if (t < k) sig[t] = sv[ord[t]];
  const int rank = info[0];
  // Pm[r][c] = sum_i V[r][i] U[c][i] / s_i = sum_i V[r][i] A[c][i] / s_i^2
  for (int e = t; e < k * k; e += blockDim.x) {
    const int r = e % k, c = e / k;
    double acc = 0.0;
    for (int ii = 0; ii < rank; ++ii) {
      const int i = ord[ii];
      const double si = sv[i];
      acc = fma(V[i * lda + r], A[i * lda + c] / (si * si), acc);
    }
    Pm[r + (int64_t)k * c] = acc;
  }
}

// ------------------------------------------------------------------ skinny GEMMs

// Out = alpha * A B + beta * Cin; A is m x k (ld lda), B is k x ncol (ld ldb,
// small), Out/Cin m x ncol.  Each thread owns one row and up to 16 columns.
__global__ void __launch_bounds__(256)
k_gemm_nn(const double* __restrict__ A, int64_t lda, int64_t m, int k, const double* __restrict__ B, int64_t ldb,
          int64_t ncol, double alpha, const double* Cin, int64_t ldci, double beta, double* Out, int64_t ldo) {
  __shared__ double bs[KMAX * 16];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v0 = (int64_t)blockIdx.y * 16;
  const int nv = (int)std::min<int64_t>(16, ncol - v0);
  for (int e = threadIdx.x; e < k * 16; e += blockDim.x) {
    const int c = e % k, v = e / k;
    bs[v * KMAX + c] = v < nv ? B[c + ldb * (v0 + v)] : 0.0;
  }
  __syncthreads();
  if (i >= m) return;
  double acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;
  for (int c = 0; c < k; ++c) {
    const double a = A[i + lda * c];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = fma(a, bs[v * KMAX + c], acc[v]);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    if (v < nv) {
      const int64_t col = v0 + v;
      const double r = alpha * acc[v];
      Out[i + ldo * col] = beta == 0.0 ? r : fma(beta, Cin[i + ldci * col], r);
    }
  }
}

constexpr int TN_ROWS = 1024;   // rows per partial-sum block

// part[blk][v][c] = sum over the block's rows of Q[i, c] * C[i, v].
__global__ void __launch_bounds__(256)
k_gemm_tn_part(const double* __restrict__ Q, int64_t ldq, int64_t m, int k, const double* __restrict__ C,
               int64_t ldc, int64_t ncol, double* __restrict__ part) {
  __shared__ double qs[32 * KMAX];
  __shared__ double cs[32 * 16];
  const int64_t r0 = (int64_t)blockIdx.x * TN_ROWS;
  const int64_t v0 = (int64_t)blockIdx.y * 16;
  const int nv = (int)std::min<int64_t>(16, ncol - v0);
  const int t = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // thread owns outputs e = t + 256*u, e -> (c = e % k, v = e / k), k*16 <= 1024
  for (int64_t rb = r0; rb < std::min<int64_t>(m, r0 + TN_ROWS); rb += 32) {
    const int nr = (int)std::min<int64_t>(32, m - rb);
    for (int e = t; e < 32 * k; e += 256) {
      const int r = e % 32, c = e / 32;
      qs[r * KMAX + c] = r < nr ? Q[rb + r + ldq * c] : 0.0;
    }
    for (int e = t; e < 32 * 16; e += 256) {
      const int r = e % 32, v = e / 32;
      cs[r * 16 + v] = (r < nr && v < nv) ? C[rb + r + ldc * (v0 + v)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u;
      if (e < k * 16) {
        const int c = e % k, v = e / k;
        double a = acc[u];
        for (int r = 0; r < 32; ++r) a = fma(qs[r * KMAX + c], cs[r * 16 + v], a);
        acc[u] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    if (e < k * 16) {
      const int c = e % k, v = e / k;
      if (v < nv) part[((int64_t)blockIdx.x * ncol + v0 + v) * k + c] = acc[u];
    }
  }
}

// T[c + k v] = sum_blk part[blk][v][c], blocks summed in order.
__global__ void k_reduce_part(const double* __restrict__ part, int64_t nblk, int k, int64_t ncol,
                              double* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * ncol) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblk; ++b) s += part[b * ncol * k + e];
  T[e] = s;
}

// Sum of squares of each column (one block per column, fixed-order tree).
__global__ void __launch_bounds__(256)
k_colnorm2(const double* __restrict__ X, int64_t ld, int64_t m, double* __restrict__ out) {
  __shared__ double red[4];
  const double* x = X + ld * (int64_t)blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) s = fma(x[i], x[i], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_ratio_sqrt(const double* num, const double* den, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = den[i] > 0.0 ? sqrt(num[i] / den[i]) : sqrt(num[i]);
}

static int gemm_nn(const double* A, int64_t lda, int64_t m, int k, const double* B, int64_t ldb, int64_t ncol,
                   double alpha, const double* Cin, int64_t ldci, double beta, double* Out, int64_t ldo,
                   hipStream_t st) {
  if (m <= 0 || ncol <= 0) return AZRBF_OK;
  const dim3 grid((unsigned)((m + 255) / 256), (unsigned)((ncol + 15) / 16));
  Prof pr("gemm_nn", 8.0 * m * (k + ncol * (beta != 0.0 ? 2.0 : 1.0)), st);
  k_gemm_nn<<<grid, 256, 0, st>>>(A, lda, m, k, B, ldb, ncol, alpha, Cin, ldci, beta, Out, ldo);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

static int64_t tn_blocks(int64_t m) { return (m + TN_ROWS - 1) / TN_ROWS; }

static int gemm_tn(const double* Q, int64_t ldq, int64_t m, int k, const double* C, int64_t ldc, int64_t ncol,
                   double* part, double* T, hipStream_t st) {
  const int64_t nb = tn_blocks(m);
  {
    Prof pr("gemm_tn", 8.0 * m * (k + ncol), st);
    k_gemm_tn_part<<<dim3((unsigned)nb, (unsigned)((ncol + 15) / 16)), 256, 0, st>>>(Q, ldq, m, k, C, ldc, ncol,
                                                                                    part);
  }
  AZ_HIP(hipGetLastError());
  const int64_t ne = (int64_t)k * ncol;
  k_reduce_part<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(part, nb, k, ncol, T);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

static int copy_cols(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols,
                     hipStream_t st) {
  if (rows <= 0 || cols <= 0) return AZRBF_OK;
  AZ_HIP(hipMemcpy2DAsync(dst, sizeof(double) * ldd, src, sizeof(double) * lds, sizeof(double) * rows, cols,
                          hipMemcpyDeviceToDevice, st));
  return AZRBF_OK;
}

// ------------------------------------------------------------------ factor

int dense_factor(Plan& P, hipStream_t st) {
  const int k = P.k;
  // the Jacobi kernel pairs k/2 columns over 256 threads: 512 / k must be a shuffle width
  if (k != 16 && k != 32 && k != 64) return AZRBF_EUNSUPPORTED;
  const int64_t N = P.N, Mt = P.Mt;
  if (!P.Om) {
    AZ_TRY(P.alloc((void**)&P.Om, sizeof(double) * N * k));
    AZ_TRY(P.alloc((void**)&P.Yf, sizeof(double) * Mt * k));
    AZ_TRY(P.alloc((void**)&P.Q, sizeof(double) * Mt * k));
    AZ_TRY(P.alloc((void**)&P.Rf, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.sig, sizeof(double) * k));
    AZ_TRY(P.alloc((void**)&P.Pm, sizeof(double) * k * k));
    const int64_t sd = N * k + Mt * k + tsqr_scratch_doubles(Mt, k) + 8;
    AZ_TRY(P.alloc((void**)&P.dscr, sizeof(double) * sd));
    P.dscr_bytes = sizeof(double) * sd;
  }
  double* Zy = P.dscr;                 // N x k
  double* W = Zy + N * k;              // Mt x k
  double* tq = W + Mt * k;             // TSQR scratch
  int* info = (int*)(tq + tsqr_scratch_doubles(Mt, k));
  AZ_TRY(dense_gaussian(P.prob.seed, N, k, P.Om, N, st));
  AZ_TRY(ops_apply_A(P, P.Om, N, k, 1.0, 0.0, P.Yf, Mt, st));        // Y = A Omega
  AZ_TRY(ops_apply_Z(P, P.Yf, Mt, k, 1.0, 0.0, Zy, N, st));          // Z* Y
  AZ_TRY(copy_cols(P.Yf, Mt, W, Mt, Mt, k, st));
  AZ_TRY(ops_apply_A(P, Zy, N, k, -1.0, 1.0, W, Mt, st));            // W = Y - A Z* Y
  AZ_TRY(tsqr(W, Mt, k, tq, P.Q, P.Rf, st));
  const double thr = P.tau * P.normA * sqrt((double)k);
  {
    Prof pj("jacobi", 8.0 * 3 * k * k, st);
    k_jacobi<<<1, 256, 0, st>>>(P.Rf, k, thr, 1e-15, 60, P.sig, P.Pm, info);
  }
  AZ_HIP(hipGetLastError());
  // Omega <- Omega Pm, Y <- Y Pm (row-wise in place: a thread reads its whole row first)
  AZ_TRY(gemm_nn(P.Om, N, N, k, P.Pm, k, k, 1.0, nullptr, 0, 0.0, Zy, N, st));
  AZ_TRY(copy_cols(Zy, N, P.Om, N, N, k, st));
  AZ_TRY(gemm_nn(P.Yf, Mt, Mt, k, P.Pm, k, k, 1.0, nullptr, 0, 0.0, W, Mt, st));
  AZ_TRY(copy_cols(W, Mt, P.Yf, Mt, Mt, k, st));
  int hinfo[2];
  AZ_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st));
  AZ_HIP(hipStreamSynchronize(st));
  P.rank = hinfo[0];
  P.factored = true;
  return P.rank >= k ? AZRBF_ERANK : AZRBF_OK;
}

// ------------------------------------------------------------------ solve

int dense_solve(Plan& P, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx, double* relres,
                hipStream_t st) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt;
  if (nrhs > P.sw_rhs) {
    const int64_t per = N + 3 * Mt + k + tn_blocks(Mt) * k + 2;
    AZ_TRY(P.alloc((void**)&P.sw, sizeof(double) * per * nrhs));
    P.sw_rhs = nrhs;
  }
  double* Zr = P.sw;                   // N x nrhs
  double* C = Zr + N * nrhs;           // Mt x nrhs
  double* R1 = C + Mt * nrhs;          // Mt x nrhs
  double* Rc = R1 + Mt * nrhs;         // Mt x nrhs
  double* Tm = Rc + Mt * nrhs;         // k x nrhs
  double* part = Tm + (int64_t)k * nrhs;
  double* nrm = part + tn_blocks(Mt) * k * nrhs;   // 2 x nrhs
  const double* rin = B;
  int64_t ldr = ldb;
  for (int it = 0; it <= P.refine; ++it) {
    AZ_TRY(ops_apply_Z(P, rin, ldr, nrhs, 1.0, 0.0, Zr, N, st));              // Z* r
    AZ_TRY(copy_cols(rin, ldr, C, Mt, Mt, nrhs, st));
    AZ_TRY(ops_apply_A(P, Zr, N, nrhs, -1.0, 1.0, C, Mt, st));                // c = (I - A Z*) r
    AZ_TRY(gemm_tn(P.Q, Mt, Mt, k, C, Mt, nrhs, part, Tm, st));               // t = Q^T c
    AZ_TRY(gemm_nn(P.Om, N, N, k, Tm, k, nrhs, 1.0, X, ldx, it == 0 ? 0.0 : 1.0, X, ldx, st));  // x1
    AZ_TRY(gemm_nn(P.Yf, Mt, Mt, k, Tm, k, nrhs, -1.0, rin, ldr, 1.0, R1, Mt, st));            // r - A x1
    AZ_TRY(ops_apply_Z(P, R1, Mt, nrhs, 1.0, 1.0, X, ldx, st));               // x += Z* (r - A x1)
    AZ_TRY(copy_cols(B, ldb, Rc, Mt, Mt, nrhs, st));
    AZ_TRY(ops_apply_A(P, X, ldx, nrhs, -1.0, 1.0, Rc, Mt, st));              // residual b - A x
    rin = Rc;
    ldr = Mt;
  }
  if (relres) {
    k_colnorm2<<<(unsigned)nrhs, 256, 0, st>>>(Rc, Mt, Mt, nrm);
    AZ_HIP(hipGetLastError());
    k_colnorm2<<<(unsigned)nrhs, 256, 0, st>>>(B, ldb, Mt, nrm + nrhs);
    AZ_HIP(hipGetLastError());
    k_ratio_sqrt<<<(unsigned)((nrhs + 255) / 256), 256, 0, st>>>(nrm, nrm + nrhs, relres, nrhs);
    AZ_HIP(hipGetLastError());
  }
  return AZRBF_OK;
}

}  // namespace az
