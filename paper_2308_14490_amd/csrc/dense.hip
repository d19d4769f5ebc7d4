// Low-rank stage of the AZ method on gfx950 (section 3.2.3, "Low-rank solver
// for Ax = b"): a Gaussian sketch Omega, the sketch W = (A - A Z* A) Omega,
// its SVD through a Householder tall-skinny QR and a one-sided Jacobi SVD of
// the small triangular factor, and the per-right-hand-side solve of
// Algorithm 1 with optional refinement passes.
//
// Sketch widths k <= 64: every TSQR block holds RB x k values in registers
// (tsqr.hip), the Jacobi SVD of the k x k factor runs in one workgroup.
#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace az {

constexpr int KMAX = 64;       // largest sketch width of this path

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

__device__ __forceinline__ void gaussian_quad(uint64_t seed, int64_t rows, int64_t cols, double* __restrict__ dst,
                                              int64_t ld, int64_t q, int64_t c) {
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

__global__ void k_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* __restrict__ dst, int64_t ld) {
  gaussian_quad(seed, rows, cols, dst, ld, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y);
}

int dense_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* dst, int64_t ld, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return AZRBF_OK;
  const int64_t nq = (rows + 3) / 4;
  Prof pr("gaussian", 8.0 * rows * cols, st);
  launch_kernel(k_gaussian, dim3((unsigned)((nq + 255) / 256), (unsigned)cols), 256, 0, st, seed, rows, cols, dst, ld);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ TSQR

// TSQR blocks (the block QR kernel lives in tsqr.hip) hold RB rows (a tile
// shape: 16384 / k by default, or the autotuner's); the Q formation below
// uses the same row blocking.
constexpr int TSQR_THREADS = 256;

// E_b = H_0 ... H_{k-1} [C_b; 0] = [C_b; 0] - V (T (V_top^T C_b)) for block b
// (compact WY; V_top = the block's first k reflector rows, unit lower
// triangular).  C_b is rows b*k.. of the level above's explicit Q (Cup), or
// the identity at the top (Cup null).  The k x k products give each thread
// several independent outputs, and each row's k outputs accumulate side by
// side, so no long chain of dependent FMAs forms.
template <int K>
__device__ __forceinline__ void formq_block(const double* __restrict__ V, int64_t ldv, const double* __restrict__ Tin,
                                            int64_t m, const double* __restrict__ Cup, int64_t ldc,
                                            double* __restrict__ E, int64_t lde, int RB, int64_t blk) {
  constexpr int LD = K + 1;
  constexpr int PER = K * K / TSQR_THREADS > 0 ? K * K / TSQR_THREADS : 1;   // outputs per thread
  __shared__ double Cb[K * LD];      // C_b[l][c] at c * LD + l
  __shared__ __align__(16) double Vt[K * LD];   // V_top[l][i] at i * LD + l
  __shared__ double Tm[K * LD];      // T[i][l] at l * LD + i
  __shared__ double Xs[K * LD];      // X = V_top^T C_b, X[l][c] at c * LD + l
  double* Mr = Vt;                   // M = T X, row-major (M[l][c] at l * K + c), over V_top once used
  const int t = threadIdx.x;
  const int64_t r0 = blk * RB;
  const double* Tb = Tin + blk * K * K;
  for (int e = t; e < K * K; e += TSQR_THREADS) {
    const int r = e % K, c = e / K;
    Cb[c * LD + r] = Cup ? Cup[blk * K + r + ldc * c] : (r == c ? 1.0 : 0.0);
    Vt[c * LD + r] = r0 + r < m ? V[r0 + r + ldv * c] : 0.0;   // unit lower, zeros above
    Tm[c * LD + r] = Tb[e];                                     // T, upper triangular
  }
  __syncthreads();
  // thread: column c = t % K, rows i = t / K + (256 / K) q
  const int c0 = t % K, i0 = t / K;
  constexpr int IS = TSQR_THREADS / K > 0 ? TSQR_THREADS / K : 1;
  if (t < K * IS) {
    double acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.0;
#pragma unroll 4
    for (int l = 0; l < K; ++l) {          // X[i][c] = sum_{l >= i} V_top[l][i] C_b[l][c]
      const double cl = Cb[c0 * LD + l];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = i0 + IS * q;
        acc[q] = fma(l >= i ? Vt[i * LD + l] : 0.0, cl, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) Xs[c0 * LD + i0 + IS * q] = acc[q];
  }
  __syncthreads();
  if (t < K * IS) {
    double acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = 0.0;
#pragma unroll 4
    for (int l = 0; l < K; ++l) {          // M[i][c] = sum_{l >= i} T[i][l] X[l][c]
      const double xl = Xs[c0 * LD + l];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = i0 + IS * q;
        acc[q] = fma(l >= i ? Tm[l * LD + i] : 0.0, xl, acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) Mr[(i0 + IS * q) * K + c0] = acc[q];
  }
  __syncthreads();
  // rows: E[r][c] = C_b[r][c] (r < K) - sum_l V[r][l] M[l][c], all c at once.
  // The row's reflector entries are streamed LC at a time, the next LC loads
  // issued before the current LC are used, so the loads' latency overlaps the
  // products instead of stalling each step.
  constexpr int CH = K < 32 ? K : 32;    // columns per pass (registers)
  constexpr int LC = 8;                  // reflector entries per load batch
#pragma unroll 1
  for (int r = t; r < RB; r += TSQR_THREADS) {
    const int64_t gi = r0 + r;
    if (gi >= m) break;
    const double* vrow = V + gi;
#pragma unroll
    for (int c0p = 0; c0p < K; c0p += CH) {
      double acc[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = r < K ? Cb[(c0p + c) * LD + r] : 0.0;
      double vb[LC];
#pragma unroll
      for (int e = 0; e < LC; ++e) vb[e] = vrow[ldv * e];
#pragma unroll 1
      for (int l0 = 0; l0 < K; l0 += LC) {
        double vn[LC];   // the next batch (wraps to the first at the end: always in bounds, unused)
#pragma unroll
        for (int e = 0; e < LC; ++e) vn[e] = vrow[ldv * ((l0 + LC + e) % K)];
#pragma unroll
        for (int e = 0; e < LC; ++e) {
          const double2* mrow = reinterpret_cast<const double2*>(Mr + (l0 + e) * K + c0p);
#pragma unroll
          for (int c = 0; c < CH; c += 2) {
            const double2 mm = mrow[c / 2];
            acc[c] = fma(-vb[e], mm.x, acc[c]);
            acc[c + 1] = fma(-vb[e], mm.y, acc[c + 1]);
          }
        }
#pragma unroll
        for (int e = 0; e < LC; ++e) vb[e] = vn[e];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) E[gi + lde * (c0p + c)] = acc[c];
    }
  }
}

template <int K>
__global__ void __launch_bounds__(TSQR_THREADS)
k_tsqr_formq(const double* __restrict__ V, int64_t ldv, const double* __restrict__ Tin, int64_t m,
             const double* __restrict__ Cup, int64_t ldc, double* __restrict__ E, int64_t lde, int RB) {
  formq_block<K>(V, ldv, Tin, m, Cup, ldc, E, lde, RB, blockIdx.x);
}

struct TsqrLevel {
  int64_t m, nb;
  double* A;     // level input; overwritten by the level's reflectors
  double* tau;   // compact-WY T factors, nb x (k x k)
  double* R;     // stacked R factors (nb*k x k): the next level's input
};

static void tsqr_plan(int64_t m, int k, int RB, std::vector<TsqrLevel>& lv, int64_t* scratch_doubles,
                      int64_t* e_doubles) {
  lv.clear();
  int64_t mm = m, tot = 0, emax = 0;
  while (true) {
    TsqrLevel L{};
    L.m = mm;
    L.nb = (mm + RB - 1) / RB;
    lv.push_back(L);
    tot += 2 * L.nb * k * k;   // T factors + stacked R
    if (lv.size() > 1) emax = std::max(emax, mm * k);
    if (L.nb == 1) break;
    mm = L.nb * k;
  }
  *scratch_doubles = tot;
  *e_doubles = emax;
}

// Scratch for every tile shape: the smallest blocks (256 rows) make the
// most of them.
static int64_t tsqr_scratch_doubles(int64_t m, int k) {
  std::vector<TsqrLevel> lv;
  int64_t s, e;
  tsqr_plan(m, k, 256, lv, &s, &e);
  return s + 2 * e;
}

__global__ void k_copy_doubles(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// W (m x k, leading dimension ld) is destroyed (level-0 reflectors); Q (m x k,
// ld) and R (k x k, ld k) out.
// after_first, if given, runs once the first level (the leaf blocks, the only
// level that spreads over the whole GPU) has been queued.
static int tsqr(double* W, int64_t m, int64_t ld, int k, int rb, double* scratch, double* Q, double* R,
                hipStream_t st, hipEvent_t r_ready = nullptr, const std::function<int()>* after_first = nullptr) {
  if (!tsqr_rows_ok(k, rb)) return AZRBF_EUNSUPPORTED;
  std::vector<TsqrLevel> lv;
  int64_t sd, ed;
  tsqr_plan(m, k, rb, lv, &sd, &ed);
  double* p = scratch;
  for (size_t l = 0; l < lv.size(); ++l) {
    lv[l].tau = p;             // T factors, nb x (k x k)
    p += lv[l].nb * k * k;
    lv[l].R = p;
    p += lv[l].nb * k * k;
    lv[l].A = l == 0 ? W : lv[l - 1].R;
  }
  double* Ebuf[2] = {p, p + ed};
  for (size_t l = 0; l < lv.size(); ++l) {
    const TsqrLevel& L = lv[l];
    Prof pr(l == 0 ? "tsqr_block" : "tsqr_block (tree)", 16.0 * L.m * k + 8.0 * L.nb * k * (k + 1), st);
    const int64_t lda = l == 0 ? ld : L.m;
    AZ_TRY(tsqr_block_qr(L.A, lda, L.m, k, rb, L.R, L.nb * k, L.A, lda, L.tau, st));
    if (l == 0 && after_first) AZ_TRY((*after_first)());
  }
  // (a kernel rather than a runtime copy: a launch does not block the host)
  launch_kernel(k_copy_doubles, (unsigned)((k * k + 255) / 256), 256, 0, st, lv.back().R, R, (int64_t)k * k);
  AZ_HIP(hipGetLastError());
  if (r_ready) AZ_HIP(hipEventRecord(r_ready, st));   // R is final; Q is formed below
  const double* up = nullptr;
  int64_t ldup = 0;
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    const TsqrLevel& L = lv[l];
    double* E = l == 0 ? Q : Ebuf[l & 1];
    const int64_t lda = l == 0 ? ld : L.m;
    Prof pr(l == 0 ? "tsqr_formq" : "tsqr_formq (tree)", 16.0 * L.m * k + 8.0 * L.nb * k * (k + 1), st);
    auto formq = k == 16 ? k_tsqr_formq<16> : k == 32 ? k_tsqr_formq<32> : k_tsqr_formq<64>;
    launch_kernel(formq, (unsigned)L.nb, TSQR_THREADS, 0, st, L.A, lda, L.tau, L.m, up, ldup, E, lda, rb);
    AZ_HIP(hipGetLastError());
    up = E;
    ldup = L.m;
  }
  return AZRBF_OK;
}

int64_t tsqr_scratch(int64_t m, int k) { return tsqr_scratch_doubles(m, k); }
int tsqr_panel(double* W, int64_t m, int k, int rb, double* scratch, double* Q, double* R, hipStream_t st) {
  return tsqr(W, m, m, k, rb, scratch, Q, R, st);
}

int plan_tsqr_rows(const Plan& P, int k) {
  const int slot = k == 16 ? 0 : k == 32 ? 1 : 2;
  const int rb = P.tsqr_rb[slot];
  return rb > 0 && tsqr_rows_ok(k, rb) ? rb : tsqr_block_rows(k);
}

// ------------------------------------------------------------------ Jacobi SVD

// 1/x and 1/sqrt(x) from the hardware estimates refined by one Newton step
// (relative error near the FP64 rounding unit).  They keep the dependency
// chain of a rotation short; the rotation stays orthogonal because c and s
// are formed from the same t.
__device__ __forceinline__ double fast_rcp(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double fast_rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Sums over groups of 8 and 16 consecutive lanes by DPP moves (quad
// permutations, then the half-row and row mirrors).  Every lane of a group
// ends with the same bits: each stage adds the same two values in either order.
template <int CTRL>
__device__ __forceinline__ double jdpp(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double sum8(double x) {
  x += jdpp<0xB1>(x);
  x += jdpp<0x4E>(x);
  return x + jdpp<0x141>(x);
}
__device__ __forceinline__ double sum16(double x) {
  x = sum8(x);
  return x + jdpp<0x140>(x);
}
// The same sums for two or three values, stage by stage, so that the
// independent DPP moves and adds of one stage overlap instead of each sum
// waiting for the previous one (bitwise the same results as separate sums).
template <int CTRL>
__device__ __forceinline__ void jstage2(double& a, double& b) {
  const double ta = jdpp<CTRL>(a), tb = jdpp<CTRL>(b);
  a += ta;
  b += tb;
}
template <int CTRL>
__device__ __forceinline__ void jstage3(double& a, double& b, double& c) {
  const double ta = jdpp<CTRL>(a), tb = jdpp<CTRL>(b), tc = jdpp<CTRL>(c);
  a += ta;
  b += tb;
  c += tc;
}
__device__ __forceinline__ void sum8x2(double& a, double& b) {
  jstage2<0xB1>(a, b);
  jstage2<0x4E>(a, b);
  jstage2<0x141>(a, b);
}
__device__ __forceinline__ void sum16x3(double& a, double& b, double& c) {
  jstage3<0xB1>(a, b, c);
  jstage3<0x4E>(a, b, c);
  jstage3<0x141>(a, b, c);
  jstage3<0x140>(a, b, c);
}

// Truncated pseudo-inverse of the k x k triangular factor R (k in {16, 32,
// 64}) by a preconditioned one-sided Jacobi SVD, in one block of 8k threads.
//
// Preconditioning: Householder QR of the transpose, R^T = Q2 R2, with Q2
// formed explicitly (k - 1 reflectors; per reflector one 16-lane group forms
// the vector, then every 8-lane slot updates one column of R2 and one row of
// Q2).  One-sided Jacobi on R2^T then converges in fewer sweeps than on R^T,
// because the QR concentrates the weight of R2's rows on the diagonal.
//
// Jacobi: the columns of A = R2^T are orthogonalised by plane rotations from
// the right, A W = U S, with W accumulated from W0 = Q2, so that
// R = U S (Q2 W)^T and the pseudo-inverse is sum_i (Q2 W)_i u_i^T / s_i.
// Round-robin (circle) schedule: in round r pair 0 is (r, k-1) and pair
// i > 0 is ((r+i) mod (k-1), (r-i) mod (k-1)); k/2 pairs per round, one
// 16-lane DPP row per pair.  A rotation is skipped when
// |a_p . a_q| <= tol sqrt(|a_p|^2 |a_q|^2); sweeps stop when none happens.
// The rotation angle theta solves tan 2theta = 2 a_p.a_q / (|a_q|^2 - |a_p|^2)
// with |theta| <= pi/4; c and s come from the half-angle identities
// c^2 = (1 + cos 2theta)/2, s = sin 2theta / (2c).
// On exit: sig (descending), info = {rank, sweeps} with rank = #{sigma > thr},
// thr = tau_k sqrt(max D) read from the device, Pm = sum_{i < rank} (Q2 W)_i u_i^T / sigma_i.
template <int K>
__device__ __forceinline__ void jacobi_block(const double* __restrict__ R, double tau_k,
                                             const double* __restrict__ dmax, double tol, int max_sweeps,
                                             double* __restrict__ sig, double* __restrict__ Pm,
                                             int* __restrict__ info) {
  constexpr int LD = K + 1;       // column stride (doubles) of the LDS matrices
  constexpr int NT = 8 * K;       // threads
  constexpr int RPL = K / 16;     // rows per lane in a rotation
  constexpr int EPL = K / 8;      // elements per lane in a reflector update
  constexpr int KM1 = K - 1;
  __shared__ double A[K * LD];    // A[c * LD + r] = entry (r, c)
  __shared__ double W[K * LD];    // Q2, then Q2 W; same layout
  __shared__ double sv[K], inv2[K];
  __shared__ int ord[K];
  const int t = threadIdx.x;
  for (int i = t; i < K * K; i += NT) {
    const int r = i % K, c = i / K;
    A[r * LD + c] = R[r + (int64_t)K * c];        // A = R^T
    W[c * LD + r] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- Householder QR of A; Q2 accumulated into W from the right
  {
    // Every 8-lane slot forms reflector j itself from column j of A (the same
    // sums in the same order in every slot, so all slots hold the same bits),
    // which saves a serial step and a barrier per reflector.  Column j is
    // still being read during step j, so its final entries (alpha, zeros)
    // are written by slot j in step j + 1, when no slot reads it.
    const int slot = t >> 3, sl = t & 7;
    double alpha_prev = 0.0;
    for (int j = 0; j < KM1; ++j) {
      if (j > 0 && slot == j - 1) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const int i = j - 1 + sl + 8 * e;
          if (i < K) A[(j - 1) * LD + i] = i == j - 1 ? alpha_prev : 0.0;
        }
      }
      const bool col = slot > j;                 // this slot's column of A needs the reflector
      double vv[EPL], ac[EPL], wr[EPL];
      double ss = 0.0;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = j + sl + 8 * e;
        const bool ok = i < K;
        vv[e] = ok ? A[j * LD + i] : 0.0;
        ac[e] = ok && col ? A[slot * LD + i] : 0.0;
        wr[e] = ok ? W[i * LD + slot] : 0.0;     // entry (slot, i) of Q2
        ss = fma(vv[e], vv[e], ss);
      }
      const double x0 = A[j * LD + j];
      ss = sum8(ss);
      const double nrm = sqrt(ss);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double beta = nrm == 0.0 ? 0.0 : 1.0 / (nrm * (nrm + fabs(x0)));
      alpha_prev = alpha;
      double dc = 0.0, dr = 0.0;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        if (sl + 8 * e == 0) vv[e] = x0 - alpha;   // the entry i = j
        dc = fma(vv[e], ac[e], dc);
        dr = fma(vv[e], wr[e], dr);
      }
      sum8x2(dc, dr);
      dc *= beta;
      dr *= beta;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = j + sl + 8 * e;
        if (i < K) {
          if (col) A[slot * LD + i] = fma(-dc, vv[e], ac[e]);
          W[i * LD + slot] = fma(-dr, vv[e], wr[e]);
        }
      }
      __syncthreads();
    }
    if (slot == KM1 - 1) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = KM1 - 1 + sl + 8 * e;
        if (i < K) A[(KM1 - 1) * LD + i] = i == KM1 - 1 ? alpha_prev : 0.0;
      }
    }
    __syncthreads();
    // A now holds R2 (column-major); the Jacobi works on its transpose
    for (int i = t; i < K * K; i += NT) {
      const int r = i % K, c = i / K;
      if (r < c) {
        const double a = A[c * LD + r];
        A[c * LD + r] = A[r * LD + c];
        A[r * LD + c] = a;
      }
    }
    __syncthreads();
  }

  // ---- one-sided Jacobi on the columns of A
  const int pi = t >> 4, gl = t & 15;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
    for (int round = 0; round < KM1; ++round) {
      const int p = pi == 0 ? round : (round + pi) % KM1;
      const int q = pi == 0 ? KM1 : (round - pi + KM1) % KM1;
      double x[RPL], y[RPL], vx[RPL], vy[RPL];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        const int r = gl + 16 * e;
        x[e] = A[p * LD + r];
        y[e] = A[q * LD + r];
        vx[e] = W[p * LD + r];
        vy[e] = W[q * LD + r];
      }
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        al = fma(x[e], x[e], al);
        be = fma(y[e], y[e], be);
        ga = fma(x[e], y[e], ga);
      }
      sum16x3(al, be, ga);
      // (|ga| > 1e-150 keeps 4 ga^2 a normal number below)
      if (ga * ga > tol2 * (al * be) && fabs(ga) > 1e-150) {
        rotated = 1;
        const double d = be - al, g2 = 2.0 * ga;
        const double rq = fast_rsq(fma(d, d, g2 * g2));
        const double cos2 = fabs(d) * rq;
        const double sin2 = (d >= 0.0 ? g2 : -g2) * rq;
        const double h = fma(0.5, cos2, 0.5);
        const double rh = fast_rsq(h);
        const double c = h * rh, s = 0.5 * sin2 * rh;
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const int r = gl + 16 * e;
          A[p * LD + r] = c * x[e] - s * y[e];
          A[q * LD + r] = s * x[e] + c * y[e];
          W[p * LD + r] = c * vx[e] - s * vy[e];
          W[q * LD + r] = s * vx[e] + c * vy[e];
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }

  if (t < K) {
    double s2 = 0.0;
    for (int r = 0; r < K; ++r) s2 = fma(A[t * LD + r], A[t * LD + r], s2);
    sv[t] = sqrt(s2);
  }
  __syncthreads();
  if (t < K) {   // position of column t in descending order (ties by index)
    int pos = 0;
    for (int j = 0; j < K; ++j) pos += (sv[j] > sv[t]) || (sv[j] == sv[t] && j < t);
    ord[pos] = t;
    inv2[t] = sv[t] > 0.0 ? 1.0 / (sv[t] * sv[t]) : 0.0;
  }
  __syncthreads();
  const double thr = tau_k * sqrt(*dmax);   // tau ||A^c|| sqrt(k), ||A^c|| = sqrt(max D)
  int rank = 0;
  for (int i = 0; i < K; ++i) rank += sv[i] > thr;
  if (t == 0) {
    info[0] = rank;
    info[1] = sweep;
  }
  if (t < K) sig[t] = sv[ord[t]];
  // Pm[r][c] = sum_i (Q2 W)[r][i] U[c][i] / s_i = sum_i (Q2 W)[r][i] A[c][i] / s_i^2
  for (int e = t; e < K * K; e += NT) {
    const int r = e % K, c = e / K;
    double acc = 0.0;
    for (int ii = 0; ii < rank; ++ii) {
      const int i = ord[ii];
      acc = fma(W[i * LD + r] * inv2[i], A[i * LD + c], acc);
    }
    Pm[r + (int64_t)K * c] = acc;
  }
}

template <int K>
__global__ void __launch_bounds__(8 * K)
k_jacobi(const double* __restrict__ R, double tau_k, const double* __restrict__ dmax, double tol, int max_sweeps,
         double* __restrict__ sig, double* __restrict__ Pm, int* __restrict__ info) {
  jacobi_block<K>(R, tau_k, dmax, tol, max_sweeps, sig, Pm, info);
}

int launch_jacobi(const double* R, int k, double tau_k, const double* dmax, double tol, int max_sweeps, double* sig,
                  double* Pm, int* info, hipStream_t st) {
  if (k == 16) launch_kernel(k_jacobi<16>, 1, 128, 0, st, R, tau_k, dmax, tol, max_sweeps, sig, Pm, info);
  else if (k == 32) launch_kernel(k_jacobi<32>, 1, 256, 0, st, R, tau_k, dmax, tol, max_sweeps, sig, Pm, info);
  else if (k == 64) launch_kernel(k_jacobi<64>, 1, 512, 0, st, R, tau_k, dmax, tol, max_sweeps, sig, Pm, info);
  else return AZRBF_EUNSUPPORTED;
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// ------------------------------------------------------------------ skinny GEMMs

// Out = alpha * A B + beta * Cin; A is m x k (ld lda), B is k x ncol (ld ldb,
// small), Out/Cin m x ncol.  Each thread owns one row and up to NC columns;
// B is staged in LDS with the columns of one reduction index contiguous.
// (NC = 16: more blocks in flight beat streaming A once with 64 accumulators
// per thread, measured on the 65536 x 32 by 32 x 64 case.)  The G column
// groups of a row block read the same 256 rows of A; blocks are numbered so
// that those G blocks are dispatched together and to the same XCD (block b
// runs on XCD b mod 8), where they share A through that XCD's L2 instead of
// each fetching it from HBM.  Out may alias Cin (each element is read and
// written by the same thread).
template <int NC>
__global__ void __launch_bounds__(256)
k_gemm_nn(const double* __restrict__ A, int64_t lda, int64_t m, int k, const double* __restrict__ B, int64_t ldb,
          int64_t ncol, double alpha, const double* Cin, int64_t ldci, double beta, double* Out, int64_t ldo,
          int64_t nrb, int G) {
  __shared__ double bs[KMAX * NC];   // bs[c * NC + v] = B(c, v0 + v)
  // linear block L = (rb / 8) (8 G) + cg 8 + rb mod 8
  const int64_t L = blockIdx.x;
  const int64_t q = L / (8 * G), rem = L % (8 * G);
  const int cg = (int)(rem / 8);
  const int64_t rb = q * 8 + rem % 8;
  if (rb >= nrb) return;
  const int64_t i = rb * 256 + threadIdx.x;
  const int64_t v0 = (int64_t)cg * NC;
  const int nv = (int)std::min<int64_t>(NC, ncol - v0);
  for (int e = threadIdx.x; e < k * NC; e += blockDim.x) {
    const int c = e % k, v = e / k;
    bs[c * NC + v] = v < nv ? B[c + ldb * (v0 + v)] : 0.0;
  }
  __syncthreads();
  if (i >= m) return;
  double acc[NC];
#pragma unroll
  for (int v = 0; v < NC; ++v) acc[v] = 0.0;
  for (int c = 0; c < k; c += 4) {   // k is a multiple of 16: four loads in flight
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = A[i + lda * (c + u)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < NC; ++v) acc[v] = fma(a[u], bs[(c + u) * NC + v], acc[v]);
  }
#pragma unroll
  for (int v = 0; v < NC; ++v) {
    if (v < nv) {
      const int64_t col = v0 + v;
      const double r = alpha * acc[v];
      Out[i + ldo * col] = beta == 0.0 ? r : fma(beta, Cin[i + ldci * col], r);
    }
  }
}

constexpr int NORM_CHUNKS = 32;
int relres_chunks() { return NORM_CHUNKS; }

// part[col * NORM_CHUNKS + chunk] = sum of squares over the chunk's rows.
__global__ void __launch_bounds__(256)
k_colnorm2_part(const double* __restrict__ X, int64_t ld, int64_t m, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t col = blockIdx.y;
  const int64_t per = (m + NORM_CHUNKS - 1) / NORM_CHUNKS;
  const int64_t lo = blockIdx.x * per, hi = std::min<int64_t>(m, lo + per);
  const double* x = X + ld * col;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = lo + threadIdx.x;
  for (; i + 256 < hi; i += 512) {
    s0 = fma(x[i], x[i], s0);
    s1 = fma(x[i + 256], x[i + 256], s1);
  }
  if (i < hi) s0 = fma(x[i], x[i], s0);
  double s = wave_sum(s0 + s1);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[col * NORM_CHUNKS + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[c] = sqrt(sum num parts / sum den parts), parts summed in order.
__global__ void k_relres(const double* __restrict__ num, const double* __restrict__ den, double* out,
                         int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < NORM_CHUNKS; ++i) {
    a += num[c * NORM_CHUNKS + i];
    b += den[c * NORM_CHUNKS + i];
  }
  out[c] = b > 0.0 ? sqrt(a / b) : sqrt(a);
}

static int gemm_nn(const double* A, int64_t lda, int64_t m, int k, const double* B, int64_t ldb, int64_t ncol,
                   double alpha, const double* Cin, int64_t ldci, double beta, double* Out, int64_t ldo,
                   hipStream_t st) {
  if (m <= 0 || ncol <= 0) return AZRBF_OK;
  const int64_t nrb = (m + 255) / 256;                 // row blocks
  const int G = (int)((ncol + 15) / 16);               // column groups of 16
  const int64_t nblk = (nrb + 7) / 8 * 8 * G;          // whole groups of eight row blocks
  Prof pr("gemm_nn", 8.0 * m * (k + ncol * (beta != 0.0 ? 2.0 : 1.0)), st);
  launch_kernel(k_gemm_nn<16>, (unsigned)nblk, 256, 0, st, A, lda, m, k, B, ldb, ncol, alpha, Cin, ldci, beta, Out,
                ldo, nrb, G);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

int relres_norms(const double* R, int64_t ldr, const double* B, int64_t ldb, int64_t m, int64_t ncol,
                        double* scratch, double* out, hipStream_t st) {
  const dim3 grid(NORM_CHUNKS, (unsigned)ncol);
  Prof pr("relres", 16.0 * m * ncol, st);
  launch_kernel(k_colnorm2_part, grid, 256, 0, st, R, ldr, m, scratch);
  AZ_HIP(hipGetLastError());
  launch_kernel(k_colnorm2_part, grid, 256, 0, st, B, ldb, m, scratch + NORM_CHUNKS * ncol);
  AZ_HIP(hipGetLastError());
  launch_kernel(k_relres, (unsigned)((ncol + 255) / 256), 256, 0, st, scratch, scratch + NORM_CHUNKS * ncol, out,
                ncol);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

// ------------------------------------------------------------------ factor

// The factor's buffers (kept across factorisations of the plan).
static int dense_factor_alloc(Plan& P) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt, Ld = P.Mtp;
  if (!P.Om) {
    AZ_TRY(P.alloc((void**)&P.Om, sizeof(double) * N * k));
    AZ_TRY(P.alloc((void**)&P.Om2, sizeof(double) * N * k));
    AZ_TRY(P.alloc((void**)&P.Yf, sizeof(double) * Ld * k));
    AZ_TRY(P.alloc((void**)&P.Yf2, sizeof(double) * Ld * k));
    AZ_TRY(P.alloc((void**)&P.Q, sizeof(double) * Ld * k));
    AZ_TRY(P.alloc((void**)&P.Rf, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.sig, sizeof(double) * k));
    AZ_TRY(P.alloc((void**)&P.Pm, sizeof(double) * k * k));
    const int64_t sd = tsqr_scratch_doubles(Mt, k) + 8;
    AZ_TRY(P.alloc((void**)&P.dscr, sizeof(double) * sd));
    P.dscr_bytes = sizeof(double) * sd;
  }
  return AZRBF_OK;
}

int dense_factor_enqueue(Plan& P, hipStream_t st, hipEvent_t after_sketch, const std::function<int()>& on_sketch,
                         const std::function<int()>& before_products) {
  const int k = P.k;
  // the Jacobi kernel pairs k/2 columns over 256 threads: 512 / k must be a shuffle width
  if (k != 16 && k != 32 && k != 64) return AZRBF_EUNSUPPORTED;
  const int64_t N = P.N, Mt = P.Mt;
  const int64_t Ld = P.Mtp;   // leading dimension of the row-space matrices (whole 128-byte lines)
  AZ_TRY(dense_factor_alloc(P));
  double* Zy = P.Om2;                  // N x k scratch, later Omega P
  double* W = P.Yf2;                   // Mt x k sketch (ld Ld), later (A Omega) P
  P.ldq = Ld;
  double* tq = P.dscr;                 // TSQR scratch
  int* info = (int*)(tq + tsqr_scratch_doubles(Mt, k));
  AZ_TRY(dense_gaussian(P.prob.seed, N, k, P.Om, N, st));
  AZ_TRY(ops_apply_A(P, P.Om, N, k, 1.0, 0.0, nullptr, 0, P.Yf, Ld, st));     // Y = A Omega
  AZ_TRY(ops_apply_AZ(P, P.Yf, Ld, k, -1.0, 1.0, P.Yf, Ld, W, Ld, Zy, st));  // W = Y - A Z* Y
  // What follows the leaf level of the TSQR is latency-bound (a few blocks
  // per level, then one workgroup for the Jacobi SVD): work on other streams
  // starts there.  (Started before the leaf level, it competed with the leaf
  // blocks for the CUs and stretched that level from 48 to 79 us.)
  const std::function<int()> after_first = [&]() -> int {
    if (after_sketch) AZ_HIP(hipEventRecord(after_sketch, st));
    if (on_sketch) AZ_TRY(on_sketch());
    return AZRBF_OK;
  };
  // TSQR destroys W; the QR is of the sketch, W is then free scratch.  The
  // Jacobi SVD needs only R: it runs on a second stream while this one forms
  // the explicit Q, and the products below (which overwrite W) wait for both.
  const double tau_k = P.tau * sqrt((double)k);   // threshold tau_k ||A^c||, ||A^c|| read on the device
  hipStream_t js = nullptr;
  hipEvent_t eR = nullptr, eJ = nullptr;
  if (!prof_enabled() && side_stream(P.device, &js) == AZRBF_OK &&
      hipEventCreateWithFlags(&eR, hipEventDisableTiming) == hipSuccess &&
      hipEventCreateWithFlags(&eJ, hipEventDisableTiming) == hipSuccess && js != st) {
  } else {
    js = st;
  }
  int rc = tsqr(W, Mt, Ld, k, plan_tsqr_rows(P, k), tq, P.Q, P.Rf, st, js != st ? eR : nullptr, &after_first);
  if (!rc && js != st && hipStreamWaitEvent(js, eR, 0) != hipSuccess) rc = AZRBF_EHIP;
  if (!rc) {
    Prof pj("jacobi", 8.0 * 3 * k * k, js);
    rc = launch_jacobi(P.Rf, k, tau_k, P.dred, 4.0 * k * 1.1102230246251565e-16, 40, P.sig, P.Pm, info, js);
  }
  if (!rc && js != st && hipEventRecord(eJ, js) != hipSuccess) rc = AZRBF_EHIP;
  if (!rc && before_products) rc = before_products();
  if (!rc && js != st && hipStreamWaitEvent(st, eJ, 0) != hipSuccess) rc = AZRBF_EHIP;
  if (eR) (void)hipEventDestroy(eR);
  if (eJ) (void)hipEventDestroy(eJ);
  if (rc) {
    if (js != st) (void)hipStreamSynchronize(js);
    return rc;
  }
  // Omega P and (A Omega) P: the solve needs only these (y = P Q^T c)
  AZ_TRY(gemm_nn(P.Om, N, N, k, P.Pm, k, k, 1.0, nullptr, 0, 0.0, Zy, N, st));
  AZ_TRY(gemm_nn(P.Yf, Ld, Mt, k, P.Pm, k, k, 1.0, nullptr, 0, 0.0, W, Ld, st));
  std::swap(P.Om, P.Om2);
  std::swap(P.Yf, P.Yf2);
  P.dinfo = info;
  return AZRBF_OK;
}

// Waits for the factor queued by dense_factor_enqueue and reads its rank (the
// copy is queued here: a copy to pageable memory can block the host).
int dense_factor_finish(Plan& P, hipStream_t st) {
  AZ_HIP(hipMemcpyAsync(P.hinfo, P.dinfo, sizeof(P.hinfo), hipMemcpyDeviceToHost, st));
  AZ_HIP(hipStreamSynchronize(st));
  P.rank = P.hinfo[0];
  P.sweeps = P.hinfo[1];
  P.factored = true;
  return 10 * (int64_t)P.rank > 9 * (int64_t)P.k ? AZRBF_ERANK : AZRBF_OK;   // too narrow: see factor_plan
}

int plan_fetch_rank(Plan& P) {
  if (!P.rank_pending) return AZRBF_OK;
  AZ_HIP(hipMemcpyAsync(P.hinfo, P.dinfo, sizeof(P.hinfo), hipMemcpyDeviceToHost, P.factor_stream));
  AZ_HIP(hipStreamSynchronize(P.factor_stream));
  P.rank = P.hinfo[0];
  P.sweeps = P.hinfo[1];
  P.rank_pending = false;
  return AZRBF_OK;
}

int dense_factor(Plan& P, hipStream_t st) {
  AZ_TRY(dense_factor_enqueue(P, st, nullptr));
  return dense_factor_finish(P, st);
}

// ------------------------------------------------------------------ grouped factor

// The factorisation of many 1D plans on the single-kernel transform as one
// launch sequence: the same kernels in the same order per plan as
// dense_factor (so the same factor bit for bit), each step one launch for all
// plans (per size class for the transforms, per sketch width and row blocking
// for the TSQR levels).  The per-plan path overlaps the Jacobi SVD with the Q
// formation on a second stream; here they follow each other.

namespace {

struct GaussOp {
  uint64_t seed;
  int64_t rows, cols;
  double* dst;
  int64_t ld;
};
struct FormqOp {
  const double* V;
  int64_t ldv;
  const double* T;
  int64_t m;
  const double* Cup;
  int64_t ldc;
  double* E;
  int64_t lde;
  int64_t nb;
  int rb;
};
struct JacOp {
  const double* R;
  double tau_k;
  const double* dmax;
  double* sig;
  double* Pm;
  int* info;
};
struct ProdOp {     // Out = A B, A m x k (ld lda), B k x k (ld k), Out ld ldo
  const double* A;
  int64_t lda, m;
  const double* B;
  double* Out;
  int64_t ldo;
  int k;
};
struct CopyOp {
  const double* src;
  double* dst;
  int64_t n;
};

__global__ void __launch_bounds__(256) k_bat_gaussian(const GaussOp* __restrict__ ops) {
  const GaussOp o = ops[blockIdx.z];
  gaussian_quad(o.seed, o.rows, o.cols, o.dst, o.ld, (int64_t)blockIdx.x * 256 + threadIdx.x, blockIdx.y);
}

template <int K>
__global__ void __launch_bounds__(TSQR_THREADS) k_bat_formq(const FormqOp* __restrict__ ops) {
  const FormqOp o = ops[blockIdx.y];
  if ((int64_t)blockIdx.x >= o.nb) return;
  formq_block<K>(o.V, o.ldv, o.T, o.m, o.Cup, o.ldc, o.E, o.lde, o.rb, blockIdx.x);
}

template <int K>
__global__ void __launch_bounds__(8 * K) k_bat_jacobi(const JacOp* __restrict__ ops, double tol, int max_sweeps) {
  const JacOp o = ops[blockIdx.x];
  jacobi_block<K>(o.R, o.tau_k, o.dmax, tol, max_sweeps, o.sig, o.Pm, o.info);
}

// as k_gemm_nn<16> with alpha = 1, beta = 0 (the same sums in the same order)
__global__ void __launch_bounds__(256) k_bat_prod(const ProdOp* __restrict__ ops) {
  const ProdOp o = ops[blockIdx.z];
  const int v0 = blockIdx.y * 16;
  if ((int64_t)blockIdx.x * 256 >= o.m || v0 >= o.k) return;
  __shared__ double bs[KMAX * 16];
  const int k = o.k;
  for (int e = threadIdx.x; e < k * 16; e += 256) {
    const int c = e % k, v = e / k;
    bs[c * 16 + v] = o.B[c + (int64_t)k * (v0 + v)];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= o.m) return;
  double acc[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0;
  for (int c = 0; c < k; c += 4) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = o.A[i + o.lda * (c + u)];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = fma(a[u], bs[(c + u) * 16 + v], acc[v]);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) o.Out[i + o.ldo * (v0 + v)] = 1.0 * acc[v];
}

__global__ void __launch_bounds__(256) k_bat_copy(const CopyOp* __restrict__ ops) {
  const CopyOp o = ops[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < o.n) o.dst[i] = o.src[i];
}

}  // namespace

bool dense_factor_batchable(const Plan& P) {
  return P.dim == 1 && P.fused && !P.generic && P.Mb == 0 && (P.k == 16 || P.k == 32 || P.k == 64);
}

int dense_factor_batched(const std::vector<Plan*>& plans, std::vector<int>& rcs, hipStream_t st) {
  const int E = (int)plans.size();
  rcs.assign(E, AZRBF_OK);
  if (E == 0) return AZRBF_OK;
  if (E > 65535) return AZRBF_EINVAL;
  for (Plan* P : plans)
    if (!dense_factor_batchable(*P)) return AZRBF_EUNSUPPORTED;
  // entries in size-class order (the transforms take one launch per (n, s))
  std::vector<int> ord(E);
  for (int i = 0; i < E; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    return plans[a]->n != plans[b]->n ? plans[a]->n < plans[b]->n : plans[a]->s < plans[b]->s;
  });
  struct Lay {
    std::vector<TsqrLevel> lv;
    double* Eb[2];
    int rb;
    int* info;
  };
  std::vector<Lay> lay(E);
  int maxL = 0;
  for (int q = 0; q < E; ++q) {
    Plan& P = *plans[ord[q]];
    AZ_TRY(dense_factor_alloc(P));
    P.ldq = P.Mtp;
    Lay& L = lay[q];
    L.rb = plan_tsqr_rows(P, P.k);
    if (!tsqr_rows_ok(P.k, L.rb)) return AZRBF_EUNSUPPORTED;
    int64_t sd = 0, ed = 0;
    tsqr_plan(P.Mt, P.k, L.rb, L.lv, &sd, &ed);
    double* p = P.dscr;          // the same layout as tsqr()
    for (size_t l = 0; l < L.lv.size(); ++l) {
      L.lv[l].tau = p;
      p += L.lv[l].nb * P.k * P.k;
      L.lv[l].R = p;
      p += L.lv[l].nb * P.k * P.k;
      L.lv[l].A = l == 0 ? P.Yf2 : L.lv[l - 1].R;
    }
    L.Eb[0] = p;
    L.Eb[1] = p + ed;
    L.info = (int*)(P.dscr + tsqr_scratch_doubles(P.Mt, P.k));
    maxL = std::max(maxL, (int)L.lv.size());
  }
  // host descriptors
  std::vector<GaussOp> gauss(E);
  std::vector<BatOp> bop(3 * (size_t)E);
  std::vector<CopyOp> cop(E);
  std::vector<ProdOp> pop(2 * (size_t)E);
  int64_t maxq = 0, maxk = 0, maxrows = 0;
  for (int q = 0; q < E; ++q) {
    Plan& P = *plans[ord[q]];
    const int k = P.k;
    const int64_t N = P.N, Ld = P.Mtp;
    gauss[q] = GaussOp{P.prob.seed, N, k, P.Om, N};
    bop[q] = BatOp{P.geo, P.tw, P.Om, N, k, 1.0, 0.0, P.Yf, Ld, P.Yf, Ld};                 // Y = A Omega
    bop[E + q] = BatOp{P.geo, P.tw, P.Yf, Ld, k, 1.0, 0.0, P.Om2, N, P.Om2, N};           // Zy = Z* Y
    bop[2 * E + q] = BatOp{P.geo, P.tw, P.Om2, N, k, -1.0, 1.0, P.Yf, Ld, P.Yf2, Ld};     // W = Y - A Zy
    cop[q] = CopyOp{lay[q].lv.back().R, P.Rf, (int64_t)k * k};
    pop[q] = ProdOp{P.Om, N, N, P.Pm, P.Om2, N, k};                                         // Omega P
    pop[E + q] = ProdOp{P.Yf, Ld, P.Mt, P.Pm, P.Yf2, Ld, k};                                // (A Omega) P
    maxq = std::max(maxq, (N + 3) / 4);
    maxk = std::max<int64_t>(maxk, k);
    maxrows = std::max(maxrows, std::max(N, P.Mt));
  }
  struct Cls {
    int n, s, first, count;
    int64_t maxvec;
  };
  std::vector<Cls> cls;
  for (int q = 0; q < E; ++q) {
    const Plan& P = *plans[ord[q]];
    if (cls.empty() || cls.back().n != P.n || cls.back().s != P.s) cls.push_back(Cls{P.n, P.s, q, 0, 0});
    ++cls.back().count;
    cls.back().maxvec = std::max<int64_t>(cls.back().maxvec, P.k);
  }
  // TSQR levels (ascending) and Q formation (descending): per level, the
  // entries that have it, grouped by (k, rb) and by k
  struct Grp {
    int level, k, rb, first, count;
    int64_t maxnb;
  };
  std::vector<TsqrOp> top;
  std::vector<Grp> tg;
  std::vector<FormqOp> fop;
  std::vector<Grp> fg;
  for (int l = 0; l < maxL; ++l) {
    std::map<std::pair<int, int>, std::vector<int>> by;
    for (int q = 0; q < E; ++q)
      if ((int)lay[q].lv.size() > l) by[{plans[ord[q]]->k, lay[q].rb}].push_back(q);
    for (auto& kv : by) {
      Grp g{l, kv.first.first, kv.first.second, (int)top.size(), (int)kv.second.size(), 0};
      for (int q : kv.second) {
        Plan& P = *plans[ord[q]];
        const TsqrLevel& L = lay[q].lv[l];
        const int64_t lda = l == 0 ? P.Mtp : L.m;
        top.push_back(TsqrOp{L.A, lda, L.m, L.R, L.nb * P.k, L.A, lda, L.tau});
        g.maxnb = std::max(g.maxnb, L.nb);
      }
      tg.push_back(g);
    }
  }
  for (int l = maxL - 1; l >= 0; --l) {
    std::map<int, std::vector<int>> by;
    for (int q = 0; q < E; ++q)
      if ((int)lay[q].lv.size() > l) by[plans[ord[q]]->k].push_back(q);
    for (auto& kv : by) {
      Grp g{l, kv.first, 0, (int)fop.size(), (int)kv.second.size(), 0};
      for (int q : kv.second) {
        Plan& P = *plans[ord[q]];
        const Lay& Y = lay[q];
        const TsqrLevel& L = Y.lv[l];
        const int64_t lda = l == 0 ? P.Mtp : L.m;
        const bool top_level = l + 1 == (int)Y.lv.size();
        const double* up = top_level ? nullptr : (l + 1 == 0 ? P.Q : Y.Eb[(l + 1) & 1]);
        const int64_t ldup = top_level ? 0 : Y.lv[l + 1].m;
        double* Eo = l == 0 ? P.Q : Y.Eb[l & 1];
        fop.push_back(FormqOp{L.A, lda, L.tau, L.m, up, ldup, Eo, lda, L.nb, Y.rb});
        g.maxnb = std::max(g.maxnb, L.nb);
      }
      fg.push_back(g);
    }
  }
  std::vector<JacOp> jop;
  std::vector<Grp> jg;
  {
    std::map<int, std::vector<int>> by;
    for (int q = 0; q < E; ++q) by[plans[ord[q]]->k].push_back(q);
    for (auto& kv : by) {
      jg.push_back(Grp{0, kv.first, 0, (int)jop.size(), (int)kv.second.size(), 0});
      for (int q : kv.second) {
        Plan& P = *plans[ord[q]];
        jop.push_back(JacOp{P.Rf, P.tau * sqrt((double)P.k), P.dred, P.sig, P.Pm, lay[q].info});
      }
    }
  }
  // one upload of every descriptor
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t o_g = 0, o_b = al(o_g + sizeof(GaussOp) * gauss.size()), o_c = al(o_b + sizeof(BatOp) * bop.size()),
               o_p = al(o_c + sizeof(CopyOp) * cop.size()), o_t = al(o_p + sizeof(ProdOp) * pop.size()),
               o_f = al(o_t + sizeof(TsqrOp) * top.size()), o_j = al(o_f + sizeof(FormqOp) * fop.size()),
               total = al(o_j + sizeof(JacOp) * jop.size());
  char* host = nullptr;
  char* dev = nullptr;
  AZ_HIP(hipHostMalloc((void**)&host, total, hipHostMallocDefault));
  if (hipMalloc((void**)&dev, total) != hipSuccess) {
    (void)hipHostFree(host);
    return AZRBF_EHIP;
  }
  std::memcpy(host + o_g, gauss.data(), sizeof(GaussOp) * gauss.size());
  std::memcpy(host + o_b, bop.data(), sizeof(BatOp) * bop.size());
  std::memcpy(host + o_c, cop.data(), sizeof(CopyOp) * cop.size());
  std::memcpy(host + o_p, pop.data(), sizeof(ProdOp) * pop.size());
  std::memcpy(host + o_t, top.data(), sizeof(TsqrOp) * top.size());
  std::memcpy(host + o_f, fop.data(), sizeof(FormqOp) * fop.size());
  std::memcpy(host + o_j, jop.data(), sizeof(JacOp) * jop.size());
  int rc = hipMemcpyAsync(dev, host, total, hipMemcpyHostToDevice, st) == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  const BatOp* dbop = (const BatOp*)(dev + o_b);
  auto grouped = [&](int which, int step) -> int {
    for (const Cls& c : cls)
      AZ_TRY(ops_batched(which, c.n, c.s, dbop + (int64_t)step * E + c.first, c.count, c.maxvec, 0.0, st));
    return AZRBF_OK;
  };
  if (!rc) {
    launch_kernel(k_bat_gaussian, dim3((unsigned)((maxq + 255) / 256), (unsigned)maxk, (unsigned)E), 256, 0, st,
                  (const GaussOp*)(dev + o_g));
    rc = hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  if (!rc) rc = grouped(0, 0);
  if (!rc) rc = grouped(1, 1);
  if (!rc) rc = grouped(0, 2);
  for (size_t i = 0; i < tg.size() && !rc; ++i)
    rc = tsqr_block_qr_batched(tg[i].k, tg[i].rb, (const TsqrOp*)(dev + o_t) + tg[i].first, tg[i].count,
                               tg[i].maxnb, st);
  if (!rc) {
    int64_t kk = maxk * maxk;
    launch_kernel(k_bat_copy, dim3((unsigned)((kk + 255) / 256), (unsigned)E), 256, 0, st, (const CopyOp*)(dev + o_c));
    rc = hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  for (size_t i = 0; i < fg.size() && !rc; ++i) {
    const FormqOp* f = (const FormqOp*)(dev + o_f) + fg[i].first;
    const dim3 grid((unsigned)fg[i].maxnb, (unsigned)fg[i].count);
    if (fg[i].k == 16) launch_kernel(k_bat_formq<16>, grid, TSQR_THREADS, 0, st, f);
    else if (fg[i].k == 32) launch_kernel(k_bat_formq<32>, grid, TSQR_THREADS, 0, st, f);
    else launch_kernel(k_bat_formq<64>, grid, TSQR_THREADS, 0, st, f);
    rc = hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  for (size_t i = 0; i < jg.size() && !rc; ++i) {
    const JacOp* j = (const JacOp*)(dev + o_j) + jg[i].first;
    const int k = jg[i].k;
    const double tol = 4.0 * k * 1.1102230246251565e-16;
    if (k == 16) launch_kernel(k_bat_jacobi<16>, jg[i].count, 128, 0, st, j, tol, 40);
    else if (k == 32) launch_kernel(k_bat_jacobi<32>, jg[i].count, 256, 0, st, j, tol, 40);
    else launch_kernel(k_bat_jacobi<64>, jg[i].count, 512, 0, st, j, tol, 40);
    rc = hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  for (int h = 0; h < 2 && !rc; ++h) {   // Omega P, then (A Omega) P: E entries per launch (grid z <= 65535)
    launch_kernel(k_bat_prod, dim3((unsigned)((maxrows + 255) / 256), (unsigned)(maxk / 16), (unsigned)E), 256, 0,
                  st, (const ProdOp*)(dev + o_p) + (int64_t)h * E);
    rc = hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  }
  for (int q = 0; q < E && !rc; ++q) {
    Plan& P = *plans[ord[q]];
    if (hipMemcpyAsync(P.hinfo, lay[q].info, sizeof(P.hinfo), hipMemcpyDeviceToHost, st) != hipSuccess)
      rc = AZRBF_EHIP;
  }
  const int rs = hipStreamSynchronize(st) == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  (void)hipFree(dev);
  (void)hipHostFree(host);
  if (rc) return rc;
  if (rs) return rs;
  for (int q = 0; q < E; ++q) {
    Plan& P = *plans[ord[q]];
    std::swap(P.Om, P.Om2);
    std::swap(P.Yf, P.Yf2);
    P.dinfo = lay[q].info;
    P.rank = P.hinfo[0];
    P.sweeps = P.hinfo[1];
    P.rank_pending = false;
    P.factored = true;
    rcs[ord[q]] = 10 * (int64_t)P.rank > 9 * (int64_t)P.k ? AZRBF_ERANK : AZRBF_OK;
  }
  return AZRBF_OK;
}

// ------------------------------------------------------------------ solve

// Solve workspace for nrhs right-hand sides (k <= 64 layout).
int dense_solve_ws(Plan& P, int64_t nrhs, hipStream_t st) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt;
  const int64_t npart = gemm_split_doubles(k, nrhs, Mt, 1);
  if (nrhs > P.sw_rhs || npart > P.sw_part) {
    const int64_t per = N + 3 * P.Mtp + k + 2 * NORM_CHUNKS;
    double* old = P.sw;
    AZ_TRY(P.alloc((void**)&P.sw, sizeof(double) * (per * nrhs + npart)));
    P.release_one_after(old, st);
    P.sw_rhs = nrhs;
    P.sw_part = npart;
  }
  return AZRBF_OK;
}

// First stage of the first pass, independent of the factor:
// Zr = Z* b, c = (I - A Z*) b, into the solve workspace.
int dense_first_stage(Plan& P, const double* B, int64_t ldb, int64_t nrhs, hipStream_t st) {
  AZ_TRY(dense_solve_ws(P, nrhs, st));
  const int64_t N = P.N;
  double* Zr = P.sw;
  double* C = Zr + N * nrhs;
  AZ_TRY(ops_apply_AZ(P, B, ldb, nrhs, -1.0, 1.0, B, ldb, C, P.Mtp, Zr, st));
  return AZRBF_OK;
}

int dense_first_qtc(Plan& P, int64_t nrhs, hipStream_t st) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt, Ld = P.Mtp;
  double* C = P.sw + N * nrhs;
  double* Tm = C + 3 * Ld * nrhs;
  double* part = Tm + (int64_t)k * nrhs + 2 * NORM_CHUNKS * nrhs;
  const int64_t npart = gemm_split_doubles(k, nrhs, Mt, 1);
  return gemm_mfma_c(true, false, k, nrhs, Mt, 1.0, P.Q, Ld, 0, C, Ld, 0, 0.0, nullptr, 0, 0, Tm, k, 0, 1, part,
                     npart, st);
}

int dense_solve(Plan& P, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx, double* relres,
                hipStream_t st, bool first_done, bool qtc_done) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt;
  const int64_t Ld = P.Mtp;   // leading dimension of the row-space matrices (whole 128-byte lines)
  AZ_TRY(dense_solve_ws(P, nrhs, st));
  double* Zr = P.sw;                   // N x nrhs
  double* C = Zr + N * nrhs;           // Mt x nrhs (ld Ld)
  double* R1 = C + Ld * nrhs;          // Mt x nrhs (ld Ld)
  double* Rc = R1 + Ld * nrhs;         // Mt x nrhs (ld Ld)
  double* Tm = Rc + Ld * nrhs;         // k x nrhs
  double* nrm = Tm + (int64_t)k * nrhs;            // 2 * NORM_CHUNKS x nrhs
  double* part = nrm + 2 * NORM_CHUNKS * nrhs;     // split-reduction partials of Q^T c
  const int64_t npart = gemm_split_doubles(k, nrhs, Mt, 1);
  const double* rin = B;
  int64_t ldr = ldb;
  for (int it = 0; it <= P.refine; ++it) {
    if (!(it == 0 && first_done)) {
      AZ_TRY(ops_apply_AZ(P, rin, ldr, nrhs, -1.0, 1.0, rin, ldr, C, Ld, Zr, st));   // c = (I - A Z*) r
    }
    if (!(it == 0 && qtc_done))
      AZ_TRY(gemm_mfma_c(true, false, k, nrhs, Mt, 1.0, P.Q, Ld, 0, C, Ld, 0, 0.0, nullptr, 0, 0, Tm, k, 0, 1, part,
                         npart, st));                                                           // t = Q^T c
    AZ_TRY(gemm_nn(P.Om, N, N, k, Tm, k, nrhs, 1.0, X, ldx, it == 0 ? 0.0 : 1.0, X, ldx, st));  // x += x1
    AZ_TRY(gemm_nn(P.Yf, Ld, Mt, k, Tm, k, nrhs, -1.0, rin, ldr, 1.0, R1, Ld, st));            // r - A x1
    AZ_TRY(ops_apply_Z(P, R1, Ld, nrhs, 1.0, 1.0, nullptr, 0, X, ldx, st));          // x += Z* (r - A x1)
    AZ_TRY(ops_apply_A(P, X, ldx, nrhs, -1.0, 1.0, B, ldb, Rc, Ld, st));            // residual b - A x
    rin = Rc;
    ldr = Ld;
  }
  if (relres) AZ_TRY(relres_norms(Rc, Ld, B, ldb, Mt, nrhs, nrm, relres, st));
  return AZRBF_OK;
}

}  // namespace az
