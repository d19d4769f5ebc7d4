// Householder QR of tall-skinny row blocks with the block held in registers
// (the leaf and tree nodes of the TSQR of section 3.2.3's sketch, widths
// k = 16, 32, 64).
//
// Thread t of the 256 owns rows t + 256 i (i < 64/k) of the block with all k
// columns in VGPRs, so the block is RB = 16384/k rows.  Column j of the
// Householder sweep needs one block-wide reduction, D_c = sum_{r>j} a_rj a_rc
// for every c: each lane forms its k partial sums, a butterfly
// reduce-scatter across the wave leaves one column sum per lane, and the four
// waves meet in LDS.  The butterfly's first two stages (lane distances 32
// and 16) exchange register halves with v_permlane32_swap / v_permlane16_swap,
// which hand each lane exactly the partner values it adds, so they need no
// per-lane selection; the last four (distances below 16) move values by DPP.  From D one gets sigma^2 = D_j, v_j^T a_c for c > j (the
// rank-one update) and v_c^T v_j for c < j (the compact-WY factor T).  The
// column loop is unrolled so that every register index is static.
#include <utility>

#include "internal.h"

namespace az {

namespace {

// RPT rows per thread (the block's tile shape, picked by the autotuner among
// the shapes whose K RPT doubles fit the registers; 64 / K by default).
template <int K, int RPT_>
struct RegQR {
  static constexpr int RPT = RPT_;     // rows per thread
  static constexpr int RB = 256 * RPT; // rows per block
};

// 1/x and 1/sqrt(x): hardware estimate and one Newton step.
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  // every lane of the permutation is valid, so no old value is needed
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// (x, y) -> lanes of the lower half of each lane pair (distance 32: lanes
// 0-31; distance 16: rows 0 and 2) get (own x, partner's x), those of the
// upper half (partner's y, own y).  x + y is then the pair sum of x in the
// lower half and of y in the upper half.
template <int D>
__device__ __forceinline__ void swap_d(double& x, double& y) {
  const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
  const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
  if constexpr (D == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
  }
}

// Stage S = 0..5 of the butterfly pairs lanes that differ in bit B_S = 5 - S
// (and agree in the bits of all earlier stages): S = 0, 1 by the swaps above
// (distance 32, 16), S = 2..5 by DPP (row mirror, half-row mirror, quad
// permutations: partner lane ^ 15, ^ 7, ^ 2, ^ 1).
template <int S>
__device__ __forceinline__ double xchg(double x) {
  if constexpr (S == 2) return dpp_d<0x140>(x);
  else if constexpr (S == 3) return dpp_d<0x141>(x);
  else if constexpr (S == 4) return dpp_d<0x4E>(x);
  else return dpp_d<0xB1>(x);
}

// Halves the N live values: the lane whose bit B_S is set keeps the upper
// half, its partner the lower half, and each adds what the other holds.
template <int S, int N>
__device__ __forceinline__ void rs_stage(double* v, int lane) {
  if constexpr (S < 2) {
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
      double x = v[q], y = v[q + N / 2];
      swap_d<S == 0 ? 32 : 16>(x, y);
      v[q] = x + y;
    }
  } else {
    const bool up = (lane >> (5 - S)) & 1;
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
      const double send = up ? v[q] : v[q + N / 2];
      const double keep = up ? v[q + N / 2] : v[q];
      v[q] = keep + xchg<S>(send);
    }
  }
}

// Once one value is left: the pair sum in both lanes.
template <int S>
__device__ __forceinline__ void ar_stage(double* v) {
  if constexpr (S < 2) {
    double x = v[0], y = v[0];
    swap_d<S == 0 ? 32 : 16>(x, y);
    v[0] = x + y;
  } else {
    v[0] += xchg<S>(v[0]);
  }
}

template <int S, int N>
__device__ __forceinline__ void rs_or_ar(double* v, int lane) {
  if constexpr (N >= 2) rs_stage<S, N>(v, lane);
  else ar_stage<S>(v);
}

// Wave-wide sums of K values per lane; the lane is left with the sum of value
// rs_col<K>(lane).
template <int K>
__device__ __forceinline__ double wave_reduce_scatter(double* v, int lane) {
  rs_or_ar<0, K>(v, lane);
  rs_or_ar<1, (K >= 2 ? K / 2 : 1)>(v, lane);
  rs_or_ar<2, (K >= 4 ? K / 4 : 1)>(v, lane);
  rs_or_ar<3, (K >= 8 ? K / 8 : 1)>(v, lane);
  rs_or_ar<4, (K >= 16 ? K / 16 : 1)>(v, lane);
  rs_or_ar<5, (K >= 32 ? K / 32 : 1)>(v, lane);
  return v[0];
}

// Column held by a lane: each halving stage S with N live values adds
// bit B_S times N/2.
template <int K>
__device__ __forceinline__ int rs_col(int lane) {
  int c = 0, n = K;
#pragma unroll
  for (int S = 0; S < 6; ++S) {
    if (n >= 2) {
      c += ((lane >> (5 - S)) & 1) * (n / 2);
      n /= 2;
    }
  }
  return c;
}

// One lane per column writes: the bits of the pair-sum (all-reduce) stages,
// the last log2(64 / K) bits, are zero.
template <int K>
__device__ __forceinline__ bool rs_writer(int lane) {
  return (lane & (64 / K - 1)) == 0;
}

template <int K>
struct QrShared {
  double (*red)[K];
  double* rowj;
  double* wv;
  double* Gm;     // Gm[j * K + l] = v_l^T v_j (l < j)
  double* scal;
  double* Tm;     // Tm[j * K + i] = T(i, j); the loop leaves tau_j on the diagonal
};

// Column J of the sweep (J static, so every register index is static).
template <int K, int RPT, int J>
__device__ __forceinline__ void qr_column(double (&a)[RPT][K], const QrShared<K>& sh, int t,
                                          int lane, int wave, int col, bool writer) {
  double p[K];
#pragma unroll
  for (int c = 0; c < K; ++c) p[c] = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const double aj = (t + 256 * i > J) ? a[i][J] : 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) p[c] = fma(aj, a[i][c], p[c]);
  }
  const double s = wave_reduce_scatter<K>(p, lane);
  if (writer) sh.red[wave][col] = s;
  __syncthreads();
  if (t < K) {
    const double sig2 = (sh.red[0][J] + sh.red[1][J]) + (sh.red[2][J] + sh.red[3][J]);
    const double dt = (sh.red[0][t] + sh.red[1][t]) + (sh.red[2][t] + sh.red[3][t]);
    const double alpha = sh.rowj[J];
    double beta = alpha, tau = 0.0, scale = 0.0;
    if (sig2 > 0.0) {
      // sqrt and reciprocals from the hardware estimates refined by Newton
      // steps: a short dependency chain on the critical path of the sweep
      const double nn = fma(alpha, alpha, sig2);
      const double rn = rsq_nr(nn);
      double nrm = nn * rn;
      nrm = fma(0.5 * rn, fma(-nrm, nrm, nn), nrm);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = fma(-alpha, rcp_nr(beta), 1.0);       // (beta - alpha) / beta
      scale = rcp_nr(alpha - beta);
    }
    if (t == J) {
      sh.scal[0] = beta;
      sh.scal[1] = tau;
      sh.scal[2] = scale;
      sh.Tm[J * K + J] = tau;
    } else if (t > J) {
      sh.wv[t] = tau * fma(dt, scale, sh.rowj[t]);
    } else {
      sh.Gm[J * K + t] = fma(dt, scale, sh.rowj[t]);   // v_t[J] = a[J][t] sits below t's diagonal
    }
  }
  __syncthreads();
  const double beta = sh.scal[0], scale = sh.scal[2];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = t + 256 * i;
    if (row >= J) {
      const double v = row == J ? 1.0 : a[i][J] * scale;
#pragma unroll
      for (int c = J + 1; c < K; ++c) a[i][c] = fma(-sh.wv[c], v, a[i][c]);
      a[i][J] = row == J ? beta : v;
    }
  }
  if constexpr (J + 1 < K) {
    if (t == J + 1) {
#pragma unroll
      for (int c = 0; c < K; ++c) sh.rowj[c] = a[0][c];
    }
  }
}

template <int K, int RPT, int... J>
__device__ __forceinline__ void qr_columns(double (&a)[RPT][K], const QrShared<K>& sh, int t,
                                           int lane, int wave, int col, bool writer,
                                           std::integer_sequence<int, J...>) {
  (qr_column<K, RPT, J>(a, sh, t, lane, wave, col, writer), ...);
}

// One block of RB rows: R (upper k x k) to rows b*k.. of Rout, the
// reflectors (unit lower trapezoid) over the block's rows of V, and the
// compact-WY T (k x k, column-major) to Tout + b*k*k, so that
// H_0 ... H_{k-1} = I - V T V^T.  Rows >= m are read as zero and not
// written.  A and V may be the same array.
template <int K, int RPT>
__device__ __forceinline__ void tsqr_reg_block(const double* A, int64_t lda, int64_t m, double* __restrict__ Rout,
                                               int64_t ldr, double* V, int64_t ldv, double* __restrict__ Tout,
                                               int64_t blk) {
  using C = RegQR<K, RPT>;
  __shared__ double red[4][K];    // per-wave column sums
  __shared__ double rowj[K];      // the pivot row
  __shared__ double wv[K];        // tau_j v_j^T a_c, c > j
  __shared__ double Gm[K * K];    // v_l^T v_j, l < j
  __shared__ double Xs[K * K];    // products of the T assembly
  __shared__ double scal[4];      // beta, tau, scale
  __shared__ double Tm[K * K];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t r0 = blk * C::RB;
  double a[C::RPT][K];
#pragma unroll
  for (int i = 0; i < C::RPT; ++i) {
    const int64_t gr = r0 + t + 256 * i;
#pragma unroll
    for (int c = 0; c < K; ++c) a[i][c] = gr < m ? A[gr + lda * c] : 0.0;
  }
  if (t == 0) {
#pragma unroll
    for (int c = 0; c < K; ++c) rowj[c] = a[0][c];
  }
  const int col = rs_col<K>(lane);
  const bool writer = rs_writer<K>(lane);
  QrShared<K> sh{red, rowj, wv, Gm, scal, Tm};
  qr_columns<K>(a, sh, t, lane, wave, col, writer, std::make_integer_sequence<int, K>{});
  __syncthreads();
  // Compact-WY T by recursive doubling (kept out of the column loop, whose
  // steps are the critical path): for adjacent blocks of b reflectors,
  // H_1 H_2 = I - V T V^T with T = [T1, -T1 (V1^T V2) T2; 0, T2], formed as
  // X = G12 T2, then T12 = -T1 X; b = 1, 2, 4, ..., K/2.
#pragma unroll 1
  for (int b = 1; b < K; b *= 2) {
    for (int e = t; e < (K / 2) * b; e += 256) {
      const int pr = e / (b * b), rem = e % (b * b);
      const int l = 2 * b * pr + rem % b, j = 2 * b * pr + b + rem / b, j0 = 2 * b * pr + b;
      double x = 0.0;
      for (int q = j0; q <= j; ++q) x = fma(Gm[q * K + l], Tm[j * K + q], x);   // G(l, q) T(q, j)
      Xs[j * K + l] = x;
    }
    __syncthreads();
    for (int e = t; e < (K / 2) * b; e += 256) {
      const int pr = e / (b * b), rem = e % (b * b);
      const int i = 2 * b * pr + rem % b, j = 2 * b * pr + b + rem / b, i1 = 2 * b * pr + b;
      double y = 0.0;
      for (int l = i; l < i1; ++l) y = fma(Tm[l * K + i], Xs[j * K + l], y);      // T(i, l) X(l, j)
      Tm[j * K + i] = -y;
    }
    __syncthreads();
  }
  for (int e = t; e < K * K; e += 256) {
    const int r = e % K, c = e / K;
    Tout[blk * K * K + e] = r <= c ? Tm[c * K + r] : 0.0;
  }
  if (t < K) {
#pragma unroll
    for (int c = 0; c < K; ++c) Rout[blk * K + t + ldr * c] = c >= t ? a[0][c] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < C::RPT; ++i) {
    const int row = t + 256 * i;
    const int64_t gr = r0 + row;
    if (gr < m) {
#pragma unroll
      for (int c = 0; c < K; ++c) V[gr + ldv * c] = row > c ? a[i][c] : (row == c ? 1.0 : 0.0);
    }
  }
}

template <int K, int RPT>
__global__ void __launch_bounds__(256)
k_tsqr_reg(const double* A, int64_t lda, int64_t m, double* __restrict__ Rout, int64_t ldr, double* V,
           int64_t ldv, double* __restrict__ Tout) {
  tsqr_reg_block<K, RPT>(A, lda, m, Rout, ldr, V, ldv, Tout, blockIdx.x);
}

// Grouped: level blockIdx.y of the list, its block blockIdx.x (blocks past
// the level's rows leave at once, the whole block).
template <int K, int RPT>
__global__ void __launch_bounds__(256) k_bat_tsqr_reg(const TsqrOp* __restrict__ ops) {
  const TsqrOp o = ops[blockIdx.y];
  if ((int64_t)blockIdx.x * RegQR<K, RPT>::RB >= o.m) return;
  tsqr_reg_block<K, RPT>(o.A, o.lda, o.m, o.R, o.ldr, o.V, o.ldv, o.T, blockIdx.x);
}

template <int K, int RPT>
int launch_bat_reg(const TsqrOp* ops, int count, int64_t maxnb, hipStream_t st) {
  launch_kernel(k_bat_tsqr_reg<K, RPT>, dim3((unsigned)maxnb, (unsigned)count), 256, 0, st, ops);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

template <int K, int RPT>
int launch_reg(const double* A, int64_t lda, int64_t m, double* R, int64_t ldr, double* V, int64_t ldv,
               double* T, hipStream_t st) {
  constexpr int RB = RegQR<K, RPT>::RB;
  const int64_t nb = (m + RB - 1) / RB;
  launch_kernel(k_tsqr_reg<K, RPT>, (unsigned)nb, 256, 0, st, A, lda, m, R, ldr, V, ldv, T);
  return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
}

}  // namespace

int tsqr_block_rows(int k) { return 16384 / k; }

// Tile shapes: RB = 256 RPT rows per block, K RPT <= 128 doubles per thread
// (k = 16: RPT 2, 4, 8; k = 32: 1, 2, 4; k = 64: 1, 2).
bool tsqr_rows_ok(int k, int rb) {
  if (rb < 256 || rb % 256) return false;
  const int rpt = rb / 256;
  if (rpt & (rpt - 1)) return false;
  return (k == 16 && rpt >= 2 && rpt <= 8) || (k == 32 && rpt <= 4) || (k == 64 && rpt <= 2);
}

int tsqr_block_qr(const double* A, int64_t lda, int64_t m, int k, int rb, double* R, int64_t ldr, double* V,
                  int64_t ldv, double* T, hipStream_t st) {
  if (m <= 0) return AZRBF_OK;
  if (!tsqr_rows_ok(k, rb)) return AZRBF_EUNSUPPORTED;
  const int rpt = rb / 256;
  switch (k * 16 + rpt) {
    case 16 * 16 + 2: return launch_reg<16, 2>(A, lda, m, R, ldr, V, ldv, T, st);
    case 16 * 16 + 4: return launch_reg<16, 4>(A, lda, m, R, ldr, V, ldv, T, st);
    case 16 * 16 + 8: return launch_reg<16, 8>(A, lda, m, R, ldr, V, ldv, T, st);
    case 32 * 16 + 1: return launch_reg<32, 1>(A, lda, m, R, ldr, V, ldv, T, st);
    case 32 * 16 + 2: return launch_reg<32, 2>(A, lda, m, R, ldr, V, ldv, T, st);
    case 32 * 16 + 4: return launch_reg<32, 4>(A, lda, m, R, ldr, V, ldv, T, st);
    case 64 * 16 + 1: return launch_reg<64, 1>(A, lda, m, R, ldr, V, ldv, T, st);
    case 64 * 16 + 2: return launch_reg<64, 2>(A, lda, m, R, ldr, V, ldv, T, st);
    default: return AZRBF_EUNSUPPORTED;
  }
}

int tsqr_block_qr_batched(int k, int rb, const TsqrOp* ops, int count, int64_t maxnb, hipStream_t st) {
  if (count <= 0 || maxnb <= 0) return AZRBF_OK;
  if (!tsqr_rows_ok(k, rb) || count > 65535) return AZRBF_EUNSUPPORTED;
  const int rpt = rb / 256;
  Prof pr("bat_tsqr_block", 0.0, st);
  switch (k * 16 + rpt) {
    case 16 * 16 + 2: return launch_bat_reg<16, 2>(ops, count, maxnb, st);
    case 16 * 16 + 4: return launch_bat_reg<16, 4>(ops, count, maxnb, st);
    case 16 * 16 + 8: return launch_bat_reg<16, 8>(ops, count, maxnb, st);
    case 32 * 16 + 1: return launch_bat_reg<32, 1>(ops, count, maxnb, st);
    case 32 * 16 + 2: return launch_bat_reg<32, 2>(ops, count, maxnb, st);
    case 32 * 16 + 4: return launch_bat_reg<32, 4>(ops, count, maxnb, st);
    case 64 * 16 + 1: return launch_bat_reg<64, 1>(ops, count, maxnb, st);
    case 64 * 16 + 2: return launch_bat_reg<64, 2>(ops, count, maxnb, st);
    default: return AZRBF_EUNSUPPORTED;
  }
}

}  // namespace az
