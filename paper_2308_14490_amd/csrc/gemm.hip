// FP64 matrix-core GEMMs of the low-rank stage (section 3.2.3) for sketch
// widths in the hundreds to thousands: the projections Q^T X and updates
// X - Q S of the block Gram-Schmidt QR, the products with the Jacobi
// rotations and the per-right-hand-side solve.
//
// One block computes a 64 x 64 tile of C with four waves (32 x 32 each, four
// 16 x 16 v_mfma_f64_16x16x4 accumulators).  op(A) and op(B) are staged in
// LDS in chunks of 16 along the reduction.  The product is formed as
// (op(A) op(B))^T = op(B)^T op(A)^T so that the accumulator lanes run along
// the rows of the column-major C and the stores are contiguous.
//
// Reductions over very long dimensions (the tall-skinny Q^T X) are split
// over blocks: each writes a partial tile, and k_sum_splits adds them in a
// fixed order, so results do not depend on scheduling.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace az {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int GT = 64;   // output tile edge
constexpr int GK = 32;   // reduction chunk staged in LDS
constexpr int GP = GT + 2;
constexpr int GL = GK * GT / 256;   // elements of each operand a thread stages per chunk

template <bool TA>
__device__ __forceinline__ double load_opA(const double* A, int64_t lda, int64_t i, int64_t kk) {
  return TA ? A[kk + lda * i] : A[i + lda * kk];
}

template <bool TB>
__device__ __forceinline__ double load_opB(const double* B, int64_t ldb, int64_t kk, int64_t j) {
  return TB ? B[j + ldb * kk] : B[kk + ldb * j];
}

// Staging coordinates of element q of a thread: contiguous global runs along
// i for A and along kk for A^T (likewise B).
template <bool T>
__device__ __forceinline__ void stage_ik(int t, int q, int* i, int* kk) {
  if (T) {
    *kk = t & (GK - 1);
    *i = (t / GK) + (256 / GK) * q;
  } else {
    *i = t & (GT - 1);
    *kk = (t / GT) + (256 / GT) * q;
  }
}

// Batch entry z / splits, reduction range [sp * kchunk, (sp + 1) * kchunk) of
// split sp = z % splits.  With splits > 1 the raw tile sums are stored at
// C + z * sC (ld ldc) and alpha, beta are applied by k_sum_splits.  The next
// chunk's operands are loaded into registers while the current one is
// multiplied from LDS.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda, int64_t sA,
       const double* __restrict__ B, int64_t ldb, int64_t sB, double beta, const double* Cin, int64_t ldci,
       int64_t sCi, double* C, int64_t ldc, int64_t sC, int splits, int64_t kchunk) {
  __shared__ double As[GK][GP];   // As[kk][i] = op(A)(i0 + i, kb + kk)
  __shared__ double Bs[GK][GP];   // Bs[kk][j] = op(B)(kb + kk, j0 + j)
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int z = blockIdx.z, bz = z / splits, sp = z % splits;
  A += (int64_t)bz * sA;
  B += (int64_t)bz * sB;
  C += (int64_t)(splits > 1 ? z : bz) * sC;
  if (Cin) Cin += (int64_t)bz * sCi;
  const int64_t i0 = (int64_t)blockIdx.x * GT, j0 = (int64_t)blockIdx.y * GT;
  const int64_t k0 = (int64_t)sp * kchunk, k1 = std::min(K, k0 + kchunk);
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  dbl4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = dbl4{0.0, 0.0, 0.0, 0.0};
  double ra[GL], rb[GL];
  auto fetch = [&](int64_t kb) {
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      int ai, ak, bj, bk;
      stage_ik<TA>(t, q, &ai, &ak);
      stage_ik<!TB>(t, q, &bj, &bk);   // B is indexed (kk, j): its "row" runs along j
      const int64_t gi = i0 + ai, gka = kb + ak, gj = j0 + bj, gkb = kb + bk;
      ra[q] = (gi < M && gka < k1) ? load_opA<TA>(A, lda, gi, gka) : 0.0;
      rb[q] = (gj < N && gkb < k1) ? load_opB<TB>(B, ldb, gkb, gj) : 0.0;
    }
  };
  if (k0 < k1) fetch(k0);
  for (int64_t kb = k0; kb < k1; kb += GK) {
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      int ai, ak, bj, bk;
      stage_ik<TA>(t, q, &ai, &ak);
      stage_ik<!TB>(t, q, &bj, &bk);
      As[ak][ai] = ra[q];
      Bs[bk][bj] = rb[q];
    }
    __syncthreads();
    if (kb + GK < k1) fetch(kb + GK);
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kk = 4 * ks + (l >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) av[mi] = As[kk][wi + 16 * mi + (l & 15)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bv[ni] = Bs[kk][wj + 16 * ni + (l & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[ni], av[mi], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
  // The accumulator of a 16 x 16 x 4 f64 product holds element (r, c) =
  // ((l >> 4) + 4 v, l & 15) in lane l, entry v; here r runs along j, c along i:
  // acc[mi][ni][v] = C(i0 + wi + 16 mi + (l & 15), j0 + wj + 16 ni + (l >> 4) + 4 v)
#pragma unroll
  for (int mi = 0; mi < 2; ++mi) {
    const int64_t i = i0 + wi + 16 * mi + (l & 15);
    if (i >= M) continue;
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = j0 + wj + 16 * ni + (l >> 4) + 4 * v;
        if (j >= N) continue;
        double* p = C + i + ldc * j;
        const double s = acc[mi][ni][v];
        if (splits > 1) *p = s;
        else *p = beta == 0.0 ? alpha * s : fma(alpha, s, beta * Cin[i + ldci * j]);
      }
    }
  }
}

// C = alpha sum_s P_s + beta C for each batch entry; P_s at P + (b*splits+s)*sP.
// One wave per output element: lane l adds the partials s = l, l + 64, ...
// in order, then the 64 lane sums are added by a fixed butterfly, so the
// result does not depend on scheduling (and the loads of a lane are
// independent, instead of one long chain of dependent round trips).
__global__ void __launch_bounds__(256)
k_sum_splits(int64_t M, int64_t N, int splits, const double* __restrict__ P, int64_t ldp, int64_t sP,
             double alpha, double beta, const double* Cin, int64_t ldci, int64_t sCi, double* C, int64_t ldc,
             int64_t sC) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t b = blockIdx.y;
  double v = 0.0;
  if (e < M * N) {
    const int64_t i = e % M, j = e / M;
    const double* p = P + (int64_t)b * splits * sP + i + ldp * j;
    for (int s = lane; s < splits; s += 64) v += p[(int64_t)s * sP];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (e < M * N && lane == 0) {
    const int64_t i = e % M, j = e / M;
    double* c = C + (int64_t)b * sC + i + ldc * j;
    *c = beta == 0.0 ? alpha * v : fma(alpha, v, beta * Cin[(int64_t)b * sCi + i + ldci * j]);
  }
}

template <bool TA, bool TB>
void launch_gemm(dim3 grid, hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                 int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, const double* Cin,
                 int64_t ldci, int64_t sCi, double* C, int64_t ldc, int64_t sC, int splits, int64_t kchunk) {
  launch_kernel(k_gemm<TA, TB>, grid, 256, 0, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cin, ldci, sCi, C,
                ldc, sC, splits, kchunk);
}

}  // namespace

// Splits of the reduction when the output has few tiles: about 1024 blocks
// in all, each reducing at least 256 rows, at most 512 splits.
static int64_t gemm_splits(int64_t M, int64_t N, int64_t K, int64_t batch) {
  const int64_t tiles = ((M + GT - 1) / GT) * ((N + GT - 1) / GT) * batch;
  if (tiles >= 256 || K < 1024) return 1;
  const int64_t sp = std::min<int64_t>({512, (1024 + tiles - 1) / tiles, K / 256});
  return sp > 1 ? sp : 1;
}

int64_t gemm_split_doubles(int64_t M, int64_t N, int64_t K, int64_t batch) {
  const int64_t sp = gemm_splits(M, N, K, batch);
  return sp > 1 ? sp * batch * M * N : 0;
}

int gemm_mfma_c(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, const double* Cin, int64_t ldci,
                int64_t sCi, double* C, int64_t ldc, int64_t sC, int64_t batch, double* part, int64_t part_doubles,
                hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return AZRBF_OK;
  if (batch > 65535) return AZRBF_EINVAL;
  if (beta != 0.0 && !Cin) return AZRBF_EINVAL;
  const int64_t tx = (M + GT - 1) / GT, ty = (N + GT - 1) / GT;
  if (tx > 0x7fffffff || ty > 65535) return AZRBF_EINVAL;
  int splits = 1;
  const int64_t need = gemm_split_doubles(M, N, K, batch);
  if (need > 0 && part && need <= part_doubles) splits = (int)gemm_splits(M, N, K, batch);
  int64_t kchunk = K;
  if (splits > 1) {
    kchunk = ((K + splits - 1) / splits + GK - 1) / GK * GK;   // whole chunks per split
    splits = (int)((K + kchunk - 1) / kchunk);
  }
  if ((int64_t)splits * batch > 65535) return AZRBF_EINVAL;
  Prof pr("gemm_mfma", 8.0 * batch * (M * K + K * N + M * N * (beta != 0.0 ? 2.0 : 1.0)), st,
          2.0 * batch * M * N * K);
  const dim3 grid((unsigned)tx, (unsigned)ty, (unsigned)(splits * batch));
  double* Cout = splits > 1 ? part : C;
  const int64_t ldo = splits > 1 ? M : ldc, so = splits > 1 ? M * N : sC;
  if (!ta && !tb)
    launch_gemm<false, false>(grid, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cin, ldci, sCi, Cout, ldo, so,
                              splits, kchunk);
  else if (ta && !tb)
    launch_gemm<true, false>(grid, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cin, ldci, sCi, Cout, ldo, so,
                             splits, kchunk);
  else if (!ta && tb)
    launch_gemm<false, true>(grid, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cin, ldci, sCi, Cout, ldo, so,
                             splits, kchunk);
  else
    launch_gemm<true, true>(grid, st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cin, ldci, sCi, Cout, ldo, so,
                            splits, kchunk);
  AZ_HIP(hipGetLastError());
  if (splits > 1) {
    const int64_t e = M * N;
    if ((e + 3) / 4 > 0x7fffffff) return AZRBF_EINVAL;
    launch_kernel(k_sum_splits, dim3((unsigned)((e + 3) / 4), (unsigned)batch), 256, 0, st, M, N, splits, part, M,
                  M * N, alpha, beta, Cin, ldci, sCi, C, ldc, sC);
    AZ_HIP(hipGetLastError());
  }
  return AZRBF_OK;
}

int gemm_mfma(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc,
              int64_t sC, int64_t batch, double* part, int64_t part_doubles, hipStream_t st) {
  return gemm_mfma_c(ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, C, ldc, sC, batch, part,
                     part_doubles, st);
}

}  // namespace az

// --------------------------------------------------------------- C ABI

namespace {

int dgemm_args(int64_t m, int64_t n, int64_t k, int32_t transa, int32_t transb, const double* A, int64_t lda,
               const double* B, int64_t ldb, const double* C, int64_t ldc) {
  if (m < 0 || n < 0 || k < 0) return AZRBF_EINVAL;
  if (m == 0 || n == 0) return AZRBF_OK;
  if (!C || ldc < m) return AZRBF_EINVAL;
  if (k > 0) {
    if (!A || !B) return AZRBF_EINVAL;
    if (lda < std::max<int64_t>(1, transa ? k : m) || ldb < std::max<int64_t>(1, transb ? n : k))
      return AZRBF_EINVAL;
  }
  return AZRBF_OK;
}

// Split-K partial tiles of azrbf_dgemm_noalloc: one fixed array per GPU.
constexpr int64_t kScratchDoubles = int64_t(1) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex scratch_mu;
double* scratch_dev[kMaxDevices];   // device address of `scratch` per device

// The address of this device's copy of `scratch`, looked up once per device
// with that device current (the host-side name is not a device address).
int scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return AZRBF_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return AZRBF_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return AZRBF_EHIP;
    }
    scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = scratch_dev[dev];
  return AZRBF_OK;
}

}  // namespace

extern "C" int azrbf_dgemm(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, double alpha,
                           const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                           int64_t ldc, void* stream) {
  const int bad = dgemm_args(m, n, k, transa, transb, A, lda, B, ldb, C, ldc);
  if (bad || m == 0 || n == 0) return bad;
  hipStream_t st = (hipStream_t)stream;
  const int64_t need = az::gemm_split_doubles(m, n, k, 1);
  double* part = nullptr;
  if (need > 0 && hipMalloc((void**)&part, sizeof(double) * need) != hipSuccess) {
    (void)hipGetLastError();
    part = nullptr;   // unsplit fallback: the same product, fewer blocks
  }
  int rc = az::gemm_mfma(transa != 0, transb != 0, m, n, k, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1,
                         part, part ? need : 0, st);
  if (part) {
    if (hipStreamSynchronize(st) != hipSuccess) rc = AZRBF_EHIP;
    (void)hipFree(part);
  }
  return rc;
}

extern "C" int azrbf_dgemm_noalloc(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k,
                                   double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                                   double beta, double* C, int64_t ldc, void* stream) {
  const int bad = dgemm_args(m, n, k, transa, transb, A, lda, B, ldb, C, ldc);
  if (bad || m == 0 || n == 0) return bad;
  const int64_t need = az::gemm_split_doubles(m, n, k, 1);
  if (need > kScratchDoubles) return AZRBF_ESCRATCH;
  double* part = nullptr;
  if (need > 0) {
    const int rc = scratch_ptr(&part);
    if (rc) return rc;
  }
  // every partial tile is written before k_sum_splits reads it: nothing to clear
  return az::gemm_mfma(transa != 0, transb != 0, m, n, k, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1,
                       part, need, (hipStream_t)stream);
}
