// Grouped solve of many uneven 1D problems (the per-right-hand-side part of
// Algorithm 1 with its refinement passes, section 3.2.3's solve phase).
//
// Every entry is a factored 1D plan on the single-kernel transform (n a power
// of two up to 8192, no boundary rows, sketch width k <= 64) with its own block
// of right-hand sides.  One pass of the solve is seven launches for the whole
// group, whatever the number of entries and their sizes:
//
//   Zr = Z* r, c = r - A Zr          grouped transforms, one launch per size class
//   t = Q^T c                         row-block partials, then a fixed-order sum
//   x (+)= (Omega P) t, r1 = r - (A Omega P) t     one launch
//   x += Z* r1, r = b - A x           grouped transforms
//
// and the residual norms once at the end.  The plain path issues the same
// steps per plan (about twenty launches per plan), so for small problems the
// group replaces a launch-bound sequence per problem by one sequence for all.
// The transforms are the per-plan kernels' own bodies; the dense products sum
// in another order, so results agree with the per-plan solve to rounding.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace az {

namespace {

constexpr int BQ_ROWS = 512;   // rows of c per partial block of Q^T c
constexpr int BQ_SUB = 64;     // rows staged in LDS at a time
constexpr int BCOLS = 16;      // right-hand sides per column block
constexpr int KMAXB = 64;      // widest sketch

// Device descriptor of one entry.
struct BatEntry {
  const double* Q;    // M x k, ld Ld
  const double* Om;   // Omega P, N x k, ld N
  const double* Yf;   // A Omega P, M x k, ld Ld
  const double* B;
  int64_t ldb;
  double* X;
  int64_t ldx;
  double* relres;     // nrhs values, or null
  double* Zr;         // N x nrhs
  double* C;          // M x nrhs, ld Ld
  double* R1;
  double* Rc;
  double* Tm;         // k x nrhs
  double* part;       // [row block][column block][k][BCOLS]
  int64_t N, M, Ld, nrhs;
  int k, refine;
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Partial products of t = Q^T c over BQ_ROWS rows of one column block:
// grid (row block, column block, entry).  Thread (i, ph) = (t mod k, t / k)
// sums column i of Q against the 16 right-hand sides over its share of each
// 64-row slice; the next slice's loads are issued before the current one is
// used (one slice in LDS, one in flight in registers).
__global__ void __launch_bounds__(256) k_bat_qtc_part(const BatEntry* __restrict__ es, int it) {
  const BatEntry e = es[blockIdx.z];
  const int64_t r0 = (int64_t)blockIdx.x * BQ_ROWS, c0 = (int64_t)blockIdx.y * BCOLS;
  if (it > e.refine || r0 >= e.M || c0 >= e.nrhs) return;
  __shared__ double qs[KMAXB][BQ_SUB + 1];
  __shared__ double cs[BCOLS][BQ_SUB + 1];
  const int tid = threadIdx.x;
  const int k = e.k;                       // 16, 32 or 64
  const int i = tid % k, ph = tid / k;
  const int nph = 256 / k, rpp = BQ_SUB / nph;
  const int nq = k * BQ_SUB / 256;         // Q elements a thread stages per slice (4, 8 or 16)
  const int64_t r1 = r0 + BQ_ROWS < e.M ? r0 + BQ_ROWS : e.M;
  double qn[KMAXB * BQ_SUB / 256], cn[BCOLS * BQ_SUB / 256];
  auto fetch = [&](int64_t rs) {
#pragma unroll
    for (int u = 0; u < KMAXB * BQ_SUB / 256; ++u) {
      if (u < nq) {
        const int idx = u * 256 + tid, col = idx / BQ_SUB, r = idx % BQ_SUB;
        qn[u] = rs + r < r1 ? e.Q[rs + r + (int64_t)col * e.Ld] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < BCOLS * BQ_SUB / 256; ++u) {
      const int idx = u * 256 + tid, j = idx / BQ_SUB, r = idx % BQ_SUB;
      cn[u] = c0 + j < e.nrhs && rs + r < r1 ? e.C[rs + r + (c0 + j) * e.Ld] : 0.0;
    }
  };
  double acc[BCOLS];
#pragma unroll
  for (int j = 0; j < BCOLS; ++j) acc[j] = 0.0;
  fetch(r0);
  for (int64_t rs = r0; rs < r1; rs += BQ_SUB) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KMAXB * BQ_SUB / 256; ++u) {
      if (u < nq) {
        const int idx = u * 256 + tid;
        qs[idx / BQ_SUB][idx % BQ_SUB] = qn[u];
      }
    }
#pragma unroll
    for (int u = 0; u < BCOLS * BQ_SUB / 256; ++u) {
      const int idx = u * 256 + tid;
      cs[idx / BQ_SUB][idx % BQ_SUB] = cn[u];
    }
    __syncthreads();
    if (rs + BQ_SUB < r1) fetch(rs + BQ_SUB);
    for (int rr = ph * rpp; rr < (ph + 1) * rpp; ++rr) {
      const double q = qs[i][rr];
#pragma unroll
      for (int j = 0; j < BCOLS; ++j) acc[j] = fma(q, cs[j][rr], acc[j]);
    }
  }
  __syncthreads();
  // the row phases, summed in a fixed order
  double* red = &qs[0][0];   // nph x k x BCOLS = 256 x BCOLS <= KMAXB x (BQ_SUB + 1)
#pragma unroll
  for (int j = 0; j < BCOLS; ++j) red[(ph * k + i) * BCOLS + j] = acc[j];
  __syncthreads();
  const int64_t ncb = (e.nrhs + BCOLS - 1) / BCOLS;
  double* out = e.part + ((int64_t)blockIdx.x * ncb + blockIdx.y) * k * BCOLS;
  for (int o = tid; o < k * BCOLS; o += 256) {
    const int ii = o / BCOLS, j = o % BCOLS;
    double sum = 0.0;
    for (int p = 0; p < nph; ++p) sum += red[(p * k + ii) * BCOLS + j];
    out[o] = sum;
  }
}

// t = sum of the row-block partials, in row-block order: grid (column block, entry).
__global__ void __launch_bounds__(256) k_bat_qtc_sum(const BatEntry* __restrict__ es, int it) {
  const BatEntry e = es[blockIdx.y];
  const int64_t c0 = (int64_t)blockIdx.x * BCOLS;
  if (it > e.refine || c0 >= e.nrhs) return;
  const int k = e.k;
  const int64_t ncb = (e.nrhs + BCOLS - 1) / BCOLS, nrb = (e.M + BQ_ROWS - 1) / BQ_ROWS;
  for (int o = threadIdx.x; o < k * BCOLS; o += 256) {
    const int i = o / BCOLS, j = o % BCOLS;
    if (c0 + j >= e.nrhs) continue;
    double s = 0.0;
    for (int64_t b = 0; b < nrb; ++b) s += e.part[(b * ncb + blockIdx.x) * k * BCOLS + o];
    e.Tm[i + (c0 + j) * k] = s;
  }
}

// x (+)= (Omega P) t on the coefficient rows, r1 = r - (A Omega P) t on the
// collocation rows: grid (row block over N then M, column block, entry).
__global__ void __launch_bounds__(256) k_bat_xr(const BatEntry* __restrict__ es, int it) {
  const BatEntry e = es[blockIdx.z];
  const int64_t c0 = (int64_t)blockIdx.y * BCOLS;
  const int64_t nbx = (e.N + 255) / 256, nbr = (e.M + 255) / 256;
  if (it > e.refine || c0 >= e.nrhs || (int64_t)blockIdx.x >= nbx + nbr) return;
  __shared__ double ts[KMAXB][BCOLS];
  const int k = e.k;
  for (int o = threadIdx.x; o < KMAXB * BCOLS; o += 256) {
    const int i = o / BCOLS, j = o % BCOLS;
    ts[i][j] = i < k && c0 + j < e.nrhs ? e.Tm[i + (c0 + j) * k] : 0.0;
  }
  __syncthreads();
  const bool xrows = (int64_t)blockIdx.x < nbx;
  const int64_t row = (xrows ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - nbx) * 256 + threadIdx.x;
  const int64_t m = xrows ? e.N : e.M;
  if (row >= m) return;
  const double* A = xrows ? e.Om : e.Yf;
  const int64_t lda = xrows ? e.N : e.Ld;
  double acc[BCOLS];
#pragma unroll
  for (int j = 0; j < BCOLS; ++j) acc[j] = 0.0;
  // (k is 16, 32 or 64: eight loads issued at a time)
#pragma unroll 8
  for (int i = 0; i < k; ++i) {
    const double a = A[row + (int64_t)i * lda];
#pragma unroll
    for (int j = 0; j < BCOLS; ++j) acc[j] = fma(a, ts[i][j], acc[j]);
  }
  const int64_t nj = e.nrhs - c0 < BCOLS ? e.nrhs - c0 : BCOLS;
  if (xrows) {
    for (int j = 0; j < nj; ++j) {
      double* x = e.X + row + (c0 + j) * e.ldx;
      *x = it == 0 ? acc[j] : *x + acc[j];
    }
  } else {
    const double* rin = it == 0 ? e.B : e.Rc;
    const int64_t ldr = it == 0 ? e.ldb : e.Ld;
    for (int j = 0; j < nj; ++j) e.R1[row + (c0 + j) * e.Ld] = rin[row + (c0 + j) * ldr] - acc[j];
  }
}

// relres = ||b - A x|| / ||b|| per right-hand side: grid (right-hand side, entry).
__global__ void __launch_bounds__(256) k_bat_relres(const BatEntry* __restrict__ es) {
  const BatEntry e = es[blockIdx.y];
  const int64_t j = blockIdx.x;
  if (!e.relres || j >= e.nrhs) return;
  __shared__ double red[2][4];
  const double* r = e.Rc + j * e.Ld;
  const double* b = e.B + j * e.ldb;
  double sn = 0.0, sd = 0.0;
  for (int64_t i = threadIdx.x; i < e.M; i += 256) {
    sn = fma(r[i], r[i], sn);
    sd = fma(b[i], b[i], sd);
  }
  sn = wsum(sn);
  sd = wsum(sd);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sn;
    red[1][threadIdx.x >> 6] = sd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double d = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    e.relres[j] = d > 0.0 ? sqrt(a / d) : sqrt(a);
  }
}

// Per-device staging: pinned host and device buffers for the descriptors and
// the entries' workspaces, in a ring of slots; a slot is reused once the GPU
// work of its previous call has finished.
struct BatSlot {
  char* host = nullptr;
  size_t hcap = 0;
  char* dev = nullptr;
  size_t dcap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
constexpr int kBatSlots = 3;
struct BatPool {
  BatSlot slot[kBatSlots];
  int next = 0;
};
std::mutex g_bat_mu;
std::map<int, BatPool> g_bat;

int64_t up16(int64_t x) { return (x + 15) / 16 * 16; }

}  // namespace

int batched_release() {
  std::lock_guard<std::mutex> lk(g_bat_mu);
  int prev = 0;
  AZ_HIP(hipGetDevice(&prev));
  int rc = AZRBF_OK;
  for (auto& kv : g_bat) {
    if (hipSetDevice(kv.first) != hipSuccess) {
      rc = AZRBF_EHIP;
      continue;
    }
    for (BatSlot& sl : kv.second.slot) {
      if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) rc = AZRBF_EHIP;
      if (sl.dev && hipFree(sl.dev) != hipSuccess) rc = AZRBF_EHIP;
      if (sl.host && hipHostFree(sl.host) != hipSuccess) rc = AZRBF_EHIP;
      sl.dev = nullptr;
      sl.host = nullptr;
      sl.dcap = sl.hcap = 0;
      sl.used = false;
    }
  }
  if (hipSetDevice(prev) != hipSuccess) rc = AZRBF_EHIP;
  return rc;
}

bool batched_eligible(const Plan& P) {
  return P.dim == 1 && P.fused && !P.generic && P.Mb == 0 && P.k <= KMAXB && P.factored && P.Om && P.Yf && P.Q;
}

int batched_solve(const std::vector<BatchItem>& items, hipStream_t st) {
  const int E = (int)items.size();
  if (E == 0) return AZRBF_OK;
  if (E > 65535) return AZRBF_EINVAL;
  int dev = 0;
  AZ_HIP(hipGetDevice(&dev));
  // entries in size-class order, so that each class is one range of operands
  std::vector<int> ord(E);
  for (int i = 0; i < E; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const Plan& A = *items[a].P;
    const Plan& B = *items[b].P;
    return A.n != B.n ? A.n < B.n : A.s < B.s;
  });
  int iters = 0;
  int64_t maxrhs = 0, maxrb = 0, maxcb = 0, maxxr = 0;
  std::vector<int64_t> wsoff(E + 1, 0);
  for (int q = 0; q < E; ++q) {
    const BatchItem& it = items[ord[q]];
    const Plan& P = *it.P;
    iters = std::max(iters, P.refine + 1);
    const int64_t ncb = (it.nrhs + BCOLS - 1) / BCOLS, nrb = (P.M + BQ_ROWS - 1) / BQ_ROWS;
    maxrhs = std::max(maxrhs, it.nrhs);
    maxrb = std::max(maxrb, nrb);
    maxcb = std::max(maxcb, ncb);
    maxxr = std::max(maxxr, (P.N + 255) / 256 + (P.M + 255) / 256);
    const int64_t w = up16(P.N * it.nrhs) + 3 * up16(P.Mtp * it.nrhs) + up16((int64_t)P.k * it.nrhs) +
                      up16(nrb * ncb * P.k * BCOLS);
    wsoff[q + 1] = wsoff[q] + w;
  }
  const int64_t nops = (int64_t)4 * iters * E;
  const size_t ent_bytes = sizeof(BatEntry) * E;
  const size_t op_off = (ent_bytes + 255) / 256 * 256;
  const size_t desc_bytes = op_off + sizeof(BatOp) * nops;
  const size_t ws_off = (desc_bytes + 255) / 256 * 256;
  const size_t dev_bytes = ws_off + sizeof(double) * wsoff[E];

  std::lock_guard<std::mutex> lk(g_bat_mu);
  BatPool& pool = g_bat[dev];
  BatSlot& sl = pool.slot[pool.next];
  pool.next = (pool.next + 1) % kBatSlots;
  if (!sl.done) AZ_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  if (sl.used) AZ_HIP(hipEventSynchronize(sl.done));
  if (sl.hcap < desc_bytes) {
    if (sl.host) AZ_HIP(hipHostFree(sl.host));
    sl.host = nullptr;
    sl.hcap = 0;
    AZ_HIP(hipHostMalloc((void**)&sl.host, desc_bytes, hipHostMallocDefault));
    sl.hcap = desc_bytes;
  }
  if (sl.dcap < dev_bytes) {
    if (sl.dev) AZ_HIP(hipFree(sl.dev));
    sl.dev = nullptr;
    sl.dcap = 0;
    AZ_HIP(hipMalloc((void**)&sl.dev, dev_bytes));
    sl.dcap = dev_bytes;
  }
  BatEntry* he = (BatEntry*)sl.host;
  BatOp* ho = (BatOp*)(sl.host + op_off);
  const BatEntry* de = (const BatEntry*)sl.dev;
  const BatOp* dop = (const BatOp*)(sl.dev + op_off);
  double* ws = (double*)(sl.dev + ws_off);
  for (int q = 0; q < E; ++q) {
    const BatchItem& it = items[ord[q]];
    const Plan& P = *it.P;
    BatEntry& e = he[q];
    double* w = ws + wsoff[q];
    const int64_t nr = it.nrhs;
    const int64_t ncb = (nr + BCOLS - 1) / BCOLS, nrb = (P.M + BQ_ROWS - 1) / BQ_ROWS;
    e.Q = P.Q;
    e.Om = P.Om;
    e.Yf = P.Yf;
    e.B = it.B;
    e.ldb = it.ldb;
    e.X = it.X;
    e.ldx = it.ldx;
    e.relres = it.relres;
    e.Zr = w;
    e.C = e.Zr + up16(P.N * nr);
    e.R1 = e.C + up16(P.Mtp * nr);
    e.Rc = e.R1 + up16(P.Mtp * nr);
    e.Tm = e.Rc + up16(P.Mtp * nr);
    e.part = e.Tm + up16((int64_t)P.k * nr);
    (void)ncb;
    (void)nrb;
    e.N = P.N;
    e.M = P.M;
    e.Ld = P.Mtp;
    e.nrhs = nr;
    e.k = P.k;
    e.refine = P.refine;
    for (int t = 0; t < iters; ++t) {
      const bool on = t <= P.refine;
      const double* rin = t == 0 ? it.B : e.Rc;
      const int64_t ldr = t == 0 ? it.ldb : e.Ld;
      BatOp* o = ho + ((int64_t)t * 4) * E + q;
      // Zr = Z* r
      o[0] = BatOp{P.geo, P.tw, rin, ldr, on ? nr : 0, 1.0, 0.0, e.Zr, P.N, e.Zr, P.N};
      // c = r - A Zr
      o[E] = BatOp{P.geo, P.tw, e.Zr, P.N, on ? nr : 0, -1.0, 1.0, rin, ldr, e.C, e.Ld};
      // x += Z* r1
      o[2 * E] = BatOp{P.geo, P.tw, e.R1, e.Ld, on ? nr : 0, 1.0, 1.0, it.X, it.ldx, it.X, it.ldx};
      // r = b - A x
      o[3 * E] = BatOp{P.geo, P.tw, it.X, it.ldx, on ? nr : 0, -1.0, 1.0, it.B, it.ldb, e.Rc, e.Ld};
    }
  }
  AZ_HIP(hipMemcpyAsync(sl.dev, sl.host, desc_bytes, hipMemcpyHostToDevice, st));
  sl.used = true;
  // size classes: ranges of equal (n, s) in the sorted order
  struct Cls {
    int n, s, first, count;
    int64_t maxvec;
    double bytes;
  };
  std::vector<Cls> cls;
  for (int q = 0; q < E; ++q) {
    const BatchItem& it = items[ord[q]];
    const Plan& P = *it.P;
    if (cls.empty() || cls.back().n != P.n || cls.back().s != P.s) cls.push_back(Cls{P.n, P.s, q, 0, 0, 0.0});
    Cls& c = cls.back();
    ++c.count;
    c.maxvec = std::max(c.maxvec, it.nrhs);
    c.bytes += 8.0 * it.nrhs * (P.N + 2.0 * P.M) + 16.0 * P.s * P.N;
  }
  int rc = AZRBF_OK;
  auto grouped = [&](int which, int64_t step) -> int {
    for (const Cls& c : cls)
      AZ_TRY(ops_batched(which, c.n, c.s, dop + step * E + c.first, c.count, c.maxvec, c.bytes, st));
    return AZRBF_OK;
  };
  for (int t = 0; t < iters && !rc; ++t) {
    const int64_t s0 = (int64_t)t * 4;
    if ((rc = grouped(1, s0)) || (rc = grouped(0, s0 + 1))) break;
    {
      Prof pr("bat_qtc", 0.0, st);
      launch_kernel(k_bat_qtc_part, dim3((unsigned)maxrb, (unsigned)maxcb, (unsigned)E), 256, 0, st, de, t);
    }
    launch_kernel(k_bat_qtc_sum, dim3((unsigned)maxcb, (unsigned)E), 256, 0, st, de, t);
    {
      Prof pr("bat_xr", 0.0, st);
      launch_kernel(k_bat_xr, dim3((unsigned)maxxr, (unsigned)maxcb, (unsigned)E), 256, 0, st, de, t);
    }
    if (hipGetLastError() != hipSuccess) {
      rc = AZRBF_EHIP;
      break;
    }
    if ((rc = grouped(1, s0 + 2)) || (rc = grouped(0, s0 + 3))) break;
  }
  if (!rc) {
    launch_kernel(k_bat_relres, dim3((unsigned)maxrhs, (unsigned)E), 256, 0, st, de);
    if (hipGetLastError() != hipSuccess) rc = AZRBF_EHIP;
  }
  // the slot is free again once everything queued above has run
  if (hipEventRecord(sl.done, st) != hipSuccess && !rc) rc = AZRBF_EHIP;
  if (rc) (void)hipStreamSynchronize(st);
  return rc;
}

}  // namespace az
