// C ABI of the azrbf library: plans, operators, factor and solve.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

struct azrbf_plan_s {
  az::Plan p;
};

namespace az {

// Device memory pool shared by all plans of the process: freed blocks are
// kept per device and size class and handed to later plans, so creating and
// destroying plans of a recurring size does not call hipMalloc / hipFree.
// Blocks return to the pool only after the owning plan's stream has drained.
namespace {
std::mutex g_pool_mu;
std::multimap<std::pair<int, int64_t>, void*> g_pool;   // (device, bytes) -> block
int64_t g_pool_bytes = 0;
constexpr int64_t kPoolCap = (int64_t)16 << 30;

// Blocks of destroyed plans whose queued work may still be running: they join
// the pool when the event has completed; until then only a plan on the same
// stream (whose work is ordered after it) may take them.
struct PendingRelease {
  int device;
  hipStream_t st;
  hipEvent_t ev;
  std::vector<std::pair<void*, int64_t>> blocks;
};
std::vector<PendingRelease> g_pending;

void pool_put_locked(int device, void* ptr, int64_t cls) {
  if (g_pool_bytes + cls > kPoolCap) {
    (void)hipFree(ptr);
    return;
  }
  g_pool.insert({{device, cls}, ptr});
  g_pool_bytes += cls;
}

void reap_locked() {
  for (size_t i = 0; i < g_pending.size();) {
    PendingRelease& r = g_pending[i];
    if (hipEventQuery(r.ev) != hipSuccess) {
      ++i;
      continue;
    }
    for (auto& b : r.blocks) pool_put_locked(r.device, b.first, b.second);
    (void)hipEventDestroy(r.ev);
    g_pending.erase(g_pending.begin() + (long)i);
  }
}

int64_t size_class(int64_t n) {
  if (n <= 4096) return 4096;
  int64_t c = 4096;
  while (c < n) c += c < ((int64_t)1 << 20) ? c : (c >> 2);   // x2 to 1 MiB, then +25%
  return c;
}
}  // namespace

int Plan::alloc(void** ptr, int64_t nbytes) {
  *ptr = nullptr;
  const int64_t cls = size_class(nbytes <= 0 ? 8 : nbytes);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    reap_locked();
    auto it = g_pool.find({device, cls});
    if (it != g_pool.end()) {
      *ptr = it->second;
      g_pool.erase(it);
      g_pool_bytes -= cls;
    }
    for (size_t i = 0; !*ptr && i < g_pending.size(); ++i) {
      PendingRelease& r = g_pending[i];
      if (r.device != device || r.st != last_stream) continue;
      for (size_t j = 0; j < r.blocks.size(); ++j) {
        if (r.blocks[j].second != cls) continue;
        *ptr = r.blocks[j].first;
        r.blocks.erase(r.blocks.begin() + (long)j);
        break;
      }
    }
  }
  if (!*ptr) {
    if (hipMalloc(ptr, (size_t)cls) != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      return AZRBF_ENOMEM;
    }
  }
  allocs.push_back({*ptr, cls});
  bytes += cls;
  return AZRBF_OK;
}

void Plan::release() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto& a : allocs) {
    if (g_pool_bytes + a.second > kPoolCap) {
      (void)hipFree(a.first);
      continue;
    }
    g_pool.insert({{device, a.second}, a.first});
    g_pool_bytes += a.second;
  }
  allocs.clear();
  bytes = 0;
}

void Plan::release_after(hipStream_t st) {
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, st) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(st);
    release();
    return;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_pending.push_back(PendingRelease{device, st, ev, allocs});
  allocs.clear();
  bytes = 0;
}

void Plan::release_one(void* ptr) {
  if (!ptr) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (size_t i = 0; i < allocs.size(); ++i) {
    if (allocs[i].first != ptr) continue;
    const int64_t cls = allocs[i].second;
    if (g_pool_bytes + cls > kPoolCap) {
      (void)hipFree(ptr);
    } else {
      g_pool.insert({{device, cls}, ptr});
      g_pool_bytes += cls;
    }
    bytes -= cls;
    allocs.erase(allocs.begin() + (long)i);
    return;
  }
}

// A block replaced by a larger one while work queued on st may still use it:
// it joins the pending releases (the pool takes it once that work is done).
void Plan::release_one_after(void* ptr, hipStream_t st) {
  if (!ptr) return;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, st) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipGetLastError();
    (void)hipStreamSynchronize(st);
    release_one(ptr);
    return;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (size_t i = 0; i < allocs.size(); ++i) {
    if (allocs[i].first != ptr) continue;
    g_pending.push_back(PendingRelease{device, st, ev, {allocs[i]}});
    bytes -= allocs[i].second;
    allocs.erase(allocs.begin() + (long)i);
    return;
  }
  (void)hipEventDestroy(ev);
}

// The stream must have drained the factor's work.
void Plan::release_factor() {
  double** bufs[] = {&Om, &Om2, &Yf, &Yf2, &Q, &Rf, &sig, &Pm, &Gj, &Vj, &dscr, &sw, &azs};
  for (double** b : bufs) {
    release_one(*b);
    *b = nullptr;
  }
  dscr_bytes = 0;
  sw_rhs = sw_part = 0;
  azs_cols = 0;
  factored = false;
  rank_pending = false;
  rank = -1;
}

int pool_trim() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto& r : g_pending) {
    (void)hipEventSynchronize(r.ev);
    for (auto& b : r.blocks) (void)hipFree(b.first);
    (void)hipEventDestroy(r.ev);
  }
  g_pending.clear();
  for (auto& kv : g_pool) (void)hipFree(kv.second);
  g_pool.clear();
  g_pool_bytes = 0;
  return AZRBF_OK;
}

// ------------------------------------------------------------------ per-launch timing

namespace {
struct ProfRec {
  std::string name;
  double bytes, flops;
  hipEvent_t a, b;    // markers around the scope
  hipEvent_t ka, kb;  // recorded by the first kernel's dispatch packet
  int kernels;        // launches made inside the scope
  bool done;
};
thread_local int tl_prof_slot = -1;
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t pool_get() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool prof_enabled() { return g_prof_on; }

int prof_begin(hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{std::string(), 0.0, 0.0, pool_get(), pool_get(), pool_get(), pool_get(), 0, false};
  if (!r.a || !r.b || !r.ka || !r.kb) {
    for (hipEvent_t e : {r.a, r.b, r.ka, r.kb})
      if (e) g_prof_pool.push_back(e);
    return -1;
  }
  (void)hipEventRecord(r.a, st);
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

int prof_enter(int slot) {
  const int prev = tl_prof_slot;
  tl_prof_slot = slot;
  return prev;
}

bool prof_kernel_events(hipEvent_t* start, hipEvent_t* stop) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  const int slot = tl_prof_slot;
  if (slot < 0 || slot >= (int)g_prof.size() || g_prof[slot].done) return false;
  ProfRec& r = g_prof[slot];
  if (r.kernels++ != 0) return false;
  *start = r.ka;
  *stop = r.kb;
  return true;
}

void prof_end(int slot, const char* name, double bytes, double flops, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (slot < 0 || slot >= (int)g_prof.size()) return;
  ProfRec& r = g_prof[slot];
  r.name = name;
  r.bytes = bytes;
  r.flops = flops;
  r.done = true;
  (void)hipEventRecord(r.b, st);
}

static bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Largest usable sketch width: a multiple of 64 (16 for tiny problems) not
// above the number of unknowns or of rows.
static int k_cap(int64_t N, int64_t Mt) {
  const int64_t m = std::min(N, Mt);
  if (m >= 64) return (int)std::min<int64_t>(m / 64 * 64, 1 << 15);
  return m >= 32 ? 32 : 16;
}

// Sketch width when the caller leaves it open.  1D: the rank of A - A Z* A
// stays near 20 whatever N (Theorem 4.6), so 32.  2D: the rank grows with the
// boundary (section 5.3.2).  Measured at s = 2 with wide sketches, the number
// of directions a sketch retains per fine-grid boundary point of the mask is
// 6.5 +- 0.2 on the disk (approximation, n = 128), the Poisson star (n = 128
// and 256, with 2.2 weak boundary rows per boundary point) and the Helmholtz
// unit disk (n = 64): the boundary rows add no rank of their own.  The
// estimate is r = 6.6 (2/s) per boundary point.  A Gaussian sketch of width k
// shrinks the smallest of r directions by about sqrt(k) - sqrt(r) instead of
// sqrt(k), so directions just above the truncation threshold are lost unless
// k exceeds r by a margin: k = 1.25 r + 10, rounded up to a multiple of 64
// (at k = 1.1 r the residual was 2-3x larger on the disk and the Helmholtz
// disk).  A sketch that still turns out too narrow is widened by the
// factorisation.
static int default_k(const azrbf_problem& q, int64_t Lax, int64_t Lay, int64_t N, int64_t Mt) {
  if (q.k > 0) return q.k;
  if (q.dim == 1) return 32;
  int64_t perim = 0;
  for (int64_t ix = 0; ix < Lax; ++ix)
    for (int64_t iy = 0; iy < Lay; ++iy) {
      if (!q.mask[ix * Lay + iy]) continue;
      const bool edge = ix == 0 || iy == 0 || ix == Lax - 1 || iy == Lay - 1 ||
                        !q.mask[(ix - 1) * Lay + iy] || !q.mask[(ix + 1) * Lay + iy] ||
                        !q.mask[ix * Lay + iy - 1] || !q.mask[ix * Lay + iy + 1];
      perim += edge;
    }
  const double r = 6.6 * 2.0 / q.s * (double)perim;
  const int64_t est = (int64_t)std::ceil(1.25 * r) + 10;
  const int cap = k_cap(N, Mt);
  if (cap <= 64) return cap;
  const int64_t k = (est + 63) / 64 * 64;
  return (int)std::max<int64_t>(64, std::min<int64_t>(k, cap));
}

// Factor with the plan's sketch width.  A sketch that retains more than 90 %
// of its directions is too narrow to resolve them all (see default_k); when
// the width was not fixed by the caller it is widened to 1.25 times the
// retained rank (at least by a quarter), up to three times.
static int factor_plan(Plan& P, hipStream_t st) {
  for (int attempt = 0;; ++attempt) {
    const int rc = P.k > 64 ? wide_factor(P, st) : dense_factor(P, st);
    if (rc != AZRBF_ERANK || P.prob.k > 0 || attempt >= 3) return rc;
    const int cap = k_cap(P.N, P.Mt);
    if (P.k >= cap) return rc;
    const int64_t want = std::max<int64_t>((int64_t)P.k * 5 / 4, ((int64_t)P.rank * 5 + 3) / 4 + 10);
    int nk = P.k < 64 && want <= 64 ? 64 : (int)((want + 63) / 64 * 64);
    if (nk > cap) nk = cap;
    if (nk <= P.k) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return AZRBF_EHIP;
    P.release_factor();
    P.k = nk;
  }
}

// Four-step split of a 1D transform of length N > 8192 (or forced): N = N1 * N2.
// Rows (the second factor) are at most 512 long; the columns take the rest,
// up to 2048 (N = 2^20).
static void split_1d(int64_t N, int* N1, int* N2) {
  int lg = 0;
  while ((1LL << lg) < N) ++lg;
  int l2 = (lg + 1) / 2;
  if (l2 > 9) l2 = 9;
  *N2 = 1 << l2;
  *N1 = (int)(N >> l2);
}

// Internal streams for azrbf_solve_many (default priority, non-blocking),
// one set per device, created on first use and kept for the process.
constexpr int kManyStreams = 4;
struct ManyPool {
  hipStream_t st[kManyStreams] = {};
  hipEvent_t done[kManyStreams] = {};
  hipEvent_t start = nullptr;
};
std::mutex g_many_mu;                 // one batched call at a time per process
std::map<int, ManyPool> g_many;

int many_pool(int dev, ManyPool** out) {
  auto it = g_many.find(dev);
  if (it == g_many.end()) {
    ManyPool mp;
    for (int w = 0; w < kManyStreams; ++w) {
      if (hipStreamCreateWithFlags(&mp.st[w], hipStreamNonBlocking) != hipSuccess) return AZRBF_EHIP;
      if (hipEventCreateWithFlags(&mp.done[w], hipEventDisableTiming) != hipSuccess) return AZRBF_EHIP;
    }
    if (hipEventCreateWithFlags(&mp.start, hipEventDisableTiming) != hipSuccess) return AZRBF_EHIP;
    it = g_many.emplace(dev, mp).first;
  }
  *out = &it->second;
  return AZRBF_OK;
}

// Side streams for work that overlaps a factorisation (default priority,
// non-blocking), a few per device, handed out in turn.
constexpr int kSideStreams = 4;
std::mutex g_side_mu;
std::map<int, std::vector<hipStream_t>> g_side;
int g_side_next = 0;

int side_stream(int dev, hipStream_t* out) {
  std::lock_guard<std::mutex> lk(g_side_mu);
  std::vector<hipStream_t>& v = g_side[dev];
  if (v.empty()) {
    for (int i = 0; i < kSideStreams; ++i) {
      hipStream_t s = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return AZRBF_EHIP;
      v.push_back(s);
    }
  }
  *out = v[(g_side_next++) % kSideStreams];
  return AZRBF_OK;
}

}  // namespace az

using az::Plan;

extern "C" {

const char* azrbf_strerror(int code) {
  switch (code) {
    case AZRBF_OK: return "ok";
    case AZRBF_EINVAL: return "invalid argument";
    case AZRBF_EUNSUPPORTED: return "unsupported problem size or option";
    case AZRBF_ENOMEM: return "device memory allocation failed";
    case AZRBF_EHIP: return "HIP runtime error";
    case AZRBF_ERANK: return "sketch too narrow: more than 90% of its directions retained";
    case AZRBF_ESTATE: return "call not valid in the plan's state";
    case AZRBF_ESCRATCH: return "needs more than the fixed scratch buffer of the allocation-free entry point";
    default: return "unknown error";
  }
}

int azrbf_plan(const azrbf_problem* pr, void* stream, azrbf_plan_t* out) {
  if (!pr || !out) return AZRBF_EINVAL;
  *out = nullptr;
  const azrbf_problem& q = *pr;
  if (q.dim != 1 && q.dim != 2) return AZRBF_EINVAL;
  if (!(q.T > 0) || !q.mask || q.n <= 0 || q.s <= 0) return AZRBF_EINVAL;
  if (q.op != AZRBF_OP_APPROX && q.op != AZRBF_OP_BVP) return AZRBF_EINVAL;
  if (q.nb < 0 || (q.nb > 0 && (!q.bpts || q.op != AZRBF_OP_BVP))) return AZRBF_EINVAL;
  if (!(q.tau > 0) || q.tauZ < 0 || q.refine < 0 || q.refine > 8 || q.k < 0) return AZRBF_EINVAL;
  if (q.eps <= 0 && !(q.tau0 > 0 && q.tau0 < 1)) return AZRBF_EINVAL;
  // centre counts: powers of two (the register-resident engine) or any
  // other count (the mixed-radix path; Bluestein for prime factors above 7)
  if (q.n < 16) return AZRBF_EUNSUPPORTED;
  if ((q.dim == 1 && q.n > (1 << 20)) || (q.dim == 2 && q.n > 512)) return AZRBF_EUNSUPPORTED;
  if (q.ny < 0 || q.Ty < 0 || (q.dim == 1 && (q.ny > 0 || q.Ty > 0))) return AZRBF_EINVAL;
  if (q.dim == 2 && q.ny > 0 && (q.ny < 16 || q.ny > 512)) return AZRBF_EUNSUPPORTED;
  const bool generic = !az::pow2(q.n) || (q.dim == 2 && q.ny > 0 && !az::pow2(q.ny));
  // a column pass puts the s phases of a column in one block of at most 256
  // threads, n1 / 16 per phase (1D: n1 = n / 512 once n > 2^18)
  if (!generic && q.dim == 1 && q.n > (1 << 18) && q.s * (q.n >> 9) / 16 > 256) return AZRBF_EUNSUPPORTED;
  if (q.s < 1 || q.s > 4) return AZRBF_EUNSUPPORTED;
  bool neumann = false;
  if (q.nb > 0 && q.btype) {
    for (int64_t i = 0; i < q.nb; ++i) {
      if (q.btype[i] > 1) return AZRBF_EINVAL;
      if (!q.btype[i]) continue;
      neumann = true;
      if (!q.bnormal) return AZRBF_EINVAL;
      double nn = 0.0;
      for (int a = 0; a < q.dim; ++a) nn += q.bnormal[i * q.dim + a] * q.bnormal[i * q.dim + a];
      if (!(std::fabs(nn - 1.0) <= 1e-8)) return AZRBF_EINVAL;   // a unit normal (NaN fails too)
    }
  }

  azrbf_plan_s* h = new (std::nothrow) azrbf_plan_s();
  if (!h) return AZRBF_ENOMEM;
  Plan& P = h->p;
  hipStream_t st = (hipStream_t)stream;
  P.last_stream = st;
  P.prob = q;
  P.prob.mask = nullptr;
  P.prob.bpts = nullptr;
  P.prob.btype = nullptr;
  P.prob.bnormal = nullptr;
  if (hipGetDevice(&P.device) != hipSuccess) { delete h; return AZRBF_EHIP; }
  P.dim = q.dim;
  P.generic = generic;
  P.n = q.n;
  P.s = q.s;
  P.ph = q.dim == 1 ? q.s : q.s * q.s;
  P.T = q.T;
  P.h = 2.0 * q.T / q.n;
  P.hL = P.h / q.s;
  P.ny = q.dim == 2 ? (q.ny > 0 ? q.ny : q.n) : 1;
  P.Ty = q.dim == 2 && q.Ty > 0 ? q.Ty : q.T;
  P.hy = 2.0 * P.Ty / P.ny;
  P.hLy = P.hy / q.s;
  if (q.eps > 0) {
    P.eps = q.eps;
  } else {   // eq. constant_shapeparam: eps = c N, c = pi / (2 T sqrt(2 log(1 + tau0^-2)))
    const double c = M_PI / (2.0 * q.T * sqrt(2.0 * log1p(1.0 / (q.tau0 * q.tau0))));
    P.eps = c * q.n;
  }
  P.tau = q.tau;
  P.tauZ = q.tauZ;
  P.refine = q.refine;
  P.bweight = q.bweight;
  P.N = q.dim == 1 ? (int64_t)q.n : (int64_t)q.n * P.ny;
  P.Lax = (int64_t)q.s * q.n;
  P.Lay = q.dim == 1 ? 1 : (int64_t)q.s * P.ny;
  P.Lg = q.dim == 1 ? P.Lax : P.Lax * P.Lay;
  P.Mb = q.nb;

  int rc = az::ops_init_twiddles(P.device, &P.tw);
  if (rc) { delete h; return rc; }

  az::Geo& g = P.geo;
  g.dim = P.dim;
  g.s = P.s;
  g.L = (int)(q.dim == 1 ? P.Lax : P.Lay);   // 2D: fine-grid points per x line
  g.N = P.N;
  g.op = q.op;
  g.k2 = q.k2;
  g.opscale = q.dim == 1 ? -1.0 / (2.0 * P.eps * P.eps) : -1.0 / (4.0 * P.eps * P.eps);

  // collocation rows: ascending fine-grid order
  int64_t M = 0;
  for (int64_t i = 0; i < P.Lg; ++i) M += q.mask[i] != 0;
  if (M == 0) { delete h; return AZRBF_EINVAL; }
  P.M = M;
  P.Mt = M + P.Mb;
  P.Mtp = (P.Mt + 15) / 16 * 16;
  g.M = M;
  if (P.dim == 1) {
    int64_t i0 = 0;
    while (!q.mask[i0]) ++i0;
    for (int64_t i = i0; i < i0 + M; ++i)
      if (!q.mask[i]) { delete h; return AZRBF_EUNSUPPORTED; }   // 1D domains are intervals
    g.i0 = i0;
    const char* force = getenv("AZRBF_ENGINE");
    P.fused = !P.generic && P.N <= 8192 && !(force && force[0] == '1' && P.N >= 256);
    if (P.fused || P.generic) {
      g.N1 = 1;
      g.N2 = (int)P.N;
    } else {
      az::split_1d(P.N, &g.N1, &g.N2);
      if (g.N1 < 16 || g.N2 < 16 || g.N1 > 2048 || g.N2 > 512) { delete h; return AZRBF_EUNSUPPORTED; }
    }
  } else {
    g.N1 = P.n;
    g.N2 = P.ny;
    std::vector<int32_t> inv(P.Lg);
    int64_t m = 0;
    for (int64_t i = 0; i < P.Lg; ++i) inv[i] = q.mask[i] ? (int32_t)m++ : -1;
    rc = P.alloc((void**)&P.inv, sizeof(int32_t) * P.Lg);
    if (!rc && hipMemcpyAsync(P.inv, inv.data(), sizeof(int32_t) * P.Lg, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = AZRBF_EHIP;
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = AZRBF_EHIP;
    if (rc) { P.release(); delete h; return rc; }
    g.inv = P.inv;
  }
  if (P.Mb > 0) {
    rc = P.alloc((void**)&P.bpts, sizeof(double) * P.Mb * P.dim);
    if (!rc && hipMemcpyAsync(P.bpts, q.bpts, sizeof(double) * P.Mb * P.dim, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = AZRBF_EHIP;
    if (!rc && neumann) {   // types and normals: read by the boundary rows and the right-hand sides
      rc = P.alloc((void**)&P.btype, P.Mb);
      if (!rc) rc = P.alloc((void**)&P.bnorm, sizeof(double) * P.Mb * P.dim);
      if (!rc && hipMemcpyAsync(P.btype, q.btype, P.Mb, hipMemcpyHostToDevice, st) != hipSuccess) rc = AZRBF_EHIP;
      if (!rc && hipMemcpyAsync(P.bnorm, q.bnormal, sizeof(double) * P.Mb * P.dim, hipMemcpyHostToDevice, st) !=
                     hipSuccess)
        rc = AZRBF_EHIP;
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = AZRBF_EHIP;
    if (rc) { P.release(); delete h; return rc; }
  }
  P.k = az::default_k(q, P.Lax, P.Lay, P.N, P.Mt);
  az::tune_apply(P);
  rc = az::ops_spectra(P, st);
  // no synchronisation: work on this stream is ordered after the set-up, work
  // on other streams waits for this event (plan_on_stream)
  P.make_stream = st;
  if (!rc) rc = az::plan_mark_ready(P, st);
  if (rc) {
    (void)hipStreamSynchronize(st);
    if (P.ready) (void)hipEventDestroy(P.ready);
    P.release();
    delete h;
    return rc;
  }
  *out = h;
  return AZRBF_OK;
}

int azrbf_plan_dims(azrbf_plan_t h, int64_t* dims) {
  if (!h || !dims) return AZRBF_EINVAL;
  const Plan& P = h->p;
  dims[0] = P.N;
  dims[1] = P.M;
  dims[2] = P.Mb;
  dims[3] = P.Lg;
  dims[4] = P.k;
  return AZRBF_OK;
}

int azrbf_plan_info(azrbf_plan_t h, azrbf_info* info) {
  if (!h || !info) return AZRBF_EINVAL;
  Plan& P = h->p;
  info->N = P.N;
  info->M = P.M;
  info->Mb = P.Mb;
  info->L = P.Lg;
  info->k = P.k;
  if (az::plan_fetch_rank(P) != AZRBF_OK) return AZRBF_EHIP;
  info->rank = P.factored ? P.rank : -1;
  info->eps = P.eps;
  if (az::ops_norms(P, P.last_stream) != AZRBF_OK) return AZRBF_EHIP;
  info->normA = P.normA;
  info->normZ = P.normZ;
  info->zeroed = P.zeroed;
  info->factored = P.factored ? 1 : 0;
  info->sweeps = P.sweeps;
  info->device_bytes = P.bytes;
  return AZRBF_OK;
}

int azrbf_apply_A(azrbf_plan_t h, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                  double* Y, int64_t ldy, void* stream) {
  if (!h || nvec < 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  if (nvec == 0) return AZRBF_OK;
  if (!X || !Y || ldx < P.N || ldy < P.Mt) return AZRBF_EINVAL;
  P.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  return az::ops_apply_A(P, X, ldx, nvec, alpha, beta, nullptr, 0, Y, ldy, (hipStream_t)stream);
}

int azrbf_rhs(azrbf_plan_t h, const double* f, int64_t ldf, const double* g, int64_t ldg, int64_t nrhs,
              double* B, int64_t ldb, void* stream) {
  if (!h || nrhs < 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  if (nrhs == 0) return AZRBF_OK;
  if (!f || !B || ldf < P.M || ldb < P.Mt || (P.Mb > 0 && (!g || ldg < P.Mb))) return AZRBF_EINVAL;
  if (f != B && ((f < B + ldb * nrhs) && (B < f + ldf * nrhs))) return AZRBF_EINVAL;   // partial overlap
  if (f == B && ldf != ldb) return AZRBF_EINVAL;
  if (g && P.Mb > 0 && (g < B + ldb * nrhs) && (B < g + ldg * nrhs)) return AZRBF_EINVAL;
  P.last_stream = (hipStream_t)stream;
  return az::ops_rhs(P, f, ldf, g, ldg, nrhs, B, ldb, (hipStream_t)stream);
}

int azrbf_apply_Zstar(azrbf_plan_t h, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                      double* Z, int64_t ldz, void* stream) {
  if (!h || nvec < 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  if (nvec == 0) return AZRBF_OK;
  if (!R || !Z || ldr < P.Mt || ldz < P.N) return AZRBF_EINVAL;
  P.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  return az::ops_apply_Z(P, R, ldr, nvec, alpha, beta, nullptr, 0, Z, ldz, (hipStream_t)stream);
}

int azrbf_apply_AZstar(azrbf_plan_t h, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                       double* Y, int64_t ldy, void* stream) {
  if (!h || nvec < 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  if (nvec == 0) return AZRBF_OK;
  if (!R || !Y || ldr < P.Mt || ldy < P.Mt) return AZRBF_EINVAL;
  if (R == Y && ldr != ldy) return AZRBF_EINVAL;
  P.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  if ((P.fused || P.generic || P.Mb > 0) && nvec > P.azs_cols) {
    // the previous scratch may still be in use by queued work on this stream
    double* old = P.azs;
    AZ_TRY(P.alloc((void**)&P.azs, sizeof(double) * P.N * nvec));
    P.release_one_after(old, (hipStream_t)stream);
    P.azs_cols = nvec;
  }
  return az::ops_apply_AZ(P, R, ldr, nvec, alpha, beta, nullptr, 0, Y, ldy, P.azs, (hipStream_t)stream);
}

int azrbf_factor(azrbf_plan_t h, void* stream) {
  if (!h) return AZRBF_EINVAL;
  h->p.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(h->p, h->p.last_stream));
  return az::factor_plan(h->p, (hipStream_t)stream);
}

int azrbf_solve(azrbf_plan_t h, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                double* relres, void* stream) {
  if (!h || nrhs < 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  if (nrhs == 0) return AZRBF_OK;
  if (!B || !X || ldb < P.Mt || ldx < P.N) return AZRBF_EINVAL;
  P.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  hipStream_t st = (hipStream_t)stream;
  // (not while per-launch timing is on: launches then run one at a time so
  // that each one's time is its own)
  if (!P.factored && P.k <= 64 && P.prob.k > 0 && !az::prof_enabled()) {
    // The first pass's c = (I - A Z*) b does not need the factor: it runs on a
    // side stream (with its own FFT workspace) while the latency-bound
    // factorisation runs on the caller's stream.  (With a fixed sketch width
    // the factor cannot be widened, so the workspace stays valid.)
    hipStream_t side = nullptr;
    AZ_TRY(az::side_stream(P.device, &side));
    hipEvent_t e_in = nullptr, e_side = nullptr;
    if (hipEventCreateWithFlags(&e_in, hipEventDisableTiming) != hipSuccess) return AZRBF_EHIP;
    if (hipEventCreateWithFlags(&e_side, hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(e_in);
      return AZRBF_EHIP;
    }
    // the side work starts once the factor's sketch (bandwidth-bound FFTs) is
    // done, so that it runs beside the latency-bound TSQR and Jacobi kernels;
    // the first pass's Q^T c is queued as soon as Q is, beside the Jacobi SVD
    auto on_sketch = [&]() -> int {
      if (hipStreamWaitEvent(side, e_in, 0) != hipSuccess) return AZRBF_EHIP;
      P.swap_ws();
      const int r = az::dense_first_stage(P, B, ldb, nrhs, side);
      P.swap_ws();
      if (r) return r;
      return hipEventRecord(e_side, side) == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
    };
    auto before_products = [&]() -> int {
      if (hipStreamWaitEvent(st, e_side, 0) != hipSuccess) return AZRBF_EHIP;
      return az::dense_first_qtc(P, nrhs, st);
    };
    int rc = az::dense_factor_enqueue(P, st, e_in, on_sketch, before_products);
    // the solve needs no host-side result of the factor: it is queued at once,
    // and the retained rank stays on the device until asked for
    // (azrbf_plan_info), so the call returns without waiting for the GPU
    if (!rc) {
      P.factored = true;
      P.rank_pending = true;
      P.factor_stream = st;
      rc = az::plan_mark_ready(P, st);
    }
    if (!rc) rc = az::dense_solve(P, B, ldb, nrhs, X, ldx, relres, st, true, true);
    if (rc) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamSynchronize(side);
    }
    (void)hipEventDestroy(e_in);
    (void)hipEventDestroy(e_side);
    return rc;
  }
  if (!P.factored) {
    const int rc = az::factor_plan(P, st);
    if (rc != AZRBF_OK && rc != AZRBF_ERANK) return rc;
  }
  if (P.k > 64) return az::wide_solve(P, B, ldb, nrhs, X, ldx, relres, st);
  return az::dense_solve(P, B, ldb, nrhs, X, ldx, relres, st);
}

int azrbf_solve_many(int32_t nprob, const azrbf_plan_t* plans, const double* const* B, const int64_t* ldb,
                     const int64_t* nrhs, double* const* X, const int64_t* ldx, double* const* relres,
                     void* stream) {
  if (nprob < 0 || (nprob > 0 && (!plans || !B || !ldb || !nrhs || !X || !ldx))) return AZRBF_EINVAL;
  if (nprob == 0) return AZRBF_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return AZRBF_EHIP;
  for (int32_t i = 0; i < nprob; ++i) {
    if (!plans[i] || nrhs[i] < 0) return AZRBF_EINVAL;
    const Plan& P = plans[i]->p;
    if (P.device != dev) return AZRBF_EINVAL;
    if (nrhs[i] > 0 && (!B[i] || !X[i] || ldb[i] < P.Mt || ldx[i] < P.N)) return AZRBF_EINVAL;
    for (int32_t j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return AZRBF_EINVAL;   // a plan serves one stream at a time
  }
  hipStream_t caller = (hipStream_t)stream;
  if (nprob == 1)
    return azrbf_solve(plans[0], B[0], ldb[0], nrhs[0], X[0], ldx[0], relres ? relres[0] : nullptr, stream);
  std::lock_guard<std::mutex> lk(az::g_many_mu);
  az::ManyPool* mp = nullptr;
  AZ_TRY(az::many_pool(dev, &mp));
  const int W = std::min<int>(az::kManyStreams, nprob);
  // largest work first, each to the least-loaded worker
  std::vector<std::pair<double, int>> cost(nprob);
  for (int32_t i = 0; i < nprob; ++i) {
    const Plan& P = plans[i]->p;
    const double lg = std::log2((double)P.N + 1.0);
    double c = (double)P.N * lg * (double)(nrhs[i] + 1);
    if (!P.factored) c += (double)P.N * lg * 3.0 * P.k + (P.k > 64 ? 8.0 * P.Mt * (double)P.k * P.k : 0.0);
    cost[i] = {c, i};
  }
  std::sort(cost.begin(), cost.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first || (a.first == b.first && a.second < b.second);
  });
  std::vector<std::vector<int>> lists(W);
  std::vector<double> load(W, 0.0);
  for (const auto& ci : cost) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lists[w].push_back(ci.second);
    load[w] += ci.first;
  }
  if (hipEventRecord(mp->start, caller) != hipSuccess) return AZRBF_EHIP;
  for (int w = 0; w < W; ++w)
    if (hipStreamWaitEvent(mp->st[w], mp->start, 0) != hipSuccess) return AZRBF_EHIP;
  std::vector<int> rcs(nprob, AZRBF_OK);
  std::vector<std::thread> th;
  for (int w = 0; w < W; ++w) {
    th.emplace_back([&, w]() {
      if (hipSetDevice(dev) != hipSuccess) {
        for (int i : lists[w]) rcs[i] = AZRBF_EHIP;
        return;
      }
      for (int i : lists[w])
        rcs[i] = azrbf_solve(plans[i], B[i], ldb[i], nrhs[i], X[i], ldx[i], relres ? relres[i] : nullptr,
                             mp->st[w]);
    });
  }
  for (auto& t : th) t.join();
  int rc = AZRBF_OK;
  for (int w = 0; w < W; ++w) {
    if (hipEventRecord(mp->done[w], mp->st[w]) != hipSuccess || hipStreamWaitEvent(caller, mp->done[w], 0) != hipSuccess)
      rc = AZRBF_EHIP;
  }
  for (int32_t i = 0; i < nprob && rc == AZRBF_OK; ++i) rc = rcs[i];
  return rc;
}

int azrbf_solve_batched(int32_t nprob, const azrbf_plan_t* plans, const double* const* B, const int64_t* ldb,
                        const int64_t* nrhs, double* const* X, const int64_t* ldx, double* const* relres,
                        void* stream) {
  if (nprob < 0 || nprob > 65535 || (nprob > 0 && (!plans || !B || !ldb || !nrhs || !X || !ldx))) return AZRBF_EINVAL;
  if (nprob == 0) return AZRBF_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return AZRBF_EHIP;
  for (int32_t i = 0; i < nprob; ++i) {
    if (!plans[i] || nrhs[i] < 0) return AZRBF_EINVAL;
    const Plan& P = plans[i]->p;
    if (P.device != dev) return AZRBF_EINVAL;
    if (nrhs[i] > 0 && (!B[i] || !X[i] || ldb[i] < P.Mt || ldx[i] < P.N)) return AZRBF_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  // set-up and factors first (each plan once: the single-kernel 1D plans in
  // one grouped factorisation, the others one by one), then the other entries
  // one by one, then the grouped entries together
  std::vector<az::BatchItem> items;
  std::vector<Plan*> grouped_factor;
  for (int32_t i = 0; i < nprob; ++i) {
    if (nrhs[i] == 0) continue;
    Plan& P = plans[i]->p;
    P.last_stream = st;
    AZ_TRY(az::plan_on_stream(P, st));
    if (P.factored) continue;
    if (az::dense_factor_batchable(P)) {
      if (std::find(grouped_factor.begin(), grouped_factor.end(), &P) == grouped_factor.end())
        grouped_factor.push_back(&P);
    } else {
      const int rc = az::factor_plan(P, st);
      if (rc != AZRBF_OK && rc != AZRBF_ERANK) return rc;
    }
  }
  {
    std::vector<int> rcs;
    AZ_TRY(az::dense_factor_batched(grouped_factor, rcs, st));
    for (size_t i = 0; i < grouped_factor.size(); ++i) {
      // too narrow with the width left open: factored again on its own, widened
      if (rcs[i] == AZRBF_ERANK && grouped_factor[i]->prob.k == 0) {
        const int rc = az::factor_plan(*grouped_factor[i], st);
        if (rc != AZRBF_OK && rc != AZRBF_ERANK) return rc;
      }
    }
  }
  for (int32_t i = 0; i < nprob; ++i) {
    if (nrhs[i] == 0) continue;
    Plan& P = plans[i]->p;
    double* rr = relres ? relres[i] : nullptr;
    if (az::batched_eligible(P)) {
      items.push_back(az::BatchItem{&P, B[i], ldb[i], nrhs[i], X[i], ldx[i], rr});
    } else if (P.k > 64) {
      AZ_TRY(az::wide_solve(P, B[i], ldb[i], nrhs[i], X[i], ldx[i], rr, st));
    } else {
      AZ_TRY(az::dense_solve(P, B[i], ldb[i], nrhs[i], X[i], ldx[i], rr, st));
    }
  }
  return az::batched_solve(items, st);
}

int64_t azrbf_footprint_bytes(const azrbf_problem* pr, int64_t max_rhs) {
  if (!pr || pr->n <= 0 || pr->s <= 0 || (pr->dim != 1 && pr->dim != 2) || max_rhs < 0) return -1;
  const int64_t n = pr->n, s = pr->s;
  const int64_t ny = pr->dim == 2 && pr->ny > 0 ? pr->ny : n;
  const int64_t N = pr->dim == 1 ? n : n * ny;
  const int64_t Lax = s * n, Lay = pr->dim == 1 ? 1 : s * ny;
  const int64_t Lg = Lax * Lay;
  const int64_t ph = pr->dim == 1 ? s : s * s;
  int64_t M = 0;
  if (pr->mask)
    for (int64_t i = 0; i < Lg; ++i) M += pr->mask[i] != 0;
  else
    M = Lg;
  const int64_t Mt = M + pr->nb;
  int k = pr->k > 0 ? pr->k : (pr->dim == 1 || !pr->mask ? 32 : az::default_k(*pr, Lax, Lay, N, Mt));
  int64_t b = 0;
  b += 2 * ph * N * 16;                                 // spectra (1D) or factors + weights (2D)
  b += pr->dim == 2 ? Lg * 4 : 0;                       // inverse map
  b += pr->nb * (16 * pr->dim + 1);                     // boundary points, normals, types
  int64_t chunk = ((int64_t)256 << 20) / (ph * N * 16);   // as engine_chunk
  chunk = chunk < 1 ? 1 : (chunk > 64 ? 64 : chunk);
  const int64_t pairs = (std::max<int64_t>(k, max_rhs) + 1) / 2;
  // FFT workspace; a 1D solve with k <= 64 keeps a second set for its side stream
  const int64_t wsets = pr->dim == 1 && k <= 64 ? 2 : 1;
  const bool generic = !az::pow2(n) || !az::pow2(ny);
  if (generic)
    b += wsets * az::gen_ws_bytes(pr->dim == 1 ? 1 : n, pr->dim == 1 ? N : ny, pairs);
  else if (!(pr->dim == 1 && N <= 8192))
    b += wsets * 2 * ph * N * 16 * std::min<int64_t>(chunk, pairs);
  if (k > 64) {
    b += 8 * az::wide_factor_doubles(N, Mt, k);
    b += 8 * (max_rhs * (2 * N + 3 * Mt + 2 * k + 64) + az::gemm_split_doubles(k, max_rhs, Mt, 1) + 1);
  } else {
    const int64_t Mtp = (Mt + 15) / 16 * 16;              // padded leading dimension
    b += 8 * (2 * N * k + 3 * Mtp * k + 2 * k * k);       // factor and its scratch
    b += 8 * (Mt * k / 4 + Mt * k / 4);                   // TSQR tree (upper bound)
    b += 8 * max_rhs * (N + 3 * Mtp + k + ((Mt + 1023) / 1024) * k + 2);
  }
  return b;
}

int azrbf_get_factor(azrbf_plan_t h, int32_t which, double* dst, int64_t ld, void* stream) {
  if (!h || !dst) return AZRBF_EINVAL;
  Plan& P = h->p;
  hipStream_t st = (hipStream_t)stream;
  if (!P.factored) return AZRBF_ESTATE;
  P.last_stream = st;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  const int k = P.k;
  switch (which) {
    case 0:
      if (ld < P.N) return AZRBF_EINVAL;
      return az::dense_gaussian(P.prob.seed, P.N, k, dst, ld, st);
    case 1:
      if (ld < P.Mt) return AZRBF_EINVAL;
      return hipMemcpy2DAsync(dst, 8 * ld, P.Q, 8 * P.ldq, 8 * P.Mt, k, hipMemcpyDeviceToDevice, st) == hipSuccess
                 ? AZRBF_OK : AZRBF_EHIP;
    case 2:
      if (ld < k) return AZRBF_EINVAL;
      return hipMemcpy2DAsync(dst, 8 * ld, P.Rf, 8 * k, 8 * k, k, hipMemcpyDeviceToDevice, st) == hipSuccess
                 ? AZRBF_OK : AZRBF_EHIP;
    case 3:
      return hipMemcpyAsync(dst, P.sig, 8 * k, hipMemcpyDeviceToDevice, st) == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
    default:
      return AZRBF_EINVAL;
  }
}

int azrbf_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* dst, int64_t ld, void* stream) {
  if (rows < 0 || cols < 0 || (rows > 0 && cols > 0 && (!dst || ld < rows))) return AZRBF_EINVAL;
  return az::dense_gaussian(seed, rows, cols, dst, ld, (hipStream_t)stream);
}

int azrbf_autotune(azrbf_plan_t h, int64_t nvec, void* stream, char* report, int64_t len) {
  if (!h || nvec <= 0) return AZRBF_EINVAL;
  Plan& P = h->p;
  P.last_stream = (hipStream_t)stream;
  AZ_TRY(az::plan_on_stream(P, P.last_stream));
  std::string rep, trep;
  int rc = az::tune_plan(P, nvec, (hipStream_t)stream, &rep);
  if (rc) return rc;
  // the TSQR tile of the low-rank stage: the plan's sketch width, or the
  // 64-column panels of the wide stage
  rc = az::tune_tsqr(P, P.k <= 64 ? P.k : 64, (hipStream_t)stream, &trep);
  if (rc) return rc;
  if (!trep.empty()) rep = rep.substr(0, rep.size() - 1) + ", \"tsqr\": " + trep + "}";
  if (report && len > 0) {
    if ((int64_t)rep.size() + 1 > len) return AZRBF_EINVAL;
    memcpy(report, rep.c_str(), rep.size() + 1);
  }
  return AZRBF_OK;
}

int azrbf_tune_table(char* buf, int64_t len) {
  if (!buf || len <= 0) return AZRBF_EINVAL;
  std::string s;
  az::tune_table(&s);
  if ((int64_t)s.size() + 1 > len) return AZRBF_EINVAL;
  memcpy(buf, s.c_str(), s.size() + 1);
  return AZRBF_OK;
}

int azrbf_tune_load(const char* text) {
  if (!text) return AZRBF_EINVAL;
  return az::tune_load(text);
}

int azrbf_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(az::g_prof_mu);
  az::g_prof_on = on != 0;
  return AZRBF_OK;
}

int azrbf_profile_report(char* buf, int64_t len) {
  if (!buf || len <= 0) return AZRBF_EINVAL;
  std::lock_guard<std::mutex> lk(az::g_prof_mu);
  struct Acc {
    int64_t calls = 0;
    double ms = 0, bytes = 0, flops = 0, max_ms = 0;
  };
  std::map<std::string, Acc> acc;
  int rc = AZRBF_OK;
  for (auto& r : az::g_prof) {
    if (!r.done) continue;
    float ms = 0.f;
    const bool own = r.kernels == 1;
    if (hipEventSynchronize(r.b) != hipSuccess ||
        hipEventElapsedTime(&ms, own ? r.ka : r.a, own ? r.kb : r.b) != hipSuccess) {
      rc = AZRBF_EHIP;
      continue;
    }
    Acc& a = acc[r.name];
    a.calls += 1;
    a.ms += ms;
    a.bytes += r.bytes;
    a.flops += r.flops;
    if (ms > a.max_ms) a.max_ms = ms;
  }
  for (auto& r : az::g_prof) {
    for (hipEvent_t e : {r.a, r.b, r.ka, r.kb})
      if (e) az::g_prof_pool.push_back(e);
  }
  az::g_prof.clear();
  std::string out = "[";
  bool first = true;
  char tmp[512];
  for (auto& kv : acc) {
    snprintf(tmp, sizeof(tmp),
             "%s{\"name\": \"%s\", \"calls\": %lld, \"ms\": %.6f, \"max_ms\": %.6f, \"bytes\": %.0f, "
             "\"flops\": %.0f}",
             first ? "" : ", ", kv.first.c_str(), (long long)kv.second.calls, kv.second.ms, kv.second.max_ms,
             kv.second.bytes, kv.second.flops);
    out += tmp;
    first = false;
  }
  out += "]";
  if ((int64_t)out.size() + 1 > len) return AZRBF_EINVAL;
  memcpy(buf, out.c_str(), out.size() + 1);
  return rc;
}

void azrbf_destroy(azrbf_plan_t h) {
  if (!h) return;
  // the plan's blocks go back to the pool once the work queued on them has
  // run: work on the plan's own stream, and on its latest stream, which first
  // waits for the former
  Plan& P = h->p;
  if (P.make_stream != P.last_stream && P.ready && hipEventRecord(P.ready, P.make_stream) == hipSuccess)
    (void)hipStreamWaitEvent(P.last_stream, P.ready, 0);
  P.release_after(P.last_stream);
  if (P.ready) (void)hipEventDestroy(P.ready);
  delete h;
}

int azrbf_release_cached_memory(void) {
  const int a = az::pool_trim();
  const int b = az::batched_release();
  return a != AZRBF_OK ? a : b;
}

}  // extern "C"
