// Autotuning of the FFT engine's tile shapes.
//
// The three passes of the engine (column FFTs, row FFTs with the spectral
// products, inverse column FFTs) take three shape parameters: C, the columns
// one block transforms (coalesced runs of C complex values per row), Lr, the
// rows one block transforms, and the number of vector pairs per chunk (how
// much of the batch one launch covers).  Which shape is fastest depends on
// the transform lengths, the oversampling and the batch, so it is measured:
// azrbf_autotune times apply_A followed by apply_Z* on the plan's own
// operator for each candidate (coordinate search: C, then Lr, then the
// chunk), keeps the fastest in the plan and in a process-wide table keyed by
// the engine shape, from which later plans of the same shape start.
//
// The TSQR of the low-rank stage has one tile parameter, the rows a block
// QR holds in registers (RB = 256 RPT): larger blocks mean fewer blocks and
// tree levels but more work per column step.  The autotuner times the whole
// TSQR (block QR tree and Q formation) of an Mt x k Gaussian matrix for each
// admissible RB and keeps the fastest under the key t<k>_<Mt>.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace az {

namespace {

struct Shape {
  int C = 0, L = 0, chunk = 0;
};

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune;

std::string engine_key(const Plan& P) {
  char b[96];
  snprintf(b, sizeof(b), "e%d_%dx%d_s%d", P.dim, P.geo.N1, P.geo.N2, P.s);
  return b;
}

bool uses_engine(const Plan& P) { return !P.fused && !P.generic; }

// Best of `reps` timings of apply_A (X -> Y) then apply_Z* (Y -> Z), in ms.
int time_ops(Plan& P, const double* X, double* Y, double* Z, int64_t nvec, hipStream_t st, int reps,
             float* best) {
  hipEvent_t a = nullptr, b = nullptr;
  AZ_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return AZRBF_EHIP;
  }
  int rc = AZRBF_OK;
  *best = 1e30f;
  for (int r = 0; r <= reps && rc == AZRBF_OK; ++r) {   // the first run warms up
    if (hipEventRecord(a, st) != hipSuccess) rc = AZRBF_EHIP;
    if (!rc) rc = ops_apply_A(P, X, P.N, nvec, 1.0, 0.0, nullptr, 0, Y, P.Mt, st);
    if (!rc) rc = ops_apply_Z(P, Y, P.Mt, nvec, 1.0, 0.0, nullptr, 0, Z, P.N, st);
    if (!rc && hipEventRecord(b, st) != hipSuccess) rc = AZRBF_EHIP;
    if (!rc && hipEventSynchronize(b) != hipSuccess) rc = AZRBF_EHIP;
    float ms = 0.f;
    if (!rc && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = AZRBF_EHIP;
    if (!rc && r > 0 && ms < *best) *best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

std::string tsqr_key(int k, int64_t m) {
  char b[64];
  snprintf(b, sizeof(b), "t%d_%lld", k, (long long)m);
  return b;
}

int tsqr_slot(int k) { return k == 16 ? 0 : k == 32 ? 1 : 2; }

void tune_apply(Plan& P) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int k : {16, 32, 64}) {
    auto t = g_tune.find(tsqr_key(k, P.Mt));
    if (t != g_tune.end() && tsqr_rows_ok(k, t->second.C)) P.tsqr_rb[tsqr_slot(k)] = t->second.C;
  }
  if (!uses_engine(P)) return;
  auto it = g_tune.find(engine_key(P));
  if (it == g_tune.end()) return;
  const Shape& s = it->second;
  if (!engine_shape_ok(P.geo.N1, P.geo.N2, s.C, s.L, s.chunk)) return;
  P.tune_C = s.C;
  P.tune_L = s.L;
  P.tune_chunk = s.chunk;
}

int tune_plan(Plan& P, int64_t nvec, hipStream_t st, std::string* report) {
  *report = "{\"engine\": false}";
  if (!uses_engine(P) || nvec <= 0) return AZRBF_OK;
  const int N1 = P.geo.N1, N2 = P.geo.N2;
  const int T1 = N1 / 16, T2 = N2 / 16;
  std::vector<int> Cs, Ls, chunks;
  for (int c = 2; c * T1 <= 256 && c <= N2; c *= 2) Cs.push_back(c);
  for (int l = 2; l * T2 <= 256 && l <= N1; l *= 2) Ls.push_back(l);
  const int64_t npairs = (nvec + 1) / 2;
  for (int ch = 4; ch <= 64; ch *= 2)
    if (ch <= npairs) chunks.push_back(ch);
  if (chunks.empty()) chunks.push_back((int)npairs);
  double *X = nullptr, *Y = nullptr, *Z = nullptr;
  AZ_TRY(P.alloc((void**)&X, sizeof(double) * P.N * nvec));
  AZ_TRY(P.alloc((void**)&Y, sizeof(double) * P.Mt * nvec));
  AZ_TRY(P.alloc((void**)&Z, sizeof(double) * P.N * nvec));
  int rc = dense_gaussian(0x5eed, P.N, nvec, X, P.N, st);
  Shape cur{P.tune_C, P.tune_L, P.tune_chunk};
  std::string log = "[";
  float best = 1e30f;
  auto trial = [&](Shape s, float* ms) -> int {
    P.tune_C = s.C;
    P.tune_L = s.L;
    P.tune_chunk = s.chunk;
    int r = time_ops(P, X, Y, Z, nvec, st, 3, ms);
    char b[128];
    snprintf(b, sizeof(b), "%s{\"C\": %d, \"L\": %d, \"chunk\": %d, \"ms\": %.4f}", log.size() > 1 ? ", " : "", s.C,
             s.L, s.chunk, r == AZRBF_OK ? *ms : -1.0f);
    log += b;
    return r;
  };
  if (!rc) rc = trial(cur, &best);
  for (int dim = 0; dim < 3 && rc == AZRBF_OK; ++dim) {
    const std::vector<int>& cand = dim == 0 ? Cs : (dim == 1 ? Ls : chunks);
    for (int v : cand) {
      Shape s = cur;
      (dim == 0 ? s.C : (dim == 1 ? s.L : s.chunk)) = v;
      float ms = 0.f;
      rc = trial(s, &ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        cur = s;
      }
    }
  }
  log += "]";
  P.tune_C = cur.C;
  P.tune_L = cur.L;
  P.tune_chunk = cur.chunk;
  (void)hipStreamSynchronize(st);
  P.release_one(X);
  P.release_one(Y);
  P.release_one(Z);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[engine_key(P)] = cur;
  }
  char b[256];
  snprintf(b, sizeof(b), "{\"engine\": true, \"key\": \"%s\", \"nvec\": %lld, \"C\": %d, \"L\": %d, \"chunk\": %d, "
           "\"ms\": %.4f, \"trials\": ",
           engine_key(P).c_str(), (long long)nvec, cur.C, cur.L, cur.chunk, best);
  *report = std::string(b) + log + "}";
  return AZRBF_OK;
}

int tune_tsqr(Plan& P, int k, hipStream_t st, std::string* report) {
  *report = "";
  if (k != 16 && k != 32 && k != 64) return AZRBF_OK;
  const int64_t m = P.Mt;
  double *W0 = nullptr, *W = nullptr, *Q = nullptr, *R = nullptr, *scr = nullptr;
  AZ_TRY(P.alloc((void**)&W0, sizeof(double) * m * k));
  AZ_TRY(P.alloc((void**)&W, sizeof(double) * m * k));
  AZ_TRY(P.alloc((void**)&Q, sizeof(double) * m * k));
  AZ_TRY(P.alloc((void**)&R, sizeof(double) * k * k));
  AZ_TRY(P.alloc((void**)&scr, sizeof(double) * tsqr_scratch(m, k)));
  int rc = dense_gaussian(0x75a1, m, k, W0, m, st);
  hipEvent_t a = nullptr, b = nullptr;
  if (!rc && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)) rc = AZRBF_EHIP;
  int best_rb = 0;
  float best = 1e30f;
  std::string log = "[";
  for (int rb = 256; rb <= 2048 && !rc; rb *= 2) {
    if (!tsqr_rows_ok(k, rb)) continue;
    float t_best = 1e30f;
    for (int rep = 0; rep < 4 && !rc; ++rep) {   // the first run warms the kernels up
      if (hipMemcpyAsync(W, W0, sizeof(double) * m * k, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipEventRecord(a, st) != hipSuccess) {
        rc = AZRBF_EHIP;
        break;
      }
      rc = tsqr_panel(W, m, k, rb, scr, Q, R, st);
      if (!rc && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess)) rc = AZRBF_EHIP;
      float ms = 0.f;
      if (!rc && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = AZRBF_EHIP;
      if (!rc && rep > 0 && ms < t_best) t_best = ms;
    }
    if (rc) break;
    char e[96];
    snprintf(e, sizeof(e), "%s{\"rows\": %d, \"ms\": %.4f}", log.size() > 1 ? ", " : "", rb, t_best);
    log += e;
    if (t_best < best) {
      best = t_best;
      best_rb = rb;
    }
  }
  log += "]";
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(st);
  for (double* p : {W0, W, Q, R, scr}) P.release_one(p);
  if (rc) return rc;
  P.tsqr_rb[tsqr_slot(k)] = best_rb;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tsqr_key(k, m)] = Shape{best_rb, 0, 0};
  }
  char h[160];
  snprintf(h, sizeof(h), "{\"key\": \"%s\", \"rows\": %d, \"ms\": %.4f, \"trials\": ", tsqr_key(k, m).c_str(),
           best_rb, best);
  *report = std::string(h) + log + "}";
  return AZRBF_OK;
}

int tune_table(std::string* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string s;
  for (const auto& kv : g_tune) {
    char b[160];
    snprintf(b, sizeof(b), "%s %d %d %d\n", kv.first.c_str(), kv.second.C, kv.second.L, kv.second.chunk);
    s += b;
  }
  *out = s;
  return AZRBF_OK;
}

int tune_load(const char* text) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const char* p = text;
  while (p && *p) {
    char key[96];
    int C = 0, L = 0, ch = 0, n = 0;
    if (sscanf(p, "%95s %d %d %d%n", key, &C, &L, &ch, &n) != 4) return AZRBF_EINVAL;
    int dim = 0, N1 = 0, N2 = 0, s = 0;
    if (key[0] == 't') {   // TSQR tile: t<k>_<rows> <RB> 0 0
      int k = 0;
      long long m = 0;
      char tail = 0;
      if (sscanf(key, "t%d_%lld%c", &k, &m, &tail) != 2 || m < 1 || !tsqr_rows_ok(k, C) || L != 0 || ch != 0)
        return AZRBF_EINVAL;
      g_tune[key] = Shape{C, 0, 0};
    } else {
      // engine shapes: rows up to 512; columns up to 512, or up to 2048 beside
      // 512-long rows (1D transforms of 2^19 and 2^20)
      if (sscanf(key, "e%d_%dx%d_s%d", &dim, &N1, &N2, &s) != 4 || N1 < 16 || N2 < 16 || N2 > 512 ||
          N1 > (dim == 1 && N2 == 512 ? 2048 : 512) || (N1 & (N1 - 1)) || (N2 & (N2 - 1)))
        return AZRBF_EINVAL;
      if (!engine_shape_ok(N1, N2, C, L, ch)) return AZRBF_EINVAL;
      g_tune[key] = Shape{C, L, ch};
    }
    p += n;
    while (*p == '\n' || *p == ' ' || *p == '\t' || *p == '\r') ++p;
  }
  return AZRBF_OK;
}

}  // namespace az
