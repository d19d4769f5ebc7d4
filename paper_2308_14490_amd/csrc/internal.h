// Internal declarations shared by the azrbf translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <functional>
#include <vector>

#include "../../include/azrbf.h"

namespace az {

#define AZ_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return AZRBF_EHIP;           \
  } while (0)

#define AZ_TRY(call)                                   \
  do {                                                 \
    int rc_ = (call);                                  \
    if (rc_ != AZRBF_OK) return rc_;                   \
  } while (0)

// Geometry and spectra of the operator as seen by the FFT kernels.
//
// Coefficients are an N1 x N2 row-major array (index a*N2 + b):
//   1D, N > 8192: the four-step split n = b + N2*a (a column index, b row
//                 element); spectra stored in transposed order k1*N2 + k2
//                 for frequency k1 + N1*k2;
//   2D:           a = jx, b = jy, N1 = N2 = n.
// Phase ph in [0, s^dim) is a shifted grid: 1D r = ph; 2D (rx, ry) =
// (ph / s, ph % s).  Coefficient (a, b) of phase ph sits at fine-grid point
//   1D: s*(a*N2 + b) + ph;   2D: (s*a + rx)*L + s*b + ry.
struct Geo {
  int dim, s, N1, N2, L;
  int64_t N;                 // N1*N2
  int64_t M;                 // collocation rows
  int64_t i0;                // 1D: fine-grid index of collocation row 0
  const int32_t* inv;        // 2D: fine-grid point -> collocation row or -1
  // 1D spectra, [phase][N], frequency layout as above, 1/N folded in:
  const double2* spA;        // d_r / N
  const double2* spZ;        // w * conj(d_r) / N
  // 2D: per-axis factors fac[deriv 0|1][phase][N1] (x) and facy[deriv
  // 0|1][phase][N2] (y) (unnormalised DFTs of the kernel and of its second
  // derivative on the shifted 1D grids of each axis), and the regularised
  // weights w2 = 1/(N D) on the N1 x N2 frequency grid.
  const double2* fac;
  const double2* facy;
  const double* w2;
  int op;                    // AZRBF_OP_*
  double k2, opscale;        // BVP: spectrum = opscale*(d2 d0 + d0 d2 + k2 d0 d0)
};

// One operand block of a grouped operator launch (1D plans on the
// single-kernel transform): out = alpha * op(in) + beta * yin, column-major
// blocks of nvec vectors, op = A (in: coefficients, out: collocation rows) or
// Z* (the reverse).  nvec = 0 leaves the entry out of the launch.
struct BatOp {
  Geo g;
  const double2* tw;
  const double* in;
  int64_t ldin, nvec;
  double alpha, beta;
  const double* yin;
  int64_t ldyi;
  double* out;
  int64_t ldo;
};

struct Plan;

// Per-launch timing (plan.hip).  When enabled, a Prof object brackets the
// kernel launches of its scope with HIP events on its stream and records the
// algorithmic bytes the launches must move (what they read and write at
// minimum).  A scope that launches exactly one kernel is timed by events that
// the kernel's own dispatch packet records (hipExtLaunchKernel), which is the
// kernel's execution time alone, as a kernel trace measures it; a scope with
// several launches is timed by the marker events around it.
bool prof_enabled();
int prof_begin(hipStream_t st);
void prof_end(int slot, const char* name, double bytes, double flops, hipStream_t st);
// Make `slot` the scope that this thread's next launches belong to; returns
// the scope it replaces.
int prof_enter(int slot);
// For a launch inside the current scope: the start and stop events for the
// kernel's dispatch packet if it is the scope's first launch, else false.
bool prof_kernel_events(hipEvent_t* start, hipEvent_t* stop);
struct Prof {
  int slot, prev;
  const char* name;
  double bytes, flops;
  hipStream_t st;
  Prof(const char* n, double b, hipStream_t s, double f = 0.0)
      : slot(-1), prev(-1), name(n), bytes(b), flops(f), st(s) {
    if (prof_enabled()) {
      slot = prof_begin(st);
      if (slot >= 0) prev = prof_enter(slot);
    }
  }
  ~Prof() {
    if (slot >= 0) {
      prof_enter(prev);
      prof_end(slot, name, bytes, flops, st);
    }
  }
};

// Every kernel of the library is launched through this, so that a timed scope
// knows how many kernels it holds.
template <typename K, typename... A>
inline void launch_kernel(K kern, dim3 grid, dim3 block, uint32_t lds, hipStream_t st, A... args) {
  hipEvent_t e0, e1;
  if (prof_enabled() && prof_kernel_events(&e0, &e1))
    hipExtLaunchKernelGGL(kern, grid, block, lds, st, e0, e1, 0, args...);
  else
    kern<<<grid, block, lds, st>>>(args...);
}

int pool_trim();
// a library stream for work that overlaps other work (plan.hip)
int side_stream(int device, hipStream_t* out);

// ops.hip
int ops_init_twiddles(int device, const double2** tw);
bool engine_shape_ok(int N1, int N2, int C, int Lr, int chunk);
int ops_spectra(Plan& P, hipStream_t st);
// Host copies of the spectral norms (synchronises the stream once per plan).
int ops_norms(Plan& P, hipStream_t st);
// Work on a stream other than the plan's own first waits for its set-up
// (and for a factor queued on another stream).
int plan_on_stream(Plan& P, hipStream_t st);
// One launch of op (0: A, 1: Z*) over count device-resident operand blocks of
// the size class (n, s); maxvec bounds their nvec.  bytes: the launch's
// algorithmic traffic (for per-launch timing).
int ops_batched(int which, int n, int s, const BatOp* ops, int count, int64_t maxvec, double bytes, hipStream_t st);
// Marks the end of set-up or factor work queued on st.
int plan_mark_ready(Plan& P, hipStream_t st);
// Reads back rank and sweeps of a factor queued without waiting.
int plan_fetch_rank(Plan& P);
// Y = alpha A X + beta Yin (Yin null: Yin = Y); Z = alpha Z* R + beta Zin likewise.
int ops_apply_A(Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st);
int ops_apply_Z(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                const double* Zin, int64_t ldzi, double* Z, int64_t ldz, hipStream_t st);
// Right-hand sides from interior data f (M x nrhs) and boundary data g (Mb x nrhs).
int ops_rhs(const Plan& P, const double* f, int64_t ldf, const double* g, int64_t ldg, int64_t nrhs, double* B,
            int64_t ldb, hipStream_t st);
// generic.hip: the operators for centre counts that are not powers of two
// (n = 2^a 3^b 5^c 7^d), by mixed-radix FFTs in global memory.
// (n = 2^a 3^b 5^c 7^d: mixed-radix passes; other n: Bluestein's chirp
// convolution through power-of-two passes)
bool gfft_supported(int64_t n);
int64_t gen_ws_bytes(int64_t N1, int64_t N2, int64_t npairs);
// Bluestein tables for the plan's axes that need them (before any transform).
int gen_tables(Plan& P, hipStream_t st);
// Forward DFTs of `lines` contiguous n-point lines, in -> out.
int gfft_lines_fwd(Plan& P, const double2* in, double2* out, int n, int64_t lines, hipStream_t st);
int gen_apply_A(Plan& P, const double* X, int64_t ldx, int64_t nvec, double alpha, double beta,
                const double* Yin, int64_t ldyi, double* Y, int64_t ldy, hipStream_t st);
int gen_apply_Z(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta, const double* Zin,
                int64_t ldzi, double* Z, int64_t ldz, hipStream_t st);
// Out = alpha A Z* R + beta Yin (Yin null: Yin = Out); Zs is N x nvec scratch
// (leading dimension N), overwritten with Z* R when the plan needs it.
int ops_apply_AZ(Plan& P, const double* R, int64_t ldr, int64_t nvec, double alpha, double beta,
                 const double* Yin, int64_t ldyi, double* Out, int64_t ldo, double* Zs, hipStream_t st);

// tsqr.hip: Householder QR of the RB-row blocks of A (m x k, k in {16, 32,
// 64}, RB = tsqr_block_rows(k)); R factors stacked at rows b*k of R, the
// reflectors over A's rows into V (may equal A), compact-WY T factors at
// T + b*k*k.
// RB: rows per block, the tile shape (tsqr_block_rows(k) by default; the
// autotuner picks among those tsqr_rows_ok accepts).
int tsqr_block_rows(int k);
bool tsqr_rows_ok(int k, int rb);
int tsqr_block_qr(const double* A, int64_t lda, int64_t m, int k, int rb, double* R, int64_t ldr, double* V,
                  int64_t ldv, double* T, hipStream_t st);

// gemm.hip: C = alpha op(A) op(B) + beta C on the FP64 matrix cores, batch
// entries at strides sA, sB, sC.  Long reductions with few output tiles are
// split over blocks when part holds gemm_split_doubles(...) doubles.
int64_t gemm_split_doubles(int64_t M, int64_t N, int64_t K, int64_t batch);
int gemm_mfma(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C, int64_t ldc,
              int64_t sC, int64_t batch, double* part, int64_t part_doubles, hipStream_t st);
// the same with a separate input Cin (C = alpha op(A) op(B) + beta Cin; Cin may be C)
int gemm_mfma_c(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, const double* Cin, int64_t ldci,
                int64_t sCi, double* C, int64_t ldc, int64_t sC, int64_t batch, double* part, int64_t part_doubles,
                hipStream_t st);

// dense.hip
int dense_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* dst, int64_t ld, hipStream_t st);
// Householder TSQR of W (m x k, ld m, destroyed): Q (m x k, ld m), R (k x k, ld k)
int64_t tsqr_scratch(int64_t m, int k);
int tsqr_panel(double* W, int64_t m, int k, int rb, double* scratch, double* Q, double* R, hipStream_t st);
// The plan's TSQR tile (rows per block) for width k: the tuned one for
// (k, Mt), else the default.
int plan_tsqr_rows(const Plan& P, int k);
// Time the TSQR (block QR tree and Q formation) of an m x k matrix for every
// tile shape and keep the fastest (tune.hip).
int tune_tsqr(Plan& P, int k, hipStream_t st, std::string* report);
// relres[c] = ||R(:, c)|| / ||B(:, c)|| over m rows; nrm holds 2 relres_chunks() x ncol
int relres_chunks();
int relres_norms(const double* R, int64_t ldr, const double* B, int64_t ldb, int64_t m, int64_t ncol,
                 double* nrm, double* out, hipStream_t st);

// tune.hip: engine tile shapes (table keyed by the engine shape)
void tune_apply(Plan& P);
int tune_plan(Plan& P, int64_t nvec, hipStream_t st, std::string* report);
int tune_table(std::string* out);
int tune_load(const char* text);

// wide.hip: sketch widths k > 64 (multiples of 64)
int64_t wide_factor_doubles(int64_t N, int64_t Mt, int k);
int wide_factor(Plan& P, hipStream_t st);
int wide_solve(Plan& P, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx, double* relres,
               hipStream_t st);
int dense_factor(Plan& P, hipStream_t st);
// the factor split in two: queue it and wait for it / read the rank.  While
// queuing, after_sketch (if set) is recorded once the sketch W is queued and
// then on_sketch (if set) runs on the host; before_products (if set) runs
// once the explicit Q is queued, before the stream waits for the Jacobi SVD
// (work that needs Q but not P can be queued there, beside the SVD).
int dense_factor_enqueue(Plan& P, hipStream_t st, hipEvent_t after_sketch,
                         const std::function<int()>& on_sketch = nullptr,
                         const std::function<int()>& before_products = nullptr);
int dense_factor_finish(Plan& P, hipStream_t st);
int dense_solve_ws(Plan& P, int64_t nrhs, hipStream_t st);
int dense_first_stage(Plan& P, const double* B, int64_t ldb, int64_t nrhs, hipStream_t st);
// t = Q^T c of the first pass (c from dense_first_stage) into the solve workspace
int dense_first_qtc(Plan& P, int64_t nrhs, hipStream_t st);
// first_done: the first pass's c = (I - A Z*) b is already in the workspace;
// qtc_done: so is its Q^T c
int dense_solve(Plan& P, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                double* relres, hipStream_t st, bool first_done = false, bool qtc_done = false);

// One block-QR level of one plan in a grouped launch (the arguments of
// tsqr_block_qr): rows m of A (ld lda) in blocks of rb, R (ld ldr), the
// reflectors over V (ld ldv), the compact-WY factors at T.
struct TsqrOp {
  const double* A;
  int64_t lda, m;
  double* R;
  int64_t ldr;
  double* V;
  int64_t ldv;
  double* T;
};
// One launch over count device-resident levels of plans with the same k and
// row blocking rb; maxnb bounds their block counts (tsqr.hip).
int tsqr_block_qr_batched(int k, int rb, const TsqrOp* ops, int count, int64_t maxnb, hipStream_t st);
// Grouped factorisation of unfactored 1D plans on the single-kernel
// transform (batched_eligible once factored); rcs[i]: the plan's code (OK or
// ERANK: retained rank above 90 % of the width).  Synchronises st.
int dense_factor_batched(const std::vector<Plan*>& plans, std::vector<int>& rcs, hipStream_t st);
bool dense_factor_batchable(const Plan& P);

// batched.hip: the grouped solve of many factored 1D plans (one entry per
// block of right-hand sides; a plan may appear in several entries).
struct BatchItem {
  Plan* P;
  const double* B;
  int64_t ldb, nrhs;
  double* X;
  int64_t ldx;
  double* relres;
};
bool batched_eligible(const Plan& P);
int batched_solve(const std::vector<BatchItem>& items, hipStream_t st);
// Frees the grouped solve's staging buffers once their last calls are done.
int batched_release();

struct Plan {
  azrbf_problem prob{};
  int device = 0;
  int dim = 1, n = 0, s = 1, ph = 1;     // ph = s^dim phases; n, T, h, hL: x axis
  int ny = 0;                             // 2D: centres along y
  double T = 1, eps = 0, h = 0, hL = 0;
  double Ty = 1, hy = 0, hLy = 0;         // 2D: y axis
  int64_t N = 0, Lax = 0, Lg = 0, M = 0, Mb = 0, Mt = 0;
  int64_t Lay = 0;                        // 2D: fine-grid points along y
  int64_t Mtp = 0;   // Mt rounded up to 16: leading dimension of internal row-space matrices
  int64_t ldq = 0;   // leading dimension of the factor's Q
  bool fused = false;                     // 1D single-kernel path
  bool generic = false;                   // a centre count is not a power of two: mixed-radix path
  Geo geo{};
  const double2* tw = nullptr;            // shared twiddle table (per device)

  hipStream_t last_stream = nullptr;      // stream of the plan's latest work
  hipStream_t make_stream = nullptr;      // stream the plan was made on
  hipEvent_t ready = nullptr;             // recorded after the latest set-up or factor work
  hipStream_t ready_stream = nullptr;     // ... on this stream

  // device memory owned by the plan (pointer, pool size class)
  std::vector<std::pair<void*, int64_t>> allocs;
  int64_t bytes = 0;
  int32_t* inv = nullptr;
  double2* spA = nullptr;
  double2* spZ = nullptr;
  double2* fac = nullptr;
  double2* facy = nullptr;                // 2D: y-axis factors (fac itself on a square box)
  double* w2 = nullptr;
  double* bpts = nullptr;                 // Mb x dim, device
  uint8_t* btype = nullptr;               // Mb, device: 1 at Neumann points (null: all Dirichlet)
  double* bnorm = nullptr;                // Mb x dim, device: unit outward normals (with btype)
  double bweight = 1;
  double normA = 0, normZ = 0;   // sqrt(max D), sqrt(max w); valid once ops_norms ran
  int zeroed = 0;
  double* dred = nullptr;          // device: max D, max w, dropped count
  bool norms_pending = false;

  // engine tile shapes (0: defaults): columns per block of the column
  // passes, rows per block of the row passes, vector pairs per chunk
  int tune_C = 0, tune_L = 0, tune_chunk = 0;
  // TSQR tile shapes (rows per block) for widths 16, 32, 64 (0: default)
  int tsqr_rb[3] = {0, 0, 0};

  // FFT-engine workspace, and a second set for work queued on a side stream
  double2* ws1 = nullptr;
  double2* ws2 = nullptr;
  int64_t ws_pairs = 0;
  double2* wsB1 = nullptr;
  double2* wsB2 = nullptr;
  int64_t wsB_pairs = 0;
  // Bluestein tables of an axis whose centre count has a prime factor above
  // 7 (mixed-radix path): M-point DFTs of the chirp filters of the forward
  // and inverse n-point transforms, M = the power of two >= 2n - 1
  struct BlueAxis {
    int n = 0, M = 0;
    double2* hf = nullptr;
    double2* hi = nullptr;
  };
  BlueAxis blue[2];
  // workspace of the mixed-radix path (three N-point buffers per pair, and
  // the Bluestein convolutions' buffers), and its second set
  double2* gws = nullptr;
  int64_t gws_pairs = 0;
  double2* gwsB = nullptr;
  int64_t gwsB_pairs = 0;
  void swap_ws() {
    std::swap(ws1, wsB1);
    std::swap(ws2, wsB2);
    std::swap(ws_pairs, wsB_pairs);
    std::swap(gws, gwsB);
    std::swap(gws_pairs, gwsB_pairs);
  }

  // factor
  int k = 0, rank = -1, refine = 0;
  double tau = 1e-12, tauZ = 1e-12;
  bool factored = false;
  int sweeps = 0;            // Jacobi sweeps of the last factor
  int hinfo[2] = {0, 0};     // rank and sweeps, copied back by the factor
  int* dinfo = nullptr;      // their device copy
  bool rank_pending = false; // the factor is queued; rank and sweeps not read back yet
  hipStream_t factor_stream = nullptr;
  double* Om = nullptr;     // N x k, then Omega * P
  double* Om2 = nullptr;    // N x k scratch
  double* Yf = nullptr;     // Mt x k, A Omega, then (A Omega) * P
  double* Yf2 = nullptr;    // Mt x k scratch (the sketch W)
  double* Q = nullptr;      // Mt x k
  double* Rf = nullptr;     // k x k
  double* sig = nullptr;    // k
  double* Pm = nullptr;     // k x k = V_r S_r^-1 U_r^T
  double* Gj = nullptr;     // k x k: R^T, rotated by the wide Jacobi (k > 64)
  double* Vj = nullptr;     // k x k: accumulated Jacobi rotations (k > 64)
  double* dscr = nullptr;   // dense scratch
  int64_t dscr_bytes = 0;

  // solve workspace
  double* sw = nullptr;
  int64_t sw_rhs = 0, sw_part = 0;
  // coefficient scratch of azrbf_apply_AZstar (N x azs_cols)
  double* azs = nullptr;
  int64_t azs_cols = 0;

  int alloc(void** p, int64_t bytes);
  void release();
  // Blocks back to the pool once the work queued on st so far has run (an
  // event guards them; plans on the same stream may take them at once).
  void release_after(hipStream_t st);
  void release_one(void* p);   // one block back to the pool
  void release_factor();       // the factor and solve workspace back to the pool
  void release_one_after(void* ptr, hipStream_t st);   // a replaced block, once st's work is done
};

}  // namespace az
