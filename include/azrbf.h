/*
 * azrbf — AZ least-squares solver for periodized Gaussian RBF approximation
 * and oversampled collocation on MI355X (gfx950), FP64 throughout.
 *
 * The method (Zhou & Huybrechs, "Efficient least squares approximation and
 * collocation methods using radial basis functions"):
 *   - N Gaussian RBFs phi(r) = exp(-eps^2 r^2) (eq. rbf), periodized with
 *     period 2T (eq. periodic_rbf), centred on a regular grid of the box
 *     [-T, T)^dim (eq. set_centers), n centres per axis, N = n^dim;
 *   - collocation points: the points of an s-times finer grid (eq. set_Xtilde,
 *     L = s n per axis) that lie in the domain (eq. set_X, eq. set_X_2d);
 *   - for boundary value problems, interior rows apply -(Laplacian + k2) to
 *     the basis (divided by 2 eps^2 in 1D, 4 eps^2 in 2D) and boundary rows
 *     evaluate the basis at boundary points with weight bweight (section 6);
 *   - the rectangular system A x = b is solved in the least-squares sense by
 *     the AZ algorithm (Algorithm 1) with Z* = F B^+ P E (section 3.2.2): a
 *     randomized low-rank solve of (A - A Z* A) x1 = (I - A Z*) b followed by
 *     x2 = Z* (b - A x1), x = x1 + x2.
 *
 * Conventions
 *   - Every function returns 0 on success or a negative AZRBF_E* code;
 *     nothing is thrown across this interface.
 *   - Matrices of vectors are column-major FP64 with a leading dimension:
 *     element (i, v) of X is X[i + ld * v].  Such pointers are DEVICE
 *     pointers owned by the caller and must not alias one another.
 *   - Coefficient vectors have N entries; in 2D entry jx * ny + jy belongs
 *     to the centre (jx, jy) (x slow, y fast; section 5.1).
 *   - Row vectors have M + Mb entries: the M collocation points in ascending
 *     fine-grid order (index ix * Ly + iy in 2D, Ly = s ny), then the Mb
 *     boundary points in the order given.
 *   - Work is queued on the given HIP stream (hipStream_t passed as void*;
 *     NULL is the default stream) and returns without synchronising, except
 *     where stated.  A plan owns its device memory.  A plan may be used from
 *     one stream at a time; calls on different streams must be ordered by the
 *     caller.  Different plans are independent.
 */
#ifndef AZRBF_H
#define AZRBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AZRBF_OK = 0,
  AZRBF_EINVAL = -1,        /* bad argument: sizes, pointers, empty domain   */
  AZRBF_EUNSUPPORTED = -2,  /* valid but not implemented (e.g. n not 2^k)    */
  AZRBF_ENOMEM = -3,        /* device allocation failed                      */
  AZRBF_EHIP = -4,          /* a HIP runtime call failed                     */
  AZRBF_ERANK = -5,         /* sketch too narrow: >90% of it retained        */
  AZRBF_ESTATE = -6,        /* call not valid in the plan's current state    */
  AZRBF_ESCRATCH = -7       /* request exceeds a fixed scratch buffer         */
};

enum {
  AZRBF_OP_APPROX = 0,      /* rows phi_j(x_i)                                */
  AZRBF_OP_BVP = 1          /* rows -(Lap + k2) phi_j(x_i)/(2 dim eps^2) and */
                            /* weighted Dirichlet rows at boundary points     */
};

typedef struct azrbf_plan_s* azrbf_plan_t;

/* Problem description (section 2.2 / 5.1 / 6).  All pointers are HOST
 * pointers, read during azrbf_plan only.  In 2D the box may be anisotropic
 * (section 5.1: its own centre count and half-width per axis, fields ny, Ty);
 * the Gaussian is radial, so eps is one value (with eps <= 0 it follows
 * eq. constant_shapeparam on the x axis). */
typedef struct {
  int32_t dim;            /* 1 or 2                                          */
  int32_t n;              /* centres per axis: a power of two, 16 <= n,      */
                          /* n <= 2^20 (1D; s <= 2 above 2^19), n <= 512     */
                          /* (2D)                                             */
  int32_t s;              /* oversampling factor per axis: 1, 2, 3 or 4      */
  double T;               /* half-width of the periodic box [-T, T)^dim      */
  double eps;             /* shape parameter; if <= 0 it follows             */
                          /* eq. constant_shapeparam from tau0               */
  double tau0;            /* used only when eps <= 0                         */
  int32_t op;             /* AZRBF_OP_*                                      */
  double k2;              /* k^2 of -(Lap + k2) for AZRBF_OP_BVP             */
  const uint8_t* mask;    /* L (1D) or Lx * Ly bytes (L = s n), nonzero     */
                          /* marks a collocation point; 2D index ix * Ly + iy */
  int64_t nb;             /* number of boundary points (BVP only)            */
  const double* bpts;     /* nb x dim coordinates, point i at bpts[i*dim+a]  */
  double bweight;         /* weight of the boundary rows                     */
  double tau;             /* step-1 truncation, relative (e.g. 1e-12)        */
  double tauZ;            /* Z* regularisation: weights whose denominator    */
                          /* is <= tauZ * max are zero (e.g. 1e-12)          */
  int32_t k;              /* sketch width; 0 = estimate from n               */
  int32_t refine;         /* extra AZ passes on the residual (0, 1, ...)     */
  uint64_t seed;          /* seed of the Gaussian sketch                     */
  int32_t ny;             /* 2D: centres along y (a power of two, 16..512);  */
                          /* 0 = n.  n and T above are then the x axis       */
  double Ty;              /* 2D: half-width of the box along y; 0 = T        */
  const uint8_t* btype;   /* nb entries or NULL (all Dirichlet): 0 marks a   */
                          /* Dirichlet point (row bweight phi_j(x_b)), 1 a   */
                          /* Neumann point (section 6.3: row bweight         */
                          /* n . grad phi_j(x_b) / eps, the 1/eps making its */
                          /* size match the Dirichlet rows)                  */
  const double* bnormal;  /* nb x dim unit outward normals n (read at        */
                          /* Neumann points; may be NULL when there are      */
                          /* none), point i at bnormal[i*dim+a]              */
} azrbf_problem;

/* Read-only facts about a plan. */
typedef struct {
  int64_t N, M, Mb, L;    /* unknowns, collocation rows, boundary rows,     */
                          /* fine-grid points (L^dim)                        */
  int32_t k;              /* sketch width                                    */
  int32_t rank;           /* retained rank after factoring (-1 before)       */
  double eps;             /* shape parameter in use                          */
  double normA;           /* ||A^c||_2 of the periodic operator              */
  double normZ;           /* ||Z*||_2 (largest regularised weight, sqrt)     */
  int32_t zeroed;         /* number of regularised (zeroed) weights          */
  int32_t factored;       /* 1 once the low-rank factor is resident          */
  int32_t sweeps;         /* Jacobi sweeps of the last factorisation         */
  int64_t device_bytes;   /* device memory currently owned by the plan       */
} azrbf_info;

/* Step 0 of section 3.2.3: collocation index list, spectra of B (Lemma 4.2:
 * DFTs of the kernel sampled on the s^dim shifted grids) and the regularised
 * weights of B^+ (eq. B_pinv; eq. B_pinv_2d; section 6.2 for BVPs).  The
 * spectra are computed on the device, queued on `stream` (1D: without
 * waiting for them; work later passed another stream first waits for them).
 * On success *out owns the plan.
 * Errors: EINVAL (bad sizes, empty mask, nb > 0 without op BVP, a Neumann
 * point without a unit normal, ...),
 * EUNSUPPORTED (n not a power of two or out of range, s not in {1,2,3,4}),
 * ENOMEM, EHIP. */
int azrbf_plan(const azrbf_problem* prob, void* stream, azrbf_plan_t* out);

/* The facts above.  normA, normZ and zeroed (computed on the device when
 * the plan is made) and rank and sweeps (of a factor queued by azrbf_solve)
 * are read back on first request, which waits for that work. */
int azrbf_plan_info(azrbf_plan_t plan, azrbf_info* info);

/* dims[0..4] = N, M, Mb, L (fine-grid points), k (current sketch width):
 * sizes known on the host, no waiting. */
int azrbf_plan_dims(azrbf_plan_t plan, int64_t* dims);

/* Y = alpha * A X + beta * Y for nvec vectors (eq. Ax_is_b, eq. Aa_is_b_2d):
 * X is N x nvec (ldx >= N), Y is (M + Mb) x nvec (ldy >= M + Mb).  A is
 * applied as R Pi^T P* B F* (section 3.2.2): FFTs of the coefficients,
 * multiplication by the spectra of the s^dim shifted grids, inverse FFTs,
 * restriction to the collocation points; boundary rows by direct summation.
 * With beta == 0, Y is not read. */
int azrbf_apply_A(azrbf_plan_t plan, const double* X, int64_t ldx, int64_t nvec,
                  double alpha, double beta, double* Y, int64_t ldy, void* stream);

/* Right-hand sides of the least-squares system from the problem's data
 * (section 2.3; for boundary value problems the section 6.1 example and
 * section 6.2): B[i, v] = c f[i, v] for the M collocation rows, where f holds
 * the data at the collocation points (the function to approximate, or the
 * source term of -(Lap + k2) u = f) and c = 1 for AZRBF_OP_APPROX, c =
 * 1 / (2 dim eps^2) for AZRBF_OP_BVP (the same normalisation as the interior
 * rows, so that the scaled equations keep their solution); B[M + j, v] =
 * bweight g[j, v] for the Mb boundary rows at Dirichlet points (g the values
 * of u) and bweight g[j, v] / eps at Neumann points (g the normal derivative
 * of u, scaled as the Neumann rows).  Device
 * pointers: f is M x nrhs (ldf >= M), g is Mb x nrhs (ldg >= Mb; unread and
 * may be NULL when Mb = 0), B is (M + Mb) x nrhs (ldb >= M + Mb).  B may be f
 * itself (same leading dimension) but must not otherwise overlap f or g.
 * Stream-ordered, no synchronisation.  Errors: EINVAL. */
int azrbf_rhs(azrbf_plan_t plan, const double* f, int64_t ldf, const double* g, int64_t ldg,
              int64_t nrhs, double* B, int64_t ldb, void* stream);

/* Z = alpha * Z* R + beta * Z with Z* = F B^+ P E (section 3.2.2); rows
 * M..M+Mb-1 of R (boundary rows) are ignored: Z* has zero columns there
 * (section 6.1.2).  R is (M + Mb) x nvec, Z is N x nvec. */
int azrbf_apply_Zstar(azrbf_plan_t plan, const double* R, int64_t ldr, int64_t nvec,
                      double alpha, double beta, double* Z, int64_t ldz, void* stream);

/* Y = alpha * A Z* R + beta * Y: the product of the two operators above, as
 * in the right-hand side (I - A Z*) b of step 1 of Algorithm 1.  Between
 * the two operators the product stays in the spectrum (one row pass does Z*'s
 * combination of the phases and A's per-phase products; Z*'s inverse and
 * A's forward transforms cancel), so it costs about half of the two calls.
 * R and Y are (M + Mb) x nvec; R may equal Y (same leading dimension); rows
 * M..M+Mb-1 of R are ignored as in azrbf_apply_Zstar.  With boundary rows or
 * on the single-kernel 1D path the plan keeps an N x nvec coefficient scratch
 * (grown on demand; the replaced one returns to the library's pool once the
 * work queued before it on the stream has run). */
int azrbf_apply_AZstar(azrbf_plan_t plan, const double* R, int64_t ldr, int64_t nvec,
                       double alpha, double beta, double* Y, int64_t ldy, void* stream);

/* Step 1 set-up (section 3.2.3, "low-rank solver"): the Gaussian sketch
 * Omega (N x k), W = (A - A Z* A) Omega, a Householder tall-skinny QR of W,
 * a one-sided Jacobi SVD of R and truncation at tau * normA * sqrt(k).  The
 * factor stays resident in the plan.  Synchronises the stream (the retained
 * rank is read back).  A sketch that retains more than 90 % of its k
 * directions is too narrow to resolve them all; with the width left open
 * (problem k = 0) the factorisation then widens it to 1.25 times the
 * retained rank and starts again (up to three times), else it returns ERANK
 * (the factor is still usable, at reduced accuracy). */
int azrbf_factor(azrbf_plan_t plan, void* stream);

/* Least-squares solve of A X = B for nrhs right-hand sides (Algorithm 1 plus
 * `refine` refinement passes on the residual).  B is (M + Mb) x nrhs, X is
 * N x nrhs.  If relres is not NULL it is a device array of nrhs doubles that
 * receives ||B - A X|| / ||B|| per column.  Factors first if needed.  With a
 * fixed sketch width k <= 64 the call queues the factor and the solve and
 * returns without waiting (the retained rank is read by azrbf_plan_info);
 * otherwise (k left open, so that it may grow, or k > 64) the factor
 * synchronises the stream. */
int azrbf_solve(azrbf_plan_t plan, const double* B, int64_t ldb, int64_t nrhs,
                double* X, int64_t ldx, double* relres, void* stream);

/* Batched form of azrbf_solve (Algorithm 1) over nprob different plans,
 * e.g. problems of uneven sizes.  The plans' work runs concurrently on the
 * library's internal streams (up to four, worker threads enqueue it; plans
 * are assigned largest first to the least-loaded stream), factoring plans
 * that are not factored yet; the work of each plan is the same as in
 * azrbf_solve, so every result equals the one-plan call bit for bit.  The
 * caller's stream waits for all of it; the call returns once everything is
 * queued (a factorisation inside synchronises its internal stream).  Arrays
 * have length nprob; relres may be NULL, or hold NULL entries.  Many
 * right-hand sides of ONE plan belong in a single azrbf_solve call instead
 * (they share every launch).  Errors: EINVAL (a plan listed twice, plans of
 * another device, bad sizes), else the first failing plan's code. */
int azrbf_solve_many(int32_t nprob, const azrbf_plan_t* plans,
                     const double* const* B, const int64_t* ldb, const int64_t* nrhs,
                     double* const* X, const int64_t* ldx, double* const* relres,
                     void* stream);

/* Grouped form of azrbf_solve (Algorithm 1 and its refinement passes, the
 * solve phase of section 3.2.3) for many small problems of uneven sizes, on
 * the caller's stream.  Entries whose plan is 1D on the single-kernel
 * transform (n a power of two <= 8192, no boundary rows, sketch width <= 64)
 * share every launch: one pass over all of them is seven launches (the
 * transforms once per size class (n, s)), however many entries and sizes
 * there are, instead of about twenty per plan.  Other entries are solved one
 * after another as by azrbf_solve.  Plans that are not factored are factored
 * first: those that qualify together, with one launch per step for all of
 * them (the same kernels in the same order per plan as azrbf_factor, so the
 * same factor bit for bit; the call then waits for the factors to read their
 * ranks), the others one after another.  Arrays have length nprob; entry
 * i solves plans[i] for nrhs[i] right-hand sides B[i] ((M + Mb) x nrhs[i],
 * ld ldb[i], device) into X[i] (N x nrhs[i], ld ldx[i], device), with
 * relres[i] (device, nrhs[i] doubles) receiving ||B - A X|| / ||B|| per
 * column when relres and relres[i] are not NULL.  A plan may appear in
 * several entries (each has its own workspace; their X must not overlap).
 * The grouped dense products sum in another order than azrbf_solve's, so the
 * results agree with it to rounding, not bit for bit.  The library keeps
 * staging buffers per device (descriptors in pinned host memory, workspace in
 * device memory, reused once the previous call's work is done) and the call
 * returns once the work is queued; a plan must not be destroyed or factored
 * again while that work is queued.  Errors: EINVAL (bad sizes or pointers,
 * plans of another device, more than 65535 entries), EHIP, else the first
 * failing plan's code. */
int azrbf_solve_batched(int32_t nprob, const azrbf_plan_t* plans,
                        const double* const* B, const int64_t* ldb, const int64_t* nrhs,
                        double* const* X, const int64_t* ldx, double* const* relres,
                        void* stream);

/* Device bytes a plan for prob needs (plan + factor + workspace for up to
 * max_rhs right-hand sides per call); used for admission by memory. */
int64_t azrbf_footprint_bytes(const azrbf_problem* prob, int64_t max_rhs);

/* Copies a resident factor matrix to a caller buffer (device pointer):
 * which = 0: Omega (N x k), 1: Q (M+Mb x k), 2: R (k x k, upper),
 * 3: singular values of R (k x 1, descending). ld is the leading dimension
 * of dst. */
int azrbf_get_factor(azrbf_plan_t plan, int32_t which, double* dst, int64_t ld,
                     void* stream);

/* The Gaussian sketch definition used by azrbf_factor, for any size:
 * dst (rows x cols, leading dimension ld) gets entry (j, c) from Philox4x32-10
 * with counter (j / 4, c, 0, 0) and key (seed mod 2^32, seed / 2^32) and the
 * Box-Muller transform (rows 4q, 4q+1 from words 0, 1; rows 4q+2, 4q+3 from
 * words 2, 3; u = (word + 1/2) / 2^32). */
int azrbf_gaussian(uint64_t seed, int64_t rows, int64_t cols, double* dst, int64_t ld,
                   void* stream);

/* Utility: C = alpha op(A) op(B) + beta C in FP64 on the matrix cores (the
 * GEMM of the low-rank stage for wide sketches, section 3.2.3).  op(A) is
 * m x k, op(B) is k x n, C is m x n; all DEVICE pointers, column-major, with
 * leading dimensions lda >= rows of A as stored (m, or k if transa), likewise
 * ldb, and ldc >= m.  transa, transb: 0 = as stored, 1 = transposed.  With
 * beta == 0, C is not read.  Long reductions that are split over blocks use a
 * temporary buffer, and then the call synchronises the stream. */
int azrbf_dgemm(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                int64_t ldc, void* stream);

/* azrbf_dgemm without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, arithmetic and split of the reduction as
 * azrbf_dgemm (so the same result bit for bit), but the split-K partial tiles
 * live in a fixed device array of the library, 2^20 doubles (8 MiB) per GPU,
 * held from the first call on that GPU until the process ends; a product
 * whose split needs more returns AZRBF_ESCRATCH and computes nothing.  The
 * call is stream-ordered and does not synchronise.  The array belongs to the
 * current device (the stream must be one of its streams); every call on that
 * GPU shares it, so calls that may overlap on one GPU (different streams,
 * host threads) race and must be ordered by the caller. */
int azrbf_dgemm_noalloc(int32_t transa, int32_t transb, int64_t m, int64_t n, int64_t k, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                        int64_t ldc, void* stream);

/* Tile shapes of the FFT passes for transforms that need the three-pass
 * engine (1D N > 8192 and all 2D plans): times apply_A followed by
 * apply_Zstar on nvec vectors of the plan's own operator for candidate
 * shapes (columns per block of the column passes, rows per block of the row
 * passes, vector pairs per launch), keeps the fastest in the plan and in a
 * process-wide table from which later plans of the same engine shape start.
 * Then the TSQR tile of the low-rank stage (section 3.2.3): the rows one
 * block QR holds (256, 512, 1024 or 2048, as registers allow for the width),
 * timed on the whole TSQR of an (M + Mb) x k Gaussian matrix (k the sketch
 * width, or the 64-column panels of wider sketches), kept the same way.
 * Synchronises the stream.  report (len bytes, may be NULL) receives a JSON
 * object with the choices and every trial's time ({"engine": false} when the
 * plan uses the single-kernel path; "tsqr": the TSQR trials).  Errors:
 * EINVAL (nvec <= 0, report too small), ENOMEM, EHIP. */
int azrbf_autotune(azrbf_plan_t plan, int64_t nvec, void* stream, char* report, int64_t len);

/* The process-wide tile-shape table as text, one shape per line: engine
 * shapes "e<dim>_<N1>x<N2>_s<s> <C> <rows> <pairs>", TSQR tiles
 * "t<k>_<rows of the matrix> <rows per block> 0 0"; and loading such text (e.g. saved
 * from an earlier process).  Loading validates every line (EINVAL on a
 * malformed or out-of-range entry) and affects plans created afterwards. */
int azrbf_tune_table(char* buf, int64_t len);
int azrbf_tune_load(const char* text);

/* Per-launch timing for measurement.  While enabled, every kernel launch of
 * the library (any plan, any stream) is bracketed by HIP events on its
 * stream and tagged with the bytes it must move at minimum (its algorithmic
 * reads and writes).  azrbf_profile_report waits for the recorded events,
 * writes a JSON array of {"name", "calls", "ms", "max_ms", "bytes", "flops"}
 * totals per kernel name into buf (len bytes, NUL-terminated; EINVAL if too
 * small) and clears the records.  While enabled, work the library would
 * otherwise overlap on its side streams runs in order on the caller's stream,
 * so that each launch's time is its own. */
int azrbf_profile_enable(int32_t on);
int azrbf_profile_report(char* buf, int64_t len);

/* Releases a plan without waiting: its device blocks return to the library's
 * memory pool once the work queued on the plan's stream and latest stream has
 * run (later plans on that same stream may reuse them at once, being ordered
 * after it). */
void azrbf_destroy(azrbf_plan_t plan);

/* Frees the pool's cached device blocks (blocks owned by live plans stay)
 * and the grouped solve's staging buffers (after waiting for the calls that
 * use them). */
int azrbf_release_cached_memory(void);
const char* azrbf_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* AZRBF_H */
