// Low-rank stage for wide sketches (k > 64, a multiple of 64), the 2D and
// boundary-value regime where the rank of A - A Z* A grows with the grid
// (section 3.2.3, section 5.3.2):
//   1. W = (A - A Z* A) Omega with the FFT operators (k columns);
//   2. W = Q R by block classical Gram-Schmidt with reorthogonalisation over
//      64-column panels: each panel is projected twice against the
//      finished Q (matrix-core GEMMs) and factored by the Householder TSQR,
//      and the panel's Q is projected once more and factored again, which
//      keeps Q orthonormal to working precision also past the numerical rank;
//   3. the SVD of R, preconditioned: the same QR of R^T = Q2 R2, then block
//      one-sided Jacobi on G = R2^T with 32-column blocks: in each round the
//      disjoint block pairs form their 64 x 64 Gram matrices (matrix-core
//      products of the current columns), a two-sided Jacobi sweep
//      diagonalises each Gram with the relative off-diagonal test
//      |h_pq| <= tol sqrt(h_pp h_qq), and the rotation is applied to the
//      pair's columns of G and of W, which starts as Q2; converged when a
//      sweep needs no rotation.  Then G_final = U Sigma (columns
//      g_i = u_i sigma_i) and R = U Sigma W^T.
//   4. truncation at sigma > tau ||A^c|| sqrt(k) and
//      P = R^+ = W_r Sigma_r^-1 U_r^T = sum w_i g_i^T / sigma_i^2, so y = P Q^T c.
// The per-right-hand-side solve then runs Algorithm 1 with GEMMs for
// Q^T c, P t and Omega y and the FFT operators for A and Z*.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"

namespace az {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// 1/sqrt(x): hardware estimate and one Newton step.
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

namespace {

constexpr int PB = 64;    // QR panel width
constexpr int JB = 32;    // Jacobi column block; a pair is 64 columns
constexpr int JP = 64;    // columns of a pair
constexpr int JINNER = 2; // Jacobi sweeps on a pair's Gram per visit
constexpr int JMAX = 40;  // outer sweeps at most

// Round-robin tournament on n slots (n even): round r in [0, n-1), pair i in
// [0, n/2).  Over the n-1 rounds every two slots meet once.
__host__ __device__ inline void tour_pair(int r, int i, int n, int* a, int* b) {
  if (i == 0) {
    *a = r;
    *b = n - 1;
  } else {
    *a = (r + i) % (n - 1);
    *b = (r - i + (n - 1)) % (n - 1);
  }
}

// column c (< 64) of block pair (I, J)
__device__ __forceinline__ int64_t pair_col(int c, int I, int J) {
  return c < JB ? (int64_t)I * JB + c : (int64_t)J * JB + (c - JB);
}

__global__ void k_transpose(int64_t k, const double* __restrict__ R, double* __restrict__ G) {
  __shared__ double tile[32][33];
  const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bx + tx, j = by + r;
    tile[r][tx] = (i < k && j < k) ? R[i + k * j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = by + tx, j = bx + r;   // G(i, j) = R(j, i)
    if (i < k && j < k) G[i + k * j] = tile[tx][r];
  }
}

// Y += X (n x m, column-major with leading dimensions)
__global__ void k_axpy(int64_t n, int64_t m, const double* __restrict__ X, int64_t ldx, double* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e % n, j = e / n;
  Y[i + ldy * j] += X[i + ldx * j];
}

// Partial Gram matrices of the round's block pairs: block (p, sr) sums rows
// [sr * rch, (sr+1) * rch) of X_p^T X_p, X_p = [G_I G_J] (k x 64), into
// Hp + (p * rsplit + sr) * 4096 (64 x 64, column-major).  Rows go through LDS
// in chunks of GR; the next chunk is loaded into registers while the current
// one is multiplied.
constexpr int GR = 32;
constexpr int GR_PER = GR * JP / 256;   // chunk elements staged per thread

__global__ void __launch_bounds__(256)
k_jac_gram(int64_t k, const double* __restrict__ G, int round, int nbj, int rsplit, int64_t rch,
           double* __restrict__ Hp) {
  __shared__ double Xs[GR][JP + 2];   // Xs[kk][c] = X(kb + kk, c)
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int p = blockIdx.x, sr = blockIdx.y;
  int I, J;
  tour_pair(round, p, nbj, &I, &J);
  const int64_t r0 = (int64_t)sr * rch, r1 = std::min(k, r0 + rch);
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  dbl4 acc[2][2];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = dbl4{0.0, 0.0, 0.0, 0.0};
  // element q of this thread: row kk = t % GR of the chunk, column c = t / GR + (256 / GR) q
  const int kk0 = t % GR, c0 = t / GR;
  double reg[GR_PER];
  auto fetch = [&](int64_t kb) {
    const int64_t row = kb + kk0;
#pragma unroll
    for (int q = 0; q < GR_PER; ++q)
      reg[q] = row < r1 ? G[row + k * pair_col(c0 + (256 / GR) * q, I, J)] : 0.0;
  };
  if (r0 < r1) fetch(r0);
  for (int64_t kb = r0; kb < r1; kb += GR) {
#pragma unroll
    for (int q = 0; q < GR_PER; ++q) Xs[kk0][c0 + (256 / GR) * q] = reg[q];
    __syncthreads();
    if (kb + GR < r1) fetch(kb + GR);
#pragma unroll
    for (int ks = 0; ks < GR / 4; ++ks) {
      const int kk = 4 * ks + (l >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) av[mi] = Xs[kk][wi + 16 * mi + (l & 15)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bv[ni] = Xs[kk][wj + 16 * ni + (l & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[ni], av[mi], acc[mi][ni], 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator entry v of lane l is (i, j) = (wi + 16 mi + (l & 15), wj + 16 ni + (l >> 4) + 4 v)
  double* out = Hp + ((int64_t)p * rsplit + sr) * (JP * JP);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(wi + 16 * mi + (l & 15)) + JP * (wj + 16 * ni + (l >> 4) + 4 * v)] = acc[mi][ni][v];
}

// Two-sided cyclic Jacobi on each pair's Gram H (sum of the partials, upper
// triangle mirrored): JINNER sweeps at most, each 63 rounds of 32 disjoint
// rotations.  Rotation of (p, q) by the angle with tan 2theta =
// 2 h_pq / (h_qq - h_pp), |theta| <= pi/4:
// columns p, q <- c col_p - s col_q, s col_p + c col_q (rows likewise).
// Out: the accumulated rotation V_p (64 x 64) and the number of rotations of
// the first sweep (the outer convergence test).
constexpr int EIG_THREADS = 1024;   // a round's 1024 2 x 2 blocks and 2048 V updates spread wide

__global__ void __launch_bounds__(EIG_THREADS)
k_jac_eig(const double* __restrict__ Hp, int rsplit, double tol, double* __restrict__ Vout,
          int* __restrict__ count) {
  extern __shared__ double sme[];
  double (*H)[JP + 1] = reinterpret_cast<double (*)[JP + 1]>(sme);
  double (*V)[JP + 1] = reinterpret_cast<double (*)[JP + 1]>(sme + JP * (JP + 1));
  __shared__ double cs[JP / 2][2];
  __shared__ int pq[JP / 2][2];
  __shared__ int nrot[JP / 2];
  __shared__ int any;
  const int t = threadIdx.x;
  const int p = blockIdx.x;
  const double* src = Hp + (int64_t)p * rsplit * (JP * JP);
  for (int e = t; e < JP * JP; e += EIG_THREADS) {
    const int i = e % JP, j = e / JP;
    const int a = i < j ? i : j, b = i < j ? j : i;   // upper triangle
    double s = 0.0;
    for (int sr = 0; sr < rsplit; ++sr) s += src[(int64_t)sr * (JP * JP) + a + JP * b];
    H[i][j] = s;
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  int first = 0;
  for (int sw = 0; sw < JINNER; ++sw) {
    if (t < JP / 2) nrot[t] = 0;
    __syncthreads();
    for (int r = 0; r < JP - 1; ++r) {
      if (t < JP / 2) {
        int a, b;
        tour_pair(r, t, JP, &a, &b);
        const double hpp = H[a][a], hqq = H[b][b], hpq = H[a][b];
        double c = 1.0, s = 0.0;
        // (|hpq| > 1e-150 keeps the squares below normal numbers)
        if (hpq * hpq > tol * tol * (hpp * hqq) && fabs(hpq) > 1e-150) {
          // the same angle from the half-angle identities: cos 2theta = |d| / r,
          // c^2 = (1 + cos 2theta) / 2, s = sin 2theta / 2c, two reciprocal
          // square roots (estimate + Newton step) on the dependency chain
          const double d = hqq - hpp, g2 = 2.0 * hpq;
          const double rq = rsq_nr(fma(d, d, g2 * g2));
          const double cos2 = fabs(d) * rq, sin2 = (d >= 0.0 ? g2 : -g2) * rq;
          const double hh = fma(0.5, cos2, 0.5);
          const double rh = rsq_nr(hh);
          c = hh * rh;
          s = 0.5 * sin2 * rh;
          nrot[t] += 1;
        }
        cs[t][0] = c;
        cs[t][1] = s;
        pq[t][0] = a;
        pq[t][1] = b;
      }
      __syncthreads();
      // H <- J^T H J by 2 x 2 blocks (row pair u, column pair v)
      for (int e = t; e < (JP / 2) * (JP / 2); e += EIG_THREADS) {
        const int v = e & (JP / 2 - 1), u = e / (JP / 2);
        const int pu = pq[u][0], qu = pq[u][1], pv = pq[v][0], qv = pq[v][1];
        const double cu = cs[u][0], su = cs[u][1], cv = cs[v][0], sv = cs[v][1];
        const double h11 = H[pu][pv], h12 = H[pu][qv], h21 = H[qu][pv], h22 = H[qu][qv];
        const double a11 = cv * h11 - sv * h12, a12 = sv * h11 + cv * h12;
        const double a21 = cv * h21 - sv * h22, a22 = sv * h21 + cv * h22;
        H[pu][pv] = cu * a11 - su * a21;
        H[qu][pv] = su * a11 + cu * a21;
        H[pu][qv] = cu * a12 - su * a22;
        H[qu][qv] = su * a12 + cu * a22;
      }
      // V <- V J
      for (int e = t; e < JP * (JP / 2); e += EIG_THREADS) {
        const int i = e % JP, v = e / JP;
        const int pv = pq[v][0], qv = pq[v][1];
        const double cv = cs[v][0], sv = cs[v][1];
        const double vp = V[i][pv], vq = V[i][qv];
        V[i][pv] = cv * vp - sv * vq;
        V[i][qv] = sv * vp + cv * vq;
      }
      __syncthreads();
    }
    if (t == 0) {
      int n = 0;
      for (int i = 0; i < JP / 2; ++i) n += nrot[i];
      any = n;
    }
    __syncthreads();
    if (sw == 0) first = any;
    if (any == 0) break;
    __syncthreads();
  }
  double* out = Vout + (int64_t)p * (JP * JP);
  for (int e = t; e < JP * JP; e += EIG_THREADS) out[e] = V[e % JP][e / JP];
  if (t == 0) count[p] = first;
}

// X_p <- X_p V_p on 64-row tiles, in place, for G (blockIdx.z = 0) and the
// accumulated V (blockIdx.z = 1); a block takes ROT_TILES consecutive tiles
// and loads V_p once.  A tile is read whole before it is written, and no
// other block touches it; the next tile's columns are loaded into registers
// while the current one is multiplied.
constexpr int ROT_TILES = 8;
constexpr int ROT_PER = JP * JP / 256;   // tile elements staged per thread

__global__ void __launch_bounds__(256)
k_jac_rot(int64_t k, double* G, double* Vm, int round, int nbj, const double* __restrict__ Vp) {
  extern __shared__ double smj[];
  double (*Xs)[JP + 2] = reinterpret_cast<double (*)[JP + 2]>(smj);                     // Xs[c][rr]
  double (*Rs)[JP + 2] = reinterpret_cast<double (*)[JP + 2]>(smj + JP * (JP + 2));      // Rs[c][j]
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int p = blockIdx.y;
  double* X = blockIdx.z == 0 ? G : Vm;
  int I, J;
  tour_pair(round, p, nbj, &I, &J);
  const double* vp = Vp + (int64_t)p * (JP * JP);
  for (int e = t; e < JP * JP; e += 256) Rs[e & 63][e >> 6] = vp[e];   // Rs[c'][j] = V_p(c', j)
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  const int64_t ntiles = k / 64;
  const int64_t tile0 = (int64_t)blockIdx.x * ROT_TILES;
  // element q of this thread: rr = t & 63 (fixed), c = (t >> 6) + 4 q
  const int rr = t & 63;
  double reg[ROT_PER];
  auto fetch = [&](int64_t tile) {
    const int64_t r0 = tile * 64;
#pragma unroll
    for (int q = 0; q < ROT_PER; ++q) reg[q] = X[r0 + rr + k * pair_col((t >> 6) + 4 * q, I, J)];
  };
  if (tile0 < ntiles) fetch(tile0);
  for (int tt = 0; tt < ROT_TILES; ++tt) {
    const int64_t tile = tile0 + tt;
    if (tile >= ntiles) break;
    const int64_t r0 = tile * 64;
#pragma unroll
    for (int q = 0; q < ROT_PER; ++q) Xs[(t >> 6) + 4 * q][rr] = reg[q];
    __syncthreads();
    if (tt + 1 < ROT_TILES && tile + 1 < ntiles) fetch(tile + 1);   // disjoint rows: in flight meanwhile
    dbl4 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ks = 0; ks < JP / 4; ++ks) {
      const int kk = 4 * ks + (l >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) av[mi] = Xs[kk][wi + 16 * mi + (l & 15)];
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) bv[ni] = Rs[kk][wj + 16 * ni + (l & 15)];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[ni], av[mi], acc[mi][ni], 0, 0, 0);
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ro = wi + 16 * mi + (l & 15), j = wj + 16 * ni + (l >> 4) + 4 * v;
          X[r0 + ro + k * pair_col(j, I, J)] = acc[mi][ni][v];
        }
    __syncthreads();   // Xs is refilled for the next tile
  }
}

// sigma_j = ||G(:, j)||
__global__ void k_colnorms(int64_t k, const double* __restrict__ G, double* __restrict__ sig) {
  __shared__ double part[256];
  const int64_t j = blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 256 < k; i += 512) {
    const double a = G[i + k * j], b = G[i + 256 + k * j];
    s0 = fma(a, a, s0);
    s1 = fma(b, b, s1);
  }
  if (i < k) {
    const double a = G[i + k * j];
    s0 = fma(a, a, s0);
  }
  part[threadIdx.x] = s0 + s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) sig[j] = sqrt(part[0]);
}

// sorted[pos_i] = sig_i, pos_i = #{j : sig_j > sig_i or (sig_j == sig_i and j < i)}
__global__ void k_rank_sort(int64_t k, const double* __restrict__ sig, double* __restrict__ sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double s = sig[i];
  int64_t pos = 0;
  for (int64_t j = 0; j < k; ++j) {
    const double x = sig[j];
    pos += (x > s) || (x == s && j < i);
  }
  sorted[pos] = s;
}

// Gs(:, j) = G(:, j) / sigma_j^2 if sigma_j > thr, else 0
__global__ void k_scale_cols(int64_t k, const double* __restrict__ G, const double* __restrict__ sig, double thr,
                             double* __restrict__ Gs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const double s = sig[e / k];
  Gs[e] = s > thr ? G[e] / (s * s) : 0.0;
}

int grid1(int64_t n) { return (int)((n + 255) / 256); }

// Split-reduction buffer for the panel projections Q(:, 0:done)^T X over
// every done = 64, 128, ..., k - 64.
int64_t panel_part(int k, int64_t Mt) {
  int64_t most = 1;
  for (int64_t done = PB; done < k; done += PB) most = std::max(most, gemm_split_doubles(done, PB, Mt, 1));
  return most;
}

struct WideScratch {
  int64_t tsqr, qpan, rpan, rpan2, part, hp, vp, cnt;   // offsets in doubles
  int64_t total;
  int rsplit;
  int64_t rch;
};

WideScratch wide_layout(int64_t Mt, int k) {
  WideScratch s{};
  const int nbj = k / JB, npairs = nbj / 2;
  int64_t off = 0;
  s.tsqr = off;
  off += tsqr_scratch(Mt, PB);
  s.qpan = off;
  off += Mt * PB;
  s.rpan = off;
  off += PB * PB;
  s.rpan2 = off;
  off += PB * PB;
  s.part = off;
  off += panel_part(k, Mt);
  s.rsplit = (int)std::max<int64_t>(1, std::min<int64_t>((512 + npairs - 1) / npairs, k / 64));
  s.rch = ((k + s.rsplit - 1) / s.rsplit + 31) / 32 * 32;   // whole Gram row chunks
  s.rsplit = (int)((k + s.rch - 1) / s.rch);
  s.hp = off;
  off += (int64_t)npairs * s.rsplit * JP * JP;
  s.vp = off;
  off += (int64_t)npairs * JP * JP;
  s.cnt = off;
  off += ((int64_t)(nbj - 1) * npairs + 1) / 2 + 1;   // ints
  s.total = off;
  return s;
}

}  // namespace

int64_t wide_factor_doubles(int64_t N, int64_t Mt, int k) {
  return 2 * N * k + Mt * k + 4 * (int64_t)k * k + 2 * k + wide_layout(Mt, k).total + 2 * (int64_t)k * PB + panel_part(k, Mt) + 8;
}

// Block classical Gram-Schmidt QR with reorthogonalisation (BCGS2) of the
// m x k matrix Xq (ld m) in place: Xq becomes Q, R (k x k, ld k) the
// triangular factor.  64-column panels: two projections against the finished
// Q (MFMA GEMMs), a TSQR of the panel, one more projection of the panel's Q
// and a second TSQR (see below).  The scratch is laid out for m <= its rows.
//
// Look-ahead: a panel's projections are split into the panels finished
// before its predecessor (the old group) and its predecessor (the new one),
// each projected twice.  The old group's projections of panel p + 1 do not
// wait for panel p, so they run on a side stream (ss, with its own partials
// part2 and coefficients rproj2) while panel p's latency-bound TSQRs run on
// st; panel p + 1 then only projects against panel p on st.  With ss == st
// the same work runs in order.
static int wide_qr(double* Xq, int64_t m, int k, double* R, double* scr, const WideScratch& L, double* rproj,
                   int rb, hipStream_t st, hipStream_t ss, double* part2, double* rproj2) {
  double* tq = scr + L.tsqr;
  double* qpan = scr + L.qpan;
  double* rpan = scr + L.rpan;
  double* r3 = scr + L.rpan2;
  double* part = scr + L.part;
  const int64_t npart = panel_part(k, m);
  const int np = k / PB;
  hipEvent_t ev_final = nullptr, ev_old = nullptr;   // panels before p final (st); old group of p + 1 done (ss)
  if (ss != st) {
    AZ_HIP(hipEventCreateWithFlags(&ev_final, hipEventDisableTiming));
    if (hipEventCreateWithFlags(&ev_old, hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(ev_final);
      return AZRBF_EHIP;
    }
  }
  int rc = AZRBF_OK;
  // projections of panel X against the done_g finished columns Qg (offset off
  // in its R column), twice: R[off..] = c1 + c2, X -= Qg (c1 + c2)
  auto project = [&](const double* Qg, int64_t done_g, int64_t off, double* X, double* Rcol, double* tmp,
                     double* prt, hipStream_t s) -> int {
    AZ_TRY(gemm_mfma(true, false, done_g, PB, m, 1.0, Qg, m, 0, X, m, 0, 0.0, Rcol + off, k, 0, 1, prt, npart, s));
    AZ_TRY(gemm_mfma(false, false, m, PB, done_g, -1.0, Qg, m, 0, Rcol + off, k, 0, 1.0, X, m, 0, 1, prt, npart, s));
    AZ_TRY(gemm_mfma(true, false, done_g, PB, m, 1.0, Qg, m, 0, X, m, 0, 0.0, tmp, done_g, 0, 1, prt, npart, s));
    AZ_TRY(gemm_mfma(false, false, m, PB, done_g, -1.0, Qg, m, 0, tmp, done_g, 0, 1.0, X, m, 0, 1, prt, npart, s));
    launch_kernel(k_axpy, grid1(done_g * PB), 256, 0, s, done_g, PB, tmp, done_g, Rcol + off, k);
    return hipGetLastError() == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  };
  rc = hipMemsetAsync(R, 0, sizeof(double) * k * k, st) == hipSuccess ? AZRBF_OK : AZRBF_EHIP;
  for (int p = 0; p < np && !rc; ++p) {
    double* X = Xq + (int64_t)p * PB * m;
    const int64_t done = (int64_t)p * PB;
    double* Rcol = R + (int64_t)p * PB * k;
    if (p > 0) {
      // panels 0 .. p - 1 are final here: the old group of panel p + 1 may start
      if (ss != st && p + 1 < np) {
        if (hipEventRecord(ev_final, st) != hipSuccess || hipStreamWaitEvent(ss, ev_final, 0) != hipSuccess) {
          rc = AZRBF_EHIP;
          break;
        }
      }
      // the old group of this panel (panels 0 .. p - 2): queued on ss during
      // the previous panel, or here when there is no side stream
      if (p >= 2) {
        if (ss != st) {
          if (hipStreamWaitEvent(st, ev_old, 0) != hipSuccess) {
            rc = AZRBF_EHIP;
            break;
          }
        } else if ((rc = project(Xq, done - PB, 0, X, Rcol, rproj, part, st)) != AZRBF_OK) {
          break;
        }
      }
      // the new group: the previous panel
      if ((rc = project(Xq + (done - PB) * m, PB, done - PB, X, Rcol, rproj, part, st)) != AZRBF_OK) break;
    }
    if ((rc = tsqr_panel(X, m, PB, rb, tq, qpan, rpan, st)) != AZRBF_OK) break;
    // queue the old group of panel p + 1 (panels 0 .. p - 1) beside this panel's TSQRs
    if (ss != st && p >= 1 && p + 1 < np) {
      double* Xn = Xq + (int64_t)(p + 1) * PB * m;
      double* Rn = R + (int64_t)(p + 1) * PB * k;
      if ((rc = project(Xq, done, 0, Xn, Rn, rproj2, part2, ss)) != AZRBF_OK) break;
      if (hipEventRecord(ev_old, ss) != hipSuccess) {
        rc = AZRBF_EHIP;
        break;
      }
    }
    if (p == 0) {
      if (hipMemcpyAsync(X, qpan, sizeof(double) * m * PB, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpy2DAsync(Rcol, sizeof(double) * k, rpan, sizeof(double) * PB, sizeof(double) * PB, PB,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = AZRBF_EHIP;
      continue;
    }
    // Past the numerical rank the projected panel is rounding noise, and
    // the Householder completion of its Q need not be orthogonal to the
    // finished Q.  One more projection of the panel's Q and a second TSQR
    // restore orthogonality:  Qp = Q S3 + Q'' R3, so the panel's R column
    // gains S3 Rpp and its diagonal block becomes R3 Rpp.
    if ((rc = gemm_mfma(true, false, done, PB, m, 1.0, Xq, m, 0, qpan, m, 0, 0.0, rproj, done, 0, 1, part, npart,
                        st)) != AZRBF_OK)
      break;
    if ((rc = gemm_mfma(false, false, m, PB, done, -1.0, Xq, m, 0, rproj, done, 0, 1.0, qpan, m, 0, 1, part, npart,
                        st)) != AZRBF_OK)
      break;
    if ((rc = tsqr_panel(qpan, m, PB, rb, tq, X, r3, st)) != AZRBF_OK) break;
    if ((rc = gemm_mfma(false, false, done, PB, PB, 1.0, rproj, done, 0, rpan, PB, 0, 1.0, Rcol, k, 0, 1, nullptr, 0,
                        st)) != AZRBF_OK)
      break;
    rc = gemm_mfma(false, false, PB, PB, PB, 1.0, r3, PB, 0, rpan, PB, 0, 0.0, Rcol + done, k, 0, 1, nullptr, 0, st);
  }
  if (rc && ss != st) {   // nothing queued on ss may outlive the call
    (void)hipStreamSynchronize(ss);
    (void)hipStreamSynchronize(st);
  }
  if (ev_final) (void)hipEventDestroy(ev_final);
  if (ev_old) (void)hipEventDestroy(ev_old);
  return rc;
}

int wide_factor(Plan& P, hipStream_t st) {
  const int k = P.k;
  if (k <= 64 || k % 64 != 0) return AZRBF_EUNSUPPORTED;
  const int64_t N = P.N, Mt = P.Mt;
  if (k > N || k > Mt) return AZRBF_EINVAL;
  const WideScratch L = wide_layout(Mt, k);
  if (!P.Om) {
    AZ_TRY(P.alloc((void**)&P.Om, sizeof(double) * N * k));
    AZ_TRY(P.alloc((void**)&P.Om2, sizeof(double) * N * k));
    AZ_TRY(P.alloc((void**)&P.Q, sizeof(double) * Mt * k));
    AZ_TRY(P.alloc((void**)&P.Rf, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.Gj, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.Vj, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.Pm, sizeof(double) * k * k));
    AZ_TRY(P.alloc((void**)&P.sig, sizeof(double) * 2 * k));
    // second-projection coefficients (k x 64), then the side stream's split-K
    // partials and coefficients
    const int64_t sd = L.total + 2 * (int64_t)k * PB + panel_part(k, Mt) + 8;
    AZ_TRY(P.alloc((void**)&P.dscr, sizeof(double) * sd));
    P.dscr_bytes = sizeof(double) * sd;
  }
  double* scr = P.dscr;
  const WideScratch& Lx = L;
  double* rproj = scr + L.total;   // second-projection coefficients, k x 64
  double* rproj2 = rproj + (int64_t)k * PB;
  double* part2 = rproj2 + (int64_t)k * PB;
  // the panels' look-ahead projections go to a side stream (not when kernels
  // are being timed one by one)
  hipStream_t ss = st;
  if (!prof_enabled() && side_stream(P.device, &ss) != AZRBF_OK) ss = st;
  // 1. sketch
  AZ_TRY(dense_gaussian(P.prob.seed, N, k, P.Om, N, st));
  AZ_TRY(ops_apply_A(P, P.Om, N, k, 1.0, 0.0, nullptr, 0, P.Q, Mt, st));        // Y = A Omega
  AZ_TRY(ops_apply_AZ(P, P.Q, Mt, k, -1.0, 1.0, P.Q, Mt, P.Q, Mt, P.Om2, st));  // W = Y - A Z* Y
  // 2. W = Q R
  P.ldq = Mt;
  AZ_TRY(wide_qr(P.Q, Mt, k, P.Rf, scr, Lx, rproj, plan_tsqr_rows(P, PB), st, ss, part2, rproj2));
  // 3. block one-sided Jacobi, preconditioned: R^T = Q2 R2 (the same QR),
  // then Jacobi on G = R2^T with the rotations accumulated onto V = Q2
  // (fewer sweeps: the QR concentrates the weight of R2's rows on its
  // diagonal); R = U S (Q2 V_J)^T with U S the rotated columns of G.
  const int nbj = k / JB, npairs = nbj / 2;
  {
    dim3 tg((unsigned)((k + 31) / 32), (unsigned)((k + 31) / 32));
    launch_kernel(k_transpose, tg, 256, 0, st, k, P.Rf, P.Vj);
    AZ_HIP(hipGetLastError());
    AZ_TRY(wide_qr(P.Vj, k, k, P.Pm, scr, Lx, rproj, plan_tsqr_rows(P, PB), st, ss, part2, rproj2));    // Vj = Q2, Pm = R2 (scratch until step 4)
    launch_kernel(k_transpose, tg, 256, 0, st, k, P.Pm, P.Gj);
    AZ_HIP(hipGetLastError());
  }
  const int rot_lds = (int)(sizeof(double) * 2 * JP * (JP + 2));
  const int eig_lds = (int)(sizeof(double) * 2 * JP * (JP + 1));
  {
    static std::mutex mu;
    static bool lds_set = false;
    std::lock_guard<std::mutex> lk(mu);
    if (!lds_set) {
      AZ_HIP(hipFuncSetAttribute((const void*)k_jac_rot, hipFuncAttributeMaxDynamicSharedMemorySize, rot_lds));
      AZ_HIP(hipFuncSetAttribute((const void*)k_jac_eig, hipFuncAttributeMaxDynamicSharedMemorySize, eig_lds));
      lds_set = true;
    }
  }
  double* Hp = scr + Lx.hp;
  double* Vp = scr + Lx.vp;
  int* cnt = (int*)(scr + Lx.cnt);
  const double tol = 4.0 * k * 1.1102230246251565e-16;
  std::vector<int> hcnt((size_t)(nbj - 1) * npairs);
  int sweeps = 0;
  for (int sw = 0; sw < JMAX; ++sw) {
    for (int r = 0; r < nbj - 1; ++r) {
      {
        Prof pr("jac_gram", 8.0 * k * 64 * npairs + 8.0 * 4096 * npairs * Lx.rsplit, st,
                2.0 * k * 64 * 64 * npairs);
        launch_kernel(k_jac_gram, dim3((unsigned)npairs, (unsigned)Lx.rsplit), 256, 0, st, k, P.Gj, r, nbj, Lx.rsplit,
                      Lx.rch, Hp);
      }
      {
        Prof pr("jac_eig", 8.0 * 4096 * npairs * (Lx.rsplit + 1), st);
        launch_kernel(k_jac_eig, npairs, EIG_THREADS, eig_lds, st, Hp, Lx.rsplit, tol, Vp, cnt + (int64_t)r * npairs);
      }
      {
        Prof pr("jac_rot", 2.0 * 16.0 * k * 64 * npairs, st, 2.0 * 2.0 * k * 64 * 64 * npairs);
        launch_kernel(k_jac_rot, dim3((unsigned)((k / 64 + ROT_TILES - 1) / ROT_TILES), (unsigned)npairs, 2), 256,
                      rot_lds, st, k, P.Gj, P.Vj, r, nbj, Vp);
      }
      AZ_HIP(hipGetLastError());
    }
    AZ_HIP(hipMemcpyAsync(hcnt.data(), cnt, sizeof(int) * hcnt.size(), hipMemcpyDeviceToHost, st));
    AZ_HIP(hipStreamSynchronize(st));
    ++sweeps;
    int64_t tot = 0;
    for (int v : hcnt) tot += v;
    if (tot == 0) break;
  }
  // 4. singular values, truncation, P = R^+ = sum_i w_i g_i^T / sigma_i^2
  // (w_i the columns of Q2 V_J, g_i = u_i sigma_i those of the rotated G)
  double* sraw = P.sig + k;
  launch_kernel(k_colnorms, k, 256, 0, st, k, P.Gj, sraw);
  launch_kernel(k_rank_sort, grid1(k), 256, 0, st, k, sraw, P.sig);
  AZ_TRY(ops_norms(P, st));
  const double thr = P.tau * P.normA * sqrt((double)k);
  launch_kernel(k_scale_cols, grid1((int64_t)k * k), 256, 0, st, k, P.Vj, sraw, thr, P.Om2);
  AZ_HIP(hipGetLastError());
  AZ_TRY(gemm_mfma(false, true, k, k, k, 1.0, P.Om2, k, 0, P.Gj, k, 0, 0.0, P.Pm, k, 0, 1, nullptr, 0, st));
  std::vector<double> hs(k);
  AZ_HIP(hipMemcpyAsync(hs.data(), P.sig, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  AZ_HIP(hipStreamSynchronize(st));
  int rank = 0;
  while (rank < k && hs[rank] > thr) ++rank;
  P.rank = rank;
  P.sweeps = sweeps;
  P.factored = true;
  return 10 * (int64_t)rank > 9 * (int64_t)k ? AZRBF_ERANK : AZRBF_OK;   // too narrow: see factor_plan
}

int wide_solve(Plan& P, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx, double* relres,
               hipStream_t st) {
  const int k = P.k;
  const int64_t N = P.N, Mt = P.Mt;
  const int64_t npart = std::max<int64_t>(gemm_split_doubles(k, nrhs, Mt, 1), 1);
  if (nrhs > P.sw_rhs || npart > P.sw_part) {
    const int64_t per = 2 * N + 3 * Mt + 2 * (int64_t)k + 2 * relres_chunks();
    double* old = P.sw;
    AZ_TRY(P.alloc((void**)&P.sw, sizeof(double) * (per * nrhs + npart)));
    P.release_one_after(old, st);
    P.sw_rhs = nrhs;
    P.sw_part = npart;
  }
  double* Zr = P.sw;                       // N x nrhs
  double* X1 = Zr + N * nrhs;              // N x nrhs
  double* C = X1 + N * nrhs;               // Mt x nrhs
  double* R1 = C + Mt * nrhs;              // Mt x nrhs
  double* Rc = R1 + Mt * nrhs;             // Mt x nrhs
  double* Tm = Rc + Mt * nrhs;             // k x nrhs
  double* Ym = Tm + (int64_t)k * nrhs;     // k x nrhs
  double* nrm = Ym + (int64_t)k * nrhs;    // 2 relres_chunks() x nrhs
  double* part = nrm + 2 * relres_chunks() * nrhs;
  const double* rin = B;
  int64_t ldr = ldb;
  for (int it = 0; it <= P.refine; ++it) {
    AZ_TRY(ops_apply_AZ(P, rin, ldr, nrhs, -1.0, 1.0, rin, ldr, C, Mt, Zr, st));             // c = (I - A Z*) r
    AZ_TRY(gemm_mfma(true, false, k, nrhs, Mt, 1.0, P.Q, Mt, 0, C, Mt, 0, 0.0, Tm, k, 0, 1, part, npart, st));
    AZ_TRY(gemm_mfma(false, false, k, nrhs, k, 1.0, P.Pm, k, 0, Tm, k, 0, 0.0, Ym, k, 0, 1, nullptr, 0, st));
    AZ_TRY(gemm_mfma(false, false, N, nrhs, k, 1.0, P.Om, N, 0, Ym, k, 0, 0.0, X1, N, 0, 1, nullptr, 0, st));
    AZ_TRY(ops_apply_A(P, X1, N, nrhs, -1.0, 1.0, rin, ldr, R1, Mt, st));                    // r - A x1
    if (it == 0) {
      AZ_TRY(ops_apply_Z(P, R1, Mt, nrhs, 1.0, 1.0, X1, N, X, ldx, st));                     // x = x1 + x2
    } else {
      AZ_TRY(ops_apply_Z(P, R1, Mt, nrhs, 1.0, 1.0, X1, N, X1, N, st));                      // x1 + x2
      launch_kernel(k_axpy, grid1(N * nrhs), 256, 0, st, N, nrhs, X1, N, X, ldx);
      AZ_HIP(hipGetLastError());
    }
    AZ_TRY(ops_apply_A(P, X, ldx, nrhs, -1.0, 1.0, B, ldb, Rc, Mt, st));                     // b - A x
    rin = Rc;
    ldr = Mt;
  }
  if (relres) AZ_TRY(relres_norms(Rc, Mt, B, ldb, Mt, nrhs, nrm, relres, st));
  return AZRBF_OK;
}

}  // namespace az
