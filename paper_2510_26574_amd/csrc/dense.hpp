// Small and medium float64 dense linear algebra used by Algorithm 1 on gfx950:
// a general tile product (C = alpha A B^T + beta C with either operand
// orientation), a blocked right-looking Cholesky, a blocked triangular solve,
// one-workgroup Cholesky+inverse, and a one-workgroup parallel-order Jacobi
// eigensolver.  All routines are stream-ordered launches; none synchronises.
#pragma once
#include "common.hpp"
#include "tile_gemm.hpp"

namespace dense {
namespace {  // internal linkage: each translation unit owns its copy

constexpr int JMAX = 96;  // largest matrix the one-workgroup Jacobi holds in LDS
constexpr int NB = 64;    // block size of the blocked Cholesky / triangular solve
constexpr int SPLITK_MAX = 16;  // most k slices of a split-K product

// Visits e = t, t + step, ... below n * n with (i, c) = (e mod n, e / n):
// the same elements in the same order as a loop over e, but with one integer
// division per call instead of two per element (a division by a run-time
// value costs some thirty instructions).
template <typename Fn>
__device__ inline void for_nn(int t, int step, int n, Fn&& fn) {
  if (n <= 0) return;
  const int di = step % n, dc = step / n;
  int i = t % n, c = t / n;
  for (int e = t; e < n * n; e += step) {
    fn(i, c);
    i += di;
    c += dc;
    if (i >= n) {
      i -= n;
      ++c;
    }
  }
}

// C(m, n) = alpha * sum_k A(m, k) B(n, k) + beta * C(m, n)
//   A(m, k) = KCA ? A[m * lda + k] : A[m + k * lda]
//   B(n, k) = KCB ? B[n * ldb + k] : B[n + k * ldb]
//   C column-major with leading dimension ldc.
template <bool KCA, bool KCB>
__global__ __launch_bounds__(256) void k_gemm64(int64_t M, int64_t N, int64_t K,
                                                const double* __restrict__ A, int64_t lda,
                                                const double* __restrict__ B, int64_t ldb,
                                                double* __restrict__ C, int64_t ldc, double alpha,
                                                double beta, const int32_t* skip) {
  if (skip && *skip) return;
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, KCA, KCB>::bytes / sizeof(double)];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  GOperand<double, KCA> a{A, lda, M, K, nullptr, (lda % 2) == 0};
  GOperand<double, KCB> b{B, ldb, N, K, nullptr, (ldb % 2) == 0};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, b, m0, n0, 0, K, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < M && n < N) {
      double* c = C + m + n * ldc;
      *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
    }
  });
}

template <bool KCA, bool KCB>
inline void gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                   double beta, const int32_t* skip = nullptr) {
  if (M <= 0 || N <= 0) return;
  dim3 g((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL((k_gemm64<KCA, KCB>), g, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc,
                     alpha, beta, skip);
}

// Zero the strict upper triangle of an n x n column-major matrix.
__global__ __launch_bounds__(256) void k_zero_upper(double* A, int64_t ld, int n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e % n), c = (int)(e / n);
  if (i < c) A[i + (int64_t)c * ld] = 0.0;
}

// ------------------------------------------------ one-workgroup Cholesky
// In-place lower Cholesky (L with the square roots applied, lower triangle of
// `a` in LDS, column-major, lda_s) for n <= 128 + 8, blocked by panels of 8
// columns: wave 0 loads a panel into registers (lane l holds panel rows
// j0 + l and j0 + l + 64), factors it
// right-looking with the pivot-row values broadcast by readlane, and writes
// it back; then every wave applies the panel to tiles of the trailing lower
// triangle on the float64 MFMA.  Two workgroup barriers per panel.  A pivot <= 0 sets
// RPC_EBREAKDOWN and is replaced by 1.
__device__ inline void chol_panel_lds(double* a, int n, int lda_s, int32_t* status) {
  constexpr int W = 8;
  const int nth = blockDim.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += W) {
    const int jw = n - j0 < W ? n - j0 : W;
    if (wave == 0) {
      double P0[W], P1[W];  // rows j0 + lane, j0 + lane + 64
      const int i0 = j0 + lane, i1 = j0 + lane + 64;
#pragma unroll
      for (int q = 0; q < W; ++q) {
        P0[q] = (q < jw && i0 < n) ? a[i0 + (j0 + q) * lda_s] : 0.0;
        P1[q] = (q < jw && i1 < n) ? a[i1 + (j0 + q) * lda_s] : 0.0;
      }
      // one column of the panel: pivot, scale, update the panel's later
      // columns; a full panel (jw == W) runs without per-column branches so
      // the columns' independent updates can interleave
      bool bad = false;
      auto column = [&](int jj, int cw) __attribute__((always_inline)) {
        double p = bcast_lane(P0[jj], jj);  // diagonal (j0 + jj, j0 + jj)
        bad |= !(p > 0.0);
        p = p > 0.0 ? p : 1.0;
        const double rd = rsqrt(p), d = p * rd;
        // column jj: rows below the diagonal scaled, the diagonal set to d
        P0[jj] = lane > jj ? P0[jj] * rd : (lane == jj ? d : P0[jj]);
        P1[jj] = P1[jj] * rd;
#pragma unroll
        for (int c2 = jj + 1; c2 < W; ++c2) {
          if (c2 < cw) {
            const double f = bcast_lane(P0[jj], c2);  // L(j0 + c2, j0 + jj)
            P0[c2] = lane >= c2 ? P0[c2] - P0[jj] * f : P0[c2];
            P1[c2] -= P1[jj] * f;
          }
        }
      };
      if (jw == W) {
#pragma unroll
        for (int jj = 0; jj < W; ++jj) column(jj, W);
      } else {
#pragma unroll
        for (int jj = 0; jj < W; ++jj)
          if (jj < jw) column(jj, jw);
      }
      if (bad && lane == 0) set_status(status, RPC_EBREAKDOWN);
#pragma unroll
      for (int q = 0; q < W; ++q) {
        if (q < jw && i0 < n && lane >= q) a[i0 + (j0 + q) * lda_s] = P0[q];
        if (q < jw && i1 < n) a[i1 + (j0 + q) * lda_s] = P1[q];
      }
    }
    __syncthreads();
    // trailing lower triangle (columns c >= j0 + jw, rows i >= c) -= P P^T,
    // P the panel's rows below it: 16 x 16 tiles of the lower triangle on the
    // float64 MFMA (two k-steps of four panel columns), one tile per wave at a
    // time; element e of lane l is row l / 16 + 4 e, column l % 16 of a tile
    const int t0 = j0 + jw;
    if (t0 < n) {
      const int nt16 = (n - t0 + 15) / 16, ntile = nt16 * (nt16 + 1) / 2;
      for (int tt = wave; tt < ntile; tt += nth / 64) {
        int bi = 0;
        while ((bi + 1) * (bi + 2) / 2 <= tt) ++bi;
        const int bj = tt - bi * (bi + 1) / 2;
        const int ra = t0 + 16 * bi + (lane & 15), cb = t0 + 16 * bj + (lane & 15);
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < W / 4; ++s4) {
          const int q = 4 * s4 + (lane >> 4);
          const double av = (ra < n && q < jw) ? a[ra + (j0 + q) * lda_s] : 0.0;
          const double bv = (cb < n && q < jw) ? a[cb + (j0 + q) * lda_s] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = t0 + 16 * bi + (lane >> 4) + 4 * e;
          if (row < n && cb < n && row >= cb) a[row + cb * lda_s] -= acc[e];
        }
      }
    }
    __syncthreads();
  }
}

// Active order of a matrix whose rows and columns from *kptr on are those of
// the identity (no coupling): its Cholesky factor is the identity there too.
__device__ inline int active_n(int n, const int32_t* kptr) {
  if (!kptr) return n;
  const int k = *kptr;
  return k < n ? (k > 0 ? k : 0) : n;
}

// Factor the NB x NB diagonal block starting at (j0, j0) of A (n x n, ld);
// only its part inside the active order.  One wave: lane i keeps row i of the
// block in registers (rows and columns past the active order are those of
// the identity); step j takes the pivot from lane j, scales column j, writes
// it to LDS and every lane subtracts L(i, j) L(c, j) from its entries c > j.
// The steps are unrolled, so the register indices are constants, and the
// wave needs no barrier (its LDS accesses complete in order).  A pivot <= 0
// sets RPC_EBREAKDOWN and is replaced by 1.
static_assert(NB == 64, "one row of the diagonal block per lane");
__global__ __launch_bounds__(64) void k_chol_diag(double* A, int64_t ld, int n, int j0,
                                                  int32_t* status, const int32_t* kptr) {
  __shared__ double col[NB];
  n = active_n(n, kptr);
  if (j0 >= n) return;
  const int nb = n - j0 < NB ? n - j0 : NB;
  const int i = threadIdx.x;
  double r[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    r[c] = (i < nb && c < nb) ? A[(j0 + i) + (int64_t)(j0 + c) * ld] : (i == c ? 1.0 : 0.0);
  bool bad = false;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double d = bcast_lane(r[j], j);
    bad |= !(d > 0.0);
    d = d > 0.0 ? d : 1.0;
    const double rs = rsqrt(d);
    const double l = i == j ? d * rs : r[j] * rs;  // L(i, j) for i >= j
    r[j] = l;
    col[i] = l;
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));  // lgkmcnt(0): the write landed
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = j + 1; c < NB; ++c) r[c] -= l * col[c];
    __builtin_amdgcn_wave_barrier();  // this step's reads come before the next step's write
  }
  if (bad && i == 0) set_status(status, RPC_EBREAKDOWN);
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (i < nb && c < nb) A[(j0 + i) + (int64_t)(j0 + c) * ld] = c <= i ? r[c] : 0.0;
}

// Panel: rows i >= j0 + NB of block column j0 solve x L_jj^T = a (forward
// substitution along the row), one thread per row, within the active order.
__global__ __launch_bounds__(256) void k_chol_panel(double* A, int64_t ld, int n, int j0,
                                                    const int32_t* kptr) {
  __shared__ double L[NB * NB];
  __shared__ double rdg[NB];  // 1 / L(c, c), taken once
  n = active_n(n, kptr);
  if (j0 >= n) return;
  const int nb = n - j0 < NB ? n - j0 : NB;
  for_nn((int)threadIdx.x, 256, nb, [&](int i, int c) {
    L[i + c * NB] = A[(j0 + i) + (int64_t)(j0 + c) * ld];
  });
  if ((int)threadIdx.x < nb) {
    const int c = threadIdx.x;
    rdg[c] = 1.0 / A[(j0 + c) + (int64_t)(j0 + c) * ld];
  }
  __syncthreads();
  const int64_t row = (int64_t)j0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = c < nb ? A[row + (int64_t)(j0 + c) * ld] : 0.0;
  // forward substitution x L^T = a; a full block runs without per-column branches
  auto column = [&](int c) __attribute__((always_inline)) {
    double s = x[c];
    for (int l = 0; l < c; ++l) s -= x[l] * L[c + l * NB];
    x[c] = s * rdg[c];
  };
  if (nb == NB) {
#pragma unroll
    for (int c = 0; c < NB; ++c) column(c);
  } else {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) column(c);
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < nb) A[row + (int64_t)(j0 + c) * ld] = x[c];
}

// skip[b] = 1 when block step b has no trailing rows inside the active order.
__global__ void k_chol_skips(int n, const int32_t* kptr, int nblk, int32_t* skip) {
  const int ne = active_n(n, kptr);
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) skip[b] = (b + 1) * NB >= ne ? 1 : 0;
}

// Blocked right-looking Cholesky A = L L^T (lower, column-major), in place.
// kptr (optional, device): rows and columns from *kptr on are those of the
// identity; the block steps past it return at once (skip holds one int per
// block step).
inline void cholesky(hipStream_t st, double* A, int64_t ld, int n, int32_t* status,
                     const int32_t* kptr = nullptr, int32_t* skip = nullptr) {
  const int nblk = (n + NB - 1) / NB;
  if (kptr && skip)
    hipLaunchKernelGGL(k_chol_skips, dim3(1), dim3(256), 0, st, n, kptr, nblk, skip);
  for (int j0 = 0; j0 < n; j0 += NB) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, A, ld, n, j0, status, kptr);
    const int rest = n - j0 - NB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3((rest + 255) / 256), dim3(256), 0, st, A, ld, n, j0,
                         kptr);
      // trailing A[j0+NB:, j0+NB:] -= P P^T, P = A[j0+NB:, j0:j0+NB]
      const double* P = A + (j0 + NB) + (int64_t)j0 * ld;
      gemm64<false, false>(st, rest, rest, NB, P, ld, P, ld, A + (j0 + NB) + (int64_t)(j0 + NB) * ld,
                           ld, -1.0, 1.0, (kptr && skip) ? skip + j0 / NB : nullptr);
    }
  }
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)(((int64_t)n * n + 255) / 256)), dim3(256), 0, st,
                     A, ld, n);
}

// Diagonal block of the back substitution L^T X = B: rows i0..i0+nb of X
// (n x m, column-major ldx) solve L_ii^T x = b.  One wave per right-hand
// side, lane l holding x_l, right-looking from the bottom: once row ii is
// solved (x_ii = b_ii / L(ii,ii) on lane ii) it is broadcast and every lane
// l < ii subtracts L(ii, l) x_ii, so a row costs one broadcast and one
// multiply-add instead of a wave reduction.
__global__ __launch_bounds__(1024) void k_trsm_ut_diag(const double* L, int64_t ld, int i0, int nb,
                                                       double* X, int64_t ldx, int m) {
  constexpr int LDS = NB + 1;  // lanes reading row ii of the block walk distinct banks
  __shared__ double Ls[NB * LDS];
  __shared__ double rd[NB];
  for_nn((int)threadIdx.x, 1024, nb, [&](int i, int c) {
    Ls[i + c * LDS] = L[(i0 + i) + (int64_t)(i0 + c) * ld];
  });
  __syncthreads();
  if (threadIdx.x < nb) rd[threadIdx.x] = 1.0 / Ls[threadIdx.x + threadIdx.x * LDS];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 16 + wave;
  if (col >= m) return;
  double* xc = X + i0 + (int64_t)col * ldx;
  double x = lane < nb ? xc[lane] : 0.0;
  for (int ii = nb - 1; ii >= 0; --ii) {
    const double xi = bcast_lane(x, ii) * rd[ii];
    if (lane == ii) x = xi;
    // (L^T)(l, ii) = L(ii, l)
    if (lane < ii) x -= Ls[ii + lane * LDS] * xi;
  }
  if (lane < nb) xc[lane] = x;
}

template <bool KCA, bool KCB>
inline void gemm64_splitk(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A,
                          int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                          double alpha, double beta, double* part, const int32_t* skip = nullptr,
                          int max_splits = SPLITK_MAX);

// Solve L^T X = B in place (L lower n x n column-major; X n x m column-major).
// `part` (SPLITK_MAX * NB * m doubles, or null) lets the block updates split
// their long k range over several workgroups.
inline void trsm_lt(hipStream_t st, const double* L, int64_t ld, int n, double* X, int64_t ldx,
                    int m, double* part = nullptr) {
  const int nblk = (n + NB - 1) / NB;
  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int i0 = ib * NB;
    const int nb = n - i0 < NB ? n - i0 : NB;
    const int below = n - (i0 + nb);
    if (below > 0) {
      // X_i -= L[below, i]^T X_below :
      //   A(i, l) = L[(i0+nb+l) + (i0+i) ld],  B(col, l) = X[(i0+nb+l) + col ldx]
      if (part)
        gemm64_splitk<true, true>(st, nb, m, below, L + (i0 + nb) + (int64_t)i0 * ld, ld,
                                  X + (i0 + nb), ldx, X + i0, ldx, -1.0, 1.0, part, nullptr);
      else
        gemm64<true, true>(st, nb, m, below, L + (i0 + nb) + (int64_t)i0 * ld, ld, X + (i0 + nb),
                           ldx, X + i0, ldx, -1.0, 1.0);
    }
    hipLaunchKernelGGL(k_trsm_ut_diag, dim3((m + 15) / 16), dim3(1024), 0, st, L, ld, i0, nb, X,
                       ldx, m);
  }
}

// ------------------------------------------------ one-workgroup Jacobi
// Eigen-decomposition of the symmetric p x p matrix A (column-major, lda),
// p <= JMAX, in one workgroup: parallel (round-robin) two-sided Jacobi with
// each step's p/2 disjoint rotations applied to all 2 x 2 blocks at once.
// Outputs eigenvalues in decreasing order and the matching eigenvectors
// (columns of W, p x p column-major, ldw).  Sets RPC_ENOCONV if the
// off-diagonal mass is not below tol after max_sweeps.
__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ A, int64_t lda, int p,
                                                 double* __restrict__ evals,
                                                 double* __restrict__ W, int64_t ldw,
                                                 int max_sweeps, double tol, int32_t* status,
                                                 const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ double a[JMAX * JMAX];
  __shared__ double v[JMAX * JMAX];
  __shared__ double cs[JMAX / 2], sn[JMAX / 2];
  __shared__ int pa[JMAX / 2], pb[JMAX / 2];
  __shared__ double red[16];
  __shared__ double thr2;
  __shared__ int done, ident[JMAX / 2];
  const int tid = threadIdx.x;
  const int n = p + (p & 1);  // even size; a padded row/column is decoupled (zero)
  for_nn(tid, 1024, n, [&](int i, int c) {
    double x = (i < p && c < p) ? 0.5 * (A[i + c * lda] + A[c + i * lda]) : 0.0;
    a[i + c * n] = x;
    v[i + c * n] = i == c ? 1.0 : 0.0;
  });
  __syncthreads();
  const int h = n / 2;
  // Each thread's 2 x 2 blocks (pairs u, w) and V entries (row i, pair u) are
  // the same in every step: their indices are taken once here, since an
  // integer division by the run-time h or n costs some thirty instructions
  // and the step loop would otherwise repeat eight of them per thread.
  constexpr int AMAX = ((JMAX / 2) * (JMAX / 2) + 1023) / 1024;
  constexpr int VMAX = (JMAX * (JMAX / 2) + 1023) / 1024;
  int au[AMAX], aw[AMAX], vi[VMAX], vu[VMAX];
#pragma unroll
  for (int q = 0; q < AMAX; ++q) {
    const int e = tid + q * 1024;
    au[q] = e < h * h ? e % h : -1;
    aw[q] = e < h * h ? e / h : 0;
  }
#pragma unroll
  for (int q = 0; q < VMAX; ++q) {
    const int e = tid + q * 1024;
    vi[q] = e < n * h ? e % n : 0;
    vu[q] = e < n * h ? e / n : -1;
  }
  for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
    // convergence: off-diagonal Frobenius mass vs total
    double off = 0.0, tot = 0.0;
    for_nn(tid, 1024, n, [&](int i, int c) {
      double x = a[i + c * n];
      tot += x * x;
      if (i != c) off += x * x;
    });
    off = wave_sum(off);
    tot = wave_sum(tot);
    if ((tid & 63) == 0) {
      red[tid >> 6] = off;
    }
    __syncthreads();
    if (tid == 0) {
      double o = 0.0;
      for (int w = 0; w < 16; ++w) o += red[w];
      red[0] = o;
    }
    __syncthreads();
    const double offs = red[0];
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = tot;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < 16; ++w) t += red[w];
      done = (offs <= tol * tol * t) ? 1 : 0;
      // rotations of pairs with a_pq^2 below tol^2 t / (4 n^2) are skipped:
      // all of them together hold less than a quarter of the mass the
      // stopping test allows, so a sweep that skips every pair ends the loop
      thr2 = tol * tol * t / (4.0 * (double)n * (double)n);
      if (sweep == max_sweeps && !done) set_status(status, RPC_ENOCONV);
    }
    __syncthreads();
    if (done || sweep == max_sweeps) break;
    // round-robin pairing: player n-1 fixed, the others rotate; for thread
    // t > 0, x = (step + t) mod (n - 1) and y = (step - t) mod (n - 1), kept
    // by increments
    int rx = tid, ry = n - 1 - tid;
    for (int step = 0; step < n - 1; ++step) {
      if (tid < h) {
        int x, y;
        if (tid == 0) {
          x = n - 1;
          y = step;
        } else {
          x = rx;
          y = ry;
        }
        const int P = x < y ? x : y, Q = x < y ? y : x;
        const double app = a[P + P * n], aqq = a[Q + Q * n], apq = a[P + Q * n];
        double c = 1.0, s = 0.0;
        const bool skip_pair = !(apq * apq > thr2);
        ident[tid] = skip_pair;
        if (!skip_pair && fabs(apq) > 1e-300) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = rsqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
        pa[tid] = P;
        pb[tid] = Q;
      }
      __syncthreads();
      rx = rx + 1 == n - 1 ? 0 : rx + 1;
      ry = ry + 1 == n - 1 ? 0 : ry + 1;
      // A <- J^T A J on every 2 x 2 block (rows of pair u, columns of pair w)
#pragma unroll
      for (int q = 0; q < AMAX; ++q) {
        const int u = au[q], w = aw[q];
        if (u < 0) continue;
        if (ident[u] & ident[w]) continue;  // both rotations are the identity
        const int P = pa[u], Q = pb[u], R = pa[w], S = pb[w];
        const double cu = cs[u], su = sn[u], cw = cs[w], sw = sn[w];
        const double aPR = a[P + R * n], aPS = a[P + S * n], aQR = a[Q + R * n], aQS = a[Q + S * n];
        // right-multiply by J_w: col R' = c R - s S, col S' = s R + c S
        const double bPR = cw * aPR - sw * aPS, bPS = sw * aPR + cw * aPS;
        const double bQR = cw * aQR - sw * aQS, bQS = sw * aQR + cw * aQS;
        // left-multiply by J_u^T: row P' = c P - s Q, row Q' = s P + c Q
        a[P + R * n] = cu * bPR - su * bQR;
        a[Q + R * n] = su * bPR + cu * bQR;
        a[P + S * n] = cu * bPS - su * bQS;
        a[Q + S * n] = su * bPS + cu * bQS;
      }
      // V <- V J
#pragma unroll
      for (int q = 0; q < VMAX; ++q) {
        const int i = vi[q], u = vu[q];
        if (u < 0) continue;
        if (ident[u]) continue;
        const int P = pa[u], Q = pb[u];
        const double c = cs[u], s = sn[u];
        const double vp = v[i + P * n], vq = v[i + Q * n];
        v[i + P * n] = c * vp - s * vq;
        v[i + Q * n] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort the p real eigenvalues in decreasing order (selection by rank; a
  // NaN ranks as -inf, so the ranks always form a permutation)
  __shared__ int order[JMAX];
  if (tid < p) {
    const double x0 = a[tid + tid * n];
    const double x = x0 == x0 ? x0 : -INFINITY;
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double y0 = a[j + j * n];
      const double y = y0 == y0 ? y0 : -INFINITY;
      if (y > x || (y == x && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < p) evals[tid] = a[order[tid] + order[tid] * n];
  for_nn(tid, 1024, p, [&](int i, int c) { W[i + c * ldw] = v[i + order[c] * n]; });
}

// One-workgroup Cholesky G = R^T R of a p x p SPD matrix (p <= JMAX); writes
// R (upper, column-major, ldr; zero below the diagonal).  With `equil` the
// factorisation runs on the equilibrated S G S, s_i = 1/sqrt(G_ii), and
// R = L^T S^{-1} is written, which is the same factor in exact arithmetic
// but keeps the pivots near 1 (Cholesky QR with column scaling).  On
// breakdown the status is set.
__global__ __launch_bounds__(1024) void k_chol_small(const double* __restrict__ G, int64_t ldg,
                                                     int p, double* __restrict__ R, int64_t ldr,
                                                     int32_t* status, const int32_t* skip,
                                                     int equil = 0, int inverse = 0) {
  if (skip && *skip) return;
  constexpr int LDS = JMAX + 1;
  __shared__ double a[JMAX * LDS];
  __shared__ double xi[JMAX * LDS];
  __shared__ double piv[JMAX];
  __shared__ double sc[JMAX];
  const int tid = threadIdx.x;
  if (tid < p) {
    const double g = G[tid + (int64_t)tid * ldg];
    sc[tid] = (equil && g > 0.0) ? 1.0 / sqrt(g) : 1.0;
  }
  __syncthreads();
  for_nn(tid, 1024, p, [&](int i, int c) { a[i + c * LDS] = G[i + c * ldg] * sc[i] * sc[c]; });
  chol_panel_lds(a, p, LDS, status);  // lower L, R = L^T S^{-1}
  if (!inverse) {
    for_nn(tid, 1024, p, [&](int i, int c) {
      R[i + c * ldr] = (i <= c) ? a[c + i * LDS] / sc[c] : 0.0;
    });
    return;
  }
  // X = L^{-1} by 16 x 16 blocks (p padded to a multiple of 16 with the
  // identity).  First each diagonal block X_bb = L_bb^{-1}, one wave per block
  // and one column per lane (forward substitution); then block row b after
  // block row (one barrier each): X_bc = -X_bb sum_{c <= d < b} L_bd X_dc for
  // c < b, one wave per block, as float64 MFMA products (16 x 16 x 4 steps).
  // The accumulator of the sum is, element s of lane l, the B operand of the
  // product with X_bb at k-step s, so it needs no trip through LDS.  Then
  // R^{-1} = S L^{-T} = S X^T.
  {
    const int lane = tid & 63, wave = tid >> 6;
    const int nb = (p + 15) / 16;
    // the identity in the padding, so that every read below is unconditional
    for_nn(tid, 1024, 16 * nb, [&](int i, int c) {
      if (i >= p || c >= p) a[i + c * LDS] = i == c ? 1.0 : 0.0;
    });
    __syncthreads();
    auto L_at = [&](int r, int c) -> double { return a[r + c * LDS]; };
    if (wave < nb && lane < 16) {
      const int b0 = 16 * wave, c = lane;  // column c of X_bb
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double s0 = i == c ? 1.0 : 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) s0 -= L_at(b0 + i, b0 + l) * x[l];
        x[i] = s0 / L_at(b0 + i, b0 + i);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) xi[(b0 + i) + (b0 + c) * LDS] = x[i];  // zero above the diagonal
    }
    __syncthreads();
    for (int b = 1; b < nb; ++b) {
      if (wave < b) {
        const int cb = wave;  // block column
        const int m = lane & 15, kq = lane >> 4;
        v4d t = {0.0, 0.0, 0.0, 0.0};
        for (int d = cb; d < b; ++d) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const double av = L_at(16 * b + m, 16 * d + 4 * s4 + kq);
            const double bv = xi[(16 * d + 4 * s4 + kq) + (16 * cb + m) * LDS];
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, t, 0, 0, 0);
          }
        }
        v4d xb = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const double av = xi[(16 * b + m) + (16 * b + 4 * s4 + kq) * LDS];
          xb = __builtin_amdgcn_mfma_f64_16x16x4f64(av, t[s4], xb, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) xi[(16 * b + kq + 4 * e) + (16 * cb + m) * LDS] = -xb[e];
      }
      __syncthreads();
    }
  }
  for_nn(tid, 1024, p, [&](int i, int c) {
    R[i + c * ldr] = (i <= c) ? sc[i] * xi[c + i * LDS] : 0.0;  // (S X^T)(i, c) = s_i X(c, i)
  });
}

// Q = Y R^{-1} for p == P (R upper P x P, Y r x P, column-major): each
// thread keeps its row of Y in registers and solves q R = y by forward
// substitution, fully unrolled, with R broadcast from LDS; four partial
// sums per dot product shorten the dependency chain.  64 rows per workgroup.
template <int P>
__global__ __launch_bounds__(64) void k_trsm_rows_reg(const double* __restrict__ Y, int64_t ldy,
                                                      int rows, const double* __restrict__ R,
                                                      int64_t ldr, double* __restrict__ Q,
                                                      int64_t ldq, const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ double Rs[P * P];
  __shared__ double rdiag[P];
  const int t = threadIdx.x;
  for (int e = t; e < P * P; e += 64) {
    const int i = e % P, c = e / P;
    Rs[i + c * P] = R[i + c * ldr];
  }
  __syncthreads();
  for (int j = t; j < P; j += 64) rdiag[j] = 1.0 / Rs[j + j * P];
  __syncthreads();
  const int row = blockIdx.x * 64 + t;
  const bool ok = row < rows;
  double q[P];
#pragma unroll
  for (int j = 0; j < P; ++j) q[j] = ok ? Y[row + (int64_t)j * ldy] : 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    double s0 = q[j], s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int l = 0; l + 3 < j; l += 4) {
      s0 -= q[l] * Rs[l + j * P];
      s1 -= q[l + 1] * Rs[l + 1 + j * P];
      s2 -= q[l + 2] * Rs[l + 2 + j * P];
      s3 -= q[l + 3] * Rs[l + 3 + j * P];
    }
#pragma unroll
    for (int l = (j / 4) * 4; l < j; ++l) s0 -= q[l] * Rs[l + j * P];
    q[j] = ((s0 + s1) + (s2 + s3)) * rdiag[j];
  }
  if (ok) {
#pragma unroll
    for (int j = 0; j < P; ++j) Q[row + (int64_t)j * ldq] = q[j];
  }
}

// Q = Y R^{-1} (R upper p x p, Y r x p, both column-major): each thread
// solves one row q R = y by forward substitution, its row staged in LDS
// (odd stride) and R broadcast from LDS.  64 rows per workgroup.
__global__ __launch_bounds__(64) void k_trsm_rows(const double* __restrict__ Y, int64_t ldy,
                                                  int rows, int p, const double* __restrict__ R,
                                                  int64_t ldr, double* __restrict__ Q,
                                                  int64_t ldq, const int32_t* skip) {
  if (skip && *skip) return;
  constexpr int LDS = JMAX + 1;
  __shared__ double Rs[JMAX * JMAX];
  __shared__ double q[64 * LDS];
  const int t = threadIdx.x;
  for_nn(t, 64, p, [&](int i, int c) { Rs[i + c * p] = R[i + c * ldr]; });
  const int row = blockIdx.x * 64 + t;
  for (int j = 0; j < p; ++j) q[t * LDS + j] = row < rows ? Y[row + (int64_t)j * ldy] : 0.0;
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    double sacc = q[t * LDS + j];
    for (int l = 0; l < j; ++l) sacc -= q[t * LDS + l] * Rs[l + j * p];
    q[t * LDS + j] = sacc / Rs[j + j * p];
  }
  if (row < rows)
    for (int j = 0; j < p; ++j) Q[row + (int64_t)j * ldq] = q[t * LDS + j];
}

// ------------------------------------------------ split-K product
// Same product as k_gemm64 for short-and-wide shapes (few output tiles, long
// K): grid.z slices K, each slice writes its float64 partial tile, and
// k_splitk_reduce adds them in a fixed order.
template <bool KCA, bool KCB>
__global__ __launch_bounds__(256) void k_gemm64_part(int64_t M, int64_t N, int64_t K, int64_t kc,
                                                     const double* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb,
                                                     double* __restrict__ part,
                                                     const int32_t* skip) {
  if (skip && *skip) return;
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, KCA, KCB>::bytes / sizeof(double)];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke = kb + kc < K ? kb + kc : K;
  GOperand<double, KCA> a{A, lda, M, K, nullptr, (lda % 2) == 0};
  GOperand<double, KCB> b{B, ldb, N, K, nullptr, (ldb % 2) == 0};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, b, m0, n0, kb, ke, smem);
  double* out = part + (int64_t)blockIdx.z * M * N;
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < M && n < N) out[m + n * M] = v;
  });
}

__global__ __launch_bounds__(256) void k_splitk_reduce(const double* __restrict__ part, int splits,
                                                       int64_t M, int64_t N, double* __restrict__ C,
                                                       int64_t ldc, double alpha, double beta,
                                                       const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * M * N + e];
  const int64_t m = e % M, n = e / M;
  double* c = C + m + n * ldc;
  *c = beta == 0.0 ? alpha * s : alpha * s + beta * *c;
}

// C = alpha A B^T + beta C with K sliced into up to max_splits (<= SPLITK_MAX)
// pieces of at least 64; `part` holds max_splits * M * N doubles.
template <bool KCA, bool KCB>
inline void gemm64_splitk(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A,
                          int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                          double alpha, double beta, double* part, const int32_t* skip,
                          int max_splits) {
  if (M <= 0 || N <= 0) return;
  int splits = (int)((K + 63) / 64);
  if (splits > max_splits) splits = max_splits;
  if (splits < 2) {
    gemm64<KCA, KCB>(st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, skip);
    return;
  }
  const int64_t kc = (K + splits - 1) / splits;
  dim3 g((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64), (unsigned)splits);
  hipLaunchKernelGGL((k_gemm64_part<KCA, KCB>), g, dim3(256), 0, st, M, N, K, kc, A, lda, B, ldb, part,
                     skip);
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, st,
                     (const double*)part, splits, M, N, C, ldc, alpha, beta, skip);
}

}  // namespace
}  // namespace dense
