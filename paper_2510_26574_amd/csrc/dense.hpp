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
// In-place lower Cholesky of the n x n (n <= NB... up to JMAX) block at A
// (column-major, ld), only the lower triangle is read and written.
// A pivot <= 0 sets *bad (and the status) and replaces the pivot by 1 so the
// rest stays finite.
__device__ inline void chol_block_lds(double* a, int n, int lda_s, int32_t* status) {
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double p = a[j + j * lda_s];
      if (!(p > 0.0)) {
        set_status(status, RPC_EBREAKDOWN);
        p = 1.0;
      }
      a[j + j * lda_s] = sqrt(p);
    }
    __syncthreads();
    const double piv = a[j + j * lda_s];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) a[i + j * lda_s] /= piv;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int c = j + 1 + e / m, i = j + 1 + e % m;
      if (i >= c) a[i + c * lda_s] -= a[i + j * lda_s] * a[c + j * lda_s];
    }
  }
  __syncthreads();
}

// Factor the NB x NB diagonal block starting at (j0, j0) of A (n x n, ld).
__global__ __launch_bounds__(256) void k_chol_diag(double* A, int64_t ld, int n, int j0,
                                                   int32_t* status) {
  __shared__ double a[NB * NB];
  const int nb = n - j0 < NB ? n - j0 : NB;
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    int i = e % nb, c = e / nb;
    a[i + c * NB] = A[(j0 + i) + (int64_t)(j0 + c) * ld];
  }
  chol_block_lds(a, nb, NB, status);
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    int i = e % nb, c = e / nb;
    A[(j0 + i) + (int64_t)(j0 + c) * ld] = i >= c ? a[i + c * NB] : 0.0;
  }
}

// Panel: rows i >= j0 + NB of block column j0 solve x L_jj^T = a (forward
// substitution along the row), one thread per row.
__global__ __launch_bounds__(256) void k_chol_panel(double* A, int64_t ld, int n, int j0) {
  __shared__ double L[NB * NB];
  const int nb = n - j0 < NB ? n - j0 : NB;
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    int i = e % nb, c = e / nb;
    L[i + c * NB] = A[(j0 + i) + (int64_t)(j0 + c) * ld];
  }
  __syncthreads();
  const int64_t row = (int64_t)j0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  double x[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = c < nb ? A[row + (int64_t)(j0 + c) * ld] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nb) {
      double s = x[c];
      for (int l = 0; l < c; ++l) s -= x[l] * L[c + l * NB];
      x[c] = s / L[c + c * NB];
    }
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < nb) A[row + (int64_t)(j0 + c) * ld] = x[c];
}

// Blocked right-looking Cholesky A = L L^T (lower, column-major), in place.
inline void cholesky(hipStream_t st, double* A, int64_t ld, int n, int32_t* status) {
  for (int j0 = 0; j0 < n; j0 += NB) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, A, ld, n, j0, status);
    const int rest = n - j0 - NB;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3((rest + 255) / 256), dim3(256), 0, st, A, ld, n, j0);
      // trailing A[j0+NB:, j0+NB:] -= P P^T, P = A[j0+NB:, j0:j0+NB]
      const double* P = A + (j0 + NB) + (int64_t)j0 * ld;
      gemm64<false, false>(st, rest, rest, NB, P, ld, P, ld, A + (j0 + NB) + (int64_t)(j0 + NB) * ld,
                           ld, -1.0, 1.0);
    }
  }
  hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)(((int64_t)n * n + 255) / 256)), dim3(256), 0, st,
                     A, ld, n);
}

// Diagonal block of the back substitution L^T X = B: rows i0..i0+nb of X
// (n x m, column-major ldx) solve L_ii^T x = b, one thread per column.
__global__ __launch_bounds__(256) void k_trsm_ut_diag(const double* L, int64_t ld, int i0, int nb,
                                                      double* X, int64_t ldx, int m) {
  __shared__ double Ls[NB * NB];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    int i = e % nb, c = e / nb;
    Ls[i + c * NB] = L[(i0 + i) + (int64_t)(i0 + c) * ld];
  }
  __syncthreads();
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= m) return;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = i < nb ? X[(i0 + i) + (int64_t)col * ldx] : 0.0;
  // (L_ii^T) is upper triangular: row i of L^T is column i of L
#pragma unroll
  for (int ii = NB - 1; ii >= 0; --ii) {
    if (ii < nb) {
      double s = x[ii];
      for (int l = ii + 1; l < nb; ++l) s -= Ls[l + ii * NB] * x[l];
      x[ii] = s / Ls[ii + ii * NB];
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < nb) X[(i0 + i) + (int64_t)col * ldx] = x[i];
}

// Solve L^T X = B in place (L lower n x n column-major; X n x m column-major).
inline void trsm_lt(hipStream_t st, const double* L, int64_t ld, int n, double* X, int64_t ldx,
                    int m) {
  const int nblk = (n + NB - 1) / NB;
  for (int ib = nblk - 1; ib >= 0; --ib) {
    const int i0 = ib * NB;
    const int nb = n - i0 < NB ? n - i0 : NB;
    const int below = n - (i0 + nb);
    if (below > 0) {
      // X_i -= L[below, i]^T X_below :
      //   A(i, l) = L[(i0+nb+l) + (i0+i) ld],  B(col, l) = X[(i0+nb+l) + col ldx]
      gemm64<true, true>(st, nb, m, below, L + (i0 + nb) + (int64_t)i0 * ld, ld, X + (i0 + nb), ldx,
                         X + i0, ldx, -1.0, 1.0);
    }
    hipLaunchKernelGGL(k_trsm_ut_diag, dim3((m + 255) / 256), dim3(256), 0, st, L, ld, i0, nb, X,
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
  __shared__ int done;
  const int tid = threadIdx.x;
  const int n = p + (p & 1);  // even size; a padded row/column is decoupled (zero)
  for (int e = tid; e < n * n; e += 1024) {
    int i = e % n, c = e / n;
    double x = (i < p && c < p) ? 0.5 * (A[i + c * lda] + A[c + i * lda]) : 0.0;
    a[i + c * n] = x;
    v[i + c * n] = i == c ? 1.0 : 0.0;
  }
  __syncthreads();
  const int h = n / 2;
  for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
    // convergence: off-diagonal Frobenius mass vs total
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += 1024) {
      int i = e % n, c = e / n;
      double x = a[i + c * n];
      tot += x * x;
      if (i != c) off += x * x;
    }
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
      if (sweep == max_sweeps && !done) set_status(status, RPC_ENOCONV);
    }
    __syncthreads();
    if (done || sweep == max_sweeps) break;
    for (int step = 0; step < n - 1; ++step) {
      if (tid < h) {
        // round-robin pairing: player n-1 fixed, the others rotate
        int x, y;
        if (tid == 0) {
          x = n - 1;
          y = step;
        } else {
          x = (step + tid) % (n - 1);
          y = (step - tid + (n - 1)) % (n - 1);
        }
        const int P = x < y ? x : y, Q = x < y ? y : x;
        const double app = a[P + P * n], aqq = a[Q + Q * n], apq = a[P + Q * n];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-300) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
        pa[tid] = P;
        pb[tid] = Q;
      }
      __syncthreads();
      // A <- J^T A J on every 2 x 2 block (rows of pair u, columns of pair w)
      for (int e = tid; e < h * h; e += 1024) {
        const int u = e % h, w = e / h;
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
      for (int e = tid; e < n * h; e += 1024) {
        const int i = e % n, u = e / n;
        const int P = pa[u], Q = pb[u];
        const double c = cs[u], s = sn[u];
        const double vp = v[i + P * n], vq = v[i + Q * n];
        v[i + P * n] = c * vp - s * vq;
        v[i + Q * n] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort the p real eigenvalues in decreasing order (selection by rank)
  __shared__ int order[JMAX];
  if (tid < p) {
    const double x = a[tid + tid * n];
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double y = a[j + j * n];
      if (y > x || (y == x && j < tid)) ++rank;
    }
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < p) evals[tid] = a[order[tid] + order[tid] * n];
  for (int e = tid; e < p * p; e += 1024) {
    int i = e % p, c = e / p;
    W[i + c * ldw] = v[i + order[c] * n];
  }
}

// One-workgroup Cholesky G = R^T R (R upper) of a p x p SPD matrix and the
// inverse R^{-1} (upper), p <= JMAX.  On breakdown the status is set.
__global__ __launch_bounds__(1024) void k_chol_inv_small(const double* __restrict__ G, int64_t ldg,
                                                         int p, double* __restrict__ Rinv,
                                                         int64_t ldr, int32_t* status,
                                                         const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ double a[JMAX * JMAX];
  __shared__ double x[JMAX * JMAX];
  const int tid = threadIdx.x;
  for (int e = tid; e < p * p; e += 1024) {
    int i = e % p, c = e / p;
    a[i + c * p] = G[i + c * ldg];
  }
  chol_block_lds(a, p, p, status);  // lower L, R = L^T
  // X = L^{-1} (lower), column c by forward substitution, one thread per column
  if (tid < p) {
    const int c = tid;
    for (int i = 0; i < c; ++i) x[i + c * p] = 0.0;
    x[c + c * p] = 1.0 / a[c + c * p];
    for (int i = c + 1; i < p; ++i) {
      double s = 0.0;
      for (int l = c; l < i; ++l) s += a[i + l * p] * x[l + c * p];
      x[i + c * p] = -s / a[i + i * p];
    }
  }
  __syncthreads();
  // R^{-1} = (L^{-1})^T
  for (int e = tid; e < p * p; e += 1024) {
    int i = e % p, c = e / p;
    Rinv[i + c * ldr] = x[c + i * p];
  }
}

}  // namespace
}  // namespace dense
