// bistoch_degrees and bistoch_eig: Algorithm 1 of the paper after the
// factorisation, on gfx950.
//
// With K~ = F F^T (F: N x r, column-major, columns >= k zero):
//   c  = F^T 1,  d~ = F c           (diag(D~) = K~ 1, asserted > 0)
//   w  = F^T (1/d~),  q~ = F w      (diag(Q~) = K~ D~^{-1} 1, asserted > 0)
//   B  = D~^{-1} F,  C = F^T Q~^{-1} F     (factored P~ = B C B^T)
//   G_B = B^T B = R^T R              (Cholesky QR: Q = B R^{-1} is never formed)
//   M  = R C R^T = V Lambda V^T      (top nev eigenpairs)
//   U  = B R^{-1} V                  (N x nev)
// The two N-long Gram products dominate; they run as MFMA tiles over row
// chunks with float64 accumulation across chunks.  Everything of size r x r
// is float64.  Unused budget columns (index >= k) are handled by padding the
// Gram with the identity there, so every launch has a static shape and no
// host synchronisation is needed.
#include <math.h>

#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "dense.hpp"
#include "kernel_rows.hpp"
#include "profile.hpp"
#include "split16.hpp"
#include "syrk.hpp"
#include "tile_gemm.hpp"

namespace {

constexpr int COLCHUNK = 8192;  // rows per partial column sum

// part[chunk][col] = sum_{n in chunk} F[n, col] * wgt[n]   (col < k; 0 beyond)
template <typename TF>
__global__ __launch_bounds__(1024) void k_coldot_partial(const TF* __restrict__ F, int64_t ldf,
                                                         int64_t N, int r, const int32_t* kptr,
                                                         const double* __restrict__ wgt,
                                                         double* __restrict__ part) {
  // one wave per (column, row chunk); 16-byte vector loads, four in flight
  // per lane, so a wave keeps 4 KB of its column outstanding
  constexpr int V = 16 / (int)sizeof(TF);
  typedef TF vt __attribute__((ext_vector_type(V)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * COLCHUNK;
  const int64_t r1 = r0 + COLCHUNK < N ? r0 + COLCHUNK : N;
  // the chunk's weights, read once per workgroup (its 16 columns share them)
  __shared__ double ws[COLCHUNK];
  if (wgt) {
    for (int64_t n = r0 + threadIdx.x; n < r1; n += 1024) ws[n - r0] = wgt[n];
    __syncthreads();
  }
  const int col = blockIdx.y * 16 + wave;
  if (col >= r) return;
  const int k = *kptr;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (col < k) {
    const TF* f = F + (int64_t)col * ldf;
    const bool vec = (ldf % V) == 0;
    int64_t i = r0;
    if (vec) {
      // full groups of 4 x 64 vectors
      const int64_t step = 4 * 64 * V;
      for (; i + step <= r1; i += step) {
        vt a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = *reinterpret_cast<const vt*>(f + i + (u * 64 + lane) * V);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double t = 0.0;
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const int64_t n = i + (u * 64 + lane) * V + e;
            t += wgt ? to_d(a[u][e]) * ws[n - r0] : to_d(a[u][e]);
          }
          if (u == 0) s0 += t;
          if (u == 1) s1 += t;
          if (u == 2) s2 += t;
          if (u == 3) s3 += t;
        }
      }
    }
    for (int64_t n = i + lane; n < r1; n += 64) {
      const double v = to_d(f[n]);
      s0 += wgt ? v * ws[n - r0] : v;
    }
  }
  double s = (s0 + s1) + (s2 + s3);
  s = wave_sum(s);
  if (lane == 0) part[(int64_t)blockIdx.x * r + col] = s;
}

__global__ void k_reduce_cols(const double* __restrict__ part, int nch, int r, double* __restrict__ out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= r) return;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < nch; ++c) s += part[(int64_t)c * r + col];  // in order, 8 loads in flight
  out[col] = s;
}

// out[n] = sum_{l<k} F[n, l] v[l]; assert out > 0 (else `code`); inv[n] = 1/out[n].
template <typename TF>
__global__ __launch_bounds__(256) void k_rowdot(const TF* __restrict__ F, int64_t ldf, int64_t N,
                                                int r, const int32_t* kptr,
                                                const double* __restrict__ v,
                                                double* __restrict__ out, double* __restrict__ inv,
                                                int32_t code, int32_t* status) {
  extern __shared__ double vs[];
  const int k = *kptr;
  for (int l = threadIdx.x; l < k; l += 256) vs[l] = v[l];
  __syncthreads();
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double s0 = 0.0, s1 = 0.0;
  int l = 0;
  for (; l + 1 < k; l += 2) {
    s0 += to_d(F[n + (int64_t)l * ldf]) * vs[l];
    s1 += to_d(F[n + (int64_t)(l + 1) * ldf]) * vs[l + 1];
  }
  if (l < k) s0 += to_d(F[n + (int64_t)l * ldf]) * vs[l];
  const double s = s0 + s1;
  if (!(s > 0.0)) set_status(status, code);
  if (out) out[n] = s;
  if (inv) inv[n] = 1.0 / s;
}

// Finalise G_B and C:
//   G_B += gamma (B[0:k,:] + B[0:k,:]^T) + gamma^2 I_k  (B = D~^{-1} F);
//   unused indices (>= k): G_B = I, C = 0;
//   equilibrate: s_i = 1/sqrt(G_B[i,i]); Gs = S G_B S; Cs = S^{-1} C S^{-1}.
template <typename TF>
__global__ __launch_bounds__(256) void k_gram_finish(double* __restrict__ GB, double* __restrict__ C,
                                                     double* __restrict__ Gs,
                                                     double* __restrict__ Cs,
                                                     double* __restrict__ s, int r,
                                                     const int32_t* kptr, const TF* __restrict__ F,
                                                     int64_t ldf, int64_t N,
                                                     const double* __restrict__ dinv, double gamma,
                                                     int phase) {
  const int k = *kptr;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  if (phase == 0) {
    double g = GB[e], c = C[e];
    if (i >= k || j >= k) {
      g = (i == j) ? 1.0 : 0.0;
      c = 0.0;
    } else if (gamma != 0.0) {
      const double bij = i < N ? to_d(F[i + (int64_t)j * ldf]) * dinv[i] : 0.0;
      const double bji = j < N ? to_d(F[j + (int64_t)i * ldf]) * dinv[j] : 0.0;
      g += gamma * (bij + bji) + (i == j ? gamma * gamma : 0.0);
    }
    GB[e] = g;
    C[e] = c;
  } else {
    // a diagonal entry <= 0 (singular G_B) keeps scale 1, so the Cholesky
    // meets a pivot <= 0, reports RPC_EBREAKDOWN and stays finite
    const double gi = GB[i + (int64_t)i * r], gj = GB[j + (int64_t)j * r];
    const double si = gi > 0.0 ? 1.0 / sqrt(gi) : 1.0;
    const double sj = gj > 0.0 ? 1.0 / sqrt(gj) : 1.0;
    Gs[e] = GB[e] * si * sj;
    Cs[e] = C[e] / (si * sj);
    if (i == j) s[i] = si;
  }
}

// delta = 1e-7 trace(M); M += delta I.  M is PSD, so M + delta I keeps its
// eigenvectors while bounding the condition of every block M Q by
// lambda_max / delta, which keeps the two-pass Cholesky QR of the subspace
// iteration stable (it needs a condition number below ~1e7).
__global__ __launch_bounds__(1024) void k_shift_diag(double* M, int r, double* delta) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < r; i += 1024) s += M[i + (int64_t)i * r];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += red[w];
  const double dl = 1e-7 * t;
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += 1024) M[i + (int64_t)i * r] += dl;
  if (threadIdx.x == 0) *delta = dl;
}

// After the first Rayleigh-Ritz step: shift the iteration matrix down by
// sigma = theta_{p-1} / 2 (half the smallest Ritz value of the block, which
// approximates the first eigenvalue outside it).  Eigenvalues near zero then
// map to magnitudes no larger than the ones just below the block, so the
// convergence ratio of the wanted eigenvalues falls from lambda_{p+1} /
// lambda_i to (lambda_{p+1} - sigma) / (lambda_i - sigma).  The total shift
// stays in *delta for the final correction of the eigenvalues.
__global__ __launch_bounds__(1024) void k_shift_down(double* M, int r, const double* theta, int p,
                                                     double* delta, const int32_t* skip) {
  if (skip && *skip) return;
  const double sg = 0.5 * theta[p - 1];
  if (!(sg > 0.0)) return;
  for (int i = threadIdx.x; i < r; i += 1024) M[i + (int64_t)i * r] -= sg;
  if (threadIdx.x == 0) *delta -= sg;
}

__global__ void k_unshift(double* theta, int n, const double* delta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) theta[i] -= *delta;
}

// Start block: the leading p coordinate vectors.  The pivoted factor orders
// the Gram-Schmidt basis of B by pivot acceptance, so the dominant
// eigenvectors of M live mostly in its leading coordinates.
__global__ void k_fill_identity(double* Q, int r, int p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * p) return;
  const int i = (int)(e % r), j = (int)(e / r);
  Q[e] = i == j ? 1.0 : 0.0;
}

// Deterministic start block for the subspace iteration (hash-based uniform in [-1, 1]).
__global__ void k_fill_start(double* Q, int r, int p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * p) return;
  unsigned long long z = (unsigned long long)e * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  Q[e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// conv = 1 if every Ritz pair i < nev has |Y_i - theta_i Q_i| <= tol |theta_0|.
__global__ __launch_bounds__(1024) void k_ritz_check(const double* __restrict__ Y,
                                                     const double* __restrict__ Q,
                                                     const double* __restrict__ theta, int r,
                                                     int nev, double tol, int32_t* conv) {
  if (*conv) return;
  __shared__ int ok;
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < nev; i += 16) {
    double s = 0.0;
    for (int l = lane; l < r; l += 64) {
      const double d = Y[l + (int64_t)i * r] - theta[i] * Q[l + (int64_t)i * r];
      s += d * d;
    }
    s = wave_sum(s);
    if (lane == 0 && !(sqrt(s) <= tol * fabs(theta[0]))) atomicAnd(&ok, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0 && ok) *conv = 1;
}

__global__ void k_copy_cols(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd, int rows, int cols, const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int i = (int)(e % rows), j = (int)(e / rows);
  dst[i + j * ldd] = src[i + j * lds];
}

// rows scaled: X[i, j] *= s[i]  (or /= s[i] when divide)
__global__ void k_scale_rows(double* X, int64_t ldx, int rows, int cols, const double* s,
                             int divide) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int i = (int)(e % rows), j = (int)(e / rows);
  X[i + j * ldx] = divide ? X[i + j * ldx] / s[i] : X[i + j * ldx] * s[i];
}

__global__ void k_recip(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = 1.0 / x[i];
}

// Row scales of the Grams in the product type: 1/d~ and 1/sqrt(q~)
// (bistochastic), or 1/sqrt(d~) alone (symmetric; qt unused).
template <typename T>
__global__ void k_gram_scales(const double* __restrict__ dt, const double* __restrict__ qt,
                              T* __restrict__ sd, T* __restrict__ sq, int64_t n, int sym) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    sd[i] = (T)(sym ? 1.0 / sqrt(dt[i]) : 1.0 / dt[i]);
    if (!sym) sq[i] = (T)(1.0 / sqrt(qt[i]));
  }
}

// y = 1 / sqrt(x)
__global__ void k_rsqrt(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = 1.0 / sqrt(x[i]);
}

// C = I on the leading k x k block, zero elsewhere (symmetric normalisation);
// the whole identity when kptr is null.
__global__ void k_eye_k(double* __restrict__ C, int r, const int32_t* kptr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  const int k = kptr ? *kptr : r;
  C[e] = (i == j && i < k) ? 1.0 : 0.0;
}

// G = I on every row and column >= k (unused budget), as for G_B.
__global__ void k_pad_eye(double* __restrict__ G, int r, const int32_t* kptr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  const int k = *kptr;
  if (i >= k || j >= k) G[e] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_set_int(int32_t* p, int32_t v) { *p = v; }

// ---- spectral-projector restart of the subspace iteration
// When the subspace iteration has not met its residual test (eigenvalues
// clustered around the edge of the block, so the block converges slowly),
// the top part of the spectrum is split off exactly: X = sign(A) by the
// Newton-Schulz iteration X <- (3 X - X^3) / 2 on A = (M - sigma I) / s, with
// sigma in the widest gap of the current Ritz values theta_{nev-1} ..
// theta_{p-1} and s a bound on |M - sigma I| (the iteration converges for
// every eigenvalue of A in (-sqrt 3, sqrt 3) other than 0; a small one grows
// by 3/2 per step until it nears +-1, then the convergence is quadratic).
// Each iterate is formed on the tiles on and below the diagonal and mirrored,
// so it is exactly symmetric.  P = (I + X) / 2 projects onto the eigenvectors
// above sigma, so
// M' = (M - eps I) P + eps I keeps those eigenpairs and maps every other
// eigenvalue to eps = 1e-3 theta_{j-1} below sigma; four block products on M'
// then converge at the ratio eps / lambda, and the final Rayleigh-Ritz step
// and residual test use
// M itself.  Every kernel returns at once when `conv` is set (the usual case),
// and the Newton-Schulz steps once X^2 = I to 1e-10 (trace deficit).
constexpr int NS_MAX = 56;
constexpr int NS_TILES = 128;  // 64-wide diagonal tiles of an r x r product, r <= 8192

// fbp: [0] sigma, [1] 1 / s, [3] eps
__global__ void k_fb_setup(const double* __restrict__ theta, int p, int nev,
                           const double* __restrict__ delta, const int32_t* conv,
                           double* __restrict__ fbp, int32_t* nsdone, int32_t* nsfinal,
                           int32_t nsfinal0) {
  if (*conv || threadIdx.x != 0) return;
  int js = nev;
  double best = -1.0;
  for (int j = nev; j < p; ++j) {
    const double g = theta[j - 1] - theta[j];
    if (g > best) {
      best = g;
      js = j;
    }
  }
  const double sg = 0.5 * (theta[js - 1] + theta[js]);
  // the eigenvalues of M lie in [*delta, lambda_max]: M is the PSD inner
  // matrix plus the accumulated diagonal shift *delta, and the top Ritz value
  // theta_0 <= lambda_max is converged (the residual test failed lower down)
  double c = fmax(theta[0] - sg, sg - *delta);
  c = c > 0.0 ? c : 1.0;
  fbp[0] = sg;
  fbp[1] = 1.0 / (1.25 * c);
  fbp[2] = 0.0;
  fbp[3] = 1e-3 * fabs(theta[js - 1]);
  *nsdone = 0;
  *nsfinal = nsfinal0;
}

// X0 = (M - sigma I) / s, symmetrised; Mc = M.
__global__ void k_fb_x0(const double* __restrict__ M, int r, const double* __restrict__ fbp,
                        double* __restrict__ X0, double* __restrict__ Mc, const int32_t* conv) {
  if (*conv) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  const double m = M[e];
  Mc[e] = m;
  X0[e] = (0.5 * (m + M[j + (int64_t)i * r]) - (i == j ? fbp[0] : 0.0)) * fbp[1];
}

// T = X X (tiles on and below the diagonal, mirrored) with the trace deficit
// sum_i (1 - T_ii) of each diagonal tile in pd[bx].
__global__ __launch_bounds__(256) void k_ns_sq(int r, const double* __restrict__ X,
                                               double* __restrict__ T, double* __restrict__ pd,
                                               const int32_t* conv, const int32_t* nsdone) {
  if (*conv || *nsdone || blockIdx.x < blockIdx.y) return;
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, false, false>::bytes / sizeof(double)];
  __shared__ double red[4];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  // T(m, n) = sum_k X(m, k) X(n, k) (X symmetric)
  GOperand<double, false> a{X, r, r, r, nullptr, (r % 2) == 0};
  GOperand<double, false> b{X, r, r, r, nullptr, (r % 2) == 0};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, b, m0, n0, 0, r, smem);
  double dsum = 0.0;
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < r && n < r && m >= n) {
      T[m + n * r] = v;
      T[n + m * r] = v;
      if (m == n) dsum += 1.0 - v;
    }
  });
  if (blockIdx.x != blockIdx.y) return;
  dsum = wave_sum(dsum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dsum;
  __syncthreads();
  if (threadIdx.x == 0) pd[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Xn = (3 X - X T) / 2, unless the deficit of T = X^2 is below 1e-10: then X
// is the sign and the iteration stops (nsdone, nsfinal = the buffer of X).
__global__ __launch_bounds__(256) void k_ns_upd(int r, const double* __restrict__ X,
                                                const double* __restrict__ T,
                                                double* __restrict__ Xn,
                                                const double* __restrict__ pd, int nt, int cur,
                                                const int32_t* conv, int32_t* nsdone,
                                                int32_t* nsfinal) {
  if (*conv || *nsdone || blockIdx.x < blockIdx.y) return;
  __shared__ double dfc;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += pd[t];
    dfc = s;
  }
  __syncthreads();
  if (dfc <= 1e-10) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {  // a lower tile: runs
      *nsdone = 1;
      *nsfinal = cur;
    }
    return;
  }
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, false, false>::bytes / sizeof(double)];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  GOperand<double, false> a{X, r, r, r, nullptr, (r % 2) == 0};
  GOperand<double, false> b{T, r, r, r, nullptr, (r % 2) == 0};  // T symmetric: T(n, k) = T(k, n)
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, b, m0, n0, 0, r, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < r && n < r && m >= n) {
      const double x = 1.5 * X[m + n * r] - 0.5 * v;
      Xn[m + n * r] = x;
      Xn[n + m * r] = x;
    }
  });
}

// T = (Mc - eps I) (I + X) / 2 + eps I, X the final Newton-Schulz iterate.
__global__ __launch_bounds__(256) void k_fb_mprime(int r, const double* __restrict__ Mc,
                                                   const double* __restrict__ X0,
                                                   const double* __restrict__ X1,
                                                   const int32_t* nsfinal,
                                                   const double* __restrict__ fbp,
                                                   double* __restrict__ T, const int32_t* conv) {
  if (*conv) return;
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, false, false>::bytes / sizeof(double)];
  const double* X = *nsfinal ? X1 : X0;
  const double eps = fbp[3];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  GOperand<double, false> a{Mc, r, r, r, nullptr, (r % 2) == 0};
  GOperand<double, false> b{X, r, r, r, nullptr, (r % 2) == 0};  // X symmetric
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, b, m0, n0, 0, r, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < r && n < r) {
      const int64_t e = m + n * r;
      T[e] = 0.5 * (v - eps * X[e] + Mc[e]) + (m == n ? 0.5 * eps : 0.0);
    }
  });
}

// M = (T + T^T) / 2
__global__ void k_sym(const double* __restrict__ T, int r, double* __restrict__ M,
                      const int32_t* conv) {
  if (*conv) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  M[e] = 0.5 * (T[e] + T[j + (int64_t)i * r]);
}

__global__ void k_flag_noconv(const int32_t* conv, int32_t* status) {
  if (!*conv) set_status(status, RPC_ENOCONV);
}

// U = diag(dinv) F Z   (F: N x r, Z: r x nev column-major; dinv may be null)
// U = D~^{-1} F Z tile: 128 rows x 64 eigenvectors, eight waves of 64 x 16,
// Z converted to the product type beforehand; U written column by column.
template <typename T>
using FormUCfg = TileCfg<T, 128, 64, (sizeof(T) == 4 ? 32 : 16), 2, 4>;

template <typename T, typename TF, typename TU>
__global__ __launch_bounds__(FormUCfg<T>::NT) void k_form_u(const TF* __restrict__ F, int64_t ldf,
                                                            int64_t N, int r,
                                                            const T* __restrict__ Zt, int nev,
                                                            const double* __restrict__ dinv,
                                                            TU* __restrict__ U, int64_t ldu,
                                                            const int32_t* kptr) {
  typedef FormUCfg<T> Cfg;
  extern __shared__ char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  const int kk = kptr ? *kptr : r;  // columns >= k of F are zero
  GOperand<T, true> B{Zt, r, nev, kk, nullptr, (r % (16 / (int)sizeof(T))) == 0};
  TileAcc<Cfg> acc;
  acc.zero();
  GOperand<TF, false> A{F, ldf, N, kk, nullptr, true};
  tile_mainloop<Cfg>(acc, A, B, m0, n0, 0, kk, smem);
  store_colmajor<Cfg, TU>(acc, smem_raw, U, ldu, m0, n0, N, nev,
                          [&](int row, int, typename Cfg::MM::acc_t v) {
                            const int64_t m = m0 + row;
                            if (m >= N) return (TU)0;
                            return (TU)(dinv ? (double)v * dinv[m] : (double)v);
                          });
}

// U = diag(dinv) F Zt^T for the split-fp16 Gram form, on the fp16 MFMA pipe
// as split pairs (the Schur operands' pipe: F column-major, Zt with
// k-contiguous rows of leading dimension r).  F is scaled by 2^12 (its rows
// have norm at most 1), Zt by the power of two zsc[0] that puts its largest
// magnitude below 2^14.  Single LDS buffer, two workgroups per CU; each lane
// writes its four consecutive rows of a column directly.
typedef TileCfg<__bf16, 128, 128, 64, 2, 4> FormUSplitCfg;
// nev <= 64: four waves on 128 x 64 tiles, 48 KB of LDS, three workgroups per
// CU (half again the operand bytes in flight per CU of the eight-wave form)
typedef TileCfg<__bf16, 128, 64, 64, 2, 2> FormUSplitCfg64;

// With cpv/cpi non-null the kernel also writes, for each column, the largest
// |U| over its 128 rows and that row (the lowest on ties) to
// cpv/cpi[col * gridDim.x + blockIdx.x], the partials of the sign rule.
template <typename TU, class Cfg>
__global__ __launch_bounds__(Cfg::NT, Cfg::NT == 512 ? 4 : 3) void k_form_u_split(
    const float* __restrict__ F, int64_t ldf,
                                                         int64_t N, int r, const float* __restrict__ Zt,
                                                         int nev, const float* __restrict__ zsc,
                                                         const double* __restrict__ dinv,
                                                         TU* __restrict__ U, int64_t ldu,
                                                         const int32_t* kptr, double* __restrict__ cpv,
                                                         int64_t* __restrict__ cpi) {
  extern __shared__ char smem_raw[];
  const int kk = *kptr;
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  const int n0 = blockIdx.y * Cfg::BN;
  TileAcc<Cfg> acc;
  acc.zero();
  const float zs = zsc[0];
  if (kk > 0) {
    SchurSplitPipe<Cfg> pipe{F, ldf, N, Zt + (int64_t)n0 * r, r, nev - n0, kk, m0, zs};
    pipe.begin1();
    pipe.run1(acc, smem_raw);
  }
  const float un = 1.0f / (SchurSplit::SC * zs);  // both powers of two
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  double bv[Cfg::NI];
  int64_t bi[Cfg::NI];
#pragma unroll
  for (int j = 0; j < Cfg::NI; ++j) {
    bv[j] = -1.0;
    bi[j] = -1;
  }
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) {
      const int col = n0 + wn * Cfg::WTN + j * 16 + (lane & 15);
      if (col >= nev) continue;
      const int64_t m = m0 + wm * Cfg::WTM + i * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (m + e < N) {
          const double v = (double)(acc.a[i][j][e] * un);
          const TU u = (TU)(dinv ? v * dinv[m + e] : v);
          U[m + e + (int64_t)col * ldu] = u;
          // rows visited in increasing order: a strict > keeps the lowest on ties
          const double a = fabs(to_d(u));
          if (a > bv[j]) {
            bv[j] = a;
            bi[j] = m + e;
          }
        }
      }
    }
  if (!cpv) return;
  // combine the four row groups of a column (lanes l, l ^ 16, l ^ 32, l ^ 48),
  // then the two waves that share the column slice, through LDS
  double* sv = reinterpret_cast<double*>(smem_raw);
  int64_t* sx = reinterpret_cast<int64_t*>(sv + Cfg::NT / 64 * Cfg::WTN);
#pragma unroll
  for (int j = 0; j < Cfg::NI; ++j) {
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
      const double v2 = __shfl_xor(bv[j], o, 64);
      const int64_t i2 = __shfl_xor(bi[j], o, 64);
      if (i2 >= 0 && (bi[j] < 0 || v2 > bv[j] || (v2 == bv[j] && i2 < bi[j]))) {
        bv[j] = v2;
        bi[j] = i2;
      }
    }
    if (lane < 16) {
      sv[wave * Cfg::WTN + j * 16 + lane] = bv[j];
      sx[wave * Cfg::WTN + j * 16 + lane] = bi[j];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < Cfg::BN) {
    const int cwn = t / Cfg::WTN, cc = t % Cfg::WTN;
    const int col = n0 + t;
    double v = -1.0;
    int64_t ix = -1;
#pragma unroll
    for (int h = 0; h < Cfg::WAVES_M; ++h) {
      const int w2 = cwn * Cfg::WAVES_M + h;  // wave = wm + WAVES_M wn
      const double v2 = sv[w2 * Cfg::WTN + cc];
      const int64_t i2 = sx[w2 * Cfg::WTN + cc];
      if (i2 >= 0 && (ix < 0 || v2 > v || (v2 == v && i2 < ix))) {
        v = v2;
        ix = i2;
      }
    }
    if (col < nev) {
      cpv[(int64_t)col * gridDim.x + blockIdx.x] = v;
      cpi[(int64_t)col * gridDim.x + blockIdx.x] = ix;
    }
  }
}

// The regularised QR factors B' = D~^{-1} F + gamma E_k (E_k: ones at (i, i),
// i < k), so U = B' R^{-1} V = D~^{-1} F Z + gamma E_k Z with Z = R^{-1} V: rows
// i < k of U gain gamma Z[i, :].
template <typename TU>
__global__ void k_gamma_rows(TU* __restrict__ U, int64_t ldu, int64_t N,
                             const double* __restrict__ Z, int r, int nev,
                             const int32_t* __restrict__ kptr, double gamma) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * nev) return;
  const int i = (int)(e % r), j = (int)(e / r);
  if (i >= *kptr || i >= N) return;
  TU* u = U + i + (int64_t)j * ldu;
  *u = (TU)(to_d(*u) + gamma * Z[e]);
}

// out[0] = 2^e with max |x| 2^e < 2^14 (1 when x is all zero), one workgroup.
__global__ __launch_bounds__(1024) void k_pow2_scale(const float* __restrict__ x, int64_t n,
                                                     float* __restrict__ out) {
  __shared__ float red[1024];
  float m = 0.0f;
  for (int64_t e = threadIdx.x; e < n; e += 1024) m = fmaxf(m, fabsf(x[e]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float mx = red[0];
    float sc = 1.0f;
    if (mx > 0.0f && mx <= 3.0e38f) {
      int ex;
      frexpf(mx, &ex);
      int q = 14 - ex;
      q = q < -100 ? -100 : (q > 100 ? 100 : q);
      sc = ldexpf(1.0f, q);
    }
    out[0] = sc;
  }
}

template <typename T>
__global__ void k_cvt(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = (T)src[e];
}

// Column sign: find the largest |U[:, j]| (lowest index on ties).
template <typename TU>
__global__ __launch_bounds__(256) void k_colmax_partial(const TU* __restrict__ U, int64_t ldu,
                                                        int64_t N, int nev, double* __restrict__ pv,
                                                        int64_t* __restrict__ pi, int nb) {
  const int j = blockIdx.y;
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int64_t base = (int64_t)blockIdx.x * 4096;
  double bv = -1.0, bs = 0.0;
  int64_t bix = -1;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int64_t i = base + e;
    if (i < N) {
      const double v = to_d(U[i + j * ldu]);
      if (fabs(v) > bv) { bv = fabs(v); bix = i; bs = v; }
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bix;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double v2 = sv[threadIdx.x + off], v1 = sv[threadIdx.x];
      const int64_t i2 = si[threadIdx.x + off], i1 = si[threadIdx.x];
      if (i2 >= 0 && (i1 < 0 || v2 > v1 || (v2 == v1 && i2 < i1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  (void)bs;
  if (threadIdx.x == 0) {
    pv[(int64_t)j * nb + blockIdx.x] = sv[0];
    pi[(int64_t)j * nb + blockIdx.x] = si[0];
  }
}

template <typename TU>
__global__ __launch_bounds__(256) void k_colsign(const TU* __restrict__ U, int64_t ldu,
                                                 const double* __restrict__ pv,
                                                 const int64_t* __restrict__ pi, int nb,
                                                 double* __restrict__ sgn) {
  const int j = blockIdx.x;
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double bv = -1.0;
  int64_t bix = -1;
  for (int e = threadIdx.x; e < nb; e += 256) {
    const double v = pv[(int64_t)j * nb + e];
    const int64_t i = pi[(int64_t)j * nb + e];
    if (i >= 0 && (v > bv || (v == bv && (bix < 0 || i < bix)))) { bv = v; bix = i; }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bix;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double v2 = sv[threadIdx.x + off], v1 = sv[threadIdx.x];
      const int64_t i2 = si[threadIdx.x + off], i1 = si[threadIdx.x];
      if (i2 >= 0 && (i1 < 0 || v2 > v1 || (v2 == v1 && i2 < i1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sgn[j] = (si[0] >= 0 && to_d(U[si[0] + j * ldu]) < 0.0) ? -1.0 : 1.0;
}

template <typename TU>
__global__ __launch_bounds__(256) void k_apply_sign(TU* __restrict__ U, int64_t ldu, int64_t N,
                                                    int nev, const double* __restrict__ sgn) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N && sgn[j] < 0.0) U[i + j * ldu] = -U[i + j * ldu];
}

template <typename TU>
__global__ void k_const_col(TU* U, int64_t N, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) U[i] = (TU)v;
}

// E[:, j] = T[:, j] * sgn[j] / lambda[j]
__global__ void k_scale_E(double* E, int r, int nev, const double* sgn, const double* lam) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * nev) return;
  const int j = (int)(e / r);
  E[e] = E[e] * sgn[j] / lam[j];
}

struct EigWs {
  double *sd, *sq, *part, *part1, *GB, *C, *Gs, *Cs, *s, *T1, *M;
  void *ssd, *ssq;
  double *Q, *Y, *H, *Wm, *theta, *Gp, *Rinv, *Qt;
  double *V, *Z, *T2, *sgn, *pv;
  int64_t* pi;
  double* Ut;
  int32_t* conv;
  int32_t* cskip;  // per block step of the r x r Cholesky: nothing left inside k
  double* delta;
  double* sk;
  double* skq;  // split-K partials of the r x p block product
  float* gsc;   // per-chunk power-of-two scales of the split-fp16 Grams
  // Cholesky QR2: Q1 = B R1^{-1} (N x r), G2 = Q1^T Q1 = L2 L2^T, R1^{-1}
  double *Q1, *G2, *R1i, *sk2;
  int64_t ldq;
  // spectral-projector restart (subspace iteration only)
  double *Xa, *Xb, *Mc, *Tn, *fbp, *pd;
  int32_t *nsdone, *nsfinal;
  size_t part_cap;
  int p;
};

// gram_rows: rows of the factor one Gram launch covers (N, or the block
// rows of the low-memory form), which sizes the chunk partial buffers.
static size_t carve_eig(WsCursor& c, EigWs& w, int64_t N, int r, int nev, bool fix_const,
                        bool cholqr2, int64_t gram_rows = 0) {
  // block of the subspace iteration (r > JMAX): twice the wanted eigenpairs,
  // at least 64 and at most JMAX (the one-workgroup Rayleigh-Ritz limit)
  int pb = 2 * nev;
  pb = pb < 64 ? 64 : pb;
  pb = pb > dense::JMAX ? dense::JMAX : pb;
  w.p = r <= dense::JMAX ? r : pb;
  const int p = w.p;
  // sign-rule partials: one per 4096 rows, or one per 128-row tile of the split U kernel
  const int nbu = (int)((N + 127) / 128);
  w.sd = c.take<double>(N);
  w.sq = c.take<double>(N);
  w.ssd = c.take<double>(N);
  w.ssq = c.take<double>(N);
  w.part_cap = syrk::part_elems_any(gram_rows > 0 && gram_rows < N ? gram_rows : N, r);
  w.part = c.take<double>(w.part_cap);
  w.part1 = c.take<double>(w.part_cap);
  w.GB = c.take<double>((size_t)r * r);
  w.C = c.take<double>((size_t)r * r);
  w.Gs = c.take<double>((size_t)r * r);
  w.Cs = c.take<double>((size_t)r * r);
  w.s = c.take<double>(r);
  w.T1 = c.take<double>((size_t)r * r);
  w.M = c.take<double>((size_t)r * r);
  w.Q = c.take<double>((size_t)r * p);
  w.Y = c.take<double>((size_t)r * p);
  w.H = c.take<double>((size_t)p * p);
  w.Wm = c.take<double>((size_t)p * p);
  w.theta = c.take<double>(p);
  w.Gp = c.take<double>((size_t)p * p);
  w.Rinv = c.take<double>((size_t)p * p);
  w.Qt = c.take<double>((size_t)r * p);
  w.V = c.take<double>((size_t)r * nev);
  w.Z = c.take<double>((size_t)r * nev);
  w.T2 = c.take<double>((size_t)r * nev);
  w.sgn = c.take<double>(nev);
  w.pv = c.take<double>((size_t)nbu * nev);
  w.pi = c.take<int64_t>((size_t)nbu * nev);
  w.Ut = fix_const ? c.take<double>((size_t)align_up((size_t)N, 8) * nev) : nullptr;
  w.conv = c.take<int32_t>(1);
  w.cskip = c.take<int32_t>((size_t)(r + dense::NB - 1) / dense::NB);
  w.delta = c.take<double>(1);
  w.sk = c.take<double>((size_t)dense::SPLITK_MAX * p * p);
  w.skq = c.take<double>((size_t)dense::SPLITK_MAX * r * p);
  w.gsc = c.take<float>(2 * syrk::MAX_CHUNKS);
  w.ldq = (int64_t)align_up((size_t)N, 8);
  w.Q1 = cholqr2 ? c.take<double>((size_t)w.ldq * r) : nullptr;
  w.G2 = cholqr2 ? c.take<double>((size_t)r * r) : nullptr;
  w.R1i = cholqr2 ? c.take<double>((size_t)r * r) : nullptr;
  w.sk2 = cholqr2 ? c.take<double>((size_t)dense::SPLITK_MAX * dense::NB * r) : nullptr;
  const bool sub = r > dense::JMAX;
  w.Xa = sub ? c.take<double>((size_t)r * r) : nullptr;
  w.Xb = sub ? c.take<double>((size_t)r * r) : nullptr;
  w.Mc = sub ? c.take<double>((size_t)r * r) : nullptr;
  w.Tn = sub ? c.take<double>((size_t)r * r) : nullptr;
  w.fbp = c.take<double>(8);
  w.pd = c.take<double>(2 * NS_TILES);
  w.nsdone = c.take<int32_t>(1);
  w.nsfinal = c.take<int32_t>(1);
  return c.used;
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---- low-memory form: rows of the factor recomputed from the points
// The low-memory factorisation keeps only L = F(S, :) (r x r, lower
// triangular in pivot order).  Since F F^T interpolates K on the pivots,
// every row of the factor follows from the points as
//   F(x, :) = K(x, X_S) L^{-T},
// so a block of rows costs one MFMA distance product with an exp epilogue
// (k_cross_kernel) and one product with T = L^{-T}, computed once per call
// (rows and columns >= k of T are zero, so are the recomputed columns >= k).
// Everything is float64.

// T[i, j] = 0 for i >= k or j >= k
__global__ void k_zero_beyond_k(double* __restrict__ T, int r, const int32_t* kptr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int k = *kptr;
  const int i = (int)(e % r), j = (int)(e / r);
  if (i >= k || j >= k) T[e] = 0.0;
}

// A += B (first: A = B) over n entries, for two pairs at once (b1 may be null)
__global__ void k_accum2(double* __restrict__ a0, const double* __restrict__ b0,
                         double* __restrict__ a1, const double* __restrict__ b1, int64_t n,
                         int first) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  a0[e] = first ? b0[e] : a0[e] + b0[e];
  if (b1) a1[e] = first ? b1[e] : a1[e] + b1[e];
}

constexpr int64_t LM_BLOCK = 65536;  // default rows per recomputed block

struct LmRows {
  const rpc_points* X;
  const int64_t* piv;
  const int32_t* k;
  const double* FSlm;
  int64_t ldfs;
  int r;
  int64_t dp, blk;
  int32_t* status;
  double *XS, *xsn, *FS, *T, *Yp, *yn, *Kb, *Fb;

  static void carve(WsCursor& c, LmRows& l, int64_t N, int64_t d, int r, int64_t blk) {
    l.dp = (int64_t)align_up((size_t)d, 16);
    l.blk = blk < N ? blk : N;
    l.XS = c.take<double>((size_t)r * l.dp);
    l.xsn = c.take<double>(r);
    l.FS = c.take<double>((size_t)r * r);
    l.T = c.take<double>((size_t)r * r);
    l.Yp = c.take<double>((size_t)l.blk * l.dp);
    l.yn = c.take<double>(l.blk);
    l.Kb = c.take<double>((size_t)l.blk * r);
    l.Fb = c.take<double>((size_t)l.blk * r);
  }
  // pivot points, L with the identity beyond k, and T = L^{-T} zeroed beyond k
  void setup(hipStream_t st) const {
    with_points_type(X->dtype, [&](auto* tx) {
      typedef typename std::remove_const<typename std::remove_pointer<decltype(tx)>::type>::type TX;
      hipLaunchKernelGGL((k_gather_pivots<double, TX>), dim3(r), dim3(256), 0, st, (const TX*)X->X,
                         X->ldx, X->d, dp, piv, k, FSlm, ldfs, r, XS, xsn, FS, 1);
      return (int)RPC_OK;
    });
    hipLaunchKernelGGL(k_fill_identity, dim3(nblk((int64_t)r * r)), dim3(256), 0, st, T, r, r);
    dense::trsm_lt(st, FS, r, r, T, r, r);
    hipLaunchKernelGGL(k_zero_beyond_k, dim3(nblk((int64_t)r * r)), dim3(256), 0, st, T, r, k);
  }
  // Fb (m x r, leading dimension m) = rows m0 .. m0 + m - 1 of the factor
  void rows(hipStream_t st, int64_t m0, int64_t m) const {
    with_points_type(X->dtype, [&](auto* tx) {
      typedef typename std::remove_const<typename std::remove_pointer<decltype(tx)>::type>::type TX;
      hipLaunchKernelGGL((k_prep_rows64<TX>), dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st,
                         (const TX*)X->X + m0 * X->ldx, X->ldx, m, X->d, dp, Yp, yn, status);
      return (int)RPC_OK;
    });
    hipLaunchKernelGGL(k_cross_kernel, dim3((unsigned)((m + 63) / 64), (unsigned)((r + 63) / 64)),
                       dim3(256), 0, st, (const double*)Yp, (const double*)yn, m, dp,
                       (const double*)XS, (const double*)xsn, r, X->eps, Kb, m);
    dense::gemm64<false, true>(st, m, r, r, Kb, m, T, r, Fb, m, 1.0, 0.0);
  }
};

// Whether the eigensolver may synchronise `st` to read its convergence flag:
// not while the stream is being captured into a graph, and not while the
// batched form issues jobs (it must never block its issuing thread).
thread_local int t_host_gate_off = 0;
static bool host_gate_allowed(hipStream_t st) {
  if (t_host_gate_off) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusNone;
}

// Orthonormalise the r x p block Y into Q by Cholesky QR (Gram, one-workgroup
// Cholesky, row-parallel triangular solve).
static void chol_qr(hipStream_t st, const double* Y, double* Q, int r, int p, EigWs& w,
                    int32_t* status, const int32_t* skip) {
  dense::gemm64_splitk<true, true>(st, p, p, r, Y, r, Y, r, w.Gp, p, 1.0, 0.0, w.sk, skip);
  // column-scaled Cholesky of the Gram and the explicit inverse of its
  // triangular factor in one workgroup; Q = Y R^{-1} as an MFMA product
  hipLaunchKernelGGL(dense::k_chol_small, dim3(1), dim3(1024), 0, st, (const double*)w.Gp, (int64_t)p,
                     p, w.Rinv, (int64_t)p, status, skip, 1, 1);
  dense::gemm64<false, true>(st, r, p, p, Y, r, w.Rinv, p, Q, r, 1.0, 0.0, skip);
}

// lm: the low-memory form (F unused; TG = TF = double; CholQR only): the
// Grams and U are formed block by block from recomputed rows.  Its
// workspace follows the caller's LmRows carve.
template <typename TG, typename TF, typename TU>
static int run_eig(const TF* F, int64_t N, int64_t ldf, int r, const int32_t* k,
                   const double* dt, const double* qt, const rpc_eig_opts* o, TU* U, int64_t ldu,
                   double* lambda, double* ext_E, void* ws, size_t ws_bytes, int32_t* status,
                   hipStream_t st, const LmRows* lm = nullptr) {
  const int nev = o->nev;
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  EigWs w;
  const bool qr2 = o->qr_mode == RPC_QR_CHOLQR2;
  carve_eig(cur, w, N, r, nev, o->fix_const != 0, qr2, lm ? lm->blk : 0);
  if (!cur.ok) return RPC_EWORKSPACE;
  if (lm && (qr2 || !std::is_same<TG, double>::value || !std::is_same<TF, double>::value))
    return RPC_EINVAL;
  const int p = w.p;
  if (!syrk::gram2_fits<TG>(lm ? lm->blk : N, r, w.part_cap) ||
      (o->fix_const && !syrk::gram2_fits<double>(N, nev, w.part_cap)) ||
      (qr2 && !syrk::gram2_fits<double>(N, r, w.part_cap)))
    return RPC_EWORKSPACE;
  const int sym = o->normalization == RPC_SYMMETRIC;
  prof::begin(prof::SMALL, st);
  // w.sd holds the row scale of B: 1/d~ (bistochastic) or 1/sqrt(d~) (symmetric)
  if (sym)
    hipLaunchKernelGGL(k_rsqrt, dim3(nblk(N)), dim3(256), 0, st, dt, w.sd, N);
  else
    hipLaunchKernelGGL(k_recip, dim3(nblk(N)), dim3(256), 0, st, dt, w.sd, N);
  hipLaunchKernelGGL((k_gram_scales<TG>), dim3(nblk(N)), dim3(256), 0, st, dt, qt, (TG*)w.ssd,
                     (TG*)w.ssq, N, sym);
  prof::end(prof::SMALL, st);

  // ---- the N-long Grams: G_B = B^T B with B = D~^{-1} F (or D~^{-1/2} F), and
  // C = (Q~^{-1/2} F)^T (Q~^{-1/2} F) (bistochastic) or C = I (symmetric)
  const int nz = sym ? 1 : 2;
  prof::begin(prof::GRAM, st);
  if (lm) {
    // block by block: partial products of the recomputed rows, reduced into
    // Gs / Cs (free until the equilibration) and added into G_B / C
    int first = 1;
    for (int64_t m0 = 0; m0 < N; m0 += lm->blk, first = 0) {
      const int64_t m = N - m0 < lm->blk ? N - m0 : lm->blk;
      lm->rows(st, m0, m);
      syrk::gram2_partial<double, double>(st, lm->Fb, m, m, r, nz, (const double*)w.ssd + m0,
                                          sym ? nullptr : (const double*)w.ssq + m0, w.part, w.part1,
                                          k);
      syrk::gram2_reduce<double>(st, m, r, nz, w.part, w.part1, w.Gs, w.Cs, k);
      hipLaunchKernelGGL(k_accum2, dim3(nblk((int64_t)r * r)), dim3(256), 0, st, w.GB,
                         (const double*)w.Gs, w.C, sym ? (const double*)nullptr : (const double*)w.Cs,
                         (int64_t)r * r, first);
    }
  } else if constexpr (std::is_same<TG, float>::value && std::is_same<TF, float>::value) {
    if (o->gram_dtype == RPC_F32_SPLIT16)
      syrk::gram2_partial_split(st, F, ldf, N, r, nz, (const float*)w.ssd, (const float*)w.ssq,
                                w.gsc, w.part, w.part1, k);
    else
      syrk::gram2_partial<TG, TF>(st, F, ldf, N, r, nz, (const TG*)w.ssd, (const TG*)w.ssq, w.part,
                                  w.part1, k);
  } else {
    syrk::gram2_partial<TG, TF>(st, F, ldf, N, r, nz, (const TG*)w.ssd, (const TG*)w.ssq, w.part,
                                w.part1, k);
  }
  prof::end(prof::GRAM, st);
  const unsigned grr = nblk((int64_t)r * r);
  RPC_LAUNCH_CHECK();
  prof::begin(prof::SMALL, st);
  if (!lm) syrk::gram2_reduce<TG>(st, N, r, nz, w.part, w.part1, w.GB, w.C, k);
  if (sym) hipLaunchKernelGGL(k_eye_k, dim3(grr), dim3(256), 0, st, w.C, r, k);
  // the regularised QR reads rows 0 .. k-1 of F (recomputed in the low-memory form)
  const TF* Fg = F;
  int64_t ldg = ldf;
  if (lm && o->gamma != 0.0) {
    const int64_t m = N < lm->blk ? N : lm->blk;
    lm->rows(st, 0, m);
    Fg = reinterpret_cast<const TF*>(lm->Fb);
    ldg = m;
  }
  hipLaunchKernelGGL((k_gram_finish<TF>), dim3(grr), dim3(256), 0, st, w.GB, w.C, w.Gs, w.Cs, w.s,
                     r, k, Fg, ldg, N, (const double*)w.sd, o->gamma, 0);
  hipLaunchKernelGGL((k_gram_finish<TF>), dim3(grr), dim3(256), 0, st, w.GB, w.C, w.Gs, w.Cs, w.s,
                     r, k, F, ldf, N, (const double*)w.sd, o->gamma, 1);
  RPC_LAUNCH_CHECK();

  // ---- Cholesky QR in Gram space: S G_B S = L' L'^T, R = L'^T S^{-1}
  dense::cholesky(st, w.Gs, r, r, status, k, w.cskip);
  // M = R C R^T = L'^T (S^{-1} C S^{-1}) L'.  The Gram partial buffers are
  // free here; when they hold four r x r slices, each product is split over
  // four k ranges (four times the workgroups of an r x r tile grid).
  if (w.part_cap >= (size_t)4 * r * r) {
    dense::gemm64_splitk<false, true>(st, r, r, r, w.Cs, r, w.Gs, r, w.T1, r, 1.0, 0.0, w.part,
                                      nullptr, 4);
    dense::gemm64_splitk<true, true>(st, r, r, r, w.Gs, r, w.T1, r, w.M, r, 1.0, 0.0, w.part,
                                     nullptr, 4);
  } else {
    dense::gemm64<false, true>(st, r, r, r, w.Cs, r, w.Gs, r, w.T1, r, 1.0, 0.0);
    dense::gemm64<true, true>(st, r, r, r, w.Gs, r, w.T1, r, w.M, r, 1.0, 0.0);
  }
  RPC_LAUNCH_CHECK();
  if (qr2) {
    // Cholesky QR2: Q1 = B R1^{-1} formed explicitly (float64), its Gram
    // G2 = Q1^T Q1 = L2 L2^T, and R = R2 R1 with R2 = L2^T, so that
    // M = R C R^T = L2^T (R1 C R1^T) L2 and U = Q1 R2^{-1} V.
    // R1^{-1} = S L'^{-T}
    hipLaunchKernelGGL(k_eye_k, dim3(grr), dim3(256), 0, st, w.R1i, r, (const int32_t*)nullptr);
    dense::trsm_lt(st, w.Gs, r, r, w.R1i, r, r, w.sk2);
    hipLaunchKernelGGL(k_scale_rows, dim3(grr), dim3(256), 0, st, w.R1i, (int64_t)r, r, r,
                       (const double*)w.s, 0);
    typedef FormUCfg<double> CfgQ;
    size_t smQ = TileSmem<CfgQ, false, true>::bytes;
    if (ColStoreSmem<CfgQ, double>::bytes > smQ) smQ = ColStoreSmem<CfgQ, double>::bytes;
    const dim3 gq((unsigned)((N + CfgQ::BM - 1) / CfgQ::BM), (unsigned)((r + CfgQ::BN - 1) / CfgQ::BN));
    hipLaunchKernelGGL((k_form_u<double, TF, double>), gq, dim3(CfgQ::NT), smQ, st, F, ldf, N, r,
                       (const double*)w.R1i, r, (const double*)w.sd, w.Q1, w.ldq, k);
    if (o->gamma != 0.0)
      hipLaunchKernelGGL((k_gamma_rows<double>), dim3(grr), dim3(256), 0, st, w.Q1, w.ldq, N,
                         (const double*)w.R1i, r, r, k, o->gamma);
    syrk::gram2_partial<double, double>(st, (const double*)w.Q1, w.ldq, N, r, 1, (const double*)nullptr,
                                        (const double*)nullptr, w.part, w.part1, k);
    syrk::gram2_reduce<double>(st, N, r, 1, w.part, w.part1, w.G2, nullptr, k);
    hipLaunchKernelGGL(k_pad_eye, dim3(grr), dim3(256), 0, st, w.G2, r, k);
    dense::cholesky(st, w.G2, r, r, status, k, w.cskip);
    dense::gemm64<false, true>(st, r, r, r, w.M, r, w.G2, r, w.T1, r, 1.0, 0.0);
    dense::gemm64<true, true>(st, r, r, r, w.G2, r, w.T1, r, w.M, r, 1.0, 0.0);
    RPC_LAUNCH_CHECK();
  }

  // ---- top-nev eigenpairs of M
  prof::end(prof::SMALL, st);
  prof::begin(prof::EIG, st);
  const double jtol = 1e-13;  // relative off-diagonal Frobenius mass
  if (r <= dense::JMAX) {
    hipLaunchKernelGGL(dense::k_jacobi, dim3(1), dim3(1024), 0, st, (const double*)w.M, (int64_t)r,
                       r, w.theta, w.Wm, (int64_t)r, 40, jtol, status, (const int32_t*)nullptr);
    hipLaunchKernelGGL(k_copy_cols, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st,
                       (const double*)w.Wm, (int64_t)r, w.V, (int64_t)r, r, nev,
                       (const int32_t*)nullptr);
  } else {
    // subspace iteration with Rayleigh-Ritz on a p-dimensional block, on
    // M + delta I, orthonormalising every product by two Cholesky QR passes
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, w.conv, 0);
    hipLaunchKernelGGL(k_shift_diag, dim3(1), dim3(1024), 0, st, w.M, r, w.delta);
    hipLaunchKernelGGL(k_fill_identity, dim3(nblk((int64_t)r * p)), dim3(256), 0, st, w.Q, r, p);
    // 12 orthonormalised products, then Rayleigh-Ritz + residual check; up to
    // 3 more rounds of 6 products if the check fails (device flag `conv`)
    // The first product (from the identity start) can be ill-conditioned and
    // gets two column-scaled Cholesky QR passes; afterwards one scaled pass
    // keeps the span of the block (its orthonormality is restored by every
    // pass and checked where it matters, at the Rayleigh-Ritz step, whose
    // residual check guards the result).
    int done = 0;
    auto products = [&](int count) {
      for (int in = 0; in < count; ++in, ++done) {
        dense::gemm64_splitk<false, true>(st, r, p, r, w.M, r, w.Q, r, w.Y, r, 1.0, 0.0, w.skq,
                                          w.conv);
        if (done < 1) {
          chol_qr(st, w.Y, w.Qt, r, p, w, status, w.conv);
          chol_qr(st, w.Qt, w.Q, r, p, w, status, w.conv);
        } else {
          chol_qr(st, w.Y, w.Q, r, p, w, status, w.conv);
        }
      }
    };
    products(12);
    // Rayleigh-Ritz on the block and the residual test (sets conv)
    auto rayleigh_ritz = [&]() {
      dense::gemm64_splitk<false, true>(st, r, p, r, w.M, r, w.Q, r, w.Y, r, 1.0, 0.0, w.skq, w.conv);
      dense::gemm64_splitk<true, true>(st, p, p, r, w.Q, r, w.Y, r, w.H, p, 1.0, 0.0, w.sk, w.conv);
      hipLaunchKernelGGL(dense::k_jacobi, dim3(1), dim3(1024), 0, st, (const double*)w.H,
                         (int64_t)p, p, w.theta, w.Wm, (int64_t)p, 40, jtol, status,
                         (const int32_t*)w.conv);
      dense::gemm64<false, true>(st, r, p, p, w.Q, r, w.Wm, p, w.Qt, r, 1.0, 0.0, w.conv);
      dense::gemm64<false, true>(st, r, p, p, w.Y, r, w.Wm, p, w.T1, r, 1.0, 0.0, w.conv);
      hipLaunchKernelGGL(k_copy_cols, dim3(nblk((int64_t)r * p)), dim3(256), 0, st,
                         (const double*)w.Qt, (int64_t)r, w.Q, (int64_t)r, r, p,
                         (const int32_t*)w.conv);
      hipLaunchKernelGGL(k_ritz_check, dim3(1), dim3(1024), 0, st, (const double*)w.T1,
                         (const double*)w.Q, (const double*)w.theta, r, nev, 1e-10, w.conv);
    };
    // Outside stream capture and the batched form, the convergence flag is
    // read back to the host after each Rayleigh-Ritz step (one stream
    // synchronisation each), so the retries and the restart below are issued
    // only when needed; otherwise they are issued unconditionally and every
    // launch returns at once once `conv` is set.
    const bool gate = host_gate_allowed(st);
    auto converged = [&]() -> bool {
      int32_t h = 0;
      if (hipMemcpyAsync(&h, w.conv, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
      if (hipStreamSynchronize(st) != hipSuccess) return false;
      return h != 0;
    };
    bool conv_host = false;
    const int max_rr = 4;
    for (int it = 0; it < max_rr && !conv_host; ++it) {
      if (it > 0) products(6);
      rayleigh_ritz();
      if (it == 0)
        hipLaunchKernelGGL(k_shift_down, dim3(1), dim3(1024), 0, st, w.M, r, (const double*)w.theta,
                           p, w.delta, (const int32_t*)w.conv);
      if (gate) conv_host = converged();
    }
    // not converged: spectral-projector restart (every launch below returns
    // at once when conv is set)
    const unsigned grr2 = nblk((int64_t)r * r);
    if (!conv_host) {
    const dim3 gt((unsigned)((r + 63) / 64), (unsigned)((r + 63) / 64));
    hipLaunchKernelGGL(k_fb_setup, dim3(1), dim3(64), 0, st, (const double*)w.theta, p, nev,
                       (const double*)w.delta, (const int32_t*)w.conv, w.fbp, w.nsdone, w.nsfinal,
                       (int32_t)(NS_MAX % 2));
    hipLaunchKernelGGL(k_fb_x0, dim3(grr2), dim3(256), 0, st, (const double*)w.M, r,
                       (const double*)w.fbp, w.Xa, w.Mc, (const int32_t*)w.conv);
    double* xbuf[2] = {w.Xa, w.Xb};
    for (int i = 0; i < NS_MAX; ++i) {
      double* pdi = w.pd + (i % 2) * NS_TILES;
      hipLaunchKernelGGL(k_ns_sq, gt, dim3(256), 0, st, r, (const double*)xbuf[i % 2], w.Tn, pdi,
                         (const int32_t*)w.conv, (const int32_t*)w.nsdone);
      hipLaunchKernelGGL(k_ns_upd, gt, dim3(256), 0, st, r, (const double*)xbuf[i % 2],
                         (const double*)w.Tn, xbuf[(i + 1) % 2], (const double*)pdi, (int)gt.x, i % 2,
                         (const int32_t*)w.conv, w.nsdone, w.nsfinal);
    }
    hipLaunchKernelGGL(k_fb_mprime, gt, dim3(256), 0, st, r, (const double*)w.Mc, (const double*)w.Xa,
                       (const double*)w.Xb, (const int32_t*)w.nsfinal, (const double*)w.fbp, w.Tn,
                       (const int32_t*)w.conv);
    hipLaunchKernelGGL(k_sym, dim3(grr2), dim3(256), 0, st, (const double*)w.Tn, r, w.M,
                       (const int32_t*)w.conv);
    products(4);
    hipLaunchKernelGGL(k_copy_cols, dim3(grr2), dim3(256), 0, st, (const double*)w.Mc, (int64_t)r,
                       w.M, (int64_t)r, r, r, (const int32_t*)w.conv);
    rayleigh_ritz();
    }
    hipLaunchKernelGGL(k_unshift, dim3(1), dim3(128), 0, st, w.theta, p, (const double*)w.delta);
    hipLaunchKernelGGL(k_flag_noconv, dim3(1), dim3(1), 0, st, (const int32_t*)w.conv, status);
    hipLaunchKernelGGL(k_copy_cols, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st,
                       (const double*)w.Q, (int64_t)r, w.V, (int64_t)r, r, nev,
                       (const int32_t*)nullptr);
  }
  hipLaunchKernelGGL(k_copy_cols, dim3(nblk(nev)), dim3(256), 0, st, (const double*)w.theta,
                     (int64_t)nev, lambda, (int64_t)nev, nev, 1, (const int32_t*)nullptr);
  RPC_LAUNCH_CHECK();

  prof::end(prof::EIG, st);
  prof::begin(prof::FORM_U, st);
  // ---- Z = R^{-1} V = S L'^{-T} V ;  U = D~^{-1} F Z
  // (Cholesky QR2: Z = R2^{-1} V = L2^{-T} V, U = Q1 Z)
  hipLaunchKernelGGL(k_copy_cols, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st,
                     (const double*)w.V, (int64_t)r, w.Z, (int64_t)r, r, nev, (const int32_t*)nullptr);
  if (qr2) {
    dense::trsm_lt(st, w.G2, r, r, w.Z, r, nev, w.sk);
  } else {
    dense::trsm_lt(st, w.Gs, r, r, w.Z, r, nev, w.sk);  // w.sk holds >= SPLITK_MAX NB nev doubles
    hipLaunchKernelGGL(k_scale_rows, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st, w.Z, (int64_t)r,
                       r, nev, (const double*)w.s, 0);
  }
  typedef FormUCfg<TG> CfgU;
  const dim3 gu((unsigned)((N + CfgU::BM - 1) / CfgU::BM), (unsigned)((nev + CfgU::BN - 1) / CfgU::BN));
  size_t smU = TileSmem<CfgU, false, true>::bytes;
  if (ColStoreSmem<CfgU, TU>::bytes > smU) smU = ColStoreSmem<CfgU, TU>::bytes;
  // Z in the product type (the scratch T2 is free until the extension matrix)
  TG* Zt = reinterpret_cast<TG*>(w.T2);
  hipLaunchKernelGGL((k_cvt<TG>), dim3(nblk((int64_t)r * nev)), dim3(256), 0, st, (const double*)w.Z,
                     Zt, (int64_t)r * nev);
  bool split_u = false;
  // the split U kernel also finds the column maxima of the sign rule when
  // nothing changes U after it (no gamma rows, no constant column)
  const bool fused_sign = o->gamma == 0.0 && !o->fix_const && !qr2 && !lm;
  const unsigned nbt = (unsigned)((N + 127) / 128);
  if (qr2) {
    typedef FormUCfg<double> CfgQ;
    size_t smQ = TileSmem<CfgQ, false, true>::bytes;
    if (ColStoreSmem<CfgQ, TU>::bytes > smQ) smQ = ColStoreSmem<CfgQ, TU>::bytes;
    const dim3 gq((unsigned)((N + CfgQ::BM - 1) / CfgQ::BM), (unsigned)((nev + CfgQ::BN - 1) / CfgQ::BN));
    hipLaunchKernelGGL((k_form_u<double, double, TU>), gq, dim3(CfgQ::NT), smQ, st, (const double*)w.Q1,
                       w.ldq, N, r, (const double*)w.Z, nev, (const double*)nullptr, U, ldu, k);
  }
  if constexpr (std::is_same<TG, float>::value && std::is_same<TF, float>::value) {
    if (!qr2 && o->gram_dtype == RPC_F32_SPLIT16) {
      // the split-fp16 form forms U on the fp16 pipe as well
      split_u = true;
      hipLaunchKernelGGL(k_pow2_scale, dim3(1), dim3(1024), 0, st, (const float*)Zt,
                         (int64_t)r * nev, w.gsc);
      auto launch_u = [&](auto cfg) {
        typedef decltype(cfg) Cfg;
        const dim3 gs((unsigned)((N + 127) / 128), (unsigned)((nev + Cfg::BN - 1) / Cfg::BN));
        hipLaunchKernelGGL((k_form_u_split<TU, Cfg>), gs, dim3(Cfg::NT),
                           SchurSplitPipe<Cfg>::single_bytes, st, (const float*)F, ldf, N, r,
                           (const float*)Zt, nev, (const float*)w.gsc, (const double*)w.sd, U, ldu, k,
                           fused_sign ? w.pv : (double*)nullptr, fused_sign ? w.pi : (int64_t*)nullptr);
      };
      if (nev <= 64)
        launch_u(FormUSplitCfg64{});
      else
        launch_u(FormUSplitCfg{});
    }
  }
  if (lm) {
    for (int64_t m0 = 0; m0 < N; m0 += lm->blk) {
      const int64_t m = N - m0 < lm->blk ? N - m0 : lm->blk;
      lm->rows(st, m0, m);
      const dim3 gm((unsigned)((m + CfgU::BM - 1) / CfgU::BM), gu.y);
      hipLaunchKernelGGL((k_form_u<TG, double, TU>), gm, dim3(CfgU::NT), smU, st,
                         (const double*)lm->Fb, m, m, r, (const TG*)Zt, nev,
                         (const double*)w.sd + m0, U + m0, ldu, k);
    }
  } else if (!split_u && !qr2) {
    hipLaunchKernelGGL((k_form_u<TG, TF, TU>), gu, dim3(CfgU::NT), smU, st, F, ldf, N, r,
                       (const TG*)Zt, nev, (const double*)w.sd, U, ldu, k);
  }
  if (o->gamma != 0.0 && !qr2)
    hipLaunchKernelGGL((k_gamma_rows<TU>), dim3(nblk((int64_t)r * nev)), dim3(256), 0, st, U, ldu, N,
                       (const double*)w.Z, r, nev, k, o->gamma);
  RPC_LAUNCH_CHECK();

  if (o->fix_const) {
    // U(:, 0) = 1/sqrt(N), then Cholesky QR with positive diag(R)
    hipLaunchKernelGGL((k_const_col<TU>), dim3(nblk(N)), dim3(256), 0, st, U, N, 1.0 / sqrt((double)N));
    syrk::gram2_partial<double, TU>(st, (const TU*)U, ldu, N, nev, 1, (const double*)nullptr,
                                    (const double*)nullptr, w.part, w.part1);
    syrk::gram2_reduce<double>(st, N, nev, 1, w.part, w.part1, w.Gp, nullptr);
    hipLaunchKernelGGL(dense::k_chol_small, dim3(1), dim3(1024), 0, st, (const double*)w.Gp,
                       (int64_t)nev, nev, w.Rinv, (int64_t)nev, status, (const int32_t*)nullptr);
    const int64_t ldut = (int64_t)align_up((size_t)N, 8);
    hipLaunchKernelGGL(k_copy_cols, dim3(nblk(N * nev)), dim3(256), 0, st, (const double*)U, ldu,
                       w.Ut, ldut, (int)N, nev, (const int32_t*)nullptr);
    if constexpr (std::is_same<TU, double>::value) {
      hipLaunchKernelGGL(dense::k_trsm_rows, dim3((unsigned)((N + 63) / 64)), dim3(64), 0, st,
                         (const double*)w.Ut, ldut, (int)N, nev, (const double*)w.Rinv,
                         (int64_t)nev, U, ldu, (const int32_t*)nullptr);
    }
    RPC_LAUNCH_CHECK();
  }

  // ---- column signs: largest-magnitude entry positive
  int nbu = (int)((N + 4095) / 4096);
  if (split_u && fused_sign) {
    nbu = (int)nbt;  // partials of the 128-row tiles, written by k_form_u_split
  } else {
    hipLaunchKernelGGL((k_colmax_partial<TU>), dim3((unsigned)nbu, (unsigned)nev), dim3(256), 0, st,
                       (const TU*)U, ldu, N, nev, w.pv, w.pi, nbu);
  }
  hipLaunchKernelGGL((k_colsign<TU>), dim3((unsigned)nev), dim3(256), 0, st, (const TU*)U, ldu,
                     (const double*)w.pv, (const int64_t*)w.pi, nbu, w.sgn);
  hipLaunchKernelGGL((k_apply_sign<TU>), dim3(nblk(N), (unsigned)nev), dim3(256), 0, st, U, ldu, N,
                     nev, (const double*)w.sgn);
  prof::end(prof::FORM_U, st);
  RPC_LAUNCH_CHECK();

  // ---- extension matrix E = C R^T V Lambda^{-1} (signed like U); R^T = S^{-1} L'
  // (Cholesky QR2: R^T V = S^{-1} L' (L2 V))
  const double* Vr = w.V;
  if (qr2) {
    dense::gemm64<false, true>(st, r, nev, r, w.G2, r, w.V, r, w.Z, r, 1.0, 0.0);
    Vr = w.Z;
  }
  dense::gemm64<false, true>(st, r, nev, r, w.Gs, r, Vr, r, w.T2, r, 1.0, 0.0);
  hipLaunchKernelGGL(k_scale_rows, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st, w.T2, (int64_t)r,
                     r, nev, (const double*)w.s, 1);
  dense::gemm64<false, true>(st, r, nev, r, w.C, r, w.T2, r, ext_E, r, 1.0, 0.0);
  hipLaunchKernelGGL(k_scale_E, dim3(nblk((int64_t)r * nev)), dim3(256), 0, st, ext_E, r, nev,
                     (const double*)w.sgn, (const double*)lambda);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

// chunks of the partial column sums
static int degree_chunks(int64_t N) { return (int)((N + COLCHUNK - 1) / COLCHUNK); }

template <typename TF>
static int run_degrees(const TF* F, int64_t N, int64_t ldf, int r, const int32_t* k, double* c,
                       double* dt, double* qt, void* ws, size_t ws_bytes, int32_t* status,
                       hipStream_t st) {
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  const int nch = degree_chunks(N);
  double* part = cur.take<double>((size_t)nch * r);
  double* inv = cur.take<double>((size_t)N);
  double* wv = cur.take<double>((size_t)r);
  if (!cur.ok) return RPC_EWORKSPACE;
  const dim3 gc((unsigned)nch, (unsigned)((r + 15) / 16));
  const size_t sh = (size_t)r * sizeof(double);
  prof::begin(prof::DEGREES, st);
  hipLaunchKernelGGL((k_coldot_partial<TF>), gc, dim3(1024), 0, st, F, ldf, N, r, k,
                     (const double*)nullptr, part);
  hipLaunchKernelGGL(k_reduce_cols, dim3((r + 255) / 256), dim3(256), 0, st, (const double*)part, nch,
                     r, c);
  hipLaunchKernelGGL((k_rowdot<TF>), dim3(nblk(N)), dim3(256), sh, st, F, ldf, N, r, k,
                     (const double*)c, dt, inv, (int32_t)RPC_EDEGREE, status);
  hipLaunchKernelGGL((k_coldot_partial<TF>), gc, dim3(1024), 0, st, F, ldf, N, r, k,
                     (const double*)inv, part);
  hipLaunchKernelGGL(k_reduce_cols, dim3((r + 255) / 256), dim3(256), 0, st, (const double*)part, nch,
                     r, wv);
  hipLaunchKernelGGL((k_rowdot<TF>), dim3(nblk(N)), dim3(256), sh, st, F, ldf, N, r, k,
                     (const double*)wv, qt, (double*)nullptr, (int32_t)RPC_EQDEGREE, status);
  prof::end(prof::DEGREES, st);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

// The degree passes of Algorithm 1 over recomputed rows: pass 1 c = F^T 1;
// pass 2 d~ = F c (asserted > 0) and w = F^T (1/d~); pass 3 q~ = F w
// (asserted > 0).  Blocks start at multiples of COLCHUNK, so the partial
// column sums of block b land at chunk m0 / COLCHUNK of one buffer and are
// reduced in the same order as in run_degrees.
static int run_degrees_lm(const LmRows& lm, int64_t N, int r, const int32_t* k, double* c,
                          double* dt, double* qt, double* part, double* inv, double* wv,
                          int32_t* status, hipStream_t st) {
  const int nch = degree_chunks(N);
  const size_t sh = (size_t)r * sizeof(double);
  prof::begin(prof::DEGREES, st);
  for (int pass = 0; pass < 3; ++pass) {
    for (int64_t m0 = 0; m0 < N; m0 += lm.blk) {
      const int64_t m = N - m0 < lm.blk ? N - m0 : lm.blk;
      lm.rows(st, m0, m);
      const dim3 gc((unsigned)((m + COLCHUNK - 1) / COLCHUNK), (unsigned)((r + 15) / 16));
      double* pb = part + (m0 / COLCHUNK) * r;
      if (pass == 0) {
        hipLaunchKernelGGL((k_coldot_partial<double>), gc, dim3(1024), 0, st, (const double*)lm.Fb, m,
                           m, r, k, (const double*)nullptr, pb);
      } else if (pass == 1) {
        hipLaunchKernelGGL((k_rowdot<double>), dim3(nblk(m)), dim3(256), sh, st, (const double*)lm.Fb,
                           m, m, r, k, (const double*)c, dt + m0, inv + m0, (int32_t)RPC_EDEGREE,
                           status);
        hipLaunchKernelGGL((k_coldot_partial<double>), gc, dim3(1024), 0, st, (const double*)lm.Fb, m,
                           m, r, k, (const double*)inv + m0, pb);
      } else {
        hipLaunchKernelGGL((k_rowdot<double>), dim3(nblk(m)), dim3(256), sh, st, (const double*)lm.Fb,
                           m, m, r, k, (const double*)wv, qt + m0, (double*)nullptr,
                           (int32_t)RPC_EQDEGREE, status);
      }
    }
    if (pass < 2)
      hipLaunchKernelGGL(k_reduce_cols, dim3((r + 255) / 256), dim3(256), 0, st, (const double*)part,
                         nch, r, pass == 0 ? c : wv);
  }
  prof::end(prof::DEGREES, st);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

static size_t degrees_ws(int64_t N, int r) {
  WsCursor c{nullptr, 0, 0, true};
  c.take<double>((size_t)degree_chunks(N) * r);
  c.take<double>((size_t)N);
  c.take<double>((size_t)r);
  return c.used;
}

static int check_eig_opts(int64_t N, int r, const rpc_eig_opts* o) {
  if (!o || N < 1 || r < 1 || r > N || r > 8192) return RPC_EINVAL;
  if (o->nev < 1 || o->nev > r) return RPC_EINVAL;
  if (r > dense::JMAX && o->nev > 64) return RPC_EINVAL;
  if (o->gram_dtype != RPC_F64 && o->gram_dtype != RPC_F32 && o->gram_dtype != RPC_F32_SPLIT16)
    return RPC_EINVAL;
  if (o->u_dtype != RPC_F64 && o->u_dtype != RPC_F32) return RPC_EINVAL;
  if (o->fix_const && o->u_dtype != RPC_F64) return RPC_EINVAL;
  if (!(o->gamma >= 0.0)) return RPC_EINVAL;
  if (o->normalization != RPC_BISTOCHASTIC && o->normalization != RPC_SYMMETRIC) return RPC_EINVAL;
  if (o->normalization == RPC_SYMMETRIC && o->fix_const) return RPC_EINVAL;
  if (o->qr_mode != RPC_QR_CHOLQR && o->qr_mode != RPC_QR_CHOLQR2) return RPC_EINVAL;
  return RPC_OK;
}

}  // namespace

extern "C" int bistoch_degrees_workspace_size(int64_t N, int32_t r, size_t* bytes) {
  if (N < 1 || r < 1 || !bytes) return RPC_EINVAL;
  *bytes = degrees_ws(N, r);
  return RPC_OK;
}

extern "C" int bistoch_degrees(const void* F, int32_t fdt, int64_t N, int64_t ldf, int32_t r,
                               const int32_t* k, double* c, double* dt, double* qt, void* ws,
                               size_t ws_bytes, int32_t* status, rpc_stream_t stream) {
  if (!F || !k || !c || !dt || !qt || !status || N < 1 || r < 1 || r > N || ldf < N) return RPC_EINVAL;
  if (r > 8192) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (fdt == RPC_F64)
    return run_degrees<double>((const double*)F, N, ldf, r, k, c, dt, qt, ws, ws_bytes, status, st);
  if (fdt == RPC_F32)
    return run_degrees<float>((const float*)F, N, ldf, r, k, c, dt, qt, ws, ws_bytes, status, st);
  return RPC_EINVAL;
}

// ---- bistoch_degrees with library-owned scratch (no workspace argument)
// The partial column sums, 1/d~ and w live in one file-scope device array,
// sized for N <= 2^20 and r <= 1024: 128 chunks x 1024 partial sums, 2^20
// reciprocals and 1024 weights, each block rounded up to 256 bytes.
namespace {
constexpr int64_t NOALLOC_MAX_N = int64_t(1) << 20;
constexpr int NOALLOC_MAX_R = 1024;
constexpr size_t NOALLOC_BYTES = size_t(128) * 1024 * 8 + (size_t(1) << 20) * 8 + 1024 * 8 + 3 * 256;
constexpr int NOALLOC_MAX_DEV = 64;
}  // namespace

static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_ptr_current(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEV) return RPC_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return RPC_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RPC_OK;
}
}  // namespace

extern "C" int bistoch_degrees_noalloc(const void* F, int32_t fdt, int64_t N, int64_t ldf, int32_t r,
                                       const int32_t* k, double* c, double* dt, double* qt,
                                       int32_t* status, rpc_stream_t stream) {
  if (!F || !k || !c || !dt || !qt || !status || N < 1 || r < 1 || r > N || ldf < N) return RPC_EINVAL;
  if (fdt != RPC_F64 && fdt != RPC_F32) return RPC_EINVAL;
  if (N > NOALLOC_MAX_N || r > NOALLOC_MAX_R || degrees_ws(N, r) > NOALLOC_BYTES) return RPC_EWORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int dev = 0;
  RPC_HIP_CHECK(hipGetDevice(&dev));
  if (st) {
    int sdev = -1;
    RPC_HIP_CHECK(hipStreamGetDevice(st, &sdev));
    if (sdev != dev) return RPC_EINVAL;
  }
  void* ws = nullptr;
  const int rc = scratch_ptr_current(&ws);
  if (rc != RPC_OK) return rc;
  // every scratch entry the kernels read is written earlier in the same call,
  // so nothing needs clearing
  if (fdt == RPC_F64)
    return run_degrees<double>((const double*)F, N, ldf, r, k, c, dt, qt, ws, NOALLOC_BYTES, status, st);
  return run_degrees<float>((const float*)F, N, ldf, r, k, c, dt, qt, ws, NOALLOC_BYTES, status, st);
}

// ---- Algorithm 1 from the low-memory factor
namespace {
struct LmLayout {
  LmRows rows;
  double *part, *inv, *wv;
  size_t eig_off;  // start of run_eig's workspace (256-aligned)
};
int64_t lm_block_rows(int64_t block_rows) { return block_rows > 0 ? block_rows : LM_BLOCK; }
size_t carve_lm(WsCursor& c, LmLayout& l, int64_t N, int64_t d, int r, int64_t blk) {
  LmRows::carve(c, l.rows, N, d, r, blk);
  const int nch = (int)((N + COLCHUNK - 1) / COLCHUNK);
  l.part = c.take<double>((size_t)nch * r);
  l.inv = c.take<double>((size_t)N);
  l.wv = c.take<double>((size_t)r);
  l.eig_off = align_up(c.used, 256);
  return l.eig_off;
}
int check_lm_args(const rpc_points* X, int r, const rpc_eig_opts* o, int64_t block_rows) {
  if (!X || !X->X || X->N < 1 || X->d < 1 || X->ldx < X->d || !(X->eps > 0.0)) return RPC_EINVAL;
  if (X->dtype != RPC_F32 && X->dtype != RPC_F64 && X->dtype != RPC_BF16) return RPC_EINVAL;
  int rc = check_eig_opts(X->N, r, o);
  if (rc) return rc;
  if (o->gram_dtype != RPC_F64 || o->qr_mode != RPC_QR_CHOLQR) return RPC_EINVAL;
  if (block_rows < 0 || block_rows % COLCHUNK != 0) return RPC_EINVAL;
  if (block_rows > 0 && block_rows < r && block_rows < X->N) return RPC_EINVAL;
  return RPC_OK;
}
}  // namespace

extern "C" int bistoch_lowmem_workspace_size(const rpc_points* X, int32_t r, const rpc_eig_opts* o,
                                             int64_t block_rows, size_t* bytes) {
  int rc = check_lm_args(X, r, o, block_rows);
  if (rc) return rc;
  if (!bytes) return RPC_EINVAL;
  const int64_t blk = lm_block_rows(block_rows);
  WsCursor c{nullptr, 0, 0, true};
  LmLayout l;
  carve_lm(c, l, X->N, X->d, r, blk);
  WsCursor e{nullptr, 0, 0, true};
  EigWs w;
  carve_eig(e, w, X->N, r, o->nev, o->fix_const != 0, false, blk < X->N ? blk : X->N);
  *bytes = l.eig_off + e.used;
  return RPC_OK;
}

extern "C" int bistoch_lowmem(const rpc_points* X, const int64_t* pivots, const int32_t* k,
                              const double* FS, int64_t ldfs, int32_t r, const rpc_eig_opts* o,
                              int64_t block_rows, double* c, double* dt, double* qt, void* U,
                              int64_t ldu, double* lambda, double* ext_E, void* ws, size_t ws_bytes,
                              int32_t* status, rpc_stream_t stream) {
  int rc = check_lm_args(X, r, o, block_rows);
  if (rc) return rc;
  const int64_t N = X->N;
  if (!pivots || !k || !FS || !c || !dt || !U || !lambda || !ext_E || !status) return RPC_EINVAL;
  if (!qt && o->normalization != RPC_SYMMETRIC) return RPC_EINVAL;
  if (ldfs < r || ldu < N || ldu % 8 != 0) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t blk = lm_block_rows(block_rows);
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  LmLayout l;
  carve_lm(cur, l, N, X->d, r, blk);
  if (!cur.ok || ws_bytes < l.eig_off) return RPC_EWORKSPACE;
  l.rows.X = X;
  l.rows.piv = pivots;
  l.rows.k = k;
  l.rows.FSlm = FS;
  l.rows.ldfs = ldfs;
  l.rows.r = r;
  l.rows.status = status;
  l.rows.setup(st);
  RPC_LAUNCH_CHECK();
  // the symmetric normalisation needs only d~; q~ is formed all the same
  double* qv = qt ? qt : l.inv;
  rc = run_degrees_lm(l.rows, N, r, k, c, dt, qv, l.part, l.inv, l.wv, status, st);
  if (rc) return rc;
  void* ews = (char*)ws + l.eig_off;
  const size_t ebytes = ws_bytes - l.eig_off;
  if (o->u_dtype == RPC_F64)
    return run_eig<double, double, double>(nullptr, N, N, r, k, dt, qt, o, (double*)U, ldu, lambda,
                                           ext_E, ews, ebytes, status, st, &l.rows);
  return run_eig<double, double, float>(nullptr, N, N, r, k, dt, qt, o, (float*)U, ldu, lambda, ext_E,
                                        ews, ebytes, status, st, &l.rows);
}

extern "C" int bistoch_eig_workspace_size(int64_t N, int32_t r, const rpc_eig_opts* o, size_t* bytes) {
  int rc = check_eig_opts(N, r, o);
  if (rc) return rc;
  if (!bytes) return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  EigWs w;
  *bytes = carve_eig(c, w, N, r, o->nev, o->fix_const != 0, o->qr_mode == RPC_QR_CHOLQR2);
  return RPC_OK;
}

extern "C" int bistoch_eig(const void* F, int32_t fdt, int64_t N, int64_t ldf, int32_t r,
                           const int32_t* k, const double* c, const double* dt, const double* qt,
                           const rpc_eig_opts* o, void* U, int64_t ldu, double* lambda,
                           double* ext_E, void* ws, size_t ws_bytes, int32_t* status,
                           rpc_stream_t stream) {
  int rc = check_eig_opts(N, r, o);
  if (rc) return rc;
  (void)c;
  if (!F || !k || !dt || !U || !lambda || !ext_E || !status) return RPC_EINVAL;
  if (!qt && !(o && o->normalization == RPC_SYMMETRIC)) return RPC_EINVAL;
  if (ldf < N || ldf % 8 != 0 || ldu < N || ldu % 8 != 0) return RPC_EINVAL;
  if (fdt != RPC_F64 && fdt != RPC_F32) return RPC_EINVAL;
  if (o->gram_dtype == RPC_F32_SPLIT16 && fdt != RPC_F32) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool g64 = o->gram_dtype == RPC_F64;
  const bool u64 = o->u_dtype == RPC_F64;
#define RPC_EIG_CALL(TG, TF, TU)                                                                  \
  return run_eig<TG, TF, TU>((const TF*)F, N, ldf, r, k, dt, qt, o, (TU*)U, ldu, lambda, ext_E, ws, \
                             ws_bytes, status, st)
  if (fdt == RPC_F64) {
    if (g64) { if (u64) RPC_EIG_CALL(double, double, double); else RPC_EIG_CALL(double, double, float); }
    if (u64) RPC_EIG_CALL(float, double, double); else RPC_EIG_CALL(float, double, float);
  } else {
    if (g64) { if (u64) RPC_EIG_CALL(double, float, double); else RPC_EIG_CALL(double, float, float); }
    if (u64) RPC_EIG_CALL(float, float, double); else RPC_EIG_CALL(float, float, float);
  }
#undef RPC_EIG_CALL
}

namespace rpc_internal {
void set_host_gate_off(bool off) { t_host_gate_off = off ? 1 : 0; }
}  // namespace rpc_internal
