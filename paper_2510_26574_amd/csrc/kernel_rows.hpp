// Rows of the kernel matrix against the accepted pivots, in float64, shared
// by the Nystrom extension and the low-memory form of Algorithm 1: gather of
// the pivot points and of F(S, :), conversion of a block of points, and the
// block K(Y, X_S) as an MFMA distance product with an exp epilogue.
#pragma once
#include <math.h>

#include "common.hpp"
#include "tile_gemm.hpp"

namespace {

// XS[i][:] = X[piv[i]][:] (i < k; zero rows beyond), xsn[i] = |XS[i]|^2;
// FS (r x r column-major) = F(S, :) on the leading k x k block, identity beyond.
// F is the N x r factor (row of pivot i at piv[i]) or, with `pivot_rows`, the
// r x r F(S, :) of the low-memory form (row of pivot i at i).
template <typename TF, typename TX>
__global__ __launch_bounds__(256) void k_gather_pivots(const TX* __restrict__ X, int64_t ldx,
                                                       int64_t d, int64_t dp,
                                                       const int64_t* __restrict__ piv,
                                                       const int32_t* kptr,
                                                       const TF* __restrict__ F, int64_t ldf,
                                                       int r, double* __restrict__ XS,
                                                       double* __restrict__ xsn,
                                                       double* __restrict__ FS,
                                                       int pivot_rows = 0) {
  const int i = blockIdx.x;
  const int k = *kptr;
  __shared__ double red[4];
  double s = 0.0;
  const int64_t p = i < k ? piv[i] : -1;
  for (int64_t c = threadIdx.x; c < dp; c += 256) {
    const double v = (p >= 0 && c < d) ? ld_point(X, p * ldx + c) : 0.0;
    XS[(int64_t)i * dp + c] = v;
    s += v * v;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) xsn[i] = red[0] + red[1] + red[2] + red[3];
  for (int j = threadIdx.x; j < r; j += 256) {
    double v;
    if (i < k && j < k)
      v = to_d(F[(pivot_rows ? (int64_t)i : p) + (int64_t)j * ldf]);
    else
      v = (i == j) ? 1.0 : 0.0;
    FS[i + (int64_t)j * r] = v;
  }
}

template <typename TX>
__global__ __launch_bounds__(256) void k_prep_rows64(const TX* __restrict__ Y, int64_t ldy,
                                                     int64_t m, int64_t d, int64_t dp,
                                                     double* __restrict__ Yp,
                                                     double* __restrict__ yn, int32_t* status) {
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= m) return;
  double s = 0.0;
  bool bad = false;
  for (int64_t j = lane; j < dp; j += 64) {
    const double v = j < d ? ld_point(Y, n * ldy + j) : 0.0;
    if (!isfinite(v)) bad = true;
    Yp[n * dp + j] = v;
    s += v * v;
  }
  s = wave_sum(s);
  if (__any(bad) && lane == 0) set_status(status, RPC_ENONFINITE);
  if (lane == 0) yn[n] = s;
}

// Kys[m][i] = exp(-max(0, yn + xsn - 2 <y, x_i>) / eps), column-major m x r.
__global__ __launch_bounds__(256) void k_cross_kernel(const double* __restrict__ Yp,
                                                      const double* __restrict__ yn, int64_t m,
                                                      int64_t dp, const double* __restrict__ XS,
                                                      const double* __restrict__ xsn, int r,
                                                      double eps, double* __restrict__ K,
                                                      int64_t ldk) {
  typedef TileCfg<double, 64, 64, 16, 2, 2> Cfg;
  __shared__ double smem[TileSmem<Cfg, true, true>::bytes / sizeof(double)];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM, n0 = (int64_t)blockIdx.y * Cfg::BN;
  GOperand<double, true> A{Yp, dp, m, dp, nullptr, true};
  GOperand<double, true> B{XS, dp, r, dp, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, A, B, m0, n0, 0, dp, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, double v) {
    const int64_t i = m0 + row, j = n0 + col;
    if (i < m && j < r) {
      double d2 = yn[i] + xsn[j] - 2.0 * v;
      d2 = d2 > 0.0 ? d2 : 0.0;
      K[i + j * ldk] = exp(-d2 / eps);
    }
  });
}

}  // namespace
