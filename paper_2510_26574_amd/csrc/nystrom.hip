// nystrom_extend: out-of-sample values of the eigenvectors of P~ (the
// extension formula of the paper's "Nystrom method connection" section,
// applied to the bistochastic approximation), on gfx950;
// nystrom_extend_symmetric: the same for L~ = D~^{-1/2} K~ D~^{-1/2} (the
// symmetric normalisation).
//
// For a new point y:  f(y) = F(S, :)^{-1} k(X_S, y),  d~(y) = c^T f(y),
// phi(y) = f(y)^T E / d~(y),  E = C R^T V Lambda^{-1} (from bistoch_eig), or
// phi(y) = f(y)^T E / sqrt(d~(y)),  E = R^T V Lambda^{-1} (symmetric).
// F(S, :) is lower triangular in pivot order, so the two triangular solves
// are folded once into E' = F(S, :)^{-T} [c | E]; each block of new points
// then costs one MFMA distance product with an exp epilogue and one product
// with E'.  Everything is float64.
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "dense.hpp"
#include "profile.hpp"
#include "kernel_rows.hpp"
#include "tile_gemm.hpp"

namespace {

constexpr int64_t MCH = 65536;  // new points per block

// rhs = [c | E] (r x (nev+1), column-major), rows >= k zero.
__global__ void k_rhs(const double* __restrict__ c, const double* __restrict__ E, int r, int nev,
                      const int32_t* kptr, double* __restrict__ B0) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * (nev + 1)) return;
  const int i = (int)(e % r), j = (int)(e / r);
  const int k = *kptr;
  double v = 0.0;
  if (i < k) v = j == 0 ? c[i] : E[i + (int64_t)(j - 1) * r];
  B0[e] = v;
}

// Phi(i, j) = P(i, j + 1) / P(i, 0) (bistochastic) or / sqrt(P(i, 0)) (symmetric)
__global__ void k_divide(const double* __restrict__ P, int64_t ldp, int64_t m, int nev,
                         double* __restrict__ Phi, int64_t ldphi, int sym) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * nev) return;
  const int64_t i = e % m;
  const int j = (int)(e / m);
  const double dy = P[i];
  Phi[i + j * ldphi] = P[i + (int64_t)(j + 1) * ldp] / (sym ? sqrt(dy) : dy);
}

struct NysWs {
  double *XS, *xsn, *FS, *B0, *Yp, *yn, *K, *P;
  int64_t dp, mch;
};

static size_t carve_nys(WsCursor& c, NysWs& w, int64_t M, int64_t d, int r, int nev) {
  w.dp = (int64_t)align_up((size_t)d, 16);
  w.mch = M < MCH ? M : MCH;
  w.XS = c.take<double>((size_t)r * w.dp);
  w.xsn = c.take<double>(r);
  w.FS = c.take<double>((size_t)r * r);
  w.B0 = c.take<double>((size_t)r * (nev + 1));
  w.Yp = c.take<double>((size_t)w.mch * w.dp);
  w.yn = c.take<double>(w.mch);
  w.K = c.take<double>((size_t)w.mch * r);
  w.P = c.take<double>((size_t)w.mch * (nev + 1));
  return c.used;
}

template <typename TF>
static int run_nys(const rpc_points* Y, const rpc_points* X, const int64_t* piv, const int32_t* k,
                   const TF* F, int64_t ldf, int r, const double* c, const double* E, int nev,
                   double* Phi, int64_t ldphi, void* ws, size_t ws_bytes, int32_t* status,
                   hipStream_t st, int sym, int pivot_rows) {
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  NysWs w;
  carve_nys(cur, w, Y->N, Y->d, r, nev);
  if (!cur.ok) return RPC_EWORKSPACE;
  prof::begin(prof::NYSTROM, st);
  with_points_type(X->dtype, [&](auto* tx) {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(tx)>::type>::type TX;
    hipLaunchKernelGGL((k_gather_pivots<TF, TX>), dim3(r), dim3(256), 0, st, (const TX*)X->X, X->ldx,
                       X->d, w.dp, piv, k, F, ldf, r, w.XS, w.xsn, w.FS, pivot_rows);
    return (int)RPC_OK;
  });
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)(((int64_t)r * (nev + 1) + 255) / 256)), dim3(256), 0, st,
                     c, E, r, nev, k, w.B0);
  dense::trsm_lt(st, w.FS, r, r, w.B0, r, nev + 1);
  RPC_LAUNCH_CHECK();
  for (int64_t m0 = 0; m0 < Y->N; m0 += w.mch) {
    const int64_t m = Y->N - m0 < w.mch ? Y->N - m0 : w.mch;
    with_points_type(Y->dtype, [&](auto* ty) {
      typedef typename std::remove_const<typename std::remove_pointer<decltype(ty)>::type>::type TY;
      hipLaunchKernelGGL((k_prep_rows64<TY>), dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st,
                         (const TY*)Y->X + m0 * Y->ldx, Y->ldx, m, Y->d, w.dp, w.Yp, w.yn, status);
      return (int)RPC_OK;
    });
    hipLaunchKernelGGL(k_cross_kernel, dim3((unsigned)((m + 63) / 64), (unsigned)((r + 63) / 64)),
                       dim3(256), 0, st, (const double*)w.Yp, (const double*)w.yn, m, w.dp,
                       (const double*)w.XS, (const double*)w.xsn, r, X->eps, w.K, m);
    dense::gemm64<false, true>(st, m, nev + 1, r, w.K, m, w.B0, r, w.P, m, 1.0, 0.0);
    hipLaunchKernelGGL(k_divide, dim3((unsigned)((m * nev + 255) / 256)), dim3(256), 0, st,
                       (const double*)w.P, m, m, nev, Phi + m0, ldphi, sym);
    RPC_LAUNCH_CHECK();
  }
  prof::end(prof::NYSTROM, st);
  return RPC_OK;
}

}  // namespace

extern "C" int nystrom_extend_workspace_size(int64_t M, int64_t d, int32_t r, int32_t nev,
                                             size_t* bytes) {
  if (M < 1 || d < 1 || r < 1 || nev < 1 || nev > r || !bytes) return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  NysWs w;
  *bytes = carve_nys(c, w, M, d, r, nev);
  return RPC_OK;
}

static int nystrom_any(const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                       const int32_t* k, const void* F, int32_t fdt, int64_t ldf, int32_t r,
                       const double* c, const double* E, int32_t nev, double* Phi, int64_t ldphi,
                       void* ws, size_t ws_bytes, int32_t* status, rpc_stream_t stream, int sym,
                       int pivot_rows = 0) {
  if (!Y || !X || !Y->X || !X->X || !pivots || !k || !F || !c || !E || !Phi || !status)
    return RPC_EINVAL;
  if (Y->N < 1 || Y->d != X->d || Y->ldx < Y->d || X->ldx < X->d || !(X->eps > 0.0)) return RPC_EINVAL;
  for (const rpc_points* P : {X, Y})
    if (P->dtype != RPC_F32 && P->dtype != RPC_F64 && P->dtype != RPC_BF16) return RPC_EINVAL;
  if (r < 1 || r > X->N || nev < 1 || nev > r || ldf < (pivot_rows ? r : X->N) || ldphi < Y->N)
    return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (fdt == RPC_F64)
    return run_nys<double>(Y, X, pivots, k, (const double*)F, ldf, r, c, E, nev, Phi, ldphi, ws,
                           ws_bytes, status, st, sym, pivot_rows);
  if (fdt == RPC_F32 && !pivot_rows)
    return run_nys<float>(Y, X, pivots, k, (const float*)F, ldf, r, c, E, nev, Phi, ldphi, ws,
                          ws_bytes, status, st, sym, 0);
  return RPC_EINVAL;
}

extern "C" int nystrom_extend(const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                              const int32_t* k, const void* F, int32_t fdt, int64_t ldf, int32_t r,
                              const double* c, const double* E, int32_t nev, double* Phi,
                              int64_t ldphi, void* ws, size_t ws_bytes, int32_t* status,
                              rpc_stream_t stream) {
  return nystrom_any(Y, X, pivots, k, F, fdt, ldf, r, c, E, nev, Phi, ldphi, ws, ws_bytes, status,
                     stream, 0);
}

extern "C" int nystrom_extend_symmetric(const rpc_points* Y, const rpc_points* X,
                                        const int64_t* pivots, const int32_t* k, const void* F,
                                        int32_t fdt, int64_t ldf, int32_t r, const double* c,
                                        const double* E, int32_t nev, double* Phi, int64_t ldphi,
                                        void* ws, size_t ws_bytes, int32_t* status,
                                        rpc_stream_t stream) {
  return nystrom_any(Y, X, pivots, k, F, fdt, ldf, r, c, E, nev, Phi, ldphi, ws, ws_bytes, status,
                     stream, 1);
}

extern "C" int nystrom_extend_lowmem(const rpc_points* Y, const rpc_points* X,
                                     const int64_t* pivots, const int32_t* k, const double* FS,
                                     int64_t ldfs, int32_t r, const double* c, const double* E,
                                     int32_t nev, int32_t normalization, double* Phi, int64_t ldphi,
                                     void* ws, size_t ws_bytes, int32_t* status,
                                     rpc_stream_t stream) {
  if (normalization != RPC_BISTOCHASTIC && normalization != RPC_SYMMETRIC) return RPC_EINVAL;
  return nystrom_any(Y, X, pivots, k, FS, RPC_F64, ldfs, r, c, E, nev, Phi, ldphi, ws, ws_bytes,
                     status, stream, normalization == RPC_SYMMETRIC, 1);
}

extern "C" int rpc_status_sync(const int32_t* dev_status, rpc_stream_t stream) {
  if (!dev_status) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return RPC_EHIP;
  int32_t v = 0;
  if (hipMemcpy(&v, dev_status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return RPC_EHIP;
  return v;
}

extern "C" const char* rpc_version(void) { return "rpchol 0.1 (gfx950)"; }
