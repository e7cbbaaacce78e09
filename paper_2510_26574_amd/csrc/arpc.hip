// rpchol_factor: accelerated randomly pivoted partial Cholesky (the paper's
// Algorithm 2, with the accept/reject check of Algorithm 3) on the Gaussian
// kernel k(x, y) = exp(-|x - y|^2 / eps), for gfx950.
//
// One round i, all on the device and without host synchronisation:
//   pivot draw      b proposals from rho / sum(rho) through an integer CDF
//                   (rho_q = floor(rho 2^40), exact and summation-order free),
//                   or argmax rho in greedy mode, or the replay list;
//   gather          proposal rows of the points and of F;
//   pivot block     H = K(S', S') - F(S', :) F(S', :)^T in float64;
//   accept/reject   Algorithm 3 on H in one workgroup (H resident in LDS),
//                   giving the accepted set T, L = chol block and L^{-1};
//   kernel columns  W = K(:, S_i): MFMA distance product
//                   |x|^2 + |s|^2 - 2 <x, s> with an exp epilogue;
//   Schur update    W -= F(:, :k) F(S_i, :k)^T (MFMA);
//   solve+downdate  G = W L^{-T} (float64 MFMA), F(:, k:k+|T|) = G,
//                   rho = max(rho - rownorms(G)^2, 0);
//   round end       rho(S_i) = 0, k += |T|.
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "dense.hpp"
#include "profile.hpp"
#include "split16.hpp"
#include "tile_gemm.hpp"

namespace {

constexpr int CHUNK = 4096;  // rho entries per partial sum (pivot draw)
constexpr int MAXB = 128;    // largest supported block size
constexpr int kStages = 4;   // LDS stages of the direct-staged products (three in flight)
constexpr int kStagesSplit = 2;  // the mixed form's fused kernel: two workgroups per CU
constexpr double QSCALE = 1099511627776.0;  // 2^40

__device__ inline unsigned long long quant_rho(double r) {
  return r > 0.0 ? (unsigned long long)floor(r * QSCALE) : 0ull;
}

struct RoundState {
  int32_t* k;      // accepted pivots so far (the caller's k_out)
  int32_t* nT;     // accepted in this round
  int32_t* stop;   // nonzero once the residual is exhausted
};

// ------------------------------------------------------------ preparation
// Xp[n][:] = points converted to the product type, zero-padded to dp columns;
// xn[n] = squared norm of the converted row (computed in float64, stored in
// the epilogue type).  Also initialises rho = 1 (diag of the Gaussian kernel),
// pivots = -1 and the counters.  xmax (optional, cleared beforehand): the
// largest finite |x| over all points, as float bits (non-negative floats
// order like their bit patterns).
// TX: element type of the points (float, double or bf16); every value is
// taken to double exactly and converted to T from there (bf16 copies of
// float64 points round through float32).
template <typename T, typename TN, typename TX>
__global__ __launch_bounds__(256) void k_prep(const TX* __restrict__ X, int64_t N, int64_t d,
                                              int64_t ldx, int64_t dp, T* __restrict__ Xp,
                                              TN* __restrict__ xn, double* __restrict__ rho,
                                              int32_t* status, unsigned* xmax) {
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  double s = 0.0;
  float amax = 0.0f;
  bool bad = false;
  // float32 rows without padding, 8-float aligned: each lane converts 8
  // consecutive columns per pass with two 16-byte loads and one vector store
  const bool vec = std::is_same<TX, float>::value && d == dp && (ldx % 8) == 0 &&
                   (((uintptr_t)X) & 31) == 0;
  if constexpr (!std::is_same<TX, float>::value) {
    for (int64_t j = lane; j < dp; j += 64) {
      const double v = j < d ? ld_point(X, n * ldx + j) : 0.0;
      if (!isfinite(v)) bad = true;
      else amax = fmaxf(amax, (float)fabs(v));
      T c = cvtd<T>(v);
      Xp[n * dp + j] = c;
      const double cd = to_d(c);
      s += cd * cd;
    }
  } else if (vec) {
    typedef T tv __attribute__((ext_vector_type(8)));
    for (int64_t j0 = (int64_t)lane * 8; j0 < dp; j0 += 512) {
      const v4f u0 = *reinterpret_cast<const v4f*>(X + n * ldx + j0);
      const v4f u1 = *reinterpret_cast<const v4f*>(X + n * ldx + j0 + 4);
      tv c;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float v = e < 4 ? u0[e] : u1[e - 4];
        if (!isfinite(v)) bad = true;
        else amax = fmaxf(amax, fabsf(v));
        c[e] = cvt<T>(v);
        const double cd = to_d(c[e]);
        s += cd * cd;
      }
      *reinterpret_cast<tv*>(Xp + n * dp + j0) = c;
    }
  } else {
    for (int64_t j = lane; j < dp; j += 64) {
      float v = j < d ? X[n * ldx + j] : 0.0f;
      if (!isfinite(v)) bad = true;
      else amax = fmaxf(amax, fabsf(v));
      T c = cvt<T>(v);
      Xp[n * dp + j] = c;
      double cd = to_d(c);
      s += cd * cd;
    }
  }
  s = wave_sum(s);
  if (__any(bad) && lane == 0) set_status(status, RPC_ENONFINITE);
  if (xmax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, RPC_WAVE));
    // the running maximum settles early: most rows skip the atomic
    if (lane == 0 && __float_as_uint(amax) > *(volatile unsigned*)xmax)
      atomicMax(xmax, __float_as_uint(amax));
  }
  if (lane == 0) {
    xn[n] = (TN)s;
    rho[n] = 1.0;
  }
}

// k_prep over the points of X (its dtype picks the loader)
template <typename T, typename TN>
static void launch_prep(const rpc_points* X, int64_t dp, T* Xp, TN* xn, double* rho,
                        int32_t* status, unsigned* xmax, hipStream_t st) {
  const dim3 g((unsigned)((X->N + 3) / 4));
  with_points_type(X->dtype, [&](auto* tx) {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(tx)>::type>::type TX;
    hipLaunchKernelGGL((k_prep<T, TN, TX>), g, dim3(256), 0, st, (const TX*)X->X, X->N, X->d,
                       X->ldx, dp, Xp, xn, rho, status, xmax);
    return (int)RPC_OK;
  });
}

__global__ void k_clear_u32(unsigned* p) { *p = 0u; }

__global__ void k_init_small(int64_t* pivots, int r, int32_t* k, int32_t* nT, int32_t* stop) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < r; i += blockDim.x * gridDim.x) pivots[i] = -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *k = 0;
    *nT = 0;
    *stop = 0;
  }
}

// ------------------------------------------------------------ pivot draw
__global__ __launch_bounds__(256) void k_rho_partial(const double* __restrict__ rho, int64_t N,
                                                     unsigned long long* __restrict__ part,
                                                     const int32_t* stop) {
  if (*stop) return;
  __shared__ unsigned long long ws[4];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  unsigned long long s = 0;
  for (int e = threadIdx.x; e < CHUNK; e += 256) {
    int64_t i = base + e;
    if (i < N) s += quant_rho(rho[i]);
  }
  s = wave_sum_u64(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// One workgroup: inclusive scan of the chunk sums in place; total in *tot.
__global__ __launch_bounds__(1024) void k_draw_scan(unsigned long long* __restrict__ part, int nb,
                                                    unsigned long long* __restrict__ tot,
                                                    int32_t* stop) {
  if (*stop) return;
  __shared__ unsigned long long tsum[1024];
  const int tid = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = tid * per;
  unsigned long long loc = 0;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) loc += part[b0 + j];
  tsum[tid] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned long long v = tid >= off ? tsum[tid - off] : 0ull;
    __syncthreads();
    tsum[tid] += v;
    __syncthreads();
  }
  unsigned long long run = tid > 0 ? tsum[tid - 1] : 0ull;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) {
      run += part[b0 + j];
      part[b0 + j] = run;
    }
  if (tid == 1023) {
    *tot = tsum[1023];
    if (tsum[1023] == 0ull) *stop = 1;
  }
}

// One workgroup per proposal j:  s = min{ i : C_i > floor(m T / 2^53) },
// m = u_j 2^53, C the inclusive prefix of rho_q = floor(rho 2^40).  The chunk
// holding the target is found by binary search over the scanned chunk sums,
// then the chunk's 4096 quantised entries are scanned in LDS.
__global__ __launch_bounds__(256) void k_draw_find(const double* __restrict__ rho, int64_t N,
                                                   const unsigned long long* __restrict__ part,
                                                   int nb, const unsigned long long* __restrict__ tot,
                                                   const double* __restrict__ u,
                                                   int64_t* __restrict__ prop,
                                                   const int32_t* stop) {
  if (*stop) return;
  __shared__ unsigned long long q[CHUNK];
  __shared__ unsigned long long tsum[256];
  __shared__ int blk_s;
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const unsigned long long T = *tot;
  const unsigned long long m = (unsigned long long)(u[j] * 9007199254740992.0);  // u * 2^53
  const unsigned long long target = (__umul64hi(m, T) << 11) | ((m * T) >> 53);
  if (tid == 0) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (part[mid] > target) hi = mid; else lo = mid + 1;
    }
    blk_s = lo;
  }
  __syncthreads();
  const int blk = blk_s;
  const unsigned long long base = blk > 0 ? part[blk - 1] : 0ull;
  const unsigned long long rem = target - base;  // < rho_q mass of this chunk
  const int64_t i0 = (int64_t)blk * CHUNK;
  for (int e = tid; e < CHUNK; e += 256) {
    const int64_t i = i0 + e;
    q[e] = i < N ? quant_rho(rho[i]) : 0ull;
  }
  __syncthreads();
  // thread t owns entries [16 t, 16 t + 16)
  unsigned long long s = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) s += q[tid * 16 + e];
  tsum[tid] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned long long v = tid >= off ? tsum[tid - off] : 0ull;
    __syncthreads();
    tsum[tid] += v;
    __syncthreads();
  }
  const unsigned long long excl = tid > 0 ? tsum[tid - 1] : 0ull;
  if (excl <= rem && rem < tsum[tid]) {
    unsigned long long c = excl;
    int e = 0;
    for (; e < 16; ++e) {
      c += q[tid * 16 + e];
      if (c > rem) break;
    }
    prop[j] = i0 + tid * 16 + e;
  }
}

// Greedy: argmax rho, lowest index on ties.
__global__ __launch_bounds__(256) void k_argmax_partial(const double* __restrict__ rho, int64_t N,
                                                        double* __restrict__ pv,
                                                        int64_t* __restrict__ pi,
                                                        const int32_t* stop) {
  if (*stop) return;
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  double bv = -1.0;
  int64_t bix = -1;
  for (int e = threadIdx.x; e < CHUNK; e += 256) {
    int64_t i = base + e;
    if (i < N) {
      double v = rho[i];
      if (v > bv) { bv = v; bix = i; }
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bix;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double v2 = sv[threadIdx.x + off];
      int64_t i2 = si[threadIdx.x + off];
      double v1 = sv[threadIdx.x];
      int64_t i1 = si[threadIdx.x];
      if (v2 > v1 || (v2 == v1 && i2 >= 0 && (i1 < 0 || i2 < i1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

__global__ __launch_bounds__(256) void k_argmax_final(const double* __restrict__ pv,
                                                      const int64_t* __restrict__ pi, int nb,
                                                      int64_t* __restrict__ prop, int32_t* stop) {
  if (*stop) return;
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double bv = -1.0;
  int64_t bix = -1;
  for (int e = threadIdx.x; e < nb; e += 256) {
    double v = pv[e];
    int64_t i = pi[e];
    if (i >= 0 && (v > bv || (v == bv && (bix < 0 || i < bix)))) { bv = v; bix = i; }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bix;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double v2 = sv[threadIdx.x + off];
      int64_t i2 = si[threadIdx.x + off];
      double v1 = sv[threadIdx.x];
      int64_t i1 = si[threadIdx.x];
      if (i2 >= 0 && (i1 < 0 || v2 > v1 || (v2 == v1 && i2 < i1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (!(sv[0] > 0.0) || si[0] < 0) {
      *stop = 1;
    } else {
      prop[0] = si[0];
    }
  }
}

__global__ void k_replay_props(const int64_t* __restrict__ replay, int64_t off, int bi, int64_t N,
                               int64_t* __restrict__ prop, int32_t* status, int32_t* stop) {
  int j = threadIdx.x;
  if (j < bi) {
    int64_t s = replay[off + j];
    if (s < 0 || s >= N) {
      set_status(status, RPC_EINVAL);
      *stop = 1;
      s = 0;
    }
    prop[j] = s;
  }
}

// ------------------------------------------------------------ gather
// XS[j][:] = Xp[prop[j]][:], ns[j] = xn[prop[j]], FS[j][l] = F[prop[j] + l ldf] (l < k).
template <typename T, typename TN, typename TF>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ Xp, const TN* __restrict__ xn,
                                                int64_t dp, const TF* __restrict__ F, int64_t ldf,
                                                int r, const int64_t* __restrict__ prop, int bi,
                                                const int32_t* kptr, const int32_t* stop,
                                                T* __restrict__ XS, TN* __restrict__ ns,
                                                TF* __restrict__ FS, int64_t N, int32_t* status) {
  if (*stop) return;
  const int j = blockIdx.x;
  if (j >= bi) return;
  int64_t s = prop[j];
  if (s < 0 || s >= N) {  // cannot happen with a consistent CDF; keep accesses in bounds
    if (threadIdx.x == 0) set_status(status, RPC_EHIP);
    s = 0;
  }
  const int k = *kptr;
  for (int64_t c = threadIdx.x; c < dp; c += 256) XS[j * dp + c] = Xp[s * dp + c];
  for (int l = threadIdx.x; l < k; l += 256) FS[(int64_t)j * r + l] = F[s + (int64_t)l * ldf];
  if (threadIdx.x == 0) ns[j] = xn[s];
}

// H[i][j] = exp(-sum_c (x_i - x_j)^2 / eps) - sum_l FS[i][l] FS[j][l], float64,
// split over the joint index range (dp coordinates, then k factor columns)
// in slices of PB_CH so that many workgroups share a block whose k reaches
// thousands: workgroup (tile of 16 x 16 pairs, slice z) writes the slice's
// two partial sums; k_pivot_block_finish adds the slices in order (the same
// order on every run) and forms H.
constexpr int PB_CH = 256;
static int pb_slices(int64_t dp, int r) { return (int)((dp + r + PB_CH - 1) / PB_CH); }

template <typename T, typename TF>
__global__ __launch_bounds__(256) void k_pivot_block_part(const T* __restrict__ XS, int64_t dp,
                                                          const TF* __restrict__ FS, int r, int bi,
                                                          const int32_t* kptr, const int32_t* stop,
                                                          double* __restrict__ pd2,
                                                          double* __restrict__ pff) {
  if (*stop) return;
  __shared__ double si_[16][65];
  __shared__ double sj_[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int i = i0 + ty, j = j0 + tx;
  const int k = *kptr;
  const int64_t e0 = (int64_t)blockIdx.z * PB_CH, e1 = e0 + PB_CH;
  double d2 = 0.0, ff = 0.0;
  const int64_t cend = e1 < dp ? e1 : dp;
  for (int64_t c0 = e0; c0 < cend; c0 += 64) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int rr = e / 64, cc = e % 64;
      const int64_t c = c0 + cc;
      si_[rr][cc] = (i0 + rr < bi && c < cend) ? to_d(XS[(int64_t)(i0 + rr) * dp + c]) : 0.0;
      sj_[rr][cc] = (j0 + rr < bi && c < cend) ? to_d(XS[(int64_t)(j0 + rr) * dp + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int cc = 0; cc < 64; ++cc) {
      const double t = si_[ty][cc] - sj_[tx][cc];
      d2 += t * t;
    }
    __syncthreads();
  }
  const int64_t lb = (e0 > dp ? e0 : dp) - dp, le = (e1 < dp + k ? e1 : dp + k) - dp;
  for (int64_t l0 = lb; l0 < le; l0 += 64) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int rr = e / 64, cc = e % 64;
      const int64_t l = l0 + cc;
      si_[rr][cc] = (i0 + rr < bi && l < le) ? to_d(FS[(int64_t)(i0 + rr) * r + l]) : 0.0;
      sj_[rr][cc] = (j0 + rr < bi && l < le) ? to_d(FS[(int64_t)(j0 + rr) * r + l]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int cc = 0; cc < 64; ++cc) ff += si_[ty][cc] * sj_[tx][cc];
    __syncthreads();
  }
  if (i < bi && j < bi) {
    const int64_t o = ((int64_t)blockIdx.z * MAXB + i) * MAXB + j;
    pd2[o] = d2;
    pff[o] = ff;
  }
}

__global__ __launch_bounds__(256) void k_pivot_block_finish(const double* __restrict__ pd2,
                                                            const double* __restrict__ pff, int ks,
                                                            int bi, const int32_t* stop, double eps,
                                                            int ldh, double* __restrict__ H) {
  if (*stop) return;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int i = e / MAXB, j = e % MAXB;
  if (i >= bi || j >= bi) return;
  double d2 = 0.0, ff = 0.0;
  for (int z = 0; z < ks; ++z) {
    d2 += pd2[((int64_t)z * MAXB + i) * MAXB + j];
    ff += pff[((int64_t)z * MAXB + i) * MAXB + j];
  }
  H[i * ldh + j] = exp(-d2 / eps) - ff;
}

template <typename T, typename TF>
static void launch_pivot_block(const T* XS, int64_t dp, const TF* FS, int r, int bi,
                               const int32_t* kptr, const int32_t* stop, double eps, double* pd2,
                               double* pff, double* H, hipStream_t st) {
  const unsigned hb = (unsigned)((bi + 15) / 16);
  const int ks = pb_slices(dp, r);
  hipLaunchKernelGGL((k_pivot_block_part<T, TF>), dim3(hb, hb, (unsigned)ks), dim3(256), 0, st, XS,
                     dp, FS, r, bi, kptr, stop, pd2, pff);
  hipLaunchKernelGGL(k_pivot_block_finish, dim3(MAXB * MAXB / 256), dim3(256), 0, st,
                     (const double*)pd2, (const double*)pff, ks, bi, stop, eps, MAXB, H);
}

// ------------------------------------------------------------ Algorithm 3
// One workgroup of 1024 threads.  H (bi x bi) lives in LDS as a packed lower
// triangle (entry (a, c), c <= a, at a (a + 1) / 2 + c).  Step i accepts
// proposal i iff it repeats no accepted proposal of this block,
// H(i,i) > tau and z_i * H0(i,i) < H(i,i) (H0 = H at block start), then
// eliminates it from the trailing triangle: H(a,c) -= H(a,i) H(c,i) / H(i,i).
// Column i is not read again after its step, so its division by
// sqrt(H(i,i)) (which makes it a Cholesky column) is deferred.  Outputs: the
// accepted pivots (appended to `pivots`), the Cholesky factor L of the
// accepted block (row-major MAXB x MAXB, zero-padded), and the block positions
// (acc) and norms (nsa) of the accepted proposals; k_copy_accepted then
// gathers their point and factor rows over many workgroups.
__device__ inline int tri(int a, int c) { return a * (a + 1) / 2 + c; }

// v from lane l of the wave (l uniform)
__device__ inline double rdlane(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename T, typename TN, typename TF>
__global__ __launch_bounds__(1024) void k_accept_reject(
    const double* __restrict__ Hg, int bi, const int64_t* __restrict__ prop,
    const double* __restrict__ z, double tau, int mode, const TN* __restrict__ ns,
    int32_t* kptr, int32_t* nTptr, const int32_t* stop, int64_t* __restrict__ pivots,
    double* __restrict__ Lc, int64_t* __restrict__ Si, int32_t* __restrict__ acc,
    TN* __restrict__ nsa, int32_t* status) {
  constexpr int PK = MAXB * (MAXB + 1) / 2;
  __shared__ double H[PK];
  __shared__ int accl[MAXB];
  __shared__ double rho_loc[MAXB];
  __shared__ double dinv[MAXB];  // 1 / sqrt(H(i,i)) of accepted pivots, by position
  __shared__ int64_t props[MAXB];
  __shared__ double zs[MAXB];
  __shared__ int first[MAXB];  // first proposal of the block with the same point
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (*stop) {
    if (tid == 0) *nTptr = 0;
    return;
  }
  const int k = *kptr;  // accepted pivots so far (position in `pivots`)
  for (int a = wave; a < bi; a += 16)
    for (int c = lane; c <= a; c += 64) H[tri(a, c)] = Hg[a * MAXB + c];
  if (tid < bi) {
    props[tid] = prop[tid];
    zs[tid] = (mode == RPC_SAMPLED) ? z[tid] : 0.0;
  }
  __syncthreads();
  if (tid < bi) {
    rho_loc[tid] = H[tri(tid, tid)];
    int f = tid;
    for (int j = 0; j < tid; ++j)
      if (props[j] == props[tid]) {
        f = j;
        break;
      }
    first[tid] = f;
  }
  __syncthreads();
  // Panels of PW steps.  The first wave holds the panel's columns for rows
  // i0 .. bi-1 in registers (lane l: rows i0 + l and i0 + l + 64) and runs
  // its steps alone, reading pivot-row entries across lanes, so a step costs
  // no barrier.  Every lane takes each decision from the same values; repeated
  // points are tracked as a bit mask over first[].  The panel's eliminated
  // columns (raw in R, scaled by 1 / H(i,i) in Q) then update the trailing
  // triangle in step order with the same multiply-adds as one step at a time,
  // so the result does not depend on the panel width.
  static_assert(MAXB <= 128, "two rows per lane, two 64-bit masks");
  constexpr int PW = 8;
  __shared__ double Qp[PW * MAXB], Rp[PW * MAXB];  // column j of the panel at j * MAXB
  __shared__ int pmask_s[2], na_s;  // pmask_s by panel parity: a panel with no
  // accepted step skips the trailing barrier, so the next panel must not
  // overwrite the mask the other waves may still be reading
  unsigned long long taken[2] = {0ull, 0ull};
  int na = 0;
  if (tid == 0) na_s = 0;  // read after the closing barrier
  for (int i0 = 0; i0 < bi; i0 += PW) {
    if (wave == 0) {
      const int ra0 = i0 + lane, ra1 = i0 + lane + 64;
      double x0[PW], x1[PW], rh[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        const int cg = i0 + c;
        const bool v0 = ra0 < bi && cg <= ra0, v1 = ra1 < bi && cg <= ra1;
        const double h0 = H[v0 ? tri(ra0, cg) : 0], h1 = H[v1 ? tri(ra1, cg) : 0];
        x0[c] = v0 ? h0 : 0.0;
        x1[c] = v1 ? h1 : 0.0;
      }
      int pm = 0;
#pragma unroll
      for (int j = 0; j < PW; ++j) {
        const int i = i0 + j;
        rh[j] = 0.0;
        if (i >= bi) continue;
        const double hii = rdlane(x0[j], j);
        const int fi = first[i];
        const bool dup = (taken[fi >> 6] >> (fi & 63)) & 1ull;
        bool ok;
        if (mode == RPC_REPLAY) {
          ok = hii > tau && !dup;
          if (!ok && lane == 0) set_status(status, RPC_EBREAKDOWN);
        } else if (mode == RPC_GREEDY) {
          ok = hii > tau;  // b = 1: z * H(0,0) < H(0,0) holds for every z in [0, 1)
        } else {
          ok = !dup && hii > tau && zs[i] * rho_loc[i] < hii;
        }
        if (!ok) continue;
        if (lane == 0) {
          dinv[na] = 1.0 / sqrt(hii);
          accl[na] = i;
        }
        taken[fi >> 6] |= 1ull << (fi & 63);
        ++na;
        pm |= 1 << j;
        rh[j] = 1.0 / hii;
        const double hai0 = x0[j] * rh[j], hai1 = x1[j] * rh[j];
#pragma unroll
        for (int c = j + 1; c < PW; ++c) {
          const double hci = rdlane(x0[j], c);
          x0[c] -= hai0 * hci;
          x1[c] -= hai1 * hci;
        }
      }
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        const int cg = i0 + c;
        if (ra0 < bi && cg <= ra0) H[tri(ra0, cg)] = x0[c];
        if (ra1 < bi && cg <= ra1) H[tri(ra1, cg)] = x1[c];
        if (ra0 < bi) {
          Rp[c * MAXB + ra0] = x0[c];
          Qp[c * MAXB + ra0] = x0[c] * rh[c];
        }
        if (ra1 < bi) {
          Rp[c * MAXB + ra1] = x1[c];
          Qp[c * MAXB + ra1] = x1[c] * rh[c];
        }
      }
      if (lane == 0) {
        pmask_s[(i0 / PW) & 1] = pm;
        na_s = na;
      }
    }
    __syncthreads();
    const int t0 = i0 + PW, pm = pmask_s[(i0 / PW) & 1];
    if (t0 < bi && pm != 0) {
      // lower trailing triangle, 32 row groups x 32 column lanes
      const int ty = tid >> 5, tx = tid & 31;
      for (int a = t0 + ty; a < bi; a += 32) {
        double q[PW];
#pragma unroll
        for (int j = 0; j < PW; ++j) q[j] = Qp[j * MAXB + a];
        const int ra = tri(a, 0);
        for (int c = t0 + tx; c <= a; c += 32) {
          double h = H[ra + c];
#pragma unroll
          for (int j = 0; j < PW; ++j)
            if ((pm >> j) & 1) h -= q[j] * Rp[j * MAXB + c];
          H[ra + c] = h;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const int nt = na_s;
  // compact L(x, y) = H(accl[x], accl[y]) dinv[y] (x >= y), row-major MAXB x MAXB
  for (int x = wave; x < MAXB; x += 16) {
    const int ax = x < nt ? accl[x] : 0;
    for (int y = lane; y < MAXB; y += 64)
      Lc[x * MAXB + y] = (x < nt && y <= x) ? H[tri(ax, accl[y])] * dinv[y] : 0.0;
  }
  if (tid < nt) {
    acc[tid] = accl[tid];
    nsa[tid] = ns[accl[tid]];
    Si[tid] = prop[accl[tid]];
    pivots[k + tid] = prop[accl[tid]];
  }
  if (tid == 0) *nTptr = nt;
}

// Accepted rows for the column kernels: workgroup a copies the point row and
// the leading kf factor entries of the a-th accepted proposal (a < nT).
template <typename T, typename TF>
__global__ __launch_bounds__(256) void k_copy_accepted(const int32_t* __restrict__ acc,
                                                       const int32_t* nTptr, const int32_t* kfptr,
                                                       const T* __restrict__ XS, int64_t dp,
                                                       const TF* __restrict__ FS, int r,
                                                       T* __restrict__ XSa, TF* __restrict__ FSa) {
  const int a = blockIdx.x;
  if (a >= *nTptr) return;
  const int64_t src = acc[a];
  const int kf = *kfptr;
  for (int64_t c = threadIdx.x; c < dp; c += 256) XSa[a * dp + c] = XS[src * dp + c];
  for (int l = threadIdx.x; l < kf; l += 256) FSa[(int64_t)a * r + l] = FS[src * r + l];
}

// L^{-1} of the accepted block, one workgroup per column c: four waves stage
// the rows of L it needs, then the first wave runs the right-looking forward
// substitution L x = e_c: lane l keeps x_l and
// x_{l+64}; once x_j = b_j / L(j,j) is known it is broadcast and every row
// i > j subtracts L(i,j) x_j, so a row costs one broadcast and two
// multiply-adds instead of a wave reduction.
__global__ __launch_bounds__(256) void k_tri_inv(const double* __restrict__ Lc,
                                                 const int32_t* nTptr, double* __restrict__ Linv) {
  constexpr int LDS = MAXB + 1;  // column walks (lane i reading L(i, j)) spread over banks
  __shared__ double Ls[MAXB * LDS];
  __shared__ double rd[MAXB];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int nt = *nTptr;
  if (c < nt) {
    // rows c .. nt-1 of L, entries c .. j of row j; whole rows are read so
    // that the four waves' loads coalesce and many are in flight at once
    const int rows = nt - c;
#pragma unroll 4
    for (int e = tid; e < rows * MAXB; e += 256) {
      const int j = c + e / MAXB, l = e % MAXB;
      const double v = Lc[j * MAXB + l];
      if (l >= c && l <= j) Ls[j * LDS + l] = v;
      if (l == j) rd[j] = 1.0 / v;
    }
  }
  __syncthreads();
  if (tid >= 64) return;  // the substitution runs in the first wave
  double x0 = 0.0, x1 = 0.0;
  if (c < nt) {
    // b = e_c
    if (lane == (c & 63)) {
      if (c < 64) x0 = 1.0; else x1 = 1.0;
    }
    for (int j = c; j < nt; ++j) {
      const double bj = bcast_lane(j < 64 ? x0 : x1, j & 63);
      const double xj = bj * rd[j];
      if (lane == (j & 63)) {
        if (j < 64) x0 = xj; else x1 = xj;
      }
      if (lane > j && lane < nt) x0 -= Ls[lane * LDS + j] * xj;
      if (lane + 64 > j && lane + 64 < nt) x1 -= Ls[(lane + 64) * LDS + j] * xj;
    }
  }
  Linv[lane * MAXB + c] = x0;
  Linv[(lane + 64) * MAXB + c] = x1;
}

// ------------------------------------------------------------ kernel columns
// W[n][j] = exp(-max(0, xn[n] + nsa[j] - 2 <Xp[n], XSa[j]>) / eps), j < nT.
// bf16 products: two direct stages and at most 128 VGPRs, so two workgroups
// share a CU and one's prologue and epilogue overlap the other's stream of X.
template <typename T>
constexpr int cols_stages() { return sizeof(T) == 2 ? kStagesSplit : kStages; }

template <typename T, typename TN, typename TW, class Cfg>
__global__ __launch_bounds__(Cfg::NT, sizeof(T) == 2 ? 4 : 1) void k_kernel_cols(const T* __restrict__ Xp,
                                                         const TN* __restrict__ xn, int64_t N,
                                                         int64_t dp, const T* __restrict__ XSa,
                                                         const TN* __restrict__ nsa,
                                                         const int32_t* nTptr, double eps,
                                                         TW* __restrict__ W, int64_t ldw) {
  const int nt = *nTptr;
  const int64_t n0 = (int64_t)blockIdx.y * Cfg::BN;
  if (n0 >= nt) return;
  extern __shared__ char smem_raw[];
  typename Cfg::T* smem = reinterpret_cast<typename Cfg::T*>(smem_raw);
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  GOperand<T, true> A{Xp, dp, N, dp, nullptr, true};
  GOperand<T, true> B{XSa, dp, nt, dp, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop_direct<Cfg, cols_stages<T>()>(acc, A, B, m0, n0, 0, dp, N, MAXB, smem, nt - (int)n0,
                                              (int)blockIdx.x);
  typedef typename Cfg::MM::acc_t AT;
  const AT ie = (AT)(1.0 / eps);
  store_colmajor<Cfg, TW>(acc, smem, W, ldw, m0, n0, N, nt, [&](int row, int col, AT v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m >= N || n >= nt) return (TW)0;
    AT d2 = (AT)xn[m] + (AT)nsa[n] - (AT)2 * v;
    d2 = d2 > (AT)0 ? d2 : (AT)0;
    return (TW)exp(-d2 * ie);
  });
}

// ------------------------------------------------------------ Schur update
// W[:, j] -= F(:, :k) FSa[j][:k]^T, j < nT.
template <typename TF, class Cfg>
__global__ __launch_bounds__(Cfg::NT) void k_schur(const TF* __restrict__ F, int64_t ldf,
                                                   int64_t N, const TF* __restrict__ FSa, int r,
                                                   const int32_t* kptr, const int32_t* nTptr,
                                                   TF* __restrict__ W, int64_t ldw) {
  const int nt = *nTptr;
  const int k = *kptr;
  const int64_t n0 = (int64_t)blockIdx.y * Cfg::BN;
  if (n0 >= nt || k == 0) return;
  extern __shared__ char smem_raw[];
  typename Cfg::T* smem = reinterpret_cast<typename Cfg::T*>(smem_raw);
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  GOperand<TF, false> A{F, ldf, N, k, nullptr, true};
  GOperand<TF, true> B{FSa, r, nt, k, nullptr, (r % (16 / (int)sizeof(TF))) == 0};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop_direct<Cfg, kStages>(acc, A, B, m0, n0, 0, k, N, MAXB, smem, nt - (int)n0,
                                     (int)blockIdx.x);
  for_each_acc<Cfg>(acc, [&](int row, int col, typename Cfg::MM::acc_t v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < N && n < nt) W[m + n * ldw] -= (TF)v;
  });
}

// ------------------------------------------------------------ fused columns + Schur
// When the distance product and the Schur update accumulate in the same
// register layout (bf16/f32 products with an f32 factor, or f64 with f64),
// one workgroup computes its 128-row tile of the kernel columns, applies the
// exp epilogue in registers, and continues accumulating -F(:, :k) F(S_i, :k)^T
// into the same accumulators: W is written once instead of written, read
// and written again.
// SPLIT: the mixed form's variant, sized for two workgroups per CU (four
// waves per SIMD: at most 128 VGPRs; two direct stages for the distance
// product, then the single-buffer split Schur product with only F in the
// register ring).
template <typename T, typename TN, typename TF, class CfgK, class CfgS, bool SPLIT>
__global__ __launch_bounds__(CfgK::NT, SPLIT ? 4 : 1) void k_cols_schur(const T* __restrict__ Xp,
                                                    const TN* __restrict__ xn, int64_t N,
                                                    int64_t dp, const T* __restrict__ XSa,
                                                    const TN* __restrict__ nsa,
                                                    const int32_t* nTptr, double eps,
                                                    const TF* __restrict__ F, int64_t ldf,
                                                    const TF* __restrict__ FSa, int r,
                                                    const int32_t* kptr, TF* __restrict__ W,
                                                    int64_t ldw) {
  static_assert(sizeof(typename CfgK::MM::acc) == sizeof(typename CfgS::MM::acc) &&
                    CfgK::MI == CfgS::MI && CfgK::NI == CfgS::NI &&
                    CfgK::WAVES_M == CfgS::WAVES_M && CfgK::BM == CfgS::BM && CfgK::BN == CfgS::BN,
                "the two products must share one accumulator layout");
  const int nt = *nTptr;
  if (nt == 0) return;
  const int k = *kptr;
  extern __shared__ char smem_raw[];
  const int64_t m0 = (int64_t)blockIdx.x * CfgK::BM;
  typedef typename CfgK::MM::acc_t AT;
  TileAcc<CfgK> acc;
  acc.zero();
  {
    GOperand<T, true> A{Xp, dp, N, dp, nullptr, true};
    GOperand<T, true> B{XSa, dp, nt, dp, nullptr, true};
    tile_mainloop_direct<CfgK, SPLIT ? kStagesSplit : kStages>(
        acc, A, B, m0, 0, 0, dp, N, MAXB, reinterpret_cast<typename CfgK::T*>(smem_raw), nt,
        (int)blockIdx.x);
  }
  // split form: the first stage of the Schur product's F reads goes out
  // before the exp epilogue, which hides its latency
  SchurSplitPipe<CfgK> pipe{(const float*)F, ldf, N, (const float*)FSa, r, nt, k, m0};
  if constexpr (SPLIT) {
    if (k > 0) pipe.begin1a();
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % CfgK::WAVES_M, wn = wave / CfgK::WAVES_M;
  const AT ie = (AT)(1.0 / eps);
  // exp epilogue, negated: acc = -K so the Schur product can accumulate on top
#pragma unroll
  for (int i = 0; i < CfgK::MI; ++i)
#pragma unroll
    for (int j = 0; j < CfgK::NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm * CfgK::WTM + i * 16 + CfgK::MM::row(lane, e);
        const int n = wn * CfgK::WTN + j * 16 + (lane & 15);
        AT v = 0;
        if (m < N && n < nt) {
          AT d2 = (AT)xn[m] + (AT)nsa[n] - (AT)2 * acc.a[i][j][e];
          d2 = d2 > (AT)0 ? d2 : (AT)0;
          v = -exp(-d2 * ie);
        }
        acc.a[i][j][e] = v;
      }
  if constexpr (SPLIT) {
    // bf16 distance product with a float32 factor: the Schur product on the
    // fp16 pipe, in units of 2^24 (exact power-of-two rescaling)
    static_assert(std::is_same<TF, float>::value && std::is_same<AT, float>::value, "split form");
    if (k > 0) {
#pragma unroll
      for (int i = 0; i < CfgK::MI; ++i)
#pragma unroll
        for (int j = 0; j < CfgK::NI; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc.a[i][j][e] *= 16777216.0f;
      pipe.run1b(acc, smem_raw);
#pragma unroll
      for (int i = 0; i < CfgK::MI; ++i)
#pragma unroll
        for (int j = 0; j < CfgK::NI; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc.a[i][j][e] *= (1.0f / 16777216.0f);
    }
    store_colmajor<CfgK, TF>(acc, smem_raw, W, ldw, m0, 0, N, nt,
                             [&](int, int, AT v) { return (TF)(-v); });
    return;
  }
  TileAcc<CfgS>& acs = reinterpret_cast<TileAcc<CfgS>&>(acc);
  if (k > 0) {
    GOperand<TF, false> A{F, ldf, N, k, nullptr, true};
    GOperand<TF, true> B{FSa, r, nt, k, nullptr, (r % (16 / (int)sizeof(TF))) == 0};
    tile_mainloop_direct<CfgS, kStages>(acs, A, B, m0, 0, 0, k, N, MAXB,
                                        reinterpret_cast<typename CfgS::T*>(smem_raw), nt,
                                        (int)blockIdx.x);
  }
  store_colmajor<CfgS, TF>(acs, smem_raw, W, ldw, m0, 0, N, nt,
                           [&](int, int, typename CfgS::MM::acc_t v) { return (TF)(-v); });
}

// ------------------------------------------------------------ split-fp16 distance product
// The split-fp16 form of the kernel columns (22 of float32's 24 significand
// bits per product, a form of its own below float32): the points stay float32 and
// the inner products <x, s> run on the fp16 MFMA pipe as split pairs (three
// products, unit roundoff 2^-22), both operands scaled by one power of two
// s_X chosen from max |x| (so that |x s_X| < 2^15; exact).  xmax is that
// maximum as float bits, from the preparation pass.
__device__ inline float point_scale(const unsigned* xmax) {
  const float am = __uint_as_float(*xmax);
  if (!(am > 0.0f) || !isfinite(am)) return 1.0f;
  int e;
  frexpf(am, &e);  // am = f 2^e, f in [0.5, 1)
  e = e < -100 ? -100 : e;
  return ldexpf(1.0f, 15 - e);
}

// SCHUR: W = K(X, X_S) - F(:, :k) F(S, :k)^T in one pass (the Schur product
// split as in the mixed form's fused kernel); otherwise W = K(X, X_S).  Two
// workgroups per CU: single-buffered split stages, at most 128 VGPRs.
template <class Cfg, bool SCHUR>
__global__ __launch_bounds__(Cfg::NT, 4) void k_cols_split(const float* __restrict__ Xp,
                                                  const float* __restrict__ xn, int64_t N,
                                                  int64_t dp, const float* __restrict__ XSa,
                                                  const float* __restrict__ nsa,
                                                  const int32_t* nTptr, double eps,
                                                  const unsigned* xmax,
                                                  const float* __restrict__ F, int64_t ldf,
                                                  const float* __restrict__ FSa, int r,
                                                  const int32_t* kptr, float* __restrict__ W,
                                                  int64_t ldw) {
  const int nt = *nTptr;
  if (nt == 0) return;
  extern __shared__ char smem_raw[];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  const float sx = point_scale(xmax), isx = 1.0f / sx;
  TileAcc<Cfg> acc;
  acc.zero();
  {
    SchurSplitPipe<Cfg, true> dist{Xp, dp, N, XSa, (int)dp, nt, (int)dp, m0, sx, sx};
    dist.begin1();
    dist.run1(acc, smem_raw);  // acc = s_X^2 <x, s>
  }
  const int k = SCHUR ? *kptr : 0;
  SchurSplitPipe<Cfg> pipe{F, ldf, N, FSa, r, nt, k, m0};
  if (k > 0) pipe.begin1a();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  const float ie = (float)(1.0 / eps);
  // exp epilogue, negated and in the Schur product's units of 2^24
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm * Cfg::WTM + i * 16 + Cfg::MM::row(lane, e);
        const int n = wn * Cfg::WTN + j * 16 + (lane & 15);
        float v = 0.0f;
        if (m < N && n < nt) {
          const float ip = acc.a[i][j][e] * isx * isx;  // two steps: s_X^-2 may underflow
          float d2 = xn[m] + nsa[n] - 2.0f * ip;
          d2 = d2 > 0.0f ? d2 : 0.0f;
          v = -exp(-d2 * ie) * 16777216.0f;
        }
        acc.a[i][j][e] = v;
      }
  if (k > 0) pipe.run1b(acc, smem_raw);
  // run1 and run1b end on a barrier, so the column staging may reuse the LDS
  store_colmajor<Cfg, float>(acc, smem_raw, W, ldw, m0, 0, N, nt,
                             [&](int, int, float v) { return -v * (1.0f / 16777216.0f); });
}

// ------------------------------------------------------------ solve + downdate
// F(:, k + j) = G(:, j), rho = max(rho - sum_j G^2, 0), with
// G = W L^{-T} tile: 128 rows x the whole block (<= 128 columns), eight
// waves of 32 x 64, float64 MFMA.  128 rows per workgroup amortise the copy
// of L^{-1} each workgroup stages.
typedef TileCfg<double, 128, 128, 16, 4, 2> SolveCfg;

template <typename TF>
__global__ __launch_bounds__(SolveCfg::NT) void k_solve_downdate(const TF* __restrict__ W, int64_t ldw,
                                                        int64_t N, const double* __restrict__ Linv,
                                                        const int32_t* kptr, const int32_t* nTptr,
                                                        TF* __restrict__ F, int64_t ldf,
                                                        double* __restrict__ rho) {
  typedef SolveCfg Cfg;
  const int nt = *nTptr;
  if (nt == 0) return;
  const int k = *kptr;
  extern __shared__ char smem_raw[];
  double* smem = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[Cfg::WAVES_N][Cfg::BM];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  GOperand<TF, false> A{W, ldw, N, nt, nullptr, true};
  GOperand<double, true> B{Linv, MAXB, nt, nt, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  // L^{-1} is lower triangular: column j of G needs k <= j only
  tile_mainloop<Cfg, TF, false, double, true, true>(acc, A, B, m0, 0, 0, nt, smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
#pragma unroll
  for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * Cfg::WTM + i * 16 + Cfg::MM::row(lane, e);
        const int col = wn * Cfg::WTN + j * 16 + (lane & 15);
        const int64_t m = m0 + row;
        const double g = acc.a[i][j][e];
        if (m < N && col < nt) F[m + (int64_t)(k + col) * ldf] = (TF)g;
      }
  // squared row norms of G: each lane sums its columns, the 16 lanes sharing
  // a row reduce by xor shuffles, then the column halves of the workgroup
  // are added in a fixed order (deterministic)
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        const int col = wn * Cfg::WTN + j * 16 + (lane & 15);
        const double g = col < nt ? acc.a[i][j][e] : 0.0;
        s += g * g;
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      const int row = wm * Cfg::WTM + i * 16 + Cfg::MM::row(lane, e);
      if ((lane & 15) == 0) red[wn][row] = s;
    }
  }
  __syncthreads();
  for (int row = threadIdx.x; row < Cfg::BM; row += Cfg::NT) {
    const int64_t m = m0 + row;
    if (m < N) {
      double s = 0.0;
#pragma unroll
      for (int h = 0; h < Cfg::WAVES_N; ++h) s += red[h][row];
      const double v = rho[m] - s;
      rho[m] = v > 0.0 ? v : 0.0;
    }
  }
}

// ------------------------------------------------------------ persistent float64 solve
// The same G = W L^{-T} (float64 MFMA), F(:, k + j) = G(:, j) and
// rho -= rownorms(G)^2 as k_solve_downdate, organised for N >> 128: one
// workgroup per CU stages L^{-1} (128 x 128, lower triangular, zero past nT)
// in LDS once; then each of its eight waves walks 16-row blocks on its own
// (no workgroup barrier after the staging).  A wave holds two blocks of W in
// registers: while it multiplies one, the whole next block (and its rho
// entries) is in flight, so a CU keeps about 48 KB of loads outstanding.  A
// block's W entries go straight from global memory into the MFMA A operand
// (lane l: row slot l % 16, k-slot l / 16); MFMA steps wholly above the
// diagonal of L^{-1} are skipped, and the loop is specialised for the number
// of 16-column tiles nT spans (the loads and MFMAs of a block are static).
//
// Row slot s of the A operand carries block row 4 (s % 4) + s / 4.  The
// accumulator element e of lane l is row slot l / 16 + 4 e, i.e. block row
// 4 (l / 16) + e: each lane ends with four consecutive rows of one column
// and writes them with one vector store.  A row's norm is summed over its 16
// lanes by xor shuffles in a fixed order (deterministic).
constexpr int SP_LDK = MAXB + 1;  // odd stride: a fragment's 16 rows on distinct banks
// threads per workgroup: eight waves, two per SIMD (twelve were no faster
// for a float32 factor)
template <typename TF>
constexpr int sp_threads() { return 512; }

// The block loop for NTL column tiles of 16 (nT <= 16 NTL): 4 NTL k-steps,
// those past nT multiplied by zero.
template <typename TF, int NTL>
__device__ __forceinline__ void solve_persist_loop(const TF* __restrict__ W, int64_t ldw, int64_t N,
                                                   const double* Ls, int nt, int k,
                                                   TF* __restrict__ F, int64_t ldf,
                                                   double* __restrict__ rho, int64_t rb, int64_t nw) {
  constexpr int NKS = 4 * NTL;
  const int lane = threadIdx.x & 63, kq = lane >> 4, sl = lane & 15;
  const int prow = 4 * (sl & 3) + (sl >> 2);  // block row of this lane's A row slot
  // 16-byte stores of four rows need 16-byte aligned columns
  constexpr int VEC = 16 / (int)sizeof(TF);
  const bool vec_ok = (ldf % VEC) == 0 && (((uintptr_t)F) & 15) == 0;
  const int64_t nrb = (N + 15) / 16;
  const int64_t step = 4 * ldw;
  const int lb0 = sl * SP_LDK + kq;

  auto load = [&](TF (&buf)[NKS], double& rh, int64_t b) __attribute__((always_inline)) {
    const int64_t m = b * 16 + prow;
    const TF* wp = W + (m < N ? m : N - 1) + (int64_t)kq * ldw;
#pragma unroll
    for (int sq = 0; sq < NKS; ++sq) {
      buf[sq] = *wp;
      wp += step;
    }
    const int64_t mr = b * 16 + 4 * kq + (sl & 3);
    rh = rho[mr < N ? mr : N - 1];
  };
  auto block = [&](const TF (&buf)[NKS], double rh, int64_t b) __attribute__((always_inline)) {
    v4d acc[NTL];
#pragma unroll
    for (int j = 0; j < NTL; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
    // the L^{-1} fragments are the same for every block: an opaque offset
    // keeps their LDS reads in the block instead of hoisted into registers
    int lb = lb0;
    asm volatile("" : "+v"(lb));
#pragma unroll
    for (int sq = 0; sq < NKS; ++sq) {
      // only the last four k-steps can reach past nT (nT > 16 (NTL - 1))
      const double av = (sq < NKS - 4 || 4 * sq + kq < nt) ? (double)buf[sq] : 0.0;
      // tiles j >= sq / 4 meet k-step sq below or on the diagonal of L^{-1}
#pragma unroll
      for (int j = sq / 4; j < NTL; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ls[lb + 16 * j * SP_LDK + 4 * sq], acc[j], 0, 0, 0);
    }
    const int64_t row0 = b * 16 + 4 * kq;
    // whole blocks with aligned columns take vector stores (wave-uniform)
    const bool full = vec_ok && b * 16 + 16 <= N;
    double s2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
      const int col = 16 * j + sl;
      const bool cok = col < nt;
      double g[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        g[e] = cok ? acc[j][e] : 0.0;
        s2[e] += g[e] * g[e];
      }
      TF* fp = F + row0 + (int64_t)(k + col) * ldf;
      if (full) {
        if (cok) {
          if constexpr (sizeof(TF) == 4) {
            *reinterpret_cast<float4*>(fp) =
                make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
          } else {
            *reinterpret_cast<v2d*>(fp) = v2d{g[0], g[1]};
            *reinterpret_cast<v2d*>(fp + 2) = v2d{g[2], g[3]};
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (cok && row0 + e < N) fp[e] = (TF)g[e];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = s2[e];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      s2[e] = v;
    }
    // lane sl < 4 of each k-slot group updates block row 4 kq + sl
    const int q = sl & 3;
    const double v = q == 0 ? s2[0] : (q == 1 ? s2[1] : (q == 2 ? s2[2] : s2[3]));
    const int64_t row = row0 + q;
    if (sl < 4 && row < N) {
      const double r2 = rh - v;
      rho[row] = r2 > 0.0 ? r2 : 0.0;
    }
  };

  // the loads are issued unconditionally (a wave's last prefetch re-reads
  // its current block) so that the waits before each block are static
  TF wa[NKS], wb[NKS];
  double ra, rbv;
  load(wa, ra, rb);
  for (;;) {
    const int64_t rb1 = rb + nw;
    load(wb, rbv, rb1 < nrb ? rb1 : rb);
    block(wa, ra, rb);
    if (rb1 >= nrb) break;
    const int64_t rb2 = rb1 + nw;
    load(wa, ra, rb2 < nrb ? rb2 : rb1);
    block(wb, rbv, rb1);
    if (rb2 >= nrb) break;
    rb = rb2;
  }
}

template <typename TF>
__global__ __launch_bounds__(sp_threads<TF>(), 1) void k_solve_persist(const TF* __restrict__ W, int64_t ldw,
                                                            int64_t N, const double* __restrict__ Linv,
                                                            const int32_t* kptr, const int32_t* nTptr,
                                                            TF* __restrict__ F, int64_t ldf,
                                                            double* __restrict__ rho) {
  const int nt = *nTptr;
  if (nt == 0) return;
  const int k = *kptr;
  __shared__ double Ls[MAXB * SP_LDK];
  constexpr int NT = sp_threads<TF>();
  for (int e = threadIdx.x; e < MAXB * MAXB; e += NT) Ls[(e / MAXB) * SP_LDK + e % MAXB] = Linv[e];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t rb = (int64_t)blockIdx.x * (NT / 64) + wave;
  if (rb >= (N + 15) / 16) return;
  const int64_t nw = (int64_t)gridDim.x * (NT / 64);
  switch ((nt + 15) / 16) {
    case 1: solve_persist_loop<TF, 1>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 2: solve_persist_loop<TF, 2>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 3: solve_persist_loop<TF, 3>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 4: solve_persist_loop<TF, 4>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 5: solve_persist_loop<TF, 5>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 6: solve_persist_loop<TF, 6>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    case 7: solve_persist_loop<TF, 7>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
    default: solve_persist_loop<TF, 8>(W, ldw, N, Ls, nt, k, F, ldf, rho, rb, nw); break;
  }
}

static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

// ------------------------------------------------------------ split-fp16 solve
// Mixed form (bf16 distance product, float32 factor): G = W L^{-T} on the
// fp16 MFMA pipe as split pairs (three products per float32 product).  W
// already carries the bf16 kernel-entry error, which the solve amplifies by
// |L^{-1}| like any rounding in W, so the 2^-22 product error of the split
// form stays below it.
//
// k_split_linv: one workgroup scales L^{-1} (MAXB x MAXB, row-major [n][k],
// zero past nT) by the power of two 2^e that puts its largest magnitude
// below 2^14 and writes the hi/lo fp16 halves and 2^e; each thread keeps its
// 16 entries in registers between the maximum and the split.
__global__ __launch_bounds__(1024) void k_split_linv(const double* __restrict__ Linv,
                                                     const int32_t* nTptr, _Float16* __restrict__ Lh,
                                                     _Float16* __restrict__ Ll, float* __restrict__ lsc) {
  static_assert(MAXB * MAXB == 1024 * 16, "16 entries per thread");
  __shared__ double red[16];
  const int nt = *nTptr;
  // thread t holds entries 16 t .. 16 t + 15 (one row segment) in registers
  // for both the maximum and the split
  const int e0 = threadIdx.x * 16, n = e0 / MAXB, k0 = e0 % MAXB;
  double x[16];
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const v2d v = *reinterpret_cast<const v2d*>(Linv + e0 + 2 * q);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = k0 + 2 * q + h;
      x[2 * q + h] = (n < nt && k < nt) ? v[h] : 0.0;
      m = fmax(m, fabs(x[2 * q + h]));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, RPC_WAVE));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double mx = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) mx = fmax(mx, red[w]);
  double sc = 1.0;
  if (mx > 0.0 && mx < 1e300) {
    int ex;
    frexp(mx, &ex);  // mx < 2^ex
    int q = 14 - ex;
    q = q < -100 ? -100 : (q > 100 ? 100 : q);
    sc = ldexp(1.0, q);
  }
  v8h_t hi[2], lo[2];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const double xs = x[e] * sc;
    const _Float16 h = (_Float16)xs;
    hi[e / 8][e % 8] = h;
    lo[e / 8][e % 8] = (_Float16)(xs - (double)h);
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    *reinterpret_cast<v8h_t*>(Lh + e0 + 8 * g) = hi[g];
    *reinterpret_cast<v8h_t*>(Ll + e0 + 8 * g) = lo[g];
  }
  if (threadIdx.x == 0) lsc[0] = (float)sc;
}

// F(:, k + j) = G(:, j) and rho -= rownorms(G)^2 like k_solve_downdate, with
// G from split pairs.  k (<= MAXB) runs in two halves of 64: W (float32,
// scaled by 2^12; |W| <= 1 up to rounding since it is a residual kernel) and
// the pre-split L^{-1} are staged as [row][k] fp16 pairs in one LDS buffer
// (SolveSplit::bytes, which lets two workgroups share a CU), the second
// half's reads in flight while the first half's MFMAs run.
struct SolveSplit {
  static constexpr int BK = 64;
  static constexpr int LDK = BK + 8;  // 144-byte rows: fragment reads on distinct 16-byte slots
  static constexpr int EL = MAXB * LDK;
  static constexpr size_t bytes = 4 * (size_t)EL * sizeof(_Float16);
};
typedef TileCfg<__bf16, 128, 128, 64, 4, 2> SolveSplitCfg;  // fp32 accumulators, 8 waves of 32 x 64

__global__ __launch_bounds__(512, 2) void k_solve_split(const float* __restrict__ W, int64_t ldw,
                                                        int64_t N, const _Float16* __restrict__ Lh,
                                                        const _Float16* __restrict__ Ll,
                                                        const float* __restrict__ lsc,
                                                        const int32_t* kptr, const int32_t* nTptr,
                                                        float* __restrict__ F, int64_t ldf,
                                                        double* __restrict__ rho) {
  typedef SolveSplitCfg Cfg;
  static_assert(Cfg::NT == 512 && Cfg::BM == MAXB && Cfg::BN == MAXB, "one 128 x 128 tile");
  constexpr int BK = SolveSplit::BK, LDK = SolveSplit::LDK, EL = SolveSplit::EL;
  const int nt = *nTptr;
  if (nt == 0) return;
  const int k = *kptr;
  extern __shared__ char smem_raw[];
  _Float16* sm = reinterpret_cast<_Float16*>(smem_raw);
  __shared__ double red[Cfg::WAVES_N][Cfg::BM];
  const int64_t m0 = (int64_t)blockIdx.x * Cfg::BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int arow = tid & 127, ag = tid >> 7;  // A: row, k groups ag and ag + 4 of a half
  const int brow = tid >> 2, bg = tid & 3;    // B: row, k groups bg and bg + 4 of a half
  const int64_t am = m0 + arow;
  float a0[2][8], a1[2][8];
  v8h_t bh0[2], bl0[2], bh1[2], bl1[2];
  auto load = [&](float (&a)[2][8], v8h_t (&bh)[2], v8h_t (&bl)[2], int kb) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k0 = kb + 8 * (ag + 4 * h);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        a[h][e] = (am < N && k0 + e < nt) ? W[am + (int64_t)(k0 + e) * ldw] : 0.0f;
      const int kk0 = kb + 8 * (bg + 4 * h);
      bh[h] = *reinterpret_cast<const v8h_t*>(Lh + brow * MAXB + kk0);
      bl[h] = *reinterpret_cast<const v8h_t*>(Ll + brow * MAXB + kk0);
    }
  };
  auto store = [&](const float (&a)[2][8], const v8h_t (&bh)[2], const v8h_t (&bl)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v8h_t hi, lo;
      split8(a[h], hi, lo);
      const int o = arow * LDK + 8 * (ag + 4 * h);
      *reinterpret_cast<v8h_t*>(sm + o) = hi;
      *reinterpret_cast<v8h_t*>(sm + EL + o) = lo;
      const int ob = brow * LDK + 8 * (bg + 4 * h);
      *reinterpret_cast<v8h_t*>(sm + 2 * EL + ob) = bh[h];
      *reinterpret_cast<v8h_t*>(sm + 3 * EL + ob) = bl[h];
    }
  };
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  TileAcc<Cfg> acc;
  acc.zero();
  auto compute = [&](int kb) {
    const int ke = nt - kb < BK ? nt - kb : BK;
    for (int kq = 0; kq < ke; kq += 32) {
      v8h_t ah[Cfg::MI], al[Cfg::MI], fh[Cfg::NI], fl[Cfg::NI];
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i) {
        const int o = (wm * Cfg::WTM + i * 16 + (lane & 15)) * LDK + kq + 8 * (lane >> 4);
        ah[i] = *reinterpret_cast<const v8h_t*>(sm + o);
        al[i] = *reinterpret_cast<const v8h_t*>(sm + EL + o);
      }
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        const int o = (wn * Cfg::WTN + j * 16 + (lane & 15)) * LDK + kq + 8 * (lane >> 4);
        fh[j] = *reinterpret_cast<const v8h_t*>(sm + 2 * EL + o);
        fl[j] = *reinterpret_cast<const v8h_t*>(sm + 3 * EL + o);
      }
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        // L^{-1} is lower triangular: columns c0 .. c0 + 15 need k <= c0 + 15
        const int c0 = wn * Cfg::WTN + j * 16;
        if (kb + kq >= c0 + 16 || c0 >= nt) continue;
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i) {
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], fh[j], acc.a[i][j], 0, 0, 0);
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], fl[j], acc.a[i][j], 0, 0, 0);
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], fh[j], acc.a[i][j], 0, 0, 0);
        }
      }
    }
  };
  load(a0, bh0, bl0, 0);
  if (nt > BK) load(a1, bh1, bl1, BK);
  store(a0, bh0, bl0);
  __syncthreads();
  compute(0);
  if (nt > BK) {
    __syncthreads();
    store(a1, bh1, bl1);
    __syncthreads();
    compute(BK);
  }
  // unscale; each lane holds rows 4 (lane / 16) .. + 3 of one column per
  // 16 x 16 block, stored as one 16-byte write (ldf and the row offset are
  // multiples of 4)
  const float un = 1.0f / (SchurSplit::SC * lsc[0]);  // both factors are powers of two
#pragma unroll
  for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc.a[i][j][e] *= un;
      const int row = wm * Cfg::WTM + i * 16 + 4 * (lane >> 4);
      const int col = wn * Cfg::WTN + j * 16 + (lane & 15);
      const int64_t m = m0 + row;
      if (col < nt) {
        float* dst = F + m + (int64_t)(k + col) * ldf;
        if (m + 4 <= N) {
          *reinterpret_cast<v4f*>(dst) = acc.a[i][j];
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (m + e < N) dst[e] = acc.a[i][j][e];
        }
      }
    }
  // squared row norms of G (float64 sums), reduced as in k_solve_downdate
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double sq = 0.0;
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        const int col = wn * Cfg::WTN + j * 16 + (lane & 15);
        const double g = col < nt ? (double)acc.a[i][j][e] : 0.0;
        sq += g * g;
      }
      sq += __shfl_xor(sq, 1, 64);
      sq += __shfl_xor(sq, 2, 64);
      sq += __shfl_xor(sq, 4, 64);
      sq += __shfl_xor(sq, 8, 64);
      const int row = wm * Cfg::WTM + i * 16 + Cfg::MM::row(lane, e);
      if ((lane & 15) == 0) red[wn][row] = sq;
    }
  }
  __syncthreads();
  for (int row = tid; row < Cfg::BM; row += Cfg::NT) {
    const int64_t m = m0 + row;
    if (m < N) {
      double sq = 0.0;
#pragma unroll
      for (int h = 0; h < Cfg::WAVES_N; ++h) sq += red[h][row];
      const double v = rho[m] - sq;
      rho[m] = v > 0.0 ? v : 0.0;
    }
  }
}

__global__ void k_round_end(const int64_t* __restrict__ Si, int32_t* kptr, const int32_t* nTptr,
                            double* __restrict__ rho, int32_t* round_acc, int round) {
  const int nt = *nTptr;
  for (int j = threadIdx.x; j < nt; j += blockDim.x) rho[Si[j]] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    *kptr += nt;
    if (round_acc) round_acc[round] = nt;
  }
}

// Trace error after a round, sum(rho) / N (the relative trace error
// tr(K - F F^T) / tr(K), tr(K) = N for the Gaussian kernel): float64 partial
// sums over CHUNK entries, then one workgroup adds them in a fixed order.
__global__ __launch_bounds__(256) void k_trace_partial(const double* __restrict__ rho, int64_t N,
                                                       double* __restrict__ part) {
  __shared__ double ws[4];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  double s = 0.0;
  for (int e = threadIdx.x; e < CHUNK; e += 256) {
    const int64_t i = base + e;
    if (i < N) s += rho[i];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ __launch_bounds__(256) void k_trace_finish(const double* __restrict__ part, int nb,
                                                      int64_t N, double* __restrict__ out) {
  __shared__ double ws[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < nb; j += 256) s += part[j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((ws[0] + ws[1]) + (ws[2] + ws[3])) / (double)N;
}

static void launch_round_trace(const double* rho, int64_t N, double* tpart, double* round_trace,
                               int round, hipStream_t st) {
  if (!round_trace) return;
  const int nb = (int)((N + CHUNK - 1) / CHUNK);
  hipLaunchKernelGGL(k_trace_partial, dim3((unsigned)nb), dim3(256), 0, st, rho, N, tpart);
  hipLaunchKernelGGL(k_trace_finish, dim3(1), dim3(256), 0, st, (const double*)tpart, nb, N,
                     round_trace + round);
}

// Zero F columns k .. r-1 (unused budget).
template <typename TF>
__global__ __launch_bounds__(256) void k_zero_tail(TF* __restrict__ F, int64_t ldf, int64_t N, int r,
                                                   const int32_t* kptr) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int k = *kptr;
  for (int c = k; c < r; ++c) F[n + (int64_t)c * ldf] = (TF)0;
}

// The fused column+Schur kernel needs both products to accumulate in the same type.
template <typename T, typename TF>
constexpr bool kFusedColsSchur = sizeof(typename Mma<T>::acc_t) == sizeof(TF);

// ------------------------------------------------------------ host driver
struct FactorWs {
  void* Xp;
  void* xn;
  void* W;
  unsigned long long* part;
  double* pv;
  int64_t* pi;
  int64_t* prop;
  void* XS;
  void* ns;
  void* FS;
  double* H;
  double* pd2;  // slice partial sums of the proposal block
  double* pff;
  double* Lc;
  double* Linv;
  _Float16* Lh;  // split-fp16 halves of L^{-1} and their power-of-two scale
  _Float16* Ll;
  float* lsc;
  int64_t* Si;
  int32_t* acc;  // block positions of the accepted proposals
  void* XSa;
  void* nsa;
  void* FSa;
  int32_t* nT;
  int32_t* stop;
  unsigned long long* tot;
  double* tpart;   // partial sums of the per-round trace error
  unsigned* xmax;  // max |x| of the points (split-fp16 distance form)
  int64_t ldw;
  int64_t dp;
};

// Workspace: the converted points (shared by jobs on the same points) and
// the per-job round state.
template <typename T, typename TN>
static void carve_shared(WsCursor& c, FactorWs& w, int64_t N, int64_t d) {
  w.dp = (int64_t)align_up((size_t)d, 32);
  w.Xp = c.take<T>((size_t)N * w.dp);
  w.xn = c.take<TN>((size_t)N);
  w.xmax = c.take<unsigned>(1);
}

template <typename T, typename TN, typename TF>
static void carve_job(WsCursor& c, FactorWs& w, int64_t N, int64_t d, int r) {
  w.dp = (int64_t)align_up((size_t)d, 32);
  w.ldw = (int64_t)align_up((size_t)N, 8);
  const int nb = (int)((N + CHUNK - 1) / CHUNK);
  w.W = c.take<TF>((size_t)w.ldw * MAXB);
  w.part = c.take<unsigned long long>((size_t)nb);
  w.pv = c.take<double>((size_t)nb);
  w.pi = c.take<int64_t>((size_t)nb);
  w.prop = c.take<int64_t>(MAXB);
  w.XS = c.take<T>((size_t)MAXB * w.dp);
  w.ns = c.take<TN>(MAXB);
  w.FS = c.take<TF>((size_t)MAXB * r);
  w.H = c.take<double>((size_t)MAXB * MAXB);
  w.pd2 = c.take<double>((size_t)pb_slices(w.dp, r) * MAXB * MAXB);
  w.pff = c.take<double>((size_t)pb_slices(w.dp, r) * MAXB * MAXB);
  w.Lc = c.take<double>((size_t)MAXB * MAXB);
  w.Linv = c.take<double>((size_t)MAXB * MAXB);
  w.Lh = c.take<_Float16>((size_t)MAXB * MAXB);
  w.Ll = c.take<_Float16>((size_t)MAXB * MAXB);
  w.lsc = c.take<float>(1);
  w.Si = c.take<int64_t>(MAXB);
  w.acc = c.take<int32_t>(MAXB);
  w.XSa = c.take<T>((size_t)MAXB * w.dp);
  w.nsa = c.take<TN>(MAXB);
  w.FSa = c.take<TF>((size_t)MAXB * r);
  w.nT = c.take<int32_t>(1);
  w.stop = c.take<int32_t>(1);
  w.tot = c.take<unsigned long long>(1);
  w.tpart = c.take<double>((size_t)nb);
}

template <typename T, typename TN, typename TF>
static size_t carve(WsCursor& c, FactorWs& w, int64_t N, int64_t d, int r) {
  carve_shared<T, TN>(c, w, N, d);
  carve_job<T, TN, TF>(c, w, N, d, r);
  return c.used;
}

// One factorisation's arguments and round state.
template <typename T, typename TN, typename TF>
struct FJob {
  rpc_points X;  // eps is this job's
  const rpc_factor_opts* o;
  TF* F;
  int64_t ldf;
  int64_t* pivots;
  double* rho;
  int32_t* k_out;
  int32_t* status;
  FactorWs w;
};

// 128 x 128 tiles, eight waves of 64 x 32 (two per SIMD at one workgroup per
// CU, which the four-stage direct pipeline's LDS allows)
template <typename T, typename TF>
struct FCfg {
  typedef TileCfg<T, 128, 128, (sizeof(T) == 2 ? 64 : (sizeof(T) == 4 ? 32 : 16)), 2, 4> K;
  typedef TileCfg<TF, 128, 128, (sizeof(TF) == 4 ? 32 : 16), 2, 4> S;
};

static int n_rounds(const rpc_factor_opts* o) {
  if (o->mode == RPC_REPLAY) return (int)((o->n_replay + o->b - 1) / o->b);
  return (o->r + o->b - 1) / o->b;
}

static int round_block(const rpc_factor_opts* o, int i) {
  const int b = o->b;
  if (o->mode == RPC_REPLAY)
    return (int)(o->n_replay - (int64_t)i * b < b ? o->n_replay - (int64_t)i * b : b);
  return o->r - i * b < b ? o->r - i * b : b;
}

// Round i: the proposals (pivot draw, greedy argmax or replay list); returns
// the accept-test uniforms of the round (sampled mode) or null.
template <typename T, typename TN, typename TF>
static const double* draw_proposals(FJob<T, TN, TF>& j, int i, hipStream_t st) {
  const rpc_factor_opts* o = j.o;
  FactorWs& w = j.w;
  const int64_t N = j.X.N;
  const int b = o->b;
  const int nb = (int)((N + CHUNK - 1) / CHUNK);
  const int bi = round_block(o, i);
  const double* z = nullptr;
  prof::begin(prof::PIVOT, st);
  if (o->mode == RPC_SAMPLED) {
    hipLaunchKernelGGL(k_rho_partial, dim3(nb), dim3(256), 0, st, j.rho, N, w.part, w.stop);
    hipLaunchKernelGGL(k_draw_scan, dim3(1), dim3(1024), 0, st, w.part, nb, w.tot, w.stop);
    hipLaunchKernelGGL(k_draw_find, dim3(bi), dim3(256), 0, st, j.rho, N,
                       (const unsigned long long*)w.part, nb, (const unsigned long long*)w.tot,
                       o->uniforms + (int64_t)2 * b * i, w.prop, w.stop);
    z = o->uniforms + (int64_t)2 * b * i + b;
  } else if (o->mode == RPC_GREEDY) {
    hipLaunchKernelGGL(k_argmax_partial, dim3(nb), dim3(256), 0, st, j.rho, N, w.pv, w.pi, w.stop);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(256), 0, st, w.pv, w.pi, nb, w.prop, w.stop);
    z = nullptr;
  } else {
    hipLaunchKernelGGL(k_replay_props, dim3(1), dim3(MAXB), 0, st, o->replay, (int64_t)i * b, bi, N,
                       w.prop, j.status, w.stop);
  }
  prof::end(prof::PIVOT, st);
  return z;
}

// Round i, part 1: proposals, the proposal block, Algorithm 3, L^{-1}.
template <typename T, typename TN, typename TF>
static void phase_select(FJob<T, TN, TF>& j, int i, hipStream_t st) {
  const rpc_factor_opts* o = j.o;
  FactorWs& w = j.w;
  const int64_t N = j.X.N;
  const int r = o->r;
  const int64_t dp = w.dp;
  const int bi = round_block(o, i);
  const double* z = draw_proposals(j, i, st);
  prof::begin(prof::ACCEPT, st);
  hipLaunchKernelGGL((k_gather<T, TN, TF>), dim3(bi), dim3(256), 0, st, (const T*)w.Xp,
                     (const TN*)w.xn, dp, (const TF*)j.F, j.ldf, r, w.prop, bi, j.k_out, w.stop,
                     (T*)w.XS, (TN*)w.ns, (TF*)w.FS, N, j.status);
  launch_pivot_block<T, TF>((const T*)w.XS, dp, (const TF*)w.FS, r, bi, j.k_out, w.stop, j.X.eps,
                            w.pd2, w.pff, w.H, st);
  hipLaunchKernelGGL((k_accept_reject<T, TN, TF>), dim3(1), dim3(1024), 0, st, w.H, bi, w.prop, z,
                     o->tau, o->mode, (const TN*)w.ns, j.k_out, w.nT, w.stop, j.pivots, w.Lc,
                     w.Si, w.acc, (TN*)w.nsa, j.status);
  hipLaunchKernelGGL((k_copy_accepted<T, TF>), dim3(MAXB), dim3(256), 0, st, (const int32_t*)w.acc,
                     (const int32_t*)w.nT, (const int32_t*)j.k_out, (const T*)w.XS, dp,
                     (const TF*)w.FS, r, (T*)w.XSa, (TF*)w.FSa);
  hipLaunchKernelGGL(k_tri_inv, dim3(MAXB), dim3(256), 0, st, (const double*)w.Lc, w.nT, w.Linv);
  prof::end(prof::ACCEPT, st);
}

// Round i, part 2 (unfused form): the Schur update W -= F(:, :k) F(S_i, :k)^T.
template <typename T, typename TN, typename TF>
static void phase_schur(FJob<T, TN, TF>& j, hipStream_t st) {
  typedef typename FCfg<T, TF>::S CfgS;
  const size_t smS = DirectSmem<CfgS, kStages, false, true>::bytes;
  const unsigned gm = (unsigned)((j.X.N + 127) / 128);
  FactorWs& w = j.w;
  prof::begin(prof::SCHUR, st);
  hipLaunchKernelGGL((k_schur<TF, CfgS>), dim3(gm, 1), dim3(CfgS::NT), smS, st, (const TF*)j.F,
                     j.ldf, j.X.N, (const TF*)w.FSa, j.o->r, j.k_out, w.nT, (TF*)w.W, w.ldw);
  prof::end(prof::SCHUR, st);
}

// Round i, part 2: W = K(X, X_{S_i}) - F(:, :k) F(S_i, :k)^T, fused in one
// kernel unless the options ask for the separate column and Schur kernels.
template <typename T, typename TN, typename TF>
static void phase_columns(FJob<T, TN, TF>& j, hipStream_t st) {
  typedef typename FCfg<T, TF>::K CfgK;
  typedef typename FCfg<T, TF>::S CfgS;
  const int64_t N = j.X.N;
  FactorWs& w = j.w;
  const size_t smK = DirectSmem<CfgK, kStages, true, true>::bytes;
  const size_t smS = DirectSmem<CfgS, kStages, false, true>::bytes;
  const size_t smKS = smK > smS ? smK : smS;
  const unsigned gm = (unsigned)((N + 127) / 128);
  if constexpr (std::is_same<T, float>::value && std::is_same<TF, float>::value) {
    if (j.o->gemm_dtype == RPC_F32_SPLIT16) {
      // float32 points, split-fp16 distance and Schur products
      typedef typename FCfg<__bf16, float>::K Cfg;
      constexpr size_t sm = SchurSplit::bytes / 2 > ColStoreSmem<Cfg, float>::bytes
                                ? SchurSplit::bytes / 2 : ColStoreSmem<Cfg, float>::bytes;
      static_assert(2 * sm <= 160 * 1024, "two workgroups per CU");
      const bool fused = !(j.o->flags & (RPC_FACTOR_UNFUSED | RPC_FACTOR_SHARED_X));
      prof::begin(prof::KERNEL_COLS, st);
      if (fused)
        hipLaunchKernelGGL((k_cols_split<Cfg, true>), dim3(gm), dim3(Cfg::NT), sm, st,
                           (const float*)w.Xp, (const float*)w.xn, N, w.dp, (const float*)w.XSa,
                           (const float*)w.nsa, w.nT, j.X.eps, (const unsigned*)w.xmax,
                           (const float*)j.F, j.ldf, (const float*)w.FSa, j.o->r, j.k_out,
                           (float*)w.W, w.ldw);
      else
        hipLaunchKernelGGL((k_cols_split<Cfg, false>), dim3(gm), dim3(Cfg::NT), sm, st,
                           (const float*)w.Xp, (const float*)w.xn, N, w.dp, (const float*)w.XSa,
                           (const float*)w.nsa, w.nT, j.X.eps, (const unsigned*)w.xmax,
                           (const float*)j.F, j.ldf, (const float*)w.FSa, j.o->r, j.k_out,
                           (float*)w.W, w.ldw);
      prof::end(prof::KERNEL_COLS, st);
      if (!fused) phase_schur(j, st);
      return;
    }
  }
  if constexpr (kFusedColsSchur<T, TF>) {
    if (!(j.o->flags & (RPC_FACTOR_UNFUSED | RPC_FACTOR_SHARED_X))) {
      prof::begin(prof::KERNEL_COLS, st);
      constexpr bool split = std::is_same<T, __bf16>::value && std::is_same<TF, float>::value;
      // the split variant needs the larger of two direct stages, one split
      // Schur buffer and the column-store staging (two workgroups per CU)
      constexpr size_t smSplit0 = DirectSmem<CfgK, kStagesSplit, true, true>::bytes;
      constexpr size_t smSplit1 = SchurSplit::bytes / 2 > ColStoreSmem<CfgK, TF>::bytes
                                      ? SchurSplit::bytes / 2 : ColStoreSmem<CfgK, TF>::bytes;
      constexpr size_t smSplit = smSplit0 > smSplit1 ? smSplit0 : smSplit1;
      static_assert(!split || 2 * smSplit <= 160 * 1024, "two workgroups per CU");
      hipLaunchKernelGGL((k_cols_schur<T, TN, TF, CfgK, CfgS, split>), dim3(gm), dim3(CfgK::NT),
                         split ? smSplit : smKS, st, (const T*)w.Xp, (const TN*)w.xn, N, w.dp,
                         (const T*)w.XSa, (const TN*)w.nsa, w.nT, j.X.eps, (const TF*)j.F, j.ldf,
                         (const TF*)w.FSa, j.o->r, j.k_out, (TF*)w.W, w.ldw);
      prof::end(prof::KERNEL_COLS, st);
      return;
    }
  }
  // LDS of the column kernel: its direct stages or the column-store staging
  constexpr size_t smC0 = DirectSmem<CfgK, cols_stages<T>(), true, true>::bytes;
  constexpr size_t smC1 = ColStoreSmem<CfgK, TF>::bytes;
  constexpr size_t smC = smC0 > smC1 ? smC0 : smC1;
  prof::begin(prof::KERNEL_COLS, st);
  hipLaunchKernelGGL((k_kernel_cols<T, TN, TF, CfgK>), dim3(gm, 1), dim3(CfgK::NT), smC, st,
                     (const T*)w.Xp, (const TN*)w.xn, N, w.dp, (const T*)w.XSa, (const TN*)w.nsa,
                     w.nT, j.X.eps, (TF*)w.W, w.ldw);
  prof::end(prof::KERNEL_COLS, st);
  phase_schur(j, st);
}

// Round i, part 3: G = W L^{-T} into F, rho -= rownorms(G)^2, rho(S_i) = 0.
template <typename T, typename TN, typename TF>
static void phase_solve(FJob<T, TN, TF>& j, int i, hipStream_t st) {
  typedef SolveCfg CfgD;
  const int64_t N = j.X.N;
  FactorWs& w = j.w;
  const size_t smD = TileSmem<CfgD, false, true>::bytes;
  prof::begin(prof::SOLVE, st);
  // The solve is float64 (MFMA) in every form by default.  Only on request
  // (RPC_FACTOR_SPLIT_SOLVE, bf16 products with a float32 factor) does it run
  // on the fp16 pipe as split pairs: the solve multiplies the columns'
  // rounding errors by up to the condition of the pivot block, and a split
  // product's 2^-22 adds to that.
  constexpr bool can_split = std::is_same<T, __bf16>::value && std::is_same<TF, float>::value;
  if (can_split && (j.o->flags & RPC_FACTOR_SPLIT_SOLVE)) {
    hipLaunchKernelGGL(k_split_linv, dim3(1), dim3(1024), 0, st, (const double*)w.Linv, w.nT, w.Lh,
                       w.Ll, w.lsc);
    hipLaunchKernelGGL(k_solve_split, dim3((unsigned)((N + MAXB - 1) / MAXB)), dim3(512),
                       SolveSplit::bytes, st, (const float*)w.W, w.ldw, N, (const _Float16*)w.Lh,
                       (const _Float16*)w.Ll, (const float*)w.lsc, j.k_out, w.nT, (float*)j.F,
                       j.ldf, j.rho);
  } else {
    const int64_t nrb = (N + 15) / 16;
    const int64_t cus = device_cus();
    constexpr int spw = sp_threads<TF>() / 64;
    const int64_t need = (nrb + spw - 1) / spw;
    const unsigned grid = (unsigned)(need < cus ? need : cus);
    hipLaunchKernelGGL((k_solve_persist<TF>), dim3(grid), dim3(sp_threads<TF>()), 0, st,
                       (const TF*)w.W, w.ldw, N, (const double*)w.Linv, (const int32_t*)j.k_out,
                       (const int32_t*)w.nT, j.F, j.ldf, j.rho);
    (void)smD;
  }
  hipLaunchKernelGGL(k_round_end, dim3(1), dim3(MAXB), 0, st, w.Si, j.k_out, w.nT, j.rho,
                     j.o->round_accepted, i);
  launch_round_trace(j.rho, N, w.tpart, j.o->round_trace, i, st);
  prof::end(prof::SOLVE, st);
}

template <typename T, typename TN, typename TF>
static int run_factor(const rpc_points* X, const rpc_factor_opts* o, TF* F, int64_t ldf,
                      int64_t* pivots, double* rho, int32_t* k_out, void* ws, size_t ws_bytes,
                      int32_t* status, hipStream_t st) {
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  FJob<T, TN, TF> j{*X, o, F, ldf, pivots, rho, k_out, status, FactorWs{}};
  carve<T, TN, TF>(cur, j.w, X->N, X->d, o->r);
  if (!cur.ok) return RPC_EWORKSPACE;
  const int64_t N = X->N;
  const bool split = o->gemm_dtype == RPC_F32_SPLIT16;
  if (split) hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(1), 0, st, j.w.xmax);
  launch_prep<T, TN>(X, j.w.dp, (T*)j.w.Xp, (TN*)j.w.xn, rho, status, split ? j.w.xmax : nullptr, st);
  hipLaunchKernelGGL(k_init_small, dim3(1), dim3(256), 0, st, pivots, o->r, k_out, j.w.nT, j.w.stop);
  RPC_LAUNCH_CHECK();
  const int t = n_rounds(o);
  for (int i = 0; i < t; ++i) {
    phase_select(j, i, st);
    phase_columns(j, st);
    phase_solve(j, i, st);
    RPC_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_zero_tail<TF>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, F, ldf,
                     N, o->r, k_out);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

// ------------------------------------------------------------ low-memory form
// The factorisation that keeps only the r x r factor F(S, :) instead of the
// N x r factor (the low-memory variant of randomly pivoted Cholesky the
// paper's appendix on it mentions): any row of F is
// F(x, :) = K(x, X_S) F(S, :)^{-T}, so every use of F in a round is
// recomputed from kernel columns.  F(S, :) and its inverse Minv are kept in
// slot coordinates: round j's pivots occupy rows and columns SW j ..
// SW j + nT_j - 1 (SW = b rounded up to 8; unused slots are zero), R = SW t.
// Round i:
//   proposal rows  FS = K(S', X_S) Minv^T                              (b x R)
//   Schur update   F F(S_i, :)^T = K(:, X_S) Z with Z = Minv^T F(S_i, :)^T, so
//                  W = K(:, S_i) - sum_{j<i} K(:, S_j) Z(slots of j, :): the
//                  kernel columns of every earlier round are evaluated again
//                  (round i makes i extra column passes);
//   block solve    G = W L_i^{-T} updates rho; G is not kept;
//   factor         F(S_i, :) = [F(S_i, :k) | L_i] and the rows of S_i in
//                  Minv = [-L_i^{-1} F(S_i, :k) Minv_< | L_i^{-1}] (block
//                  inverse of a lower triangular matrix).
// Memory beyond the points: rho, two N x b column blocks and O(R^2).
__global__ void k_fill_f64(double* __restrict__ p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0.0;
}

__global__ void k_lm_init(int32_t* pads, int t, int sw, int32_t* zero) {
  for (int i = threadIdx.x; i < t; i += blockDim.x) pads[i] = sw * i;
  if (threadIdx.x == 0) *zero = 0;
}

// KP[j][m] = exp(-|XS_j - XSall_m|^2 / eps) in float64 for proposal j < bi
// and slot m < R; zero for slots of rounds not yet taken (>= rounds) or past
// their round's accepted count.  16 x 16 pairs per workgroup, 64 coordinates
// staged at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_lm_kp(const T* __restrict__ XS, const T* __restrict__ XSall,
                                               int64_t dp, int bi, int R, int sw, int rounds,
                                               const int32_t* __restrict__ round_nT, double eps,
                                               double* __restrict__ KP) {
  __shared__ double sa[16][65];
  __shared__ double sb[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int m = m0 + tx, j = j0 + ty;
  auto valid = [&](int mm) {
    const int jr = mm / sw, a = mm % sw;
    return mm < R && jr < rounds && a < round_nT[jr];
  };
  double d2 = 0.0;
  for (int64_t c0 = 0; c0 < dp; c0 += 64) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int rr = e / 64, cc = e % 64;
      const int64_t c = c0 + cc;
      sa[rr][cc] = (valid(m0 + rr) && c < dp) ? to_d(XSall[(int64_t)(m0 + rr) * dp + c]) : 0.0;
      sb[rr][cc] = (j0 + rr < bi && c < dp) ? to_d(XS[(int64_t)(j0 + rr) * dp + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int cc = 0; cc < 64; ++cc) {
      const double t = sa[tx][cc] - sb[ty][cc];
      d2 += t * t;
    }
    __syncthreads();
  }
  if (m < R && j < bi) KP[(int64_t)j * R + m] = valid(m) ? exp(-d2 / eps) : 0.0;
}

// FSa rows a >= nT (not written by this round's Algorithm 3) set to zero.
__global__ void k_lm_zero_rows(double* __restrict__ A, int R, const int32_t* nTptr) {
  const int nt = *nTptr;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)MAXB * R;
       e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e / R);
    if (a >= nt) A[e] = 0.0;
  }
}

// Slots SW i .. SW i + SW - 1 of F(S, :) and the diagonal block of Minv:
// FSp(SW i + a, l) = F(S_i, :)(a, l) for l < SW i, L_i(a, l - SW i) after;
// Minv(SW i + a, SW i + c) = L_i^{-1}(a, c); rows a >= nT are zero.  Both
// column-major R x R.
__global__ void k_lm_rows(double* __restrict__ FSp, double* __restrict__ Minv,
                          const double* __restrict__ FSa, const double* __restrict__ Lc,
                          const double* __restrict__ Linv, const int32_t* nTptr, int i, int sw,
                          int R) {
  const int nt = *nTptr;
  const int s0 = sw * i;
  const int64_t n = (int64_t)sw * (s0 + sw);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int a = (int)(e % sw), l = (int)(e / sw);
    double f = 0.0, v = 0.0;
    if (a < nt) {
      if (l < s0) {
        f = FSa[(int64_t)a * R + l];
      } else {
        const int c = l - s0;
        f = c <= a ? Lc[a * MAXB + c] : 0.0;
        v = Linv[a * MAXB + c];
      }
    }
    FSp[(s0 + a) + (int64_t)l * R] = f;
    if (l >= s0) Minv[(s0 + a) + (int64_t)l * R] = v;
  }
}

// Keep round i's accepted point rows, norms, count and offset.
template <typename T, typename TN>
__global__ void k_lm_save(const T* __restrict__ XSa, const TN* __restrict__ nsa, int64_t dp,
                          const int32_t* nTptr, const int32_t* kptr, int sw, T* __restrict__ XSall,
                          TN* __restrict__ nsall, int32_t* round_nT, int32_t* round_k, int i) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)sw * dp;
       e += (int64_t)gridDim.x * 256)
    XSall[e] = XSa[e];
  if (blockIdx.x == 0) {
    for (int a = threadIdx.x; a < sw; a += 256) nsall[a] = nsa[a];
    if (threadIdx.x == 0) {
      round_nT[i] = *nTptr;
      round_k[i] = *kptr;
    }
  }
}

// F(p, q) = FSp(slot p, slot q) in compact pivot order (round j's slot a is
// pivot round_k[j] + a); F is r x r column-major, cleared beforehand.
__global__ void k_lm_compact(const double* __restrict__ FSp, int R, int sw,
                             const int32_t* __restrict__ round_nT,
                             const int32_t* __restrict__ round_k, int t, double* __restrict__ F,
                             int64_t ldf) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)R * R;
       e += (int64_t)gridDim.x * 256) {
    const int pr = (int)(e % R), pc = (int)(e / R);
    const int jr = pr / sw, a = pr % sw, jc = pc / sw, c = pc % sw;
    if (jr >= t || jc >= t || a >= round_nT[jr] || c >= round_nT[jc]) continue;
    F[(int64_t)(round_k[jr] + a) + (int64_t)(round_k[jc] + c) * ldf] = FSp[e];
  }
}

__global__ void k_clear_square(double* __restrict__ F, int r, int64_t ldf) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)r * r;
       e += (int64_t)gridDim.x * 256)
    F[(e % r) + (e / r) * ldf] = 0.0;
}

struct LowMemWs {
  double* Minv;
  double* FSp;
  double* Z;
  double* KP;
  double* Wt;
  void* XSall;
  void* nsall;
  int32_t* round_nT;
  int32_t* round_k;
  int32_t* pads;
  int32_t* zero;
};

static int lm_slot(const rpc_factor_opts* o) { return (int)align_up((size_t)o->b, 8); }

template <typename T, typename TN>
static size_t carve_lowmem(WsCursor& c, FactorWs& w, LowMemWs& l, int64_t N, int64_t d,
                           const rpc_factor_opts* o) {
  const int t = n_rounds(o), sw = lm_slot(o), R = sw * t;
  carve<T, TN, double>(c, w, N, d, R);  // FS / FSa rows have R entries (slot coordinates)
  l.Minv = c.take<double>((size_t)R * R);
  l.FSp = c.take<double>((size_t)R * R);
  l.Z = c.take<double>((size_t)R * MAXB);
  l.KP = c.take<double>((size_t)MAXB * R);
  l.Wt = c.take<double>((size_t)w.ldw * MAXB);
  // + MAXB rows: the column kernel's direct loads read whole 128-row tiles of
  // a round's block, which for the last rounds' blocks run past R
  l.XSall = c.take<T>((size_t)(R + MAXB) * w.dp);
  l.nsall = c.take<TN>((size_t)R);
  l.round_nT = c.take<int32_t>((size_t)t);
  l.round_k = c.take<int32_t>((size_t)t);
  l.pads = c.take<int32_t>((size_t)t);
  l.zero = c.take<int32_t>(1);
  return c.used;
}

template <typename T, typename TN>
static int run_factor_lowmem(const rpc_points* X, const rpc_factor_opts* o, double* F, int64_t ldf,
                             int64_t* pivots, double* rho, int32_t* k_out, void* ws,
                             size_t ws_bytes, int32_t* status, hipStream_t st) {
  typedef typename FCfg<T, double>::K CfgK;
  typedef typename FCfg<T, double>::S CfgS;
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  FJob<T, TN, double> j{*X, o, nullptr, 0, pivots, rho, k_out, status, FactorWs{}};
  LowMemWs l;
  carve_lowmem<T, TN>(cur, j.w, l, X->N, X->d, o);
  if (!cur.ok) return RPC_EWORKSPACE;
  FactorWs& w = j.w;
  const int64_t N = X->N, dp = w.dp;
  const int t = n_rounds(o), sw = lm_slot(o), R = sw * t;
  auto clear = [&](double* p, int64_t n) {
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  };
  clear(l.Minv, (int64_t)R * R);
  clear(l.FSp, (int64_t)R * R);
  clear((double*)w.FS, (int64_t)MAXB * R);
  clear((double*)w.FSa, (int64_t)MAXB * R);
  hipLaunchKernelGGL(k_lm_init, dim3(1), dim3(256), 0, st, l.pads, t, sw, l.zero);
  launch_prep<T, TN>(X, dp, (T*)w.Xp, (TN*)w.xn, rho, status, nullptr, st);
  hipLaunchKernelGGL(k_init_small, dim3(1), dim3(256), 0, st, pivots, o->r, k_out, w.nT, w.stop);
  RPC_LAUNCH_CHECK();
  constexpr size_t smC0 = DirectSmem<CfgK, cols_stages<T>(), true, true>::bytes;
  constexpr size_t smC1 = ColStoreSmem<CfgK, double>::bytes;
  constexpr size_t smC = smC0 > smC1 ? smC0 : smC1;
  const size_t smS = DirectSmem<CfgS, kStages, false, true>::bytes;
  const size_t smD = TileSmem<SolveCfg, false, true>::bytes;
  const unsigned gm = (unsigned)((N + 127) / 128);
  const unsigned gs = (unsigned)((N + SolveCfg::BM - 1) / SolveCfg::BM);
  for (int i = 0; i < t; ++i) {
    const int bi = round_block(o, i);
    const double* z = draw_proposals(j, i, st);
    prof::begin(prof::ACCEPT, st);
    // proposal rows: points and norms gathered, F rows from the kernel
    hipLaunchKernelGGL((k_gather<T, TN, double>), dim3(bi), dim3(256), 0, st, (const T*)w.Xp,
                       (const TN*)w.xn, dp, (const double*)nullptr, (int64_t)0, R, w.prop, bi,
                       (const int32_t*)l.zero, w.stop, (T*)w.XS, (TN*)w.ns, (double*)w.FS, N,
                       status);
    hipLaunchKernelGGL((k_lm_kp<T>), dim3((unsigned)((R + 15) / 16), (unsigned)((bi + 15) / 16)),
                       dim3(256), 0, st, (const T*)w.XS, (const T*)l.XSall, dp, bi, R, sw, i,
                       (const int32_t*)l.round_nT, X->eps, l.KP);
    dense::gemm64<false, true>(st, R, bi, R, l.Minv, R, l.KP, R, (double*)w.FS, R, 1.0, 0.0);
    launch_pivot_block<T, double>((const T*)w.XS, dp, (const double*)w.FS, R, bi,
                                  (const int32_t*)(l.pads + i), w.stop, X->eps, w.pd2, w.pff, w.H,
                                  st);
    hipLaunchKernelGGL((k_accept_reject<T, TN, double>), dim3(1), dim3(1024), 0, st, w.H, bi,
                       w.prop, z, o->tau, o->mode, (const TN*)w.ns, k_out, w.nT, w.stop, pivots,
                       w.Lc, w.Si, w.acc, (TN*)w.nsa, status);
    hipLaunchKernelGGL((k_copy_accepted<T, double>), dim3(MAXB), dim3(256), 0, st,
                       (const int32_t*)w.acc, (const int32_t*)w.nT,
                       (const int32_t*)(l.pads + i), (const T*)w.XS, dp, (const double*)w.FS, R,
                       (T*)w.XSa, (double*)w.FSa);
    hipLaunchKernelGGL(k_lm_zero_rows, dim3((unsigned)((MAXB * R + 255) / 256)), dim3(256), 0, st,
                       (double*)w.FSa, R, (const int32_t*)w.nT);
    hipLaunchKernelGGL(k_tri_inv, dim3(MAXB), dim3(256), 0, st, (const double*)w.Lc, w.nT, w.Linv);
    prof::end(prof::ACCEPT, st);
    // W = K(:, S_i) - sum_{j<i} K(:, S_j) Z(slots of j, :)
    prof::begin(prof::KERNEL_COLS, st);
    dense::gemm64<true, true>(st, R, MAXB, R, l.Minv, R, (const double*)w.FSa, R, l.Z, R, 1.0, 0.0);
    hipLaunchKernelGGL((k_kernel_cols<T, TN, double, CfgK>), dim3(gm, 1), dim3(CfgK::NT), smC, st,
                       (const T*)w.Xp, (const TN*)w.xn, N, dp, (const T*)w.XSa, (const TN*)w.nsa,
                       w.nT, X->eps, (double*)w.W, w.ldw);
    for (int jj = 0; jj < i; ++jj) {
      hipLaunchKernelGGL((k_kernel_cols<T, TN, double, CfgK>), dim3(gm, 1), dim3(CfgK::NT), smC,
                         st, (const T*)w.Xp, (const TN*)w.xn, N, dp,
                         (const T*)l.XSall + (int64_t)sw * jj * dp, (const TN*)l.nsall + sw * jj,
                         (const int32_t*)(l.round_nT + jj), X->eps, l.Wt, w.ldw);
      hipLaunchKernelGGL((k_schur<double, CfgS>), dim3(gm, 1), dim3(CfgS::NT), smS, st,
                         (const double*)l.Wt, w.ldw, N, (const double*)(l.Z + sw * jj), R,
                         (const int32_t*)(l.round_nT + jj), w.nT, (double*)w.W, w.ldw);
    }
    prof::end(prof::KERNEL_COLS, st);
    // rho -= rownorms(W L_i^{-T})^2 (the block of F itself goes to scratch)
    prof::begin(prof::SOLVE, st);
    hipLaunchKernelGGL((k_solve_downdate<double>), dim3(gs), dim3(SolveCfg::NT), smD, st,
                       (const double*)w.W, w.ldw, N, w.Linv, (const int32_t*)l.zero, w.nT, l.Wt,
                       w.ldw, rho);
    // F(S_i, :), Minv's rows of S_i
    hipLaunchKernelGGL(k_lm_rows, dim3((unsigned)(((int64_t)sw * sw * (i + 1) + 255) / 256)),
                       dim3(256), 0, st, l.FSp, l.Minv, (const double*)w.FSa, (const double*)w.Lc,
                       (const double*)w.Linv, (const int32_t*)w.nT, i, sw, R);
    if (i > 0)
      dense::gemm64<true, false>(st, sw, (int64_t)sw * i, MAXB, w.Linv, MAXB, l.Z, R,
                                 l.Minv + (int64_t)sw * i, R, -1.0, 0.0);
    hipLaunchKernelGGL((k_lm_save<T, TN>), dim3((unsigned)((sw * dp + 255) / 256)), dim3(256), 0, st,
                       (const T*)w.XSa, (const TN*)w.nsa, dp, (const int32_t*)w.nT,
                       (const int32_t*)k_out, sw, (T*)l.XSall + (int64_t)sw * i * dp,
                       (TN*)l.nsall + sw * i, l.round_nT, l.round_k, i);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(MAXB), 0, st, w.Si, k_out, w.nT, rho,
                       o->round_accepted, i);
    launch_round_trace(rho, N, w.tpart, o->round_trace, i, st);
    prof::end(prof::SOLVE, st);
    RPC_LAUNCH_CHECK();
  }
  const unsigned gc = (unsigned)(((int64_t)R * R + 255) / 256 < 4096 ? ((int64_t)R * R + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_clear_square, dim3(gc), dim3(256), 0, st, F, o->r, ldf);
  hipLaunchKernelGGL(k_lm_compact, dim3(gc), dim3(256), 0, st, (const double*)l.FSp, R, sw,
                     (const int32_t*)l.round_nT, (const int32_t*)l.round_k, t, F, ldf);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

// ------------------------------------------------------------ shared points
// Kernel columns of a group of factorisations of the same points at
// different bandwidths, in one launch per round: workgroup (job g, row tile)
// computes W_g = K_g(X tile, X_{S_g}) exactly as k_kernel_cols does for job g
// alone (same main loop and epilogue, job g's eps per column).  The
// workgroups of all jobs for one row tile are adjacent and on the same XCD,
// so each tile of X is fetched from HBM once per round for the group and
// served from that XCD's L2 to the other bandwidths.
constexpr int MAX_GROUP = 16;

template <typename T, typename TN, typename TW>
struct ColGroup {
  const T* XSa[MAX_GROUP];
  const TN* nsa[MAX_GROUP];
  const int32_t* nT[MAX_GROUP];
  TW* W[MAX_GROUP];
  double eps[MAX_GROUP];
  int G;
};

template <typename T, typename TN, typename TW, class Cfg>
__global__ __launch_bounds__(Cfg::NT, sizeof(T) == 2 ? 4 : 1) void k_kernel_cols_group(const T* __restrict__ Xp,
                                                               const TN* __restrict__ xn, int64_t N,
                                                               int64_t dp, int tiles,
                                                               ColGroup<T, TN, TW> grp, int64_t ldw) {
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int g = slot % grp.G;
  const int tile = (slot / grp.G) * 8 + xcd;
  if (tile >= tiles) return;
  const int nt = *grp.nT[g];
  if (nt == 0) return;
  extern __shared__ char smem_raw[];
  typename Cfg::T* smem = reinterpret_cast<typename Cfg::T*>(smem_raw);
  const int64_t m0 = (int64_t)tile * Cfg::BM;
  GOperand<T, true> A{Xp, dp, N, dp, nullptr, true};
  GOperand<T, true> B{grp.XSa[g], dp, nt, dp, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop_direct<Cfg, cols_stages<T>()>(acc, A, B, m0, 0, 0, dp, N, MAXB, smem, nt, tile);
  typedef typename Cfg::MM::acc_t AT;
  const AT ie = (AT)(1.0 / grp.eps[g]);
  const TN* nsa = grp.nsa[g];
  store_colmajor<Cfg, TW>(acc, smem, grp.W[g], ldw, m0, 0, N, nt, [&](int row, int col, AT v) {
    const int64_t m = m0 + row, n = col;
    if (m >= N || n >= nt) return (TW)0;
    AT d2 = (AT)xn[m] + (AT)nsa[n] - (AT)2 * v;
    d2 = d2 > (AT)0 ? d2 : (AT)0;
    return (TW)exp(-d2 * ie);
  });
}

__global__ void k_fill_rho(double* rho, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < N) rho[i] = 1.0;
}

__global__ void k_status_from(const int32_t* src, int32_t* dst) {
  if (*src != RPC_OK) set_status(dst, *src);
}

template <typename T, typename TN, typename TF>
static size_t group_ws(int64_t N, int64_t d, int r, int G) {
  WsCursor c{nullptr, 0, 0, true};
  FactorWs w;
  carve_shared<T, TN>(c, w, N, d);
  for (int g = 0; g < G; ++g) carve_job<T, TN, TF>(c, w, N, d, r);
  return c.used;
}

template <typename T, typename TN, typename TF>
static int run_factor_group(const rpc_points* X, const double* eps, const rpc_factor_opts* const* opts,
                            int G, void* const* F, int64_t ldf, int64_t* const* pivots,
                            double* const* rho, int32_t* const* k_out, int32_t* const* status,
                            void* ws, size_t ws_bytes, hipStream_t st) {
  typedef typename FCfg<T, TF>::K CfgK;
  WsCursor cur{(char*)ws, 0, ws_bytes, true};
  FactorWs shared;
  carve_shared<T, TN>(cur, shared, X->N, X->d);
  FJob<T, TN, TF> jobs[MAX_GROUP];
  for (int g = 0; g < G; ++g) {
    jobs[g] = FJob<T, TN, TF>{*X, opts[g], (TF*)F[g], ldf, pivots[g], rho[g], k_out[g], status[g],
                              FactorWs{}};
    jobs[g].X.eps = eps[g];
    carve_job<T, TN, TF>(cur, jobs[g].w, X->N, X->d, opts[g]->r);
    jobs[g].w.Xp = shared.Xp;
    jobs[g].w.xn = shared.xn;
  }
  if (!cur.ok) return RPC_EWORKSPACE;
  const int64_t N = X->N;
  const int64_t dp = shared.dp;
  // the points are converted once; every job starts from rho = 1
  launch_prep<T, TN>(X, dp, (T*)shared.Xp, (TN*)shared.xn, rho[0], status[0], nullptr, st);
  for (int g = 0; g < G; ++g) {
    if (g > 0) {
      hipLaunchKernelGGL(k_fill_rho, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, rho[g], N);
      hipLaunchKernelGGL(k_status_from, dim3(1), dim3(1), 0, st, (const int32_t*)status[0], status[g]);
    }
    hipLaunchKernelGGL(k_init_small, dim3(1), dim3(256), 0, st, pivots[g], opts[g]->r, k_out[g],
                       jobs[g].w.nT, jobs[g].w.stop);
  }
  RPC_LAUNCH_CHECK();
  ColGroup<T, TN, TF> grp{};
  grp.G = G;
  for (int g = 0; g < G; ++g) {
    grp.XSa[g] = (const T*)jobs[g].w.XSa;
    grp.nsa[g] = (const TN*)jobs[g].w.nsa;
    grp.nT[g] = jobs[g].w.nT;
    grp.W[g] = (TF*)jobs[g].w.W;
    grp.eps[g] = eps[g];
  }
  const int tiles = (int)((N + 127) / 128);
  const unsigned blocks = (unsigned)(8 * ((tiles + 7) / 8) * G);
  constexpr size_t smC0 = DirectSmem<CfgK, cols_stages<T>(), true, true>::bytes;
  constexpr size_t smC1 = ColStoreSmem<CfgK, TF>::bytes;
  constexpr size_t smK = smC0 > smC1 ? smC0 : smC1;
  const int t = n_rounds(opts[0]);
  for (int i = 0; i < t; ++i) {
    for (int g = 0; g < G; ++g) phase_select(jobs[g], i, st);
    prof::begin(prof::KERNEL_COLS, st);
    hipLaunchKernelGGL((k_kernel_cols_group<T, TN, TF, CfgK>), dim3(blocks), dim3(CfgK::NT), smK, st,
                       (const T*)shared.Xp, (const TN*)shared.xn, N, dp, tiles, grp, jobs[0].w.ldw);
    prof::end(prof::KERNEL_COLS, st);
    for (int g = 0; g < G; ++g) phase_schur(jobs[g], st);
    for (int g = 0; g < G; ++g) phase_solve(jobs[g], i, st);
    RPC_LAUNCH_CHECK();
  }
  for (int g = 0; g < G; ++g)
    hipLaunchKernelGGL((k_zero_tail<TF>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       (TF*)F[g], ldf, N, opts[g]->r, k_out[g]);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

static int check_factor_args(const rpc_points* X, const rpc_factor_opts* o) {
  if (!X || !o || !X->X) return RPC_EINVAL;
  if (X->dtype != RPC_F32 && X->dtype != RPC_F64 && X->dtype != RPC_BF16) return RPC_EINVAL;
  if (X->N < 1 || X->d < 1 || X->ldx < X->d || !(X->eps > 0.0)) return RPC_EINVAL;
  if (o->r < 1 || o->r > X->N || o->b < 1 || o->b > MAXB) return RPC_EINVAL;
  if (o->mode == RPC_GREEDY && o->b != 1) return RPC_EINVAL;
  if (o->mode != RPC_SAMPLED && o->mode != RPC_GREEDY && o->mode != RPC_REPLAY) return RPC_EINVAL;
  if (o->gemm_dtype != RPC_F64 && o->gemm_dtype != RPC_F32 && o->gemm_dtype != RPC_BF16 &&
      o->gemm_dtype != RPC_F32_SPLIT16)
    return RPC_EINVAL;
  if (o->factor_dtype != RPC_F64 && o->factor_dtype != RPC_F32) return RPC_EINVAL;
  if (o->gemm_dtype == RPC_F64 && o->factor_dtype != RPC_F64) return RPC_EINVAL;
  if (o->gemm_dtype == RPC_F32_SPLIT16 && o->factor_dtype != RPC_F32) return RPC_EINVAL;
  if (o->mode == RPC_SAMPLED) {
    const int64_t t = (o->r + o->b - 1) / o->b;
    if (!o->uniforms || o->n_uniforms < 2 * (int64_t)o->b * t) return RPC_EINVAL;
  }
  if (o->mode == RPC_REPLAY) {
    if (!o->replay || o->n_replay < 1 || o->n_replay > o->r) return RPC_EINVAL;
  }
  if (!(o->tau >= 0.0)) return RPC_EINVAL;
  if (o->flags &
      ~(RPC_FACTOR_UNFUSED | RPC_FACTOR_SHARED_X | RPC_FACTOR_LOW_MEMORY | RPC_FACTOR_SPLIT_SOLVE))
    return RPC_EINVAL;
  if ((o->flags & RPC_FACTOR_SPLIT_SOLVE) &&
      (o->gemm_dtype != RPC_BF16 || o->factor_dtype != RPC_F32 || (o->flags & RPC_FACTOR_LOW_MEMORY)))
    return RPC_EINVAL;
  if ((o->flags & RPC_FACTOR_LOW_MEMORY) &&
      (o->factor_dtype != RPC_F64 || (o->flags & RPC_FACTOR_SHARED_X)))
    return RPC_EINVAL;
  if (X->N > (int64_t)1 << 23) return RPC_EINVAL;  // keeps sum(rho_q) < 2^63
  return RPC_OK;
}

template <typename Fn>
static int dispatch(const rpc_factor_opts* o, Fn&& fn) {
  if (o->gemm_dtype == RPC_F64) return fn((double*)0, (double*)0, (double*)0);
  if (o->gemm_dtype == RPC_F32_SPLIT16) return fn((float*)0, (float*)0, (float*)0);
  if (o->gemm_dtype == RPC_F32) {
    if (o->factor_dtype == RPC_F32) return fn((float*)0, (float*)0, (float*)0);
    return fn((float*)0, (float*)0, (double*)0);
  }
  if (o->factor_dtype == RPC_F32) return fn((__bf16*)0, (float*)0, (float*)0);
  return fn((__bf16*)0, (float*)0, (double*)0);
}

}  // namespace

extern "C" int rpchol_factor_workspace_size(const rpc_points* X, const rpc_factor_opts* o,
                                            size_t* bytes) {
  int rc = check_factor_args(X, o);
  if (rc) return rc;
  if (!bytes) return RPC_EINVAL;
  return dispatch(o, [&](auto* t, auto* tn, auto* tf) {
    typedef typename std::remove_pointer<decltype(t)>::type T;
    typedef typename std::remove_pointer<decltype(tn)>::type TN;
    typedef typename std::remove_pointer<decltype(tf)>::type TF;
    WsCursor c{nullptr, 0, 0, true};
    FactorWs w;
    if (o->flags & RPC_FACTOR_LOW_MEMORY) {
      LowMemWs l;
      *bytes = carve_lowmem<T, TN>(c, w, l, X->N, X->d, o);
    } else {
      *bytes = carve<T, TN, TF>(c, w, X->N, X->d, o->r);
    }
    return (int)RPC_OK;
  });
}

extern "C" int rpchol_factor(const rpc_points* X, const rpc_factor_opts* o, void* F, int64_t ldf,
                             int64_t* pivots, double* rho, int32_t* k_out, void* ws,
                             size_t ws_bytes, int32_t* status, rpc_stream_t stream) {
  int rc = check_factor_args(X, o);
  if (rc) return rc;
  const bool lowmem = (o->flags & RPC_FACTOR_LOW_MEMORY) != 0;
  if (!F || !pivots || !rho || !k_out || !status || ldf < (lowmem ? o->r : X->N) || ldf % 8 != 0)
    return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return dispatch(o, [&](auto* t, auto* tn, auto* tf) {
    typedef typename std::remove_pointer<decltype(t)>::type T;
    typedef typename std::remove_pointer<decltype(tn)>::type TN;
    typedef typename std::remove_pointer<decltype(tf)>::type TF;
    if constexpr (std::is_same<TF, double>::value) {
      if (lowmem)
        return run_factor_lowmem<T, TN>(X, o, (double*)F, ldf, pivots, rho, k_out, ws, ws_bytes,
                                        status, st);
    }
    return run_factor<T, TN, TF>(X, o, (TF*)F, ldf, pivots, rho, k_out, ws, ws_bytes, status, st);
  });
}

namespace {
// Group options: every job as rpchol_factor accepts it, sharing everything
// but the uniforms and round_accepted, SAMPLED or GREEDY, with SHARED_X set.
int check_group_args(const rpc_points* X, const double* eps, const rpc_factor_opts* const* opts,
                     int32_t G) {
  if (!X || !opts || !eps || G < 1 || G > MAX_GROUP) return RPC_EINVAL;
  for (int g = 0; g < G; ++g) {
    if (!opts[g]) return RPC_EINVAL;
    rpc_points Xg = *X;
    Xg.eps = eps[g];
    const int rc = check_factor_args(&Xg, opts[g]);
    if (rc) return rc;
    const rpc_factor_opts* a = opts[0];
    const rpc_factor_opts* o = opts[g];
    if (!(o->flags & RPC_FACTOR_SHARED_X)) return RPC_EINVAL;
    if (o->mode == RPC_REPLAY || o->gemm_dtype == RPC_F32_SPLIT16) return RPC_EINVAL;
    if (o->flags & RPC_FACTOR_LOW_MEMORY) return RPC_EINVAL;
    if (o->r != a->r || o->b != a->b || o->mode != a->mode || o->gemm_dtype != a->gemm_dtype ||
        o->factor_dtype != a->factor_dtype || o->tau != a->tau || o->flags != a->flags)
      return RPC_EINVAL;
  }
  return RPC_OK;
}
}  // namespace

extern "C" int rpchol_factor_group_workspace_size(const rpc_points* X, const rpc_factor_opts* o,
                                                  int32_t n_group, size_t* bytes) {
  if (!X || !o || !bytes || n_group < 1 || n_group > MAX_GROUP) return RPC_EINVAL;
  rpc_points X1 = *X;  // the points' eps is not used by a group
  X1.eps = 1.0;
  int rc = check_factor_args(&X1, o);
  if (rc) return rc;
  if (o->gemm_dtype == RPC_F32_SPLIT16) return RPC_EINVAL;  // not offered for groups
  return dispatch(o, [&](auto* t, auto* tn, auto* tf) {
    typedef typename std::remove_pointer<decltype(t)>::type T;
    typedef typename std::remove_pointer<decltype(tn)>::type TN;
    typedef typename std::remove_pointer<decltype(tf)>::type TF;
    *bytes = group_ws<T, TN, TF>(X->N, X->d, o->r, n_group);
    return (int)RPC_OK;
  });
}

extern "C" int rpchol_factor_group(const rpc_points* X, const double* eps,
                                   const rpc_factor_opts* const* opts, int32_t n_group,
                                   void* const* F, int64_t ldf, int64_t* const* pivots,
                                   double* const* rho, int32_t* const* k_out,
                                   int32_t* const* status, void* ws, size_t ws_bytes,
                                   rpc_stream_t stream) {
  int rc = check_group_args(X, eps, opts, n_group);
  if (rc) return rc;
  if (!F || !pivots || !rho || !k_out || !status || ldf < X->N || ldf % 8 != 0) return RPC_EINVAL;
  for (int g = 0; g < n_group; ++g)
    if (!F[g] || !pivots[g] || !rho[g] || !k_out[g] || !status[g]) return RPC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return dispatch(opts[0], [&](auto* t, auto* tn, auto* tf) {
    typedef typename std::remove_pointer<decltype(t)>::type T;
    typedef typename std::remove_pointer<decltype(tn)>::type TN;
    typedef typename std::remove_pointer<decltype(tf)>::type TF;
    return run_factor_group<T, TN, TF>(X, eps, opts, n_group, F, ldf, pivots, rho, k_out, status,
                                       ws, ws_bytes, st);
  });
}
