// Symmetric Gram products of a tall column-major factor, as MFMA tiles.
//
//   G_z = (diag(s_z) A)^T (diag(s_z) A),   A: N x r column-major (lda),
//
// for one or two row scalings z at once.  The reduction runs over N, so the
// work is split into row chunks; each workgroup owns one 128 x 128 tile of
// the upper triangle for one chunk and writes its float64 partial sum, and a
// second kernel adds the chunk partials in a fixed order (deterministic).
//
// Layout choices for gfx950:
//   * only upper-triangle tiles are launched; a diagonal tile loads its
//     operand once and uses it on both sides;
//   * the workgroup -> (chunk, tile) map sends every tile of one chunk to the
//     same XCD, so the chunk's rows are fetched into that XCD's L2 once;
//   * operands are read as 128-byte column segments (A^T is k-contiguous),
//     staged through LDS with the next segment prefetched into registers
//     while the current one feeds the MFMAs;
//   * float32 tiles are flushed into float64 accumulators every 256 rows, so a
//     float32 run sums at most 64 MFMA steps; eight waves of 64 x 32 keep the
//     float64 copy within two waves per SIMD of register budget.
#pragma once
#include "common.hpp"

namespace syrk {
namespace {

constexpr int TILE = 128;
constexpr int NTH = 512;  // 8 waves: 2 along rows x 4 along columns, 64 x 32 each
constexpr int WTM = 64, WTN = 32, MI = WTM / 16, NI = WTN / 16;
constexpr int FLUSH_ROWS = 256;  // float32 runs joined into float64 accumulators

__host__ __device__ inline int n_tiles(int r) { return (r + TILE - 1) / TILE; }
__host__ __device__ inline int n_upper(int nt) { return nt * (nt + 1) / 2; }
__host__ __device__ inline int upper_index(int ti, int tj, int nt) {
  return ti * nt - ti * (ti - 1) / 2 + (tj - ti);
}
__device__ inline void upper_decode(int t, int nt, int& ti, int& tj) {
  int a = 0;
  while (t >= nt - a) {
    t -= nt - a;
    ++a;
  }
  ti = a;
  tj = a + t;
}

template <typename T>
struct SyrkTraits;
// BK is a multiple of 16 k (four MFMA k-steps); the row stride LDK = BK + PAD
// (272 bytes for float32, 144 for float64) puts the 16 rows of a vector
// fragment read on distinct banks.
template <>
struct SyrkTraits<float> {
  static constexpr int BK = 64;
  static constexpr int PAD = 4;
};
template <>
struct SyrkTraits<double> {
  static constexpr int BK = 16;
  static constexpr int PAD = 2;
};

template <typename T, typename TF>
struct SyrkLoader {
  static constexpr int BK = SyrkTraits<T>::BK;
  static constexpr int V = 16 / sizeof(TF);
  static constexpr int VPC = BK / V;             // vectors per column segment
  static constexpr int PER = TILE * VPC / NTH;   // vectors per thread
  typedef TF vt __attribute__((ext_vector_type(V)));
  static_assert(NTH % VPC == 0, "every vector of a thread covers the same rows n");
  vt buf[PER];
  T sc[V];  // row scales: the same n offsets for all PER vectors of a thread

  __device__ inline void load(const TF* __restrict__ A, int64_t lda, int r, int c0,
                              const T* __restrict__ s, int64_t n0, int64_t n1, int tid) {
    typedef T st __attribute__((ext_vector_type(V)));
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * NTH;
      const int col = vid / VPC;
      const int64_t n = n0 + (vid % VPC) * V;
      const int gc = c0 + col;
      if (gc < r && n + V <= n1) {
        buf[p] = *reinterpret_cast<const vt*>(A + (int64_t)gc * lda + n);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const bool ok = gc < r && n + e < n1;
          buf[p][e] = ok ? A[(int64_t)gc * lda + n + e] : (TF)0;
        }
      }
      if (p == 0) {
        if (s && n + V <= n1) {
          if constexpr (sizeof(T) == sizeof(TF)) {
            const st sv = *reinterpret_cast<const st*>(s + n);
#pragma unroll
            for (int e = 0; e < V; ++e) sc[e] = sv[e];
          } else {
#pragma unroll
            for (int e = 0; e < V; ++e) sc[e] = s[n + e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) sc[e] = (n + e < n1) ? (s ? s[n + e] : (T)1) : (T)0;
        }
      }
    }
  }
  __device__ inline void store(T* __restrict__ lds, int tid) const {
    constexpr int LDK = BK + SyrkTraits<T>::PAD;
    typedef T st __attribute__((ext_vector_type(V)));
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * NTH;
      const int col = vid / VPC;
      const int kv = (vid % VPC) * V;
      st v;
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] = (T)buf[p][e] * sc[e];
      if constexpr (sizeof(T) == sizeof(TF)) {
        *reinterpret_cast<st*>(lds + col * LDK + kv) = v;
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) lds[col * LDK + kv + e] = v[e];
      }
    }
  }
};

// grid.x = 8 * ceil(groups / 8) * n_upper, groups = nz * nch (z-major).
// Group g of a Gram launch -> (Gram z, row chunk ch).  Workgroups are
// dealt to the 8 XCDs in turn, so groups g and g + 8 run on the same XCD one
// after the other; the nz Grams of one row chunk are placed there, and the
// second reads the chunk's F panels while the first has them in that XCD's
// L2.  g covers group_slots(nz, nch) groups; false for the padding ones.
__device__ inline bool group_decode(int g, int nz, int nch, int& z, int& ch) {
  const int blk = g / (8 * nz), w = g % (8 * nz);
  z = w / 8;
  ch = blk * 8 + w % 8;
  return ch < nch;
}
__host__ __device__ inline int group_slots(int nz, int nch) { return 8 * nz * ((nch + 7) / 8); }

template <typename T, typename TF>
__global__ __launch_bounds__(NTH, 2) void k_syrk_partial(const TF* __restrict__ A, int64_t lda,
                                                         int64_t N, int r, const T* __restrict__ s0,
                                                         const T* __restrict__ s1, int nz,
                                                         int64_t chunk, int nch,
                                                         double* __restrict__ part0,
                                                         double* __restrict__ part1,
                                                         const int32_t* kptr) {
  typedef Mma<T> MM;
  constexpr int BK = SyrkTraits<T>::BK;
  constexpr int LDK = BK + SyrkTraits<T>::PAD;
  constexpr bool F32 = sizeof(T) == 4;
  static_assert(BK % (4 * Mma<T>::KS) == 0 && (LDK * sizeof(T)) % 16 == 0, "vector fragment reads");
  __shared__ __attribute__((aligned(16))) T As[2][TILE * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][TILE * LDK];
  const int nt = n_tiles(r);
  const int nu = n_upper(nt);
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int g = (slot / nu) * 8 + xcd;
  int z, ch;
  if (g >= group_slots(nz, nch) || !group_decode(g, nz, nch, z, ch)) return;
  const int tile = slot % nu;
  int ti, tj;
  upper_decode(tile, nt, ti, tj);
  // columns >= k are zero: tiles entirely beyond k are skipped (the reduce
  // writes zeros there)
  const int kk = kptr ? *kptr : r;
  if (tj * TILE >= kk) return;
  const bool diag = ti == tj;
  const T* s = z ? s1 : s0;
  double* out = (z ? part1 : part0) + ((int64_t)ch * nu + tile) * TILE * TILE;
  const int64_t n0 = (int64_t)ch * chunk;
  const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  typename MM::acc acc[MI][NI];
  double acc64[F32 ? MI : 1][F32 ? NI : 1][4];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;
  if constexpr (F32) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc64[i][j][e] = 0.0;
  }
  SyrkLoader<T, TF> la, lb;
  la.load(A, lda, r, ti * TILE, s, n0, n1, tid);
  if (!diag) lb.load(A, lda, r, tj * TILE, s, n0, n1, tid);
  la.store(As[0], tid);
  if (!diag) lb.store(Bs[0], tid);
  __syncthreads();
  int buf = 0;
  int run = 0;
  for (int64_t k0 = n0; k0 < n1; k0 += BK) {
    const bool more = k0 + BK < n1;
    if (more) {
      la.load(A, lda, r, ti * TILE, s, k0 + BK, n1, tid);
      if (!diag) lb.load(A, lda, r, tj * TILE, s, k0 + BK, n1, tid);
    }
    const T* Ac = As[buf];
    const T* Bc = diag ? As[buf] : Bs[buf];
    // Four MFMA k-steps per LDS read: in step t lane group g = lane / 16
    // takes k = kq + 4 g + t on both operands (only the pairing of A and B
    // k-slots matters), so each lane reads its four k values as one vector.
    typedef T v4t __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4 * MM::KS) {
      v4t fa[MI], fb[NI];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        fa[i] = *reinterpret_cast<const v4t*>(Ac + (wm * WTM + i * 16 + (lane & 15)) * LDK + kq +
                                               4 * (lane >> 4));
#pragma unroll
      for (int j = 0; j < NI; ++j)
        fb[j] = *reinterpret_cast<const v4t*>(Bc + (wn * WTN + j * 16 + (lane & 15)) * LDK + kq +
                                               4 * (lane >> 4));
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j) acc[i][j] = MM::mma(fa[i][t], fb[j][t], acc[i][j]);
    }
    if (more) {
      la.store(As[buf ^ 1], tid);
      if (!diag) lb.store(Bs[buf ^ 1], tid);
    }
    if constexpr (F32) {
      run += BK;
      if (run >= FLUSH_ROWS) {
        run = 0;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              acc64[i][j][e] += (double)acc[i][j][e];
              acc[i][j][e] = 0;
            }
      }
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double v;
        if constexpr (F32)
          v = acc64[i][j][e] + (double)acc[i][j][e];
        else
          v = acc[i][j][e];
        const int row = wm * WTM + i * 16 + MM::row(lane, e);
        const int col = wn * WTN + j * 16 + (lane & 15);
        out[row + col * TILE] = v;
      }
}

// ---------------------------------------------------------------------------
// float32 Grams on the fp16 MFMA pipe.  Each scaled operand x (float32) is
// split as hi = fp16(x), lo = fp16(x - hi), so x = hi + lo to 22 bits, and a
// product x y is taken as hi_x hi_y + hi_x lo_y + lo_x hi_y (the dropped
// lo_x lo_y is below 2^-22 |x y|); fp16 products are exact in the float32
// accumulator.  This is the three-product fp32 emulation of Ootomo and
// Yokota (2022), here on v_mfma_f32_16x16x32_f16, at three fp16 MFMAs per
// float32 product instead of one float32 MFMA of a fifth of the rate.
//
// fp16 has a narrow exponent range, so every row chunk is multiplied by a
// power of two 2^e (exact) chosen from the chunk's largest row scale so that
// the scaled operands stay below 2^14; the chunk partial is multiplied by
// 2^-2e on the way out.  This bounds the operands because the rows of the
// factor have norm at most 1 (unit kernel diagonal minus a non-negative
// residual); an operand beyond fp16 range turns into inf and surfaces as a
// non-finite Gram, never as a silently wrong one.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
constexpr int SPLIT_LDK = 64 + 8;  // halfs per staged column: 144 bytes puts the 16
                                   // rows of a fragment read on distinct 16-byte slots

// scl[z * nch + ch] = 2^e with max_{n in chunk} |s_z[n]| 2^e < 2^14 (1 when the
// chunk's scales are all zero or s_z is null).
__global__ __launch_bounds__(256) void k_split_scales(const float* __restrict__ s0,
                                                      const float* __restrict__ s1, int64_t N,
                                                      int64_t chunk, int nch,
                                                      float* __restrict__ scl) {
  const int z = blockIdx.x / nch, ch = blockIdx.x % nch;
  const float* s = z ? s1 : s0;
  const int64_t n0 = (int64_t)ch * chunk;
  const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;
  float m = 0.0f;
  if (s) {
    for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) m = fmaxf(m, fabsf(s[n]));
  } else {
    m = 1.0f;
  }
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float mx = red[0];
    float sc = 1.0f;
    if (mx > 0.0f && mx <= 3.0e38f) {
      int e;
      frexpf(mx, &e);  // mx < 2^e
      int p = 14 - e;
      p = p < -100 ? -100 : (p > 100 ? 100 : p);
      sc = ldexpf(1.0f, p);
    }
    scl[blockIdx.x] = sc;
  }
}

struct SplitLoader {
  SyrkLoader<float, float> ld;  // 128 columns x 64 rows of float32 per stage
  static constexpr int PER = SyrkLoader<float, float>::PER;
  static constexpr int VPC = SyrkLoader<float, float>::VPC;
  __device__ inline void load(const float* __restrict__ A, int64_t lda, int r, int c0,
                              const float* __restrict__ s, int64_t n0, int64_t n1, int tid) {
    ld.load(A, lda, r, c0, s, n0, n1, tid);
  }
  __device__ inline void store(_Float16* __restrict__ hi, _Float16* __restrict__ lo, float scale,
                               int tid) const {
    float ss[4];  // row scale times the chunk's power of two (the same rows for every p)
#pragma unroll
    for (int e = 0; e < 4; ++e) ss[e] = ld.sc[e] * scale;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * NTH;
      const int col = vid / VPC;
      const int kv = (vid % VPC) * 4;
      // v = x s rounded to float32, split into fp16 hi and lo
      uint32_t hw[2], lw[2];
#pragma unroll
      for (int e = 0; e < 4; e += 2)
        split_pair_f16(ld.buf[p][e] * ss[e], ld.buf[p][e + 1] * ss[e + 1], hw[e >> 1], lw[e >> 1]);
      *reinterpret_cast<uint2*>(hi + col * SPLIT_LDK + kv) = make_uint2(hw[0], hw[1]);
      *reinterpret_cast<uint2*>(lo + col * SPLIT_LDK + kv) = make_uint2(lw[0], lw[1]);
    }
  }
};

// Same grid, chunking and partial layout as k_syrk_partial<float, float>.
__global__ __launch_bounds__(NTH, 2) void k_syrk_split_partial(
    const float* __restrict__ A, int64_t lda, int64_t N, int r, const float* __restrict__ s0,
    const float* __restrict__ s1, const float* __restrict__ scl, int nz, int64_t chunk, int nch,
    double* __restrict__ part0, double* __restrict__ part1, const int32_t* kptr) {
  constexpr int BK = 64;
  constexpr int LDK = SPLIT_LDK;
  __shared__ __attribute__((aligned(16))) _Float16 Ah[2][TILE * LDK];
  __shared__ __attribute__((aligned(16))) _Float16 Al[2][TILE * LDK];
  __shared__ __attribute__((aligned(16))) _Float16 Bh[2][TILE * LDK];
  __shared__ __attribute__((aligned(16))) _Float16 Bl[2][TILE * LDK];
  const int nt = n_tiles(r);
  const int nu = n_upper(nt);
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int g = (slot / nu) * 8 + xcd;
  int z, ch;
  if (g >= group_slots(nz, nch) || !group_decode(g, nz, nch, z, ch)) return;
  const int tile = slot % nu;
  int ti, tj;
  upper_decode(tile, nt, ti, tj);
  const int kk = kptr ? *kptr : r;
  if (tj * TILE >= kk) return;
  const bool diag = ti == tj;
  const float* s = z ? s1 : s0;
  const float scale = scl[z * nch + ch];
  double* out = (z ? part1 : part0) + ((int64_t)ch * nu + tile) * TILE * TILE;
  const int64_t n0 = (int64_t)ch * chunk;
  const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  v4f acc[MI][NI];
  double acc64[MI][NI][4];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[i][j][e] = 0.0f;
        acc64[i][j][e] = 0.0;
      }
  // register ring of two stages: the reads of stage q + 2 are issued while
  // the MFMAs consume stage q; stage q sits in LDS buffer q & 1 and passes
  // through loader set q & 1
  SplitLoader la0, lb0, la1, lb1;
  const int nst = (int)((n1 - n0 + BK - 1) / BK);
  auto compute = [&](int buf) {
    const _Float16* ah_s = Ah[buf];
    const _Float16* al_s = Al[buf];
    const _Float16* bh_s = diag ? Ah[buf] : Bh[buf];
    const _Float16* bl_s = diag ? Al[buf] : Bl[buf];
    // lane group g = lane / 16 takes k = kq + 8 g .. kq + 8 g + 7 on both operands;
    // B fragments for the whole k-step, A fragments one row block at a time
#pragma unroll
    for (int kq = 0; kq < BK; kq += 32) {
      v8h bh[NI], bl[NI];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int o = (wn * WTN + j * 16 + (lane & 15)) * LDK + kq + 8 * (lane >> 4);
        bh[j] = *reinterpret_cast<const v8h*>(bh_s + o);
        bl[j] = *reinterpret_cast<const v8h*>(bl_s + o);
      }
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int o = (wm * WTM + i * 16 + (lane & 15)) * LDK + kq + 8 * (lane >> 4);
        const v8h ah = *reinterpret_cast<const v8h*>(ah_s + o);
        const v8h al = *reinterpret_cast<const v8h*>(al_s + o);
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc[i][j], 0, 0, 0);
        }
      }
    }
  };
  int run = 0;
  auto flush = [&]() {
    run += BK;
    if (run >= FLUSH_ROWS) {
      run = 0;
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc64[i][j][e] += (double)acc[i][j][e];
            acc[i][j][e] = 0.0f;
          }
    }
  };
  la0.load(A, lda, r, ti * TILE, s, n0, n1, tid);
  if (!diag) lb0.load(A, lda, r, tj * TILE, s, n0, n1, tid);
  if (nst > 1) {
    la1.load(A, lda, r, ti * TILE, s, n0 + BK, n1, tid);
    if (!diag) lb1.load(A, lda, r, tj * TILE, s, n0 + BK, n1, tid);
  }
  la0.store(Ah[0], Al[0], scale, tid);
  if (!diag) lb0.store(Bh[0], Bl[0], scale, tid);
  __syncthreads();
  for (int q = 0; q < nst; q += 2) {
    if (q + 2 < nst) {
      la0.load(A, lda, r, ti * TILE, s, n0 + (int64_t)(q + 2) * BK, n1, tid);
      if (!diag) lb0.load(A, lda, r, tj * TILE, s, n0 + (int64_t)(q + 2) * BK, n1, tid);
    }
    compute(0);
    if (q + 1 < nst) {
      la1.store(Ah[1], Al[1], scale, tid);
      if (!diag) lb1.store(Bh[1], Bl[1], scale, tid);
    }
    flush();
    __syncthreads();
    if (q + 1 >= nst) break;
    if (q + 3 < nst) {
      la1.load(A, lda, r, ti * TILE, s, n0 + (int64_t)(q + 3) * BK, n1, tid);
      if (!diag) lb1.load(A, lda, r, tj * TILE, s, n0 + (int64_t)(q + 3) * BK, n1, tid);
    }
    compute(1);
    if (q + 2 < nst) {
      la0.store(Ah[0], Al[0], scale, tid);
      if (!diag) lb0.store(Bh[0], Bl[0], scale, tid);
    }
    flush();
    __syncthreads();
  }
  const double unscale = 1.0 / ((double)scale * (double)scale);
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double v = (acc64[i][j][e] + (double)acc[i][j][e]) * unscale;
        const int row = wm * WTM + i * 16 + 4 * (lane >> 4) + e;
        const int col = wn * WTN + j * 16 + (lane & 15);
        out[row + col * TILE] = v;
      }
}

// Both Grams of one row chunk (nz = 2) in one launch, each (chunk, tile) as
// two adjacent four-wave workgroups on the same XCD, one per Gram, so the
// second finds the panels the first fetched in L2.  The two accumulator sets
// of a wave fit its register budget because the runs are joined in float32
// rather than float64: a float32 run covers 256 rows (as above) and a float32
// second-level sum joins the runs of the chunk, at most PAIR_RUNS of them
// (the launcher takes this kernel only for such chunks), before the float64
// partial tile is written.  Stages are 32 rows deep: two stage buffers of the
// four hi/lo operand tiles take 64 KB of LDS, so two workgroups share a CU.
// Each wave computes a 64 x 64 quarter of its Gram's tile, which reads a third
// fewer fragment bytes per MFMA than a 64 x 32 one.  One workgroup per Gram (rather than
// eight waves taking both Grams from one staging) lets the two workgroups on a
// CU drift out of phase, so one's split conversion and LDS writes overlap the
// other's MFMAs; a workgroup's stage barrier holds only its own four waves.
constexpr int PAIR_BK = 32;
constexpr int PAIR_LDK = PAIR_BK;  // 64-byte columns, 16-byte k-slots permuted per column
constexpr int PAIR_RUNS = 64;          // most 256-row runs in one chunk
constexpr int PAIR_NTH = 256;          // four waves, 2 x 2 quarters of the tile

// Half offset of k-slot q (8 rows, 16 bytes) of staged column c.  A 16-byte
// LDS read serves a wave in four passes of 16 lanes; the lanes of one pass are
// the four-lane groups g = lane / 4 of one half-wave whose three low bits have
// the same parity (counted on this chip: lanes 0-3, 12-15, 20-23 and 24-27
// share a pass).  A fragment read (lane: column lane % 16, slot lane / 16)
// then puts columns c and c + 4 of adjacent slots in one pass, and with 64-byte
// columns those meet on the same banks; XORing the slot with 2 on every other
// group of four columns moves them apart, so each pass covers all 64 banks.
// The stage writes stay conflict-free: two adjacent columns are one 128-byte
// row of the 32 banks an 8-byte write pass covers.
__device__ inline int pair_at(int c, int q) { return c * PAIR_LDK + 8 * (q ^ (c & 4) >> 1); }

struct PairLoader {  // 128 columns x 32 rows of float32, four 4-row vectors per thread
  static constexpr int VPC = PAIR_BK / 4;
  static constexpr int PER = TILE * VPC / PAIR_NTH;
  static_assert(PAIR_NTH % VPC == 0, "every vector of a thread covers the same rows");
  v4f buf[PER];
  __device__ inline void load(const float* __restrict__ A, int64_t lda, int r, int c0,
                              int64_t n0, int64_t n1, int tid) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * PAIR_NTH;
      const int col = vid / VPC;
      const int64_t n = n0 + (vid % VPC) * 4;
      const int gc = c0 + col;
      if (gc < r && n + 4 <= n1) {
        buf[p] = *reinterpret_cast<const v4f*>(A + (int64_t)gc * lda + n);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          buf[p][e] = (gc < r && n + e < n1) ? A[(int64_t)gc * lda + n + e] : 0.0f;
      }
    }
  }
  // v = x s rounded to float32 (s the row scale times the chunk's 2^e), hi = fp16(v), lo = fp16(v - hi)
  __device__ inline void store(_Float16* __restrict__ hi, _Float16* __restrict__ lo,
                               const float (&ss)[4], int tid) const {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * PAIR_NTH;
      const int col = vid / VPC;
      const int kv = vid % VPC;  // rows 4 kv .. 4 kv + 3: half kv & 1 of slot kv / 2
      uint32_t hw[2], lw[2];
#pragma unroll
      for (int e = 0; e < 4; e += 2)
        split_pair_f16(buf[p][e] * ss[e], buf[p][e + 1] * ss[e + 1], hw[e >> 1], lw[e >> 1]);
      const int o = pair_at(col, kv >> 1) + 4 * (kv & 1);
      *reinterpret_cast<uint2*>(hi + o) = make_uint2(hw[0], hw[1]);
      *reinterpret_cast<uint2*>(lo + o) = make_uint2(lw[0], lw[1]);
    }
  }
};

// Row scales of the 4 rows n .. n + 3 a thread stages (zero past n1).
__device__ inline void pair_row_scales(const float* __restrict__ s, int64_t n, int64_t n1,
                                       float (&out)[4]) {
  if (n + 4 <= n1) {
    const v4f v = *reinterpret_cast<const v4f*>(s + n);
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = v[e];
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = n + e < n1 ? s[n + e] : 0.0f;
  }
}

// grid.x = 2 * 8 * ceil(nch / 8) * n_upper: slot pairs (2 t, 2 t + 1) on XCD
// blockIdx % 8 are Grams 0 and 1 of chunk (t / n_upper) * 8 + XCD, tile
// t % n_upper.  s0 and s1 are both required; scl as for k_syrk_split_partial
// with nz = 2.
__global__ __launch_bounds__(PAIR_NTH, 2) void k_syrk_split_pair_partial(
    const float* __restrict__ A, int64_t lda, int64_t N, int r, const float* __restrict__ s0,
    const float* __restrict__ s1, const float* __restrict__ scl, int64_t chunk, int nch,
    double* __restrict__ part0, double* __restrict__ part1, const int32_t* kptr) {
  constexpr int BK = PAIR_BK;
  constexpr int LDK = PAIR_LDK;
  constexpr int TS = TILE * LDK;
  // [stage buffer][A hi, A lo, B hi, B lo]
  __shared__ __attribute__((aligned(16))) _Float16 lds[2][4][TS];
  const int nt = n_tiles(r);
  const int nu = n_upper(nt);
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int z = slot & 1, pslot = slot >> 1;
  const int ch = (pslot / nu) * 8 + xcd;
  if (ch >= nch) return;
  const int tile = pslot % nu;
  int ti, tj;
  upper_decode(tile, nt, ti, tj);
  const int kk = kptr ? *kptr : r;
  if (tj * TILE >= kk) return;
  const bool diag = ti == tj;
  const float scale = scl[z * nch + ch];
  const float* sz = z ? s1 : s0;
  double* o = (z ? part1 : part0) + ((int64_t)ch * nu + tile) * TILE * TILE;
  const int64_t n0 = (int64_t)ch * chunk;
  const int64_t n1 = n0 + chunk < N ? n0 + chunk : N;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t nrow = (tid % PairLoader::VPC) * 4;  // this thread's rows within a stage
  constexpr int PM = 4, PN = 4;                     // 16 x 16 blocks per wave
  v4f acc[PM][PN], acc2[PM][PN];
#pragma unroll
  for (int i = 0; i < PM; ++i)
#pragma unroll
    for (int j = 0; j < PN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[i][j][e] = 0.0f;
        acc2[i][j][e] = 0.0f;
      }
  PairLoader la, lb;
  float w[4];  // s_z at the staged rows
  auto stage = [&](int b) __attribute__((always_inline)) {
    float ss[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) ss[e] = w[e] * scale;
    la.store(lds[b][0], lds[b][1], ss, tid);
    if (!diag) lb.store(lds[b][2], lds[b][3], ss, tid);
  };
  auto compute = [&](int b) __attribute__((always_inline)) {
    const _Float16* ah_s = lds[b][0];
    const _Float16* al_s = lds[b][1];
    const _Float16* bh_s = diag ? lds[b][0] : lds[b][2];
    const _Float16* bl_s = diag ? lds[b][1] : lds[b][3];
    // lane group lane / 16 takes k = 8 (lane / 16) .. + 7 of the 32-row stage
    v8h bh[PN], bl[PN];
#pragma unroll
    for (int j = 0; j < PN; ++j) {
      const int o2 = pair_at(wn * 64 + j * 16 + (lane & 15), lane >> 4);
      bh[j] = *reinterpret_cast<const v8h*>(bh_s + o2);
      bl[j] = *reinterpret_cast<const v8h*>(bl_s + o2);
    }
#pragma unroll
    for (int i = 0; i < PM; ++i) {
      const int o2 = pair_at(wm * 64 + i * 16 + (lane & 15), lane >> 4);
      const v8h ah = *reinterpret_cast<const v8h*>(ah_s + o2);
      const v8h al = *reinterpret_cast<const v8h*>(al_s + o2);
#pragma unroll
      for (int j = 0; j < PN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  int rows = 0;
  auto flush = [&]() __attribute__((always_inline)) {
    rows += BK;
    if (rows < FLUSH_ROWS) return;
    rows = 0;
#pragma unroll
    for (int i = 0; i < PM; ++i)
#pragma unroll
      for (int j = 0; j < PN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc2[i][j][e] += acc[i][j][e];
          acc[i][j][e] = 0.0f;
        }
  };
  const int nst = (int)((n1 - n0 + BK - 1) / BK);
  auto fetch = [&](int q) __attribute__((always_inline)) {
    const int64_t p0 = n0 + (int64_t)q * BK;
    la.load(A, lda, r, ti * TILE, p0, n1, tid);
    if (!diag) lb.load(A, lda, r, tj * TILE, p0, n1, tid);
    pair_row_scales(sz, p0 + nrow, n1, w);
  };
  // one stage in registers: stage q + 1's panels are read during stage q's
  // MFMAs and split into the other buffer after them
  fetch(0);
  stage(0);
  if (nst > 1) fetch(1);
  __syncthreads();
  for (int q = 0; q < nst; ++q) {
    const int b = q & 1;
    compute(b);
    if (q + 1 < nst) {
      stage(b ^ 1);
      if (q + 2 < nst) fetch(q + 2);
    }
    flush();
    __syncthreads();
  }
  const double unscale = 1.0 / ((double)scale * (double)scale);
#pragma unroll
  for (int i = 0; i < PM; ++i)
#pragma unroll
    for (int j = 0; j < PN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double v = ((double)acc2[i][j][e] + (double)acc[i][j][e]) * unscale;
        const int row = wm * 64 + i * 16 + 4 * (lane >> 4) + e;
        const int col = wn * 64 + j * 16 + (lane & 15);
        o[row + col * TILE] = v;
      }
}

// G[i + j r] = sum over chunks of the partial tile entry (min(i,j), max(i,j)):
// workgroups run over the upper tiles (blockIdx.y) and each thread sums two
// adjacent entries of its tile over the chunks (16-byte loads, chunks in
// order, eight in flight), then writes them and their mirror images.  Inside a
// diagonal tile only the upper entry is used for both, so G is exactly
// symmetric; entries with an index >= k are zero.
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ part, int nch, int r,
                                                     double* __restrict__ G, const int32_t* kptr) {
  const int nt = n_tiles(r), nu = n_upper(nt);
  const int u = blockIdx.y;
  int ti, tj;
  upper_decode(u, nt, ti, tj);
  const int e = (blockIdx.x * 256 + threadIdx.x) * 2;  // entries e, e + 1: rows a, a + 1 of column b
  if (e >= TILE * TILE) return;
  const int a = e % TILE, b = e / TILE;
  const int kk = kptr ? *kptr : r;
  double s0 = 0.0, s1 = 0.0;
  if (tj * TILE < kk) {  // tiles wholly past k were not computed
    const double* p = part + (int64_t)u * TILE * TILE + e;
    const int64_t step = (int64_t)nu * TILE * TILE;
#pragma unroll 8
    for (int c = 0; c < nch; ++c) {
      const v2d v = *reinterpret_cast<const v2d*>(p + c * step);
      s0 += v[0];
      s1 += v[1];
    }
  }
  const int j = tj * TILE + b;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = ti * TILE + a + h;
    if (i >= r || j >= r) continue;
    if (ti == tj && a + h > b) continue;  // the mirror of an upper entry of this tile
    const double v = (i < kk && j < kk) ? (h ? s1 : s0) : 0.0;
    G[i + (int64_t)j * r] = v;
    G[j + (int64_t)i * r] = v;
  }
}

// Row chunks of the Gram partial products: about 4096 workgroups per Gram
// (chunks x upper tiles), at least 256 rows per chunk, at most MAX_CHUNKS
// chunks; the partial buffers then hold about 4096 tiles of 128 x 128 doubles
// per Gram.  Many short workgroups keep the ones that share a chunk's panels
// close together in time, so more of the panel re-reads hit L2.
constexpr int MAX_CHUNKS = 128;
inline void plan(int64_t N, int r, int& nch, int64_t& chunk) {
  const int nu = n_upper(n_tiles(r));
  int64_t want = (4096 + nu - 1) / nu;
  const int64_t rows_cap = (N + 255) / 256;
  if (want > rows_cap) want = rows_cap;
  int c = (int)(want < MAX_CHUNKS ? want : MAX_CHUNKS);
  if (c < 1) c = 1;
  chunk = (int64_t)align_up((size_t)((N + c - 1) / c), 256);
  nch = (int)((N + chunk - 1) / chunk);
}

inline size_t part_elems(int64_t N, int r, bool f32) {
  int nch;
  int64_t chunk;
  plan(N, r, nch, chunk);
  const int nu = n_upper(n_tiles(r));
  return (size_t)nch * nu * TILE * TILE;
}

// Partial-buffer size that serves any rank <= r (the chunk count depends on
// the tile count, so the largest product of the two is taken).
inline size_t part_elems_any(int64_t N, int r) {
  size_t m = 0;
  for (int t = 1; t <= n_tiles(r); ++t) {
    const size_t e = part_elems(N, t * TILE < r ? t * TILE : r, true);
    m = e > m ? e : m;
  }
  return m;
}

// part0/part1 each hold part_cap doubles, enough when gram2_fits holds
// (part_elems(N, r, sizeof(T) == 4)); G0/G1 are r x r.
// nz = 1: only G0 (s0 may be null = no scaling); nz = 2: G0 and G1.
template <typename T>
inline bool gram2_fits(int64_t N, int r, size_t part_cap) {
  int nch;
  int64_t chunk;
  plan(N, r, nch, chunk);
  return (size_t)nch * n_upper(n_tiles(r)) * TILE * TILE <= part_cap;
}

// Chunked partial products of nz (1 or 2) Grams; the caller checked
// gram2_fits.  gram2_reduce then sums the chunks into the r x r results.
template <typename T, typename TF>
inline void gram2_partial(hipStream_t st, const TF* A, int64_t lda, int64_t N, int r, int nz,
                          const T* s0, const T* s1, double* part0, double* part1,
                          const int32_t* kptr = nullptr) {
  int nch;
  int64_t chunk;
  plan(N, r, nch, chunk);
  const int nu = n_upper(n_tiles(r));
  const unsigned blocks = (unsigned)(group_slots(nz, nch) * nu);
  hipLaunchKernelGGL((k_syrk_partial<T, TF>), dim3(blocks), dim3(NTH), 0, st, A, lda, N, r, s0, s1, nz,
                     chunk, nch, part0, part1, kptr);
}

// Split-fp16 form of gram2_partial for float32 operands and scales; scl
// holds at least nz * nch floats (nch <= MAX_CHUNKS).
inline void gram2_partial_split(hipStream_t st, const float* A, int64_t lda, int64_t N, int r,
                                int nz, const float* s0, const float* s1, float* scl,
                                double* part0, double* part1, const int32_t* kptr = nullptr) {
  int nch;
  int64_t chunk;
  plan(N, r, nch, chunk);
  const int nu = n_upper(n_tiles(r));
  const int groups = nz * nch;
  hipLaunchKernelGGL(k_split_scales, dim3(groups), dim3(256), 0, st, s0, s1, N, chunk, nch, scl);
  if (nz == 2 && s0 && s1 && chunk <= (int64_t)PAIR_RUNS * FLUSH_ROWS) {
    const unsigned blocks = (unsigned)(2 * 8 * ((nch + 7) / 8) * nu);
    hipLaunchKernelGGL(k_syrk_split_pair_partial, dim3(blocks), dim3(PAIR_NTH), 0, st, A, lda, N, r,
                       s0, s1, (const float*)scl, chunk, nch, part0, part1, kptr);
    return;
  }
  const unsigned blocks = (unsigned)(group_slots(nz, nch) * nu);
  hipLaunchKernelGGL(k_syrk_split_partial, dim3(blocks), dim3(NTH), 0, st, A, lda, N, r, s0, s1,
                     (const float*)scl, nz, chunk, nch, part0, part1, kptr);
}

template <typename T>
inline void gram2_reduce(hipStream_t st, int64_t N, int r, int nz, const double* part0,
                         const double* part1, double* G0, double* G1,
                         const int32_t* kptr = nullptr) {
  int nch;
  int64_t chunk;
  plan(N, r, nch, chunk);
  const dim3 gr(TILE * TILE / 512, (unsigned)n_upper(n_tiles(r)));
  hipLaunchKernelGGL(k_syrk_reduce, gr, dim3(256), 0, st, part0, nch, r, G0, kptr);
  if (nz == 2) hipLaunchKernelGGL(k_syrk_reduce, gr, dim3(256), 0, st, part1, nch, r, G1, kptr);
}

}  // namespace
}  // namespace syrk
