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
  const int groups = nz * nch;
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int g = (slot / nu) * 8 + xcd;
  if (g >= groups) return;
  const int tile = slot % nu;
  const int z = g / nch, ch = g % nch;
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

// G[i + j r] = sum over chunks of the partial tile holding (i, j) (or (j, i)).
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ part, int nch, int r,
                                                     double* __restrict__ G, const int32_t* kptr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int i = (int)(e % r), j = (int)(e / r);
  const int kk = kptr ? *kptr : r;
  if (i >= kk || j >= kk) {
    G[e] = 0.0;
    return;
  }
  const int nt = n_tiles(r), nu = n_upper(nt);
  int a = i, b = j;
  if (i / TILE > j / TILE) {
    a = j;
    b = i;
  }
  const int t = upper_index(a / TILE, b / TILE, nt);
  const int64_t off = (int64_t)t * TILE * TILE + (a % TILE) + (int64_t)(b % TILE) * TILE;
  double acc = 0.0;
  for (int c = 0; c < nch; ++c) acc += part[(int64_t)c * nu * TILE * TILE + off];
  G[e] = acc;
}

// Row chunking: about 32 chunks of whole 256-row flush runs (both types).
inline void plan(int64_t N, int& nch, int64_t& chunk, bool f32) {
  (void)f32;
  int64_t want = (N + 255) / 256;
  int c = (int)(want < 32 ? want : 32);
  if (c < 1) c = 1;
  chunk = (int64_t)align_up((size_t)((N + c - 1) / c), 256);
  nch = (int)((N + chunk - 1) / chunk);
}

inline size_t part_elems(int64_t N, int r, bool f32) {
  int nch;
  int64_t chunk;
  plan(N, nch, chunk, f32);
  const int nu = n_upper(n_tiles(r));
  return (size_t)nch * nu * TILE * TILE;
}

// Partial-buffer size that serves both product types (and any rank <= r).
inline size_t part_elems_any(int64_t N, int r) {
  const size_t a = part_elems(N, r, true), b = part_elems(N, r, false);
  return a > b ? a : b;
}

// part0/part1 each hold part_cap doubles, enough when gram2_fits holds
// (part_elems(N, r, sizeof(T) == 4)); G0/G1 are r x r.
// nz = 1: only G0 (s0 may be null = no scaling); nz = 2: G0 and G1.
template <typename T>
inline bool gram2_fits(int64_t N, int r, size_t part_cap) {
  int nch;
  int64_t chunk;
  plan(N, nch, chunk, sizeof(T) == 4);
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
  plan(N, nch, chunk, sizeof(T) == 4);
  const int nu = n_upper(n_tiles(r));
  const int groups = nz * nch;
  const unsigned blocks = (unsigned)(8 * ((groups + 7) / 8) * nu);
  hipLaunchKernelGGL((k_syrk_partial<T, TF>), dim3(blocks), dim3(NTH), 0, st, A, lda, N, r, s0, s1, nz,
                     chunk, nch, part0, part1, kptr);
}

template <typename T>
inline void gram2_reduce(hipStream_t st, int64_t N, int r, int nz, const double* part0,
                         const double* part1, double* G0, double* G1,
                         const int32_t* kptr = nullptr) {
  int nch;
  int64_t chunk;
  plan(N, nch, chunk, sizeof(T) == 4);
  const unsigned gr = (unsigned)(((int64_t)r * r + 255) / 256);
  hipLaunchKernelGGL(k_syrk_reduce, dim3(gr), dim3(256), 0, st, part0, nch, r, G0, kptr);
  if (nz == 2) hipLaunchKernelGGL(k_syrk_reduce, dim3(gr), dim3(256), 0, st, part1, nch, r, G1, kptr);
}

}  // namespace
}  // namespace syrk
