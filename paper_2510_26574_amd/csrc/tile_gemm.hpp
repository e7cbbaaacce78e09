// Block-tiled MFMA product engine for gfx950.
//
// Computes, for one workgroup, the BM x BN tile  acc = A(m0:, kb:ke) * B(n0:, kb:ke)^T
// where A is (rows x K) and B is (cols x K).  Each operand is read from global
// memory in whichever orientation it is stored (k-contiguous: element (i, k)
// at p[i * ld + k]; or row-contiguous: element (i, k) at p[i + k * ld]),
// converted to the MFMA input type T, optionally scaled by a per-k weight,
// and staged in LDS as [row][k].  Four waves split the tile; each wave holds
// (BM / WAVES_M) x (BN / WAVES_N) of 16 x 16 MFMA accumulators.
//
// Callers own the epilogue: `for_each_acc` walks the accumulators with their
// global (row, col) coordinates.
#pragma once
#include "common.hpp"

template <typename TG, bool KCONTIG>
struct GOperand {
  const TG* p;
  int64_t ld;     // stride of the non-contiguous index
  int64_t rows;   // valid rows
  int64_t K;      // valid k
  const double* kscale;  // optional per-k weight (nullptr = none)
  bool vec;       // 16-byte loads allowed (aligned base and ld)
};

template <typename T_, int BM_, int BN_, int BK_, int WAVES_M_, int WAVES_N_>
struct TileCfg {
  typedef T_ T;
  typedef Mma<T_> MM;
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int NT = 64 * WAVES_M * WAVES_N;
  static constexpr int WTM = BM / WAVES_M, WTN = BN / WAVES_N;
  static constexpr int MI = WTM / 16, NI = WTN / 16;
  // LDS row padding: keeps 16-byte alignment for bf16 fragments and spreads
  // the 16 rows of a fragment over distinct banks.
  static constexpr int PAD = (sizeof(T_) == 2) ? 8 : 1;
  static constexpr int LDK = BK + PAD;
  static constexpr size_t smem_bytes = (size_t)(BM + BN) * LDK * sizeof(T_);
  static_assert(BM % (16 * WAVES_M) == 0 && BN % (16 * WAVES_N) == 0, "tile");
  static_assert(BK % MM::KS == 0, "BK must be a multiple of the MFMA k");
};

template <typename T, typename TG>
__device__ inline T scale_cvt(TG v, const double* ks, int64_t k) {
  if (ks) return cvtd<T>(to_d(v) * ks[k]);
  if constexpr (sizeof(TG) == sizeof(T)) {
    return (T)v;
  } else {
    return cvtd<T>(to_d(v));
  }
}

// Stage a ROWS x BK slice (rows r0.., k k0..) of operand `op` into s[row][k].
template <typename T, int ROWS, int BK, int LDK, int NT, typename TG, bool KC>
__device__ inline void stage_tile(T* __restrict__ s, const GOperand<TG, KC>& op, int64_t r0,
                                  int64_t k0, int tid) {
  constexpr int V = 16 / sizeof(TG);
  if constexpr (KC) {
    constexpr int VPR = BK / V;  // vectors per row
    static_assert(BK % V == 0, "BK");
    constexpr int NV = ROWS * VPR;
    for (int vid = tid; vid < NV; vid += NT) {
      const int row = vid / VPR;
      const int kv = (vid % VPR) * V;
      const int64_t gr = r0 + row, gk = k0 + kv;
      T* dst = s + row * LDK + kv;
      if (gr < op.rows && gk + V <= op.K && op.vec) {
        typedef TG vt __attribute__((ext_vector_type(V)));
        vt v = *reinterpret_cast<const vt*>(op.p + gr * op.ld + gk);
#pragma unroll
        for (int j = 0; j < V; ++j) dst[j] = scale_cvt<T>(v[j], op.kscale, gk + j);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const int64_t kk = gk + j;
          dst[j] = (gr < op.rows && kk < op.K) ? scale_cvt<T>(op.p[gr * op.ld + kk], op.kscale, kk)
                                               : cvtd<T>(0.0);
        }
      }
    }
  } else {
    constexpr int VPC = ROWS / V;  // vectors per k-column
    static_assert(ROWS % V == 0, "ROWS");
    constexpr int NV = BK * VPC;
    for (int vid = tid; vid < NV; vid += NT) {
      const int kc = vid / VPC;
      const int rv = (vid % VPC) * V;
      const int64_t gr = r0 + rv, gk = k0 + kc;
      if (gk < op.K && gr + V <= op.rows && op.vec) {
        typedef TG vt __attribute__((ext_vector_type(V)));
        vt v = *reinterpret_cast<const vt*>(op.p + gr + gk * op.ld);
#pragma unroll
        for (int j = 0; j < V; ++j) s[(rv + j) * LDK + kc] = scale_cvt<T>(v[j], op.kscale, gk);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const int64_t rr = gr + j;
          s[(rv + j) * LDK + kc] = (rr < op.rows && gk < op.K)
                                       ? scale_cvt<T>(op.p[rr + gk * op.ld], op.kscale, gk)
                                       : cvtd<T>(0.0);
        }
      }
    }
  }
}

template <class Cfg>
struct TileAcc {
  typename Cfg::MM::acc a[Cfg::MI][Cfg::NI];
  __device__ inline void zero() {
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) a[i][j][e] = 0;
  }
};

template <class Cfg>
__device__ inline typename Cfg::MM::frag load_frag(const typename Cfg::T* s, int row, int kk,
                                                   int lane) {
  typedef typename Cfg::MM MM;
  const typename Cfg::T* p = s + row * Cfg::LDK + kk + (lane >> 4) * MM::EPL;
  if constexpr (MM::EPL == 1) {
    return *p;
  } else {
    return *reinterpret_cast<const typename MM::frag*>(p);
  }
}

// acc += A(m0.., kb..ke) * B(n0.., kb..ke)^T over the k range [kb, ke).
template <class Cfg, typename TGA, bool KCA, typename TGB, bool KCB>
__device__ inline void tile_mainloop(TileAcc<Cfg>& acc, const GOperand<TGA, KCA>& A,
                                     const GOperand<TGB, KCB>& B, int64_t m0, int64_t n0,
                                     int64_t kb, int64_t ke, typename Cfg::T* smem) {
  typedef typename Cfg::T T;
  typedef typename Cfg::MM MM;
  T* As = smem;
  T* Bs = smem + Cfg::BM * Cfg::LDK;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  for (int64_t k0 = kb; k0 < ke; k0 += Cfg::BK) {
    GOperand<TGA, KCA> a = A;
    GOperand<TGB, KCB> b = B;
    a.K = ke < A.K ? ke : A.K;
    b.K = ke < B.K ? ke : B.K;
    stage_tile<T, Cfg::BM, Cfg::BK, Cfg::LDK, Cfg::NT>(As, a, m0, k0, tid);
    stage_tile<T, Cfg::BN, Cfg::BK, Cfg::LDK, Cfg::NT>(Bs, b, n0, k0, tid);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < Cfg::BK; kk += MM::KS) {
      typename MM::frag fa[Cfg::MI], fb[Cfg::NI];
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
        fa[i] = load_frag<Cfg>(As, wm * Cfg::WTM + i * 16 + (lane & 15), kk, lane);
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
        fb[j] = load_frag<Cfg>(Bs, wn * Cfg::WTN + j * 16 + (lane & 15), kk, lane);
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) acc.a[i][j] = MM::mma(fa[i], fb[j], acc.a[i][j]);
    }
    __syncthreads();
  }
}

// Visit every accumulator element with its tile-local (row, col).
template <class Cfg, typename Fn>
__device__ inline void for_each_acc(TileAcc<Cfg>& acc, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * Cfg::WTM + i * 16 + Cfg::MM::row(lane, e);
        const int col = wn * Cfg::WTN + j * 16 + (lane & 15);
        fn(row, col, acc.a[i][j][e]);
      }
}
