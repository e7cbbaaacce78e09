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
  static_assert(BM % (16 * WAVES_M) == 0 && BN % (16 * WAVES_N) == 0, "tile");
  static_assert(BK % MM::KS == 0, "BK must be a multiple of the MFMA k");
};

// Whether a staged slice is k-contiguous in LDS: always for k-contiguous
// global operands, and also for row-contiguous ones when the MFMA fragment
// holds several consecutive k (bf16), in which case staging transposes.
template <typename T, bool KC>
struct LdsKC {
  static constexpr bool value = KC || Mma<T>::EPL > 1;
};

// LDS layout of one staged operand slice (ROWS x BK):
//   k-contiguous operand   -> s[row * LDK + k],  LDK = BK + 16 bytes of pad
//   row-contiguous operand -> s[k * LDR + row],  LDR = ROWS + 16 elements of pad
// Both keep 16-byte aligned vector stores (the staged vectors run along the
// contiguous index) and spread a fragment's 16 rows over distinct banks.
template <typename T, int ROWS, int BK, bool KC>
struct SliceLayout {
  static constexpr int LDK = BK + 16 / (int)sizeof(T);
  static constexpr int LDR = ROWS + 16;
  static constexpr int ELEMS = KC ? ROWS * LDK : BK * LDR;
  __device__ static inline int at(int row, int k) { return KC ? row * LDK + k : k * LDR + row; }
};

template <class Cfg, bool KCA, bool KCB>
struct TileSmem {
  typedef SliceLayout<typename Cfg::T, Cfg::BM, Cfg::BK, LdsKC<typename Cfg::T, KCA>::value> LA;
  typedef SliceLayout<typename Cfg::T, Cfg::BN, Cfg::BK, LdsKC<typename Cfg::T, KCB>::value> LB;
  static constexpr int STAGE = LA::ELEMS + LB::ELEMS;  // one buffer (A then B)
  static constexpr size_t bytes = 2 * (size_t)STAGE * sizeof(typename Cfg::T);  // double buffered
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

// Register-staged copy of a ROWS x BK slice (rows r0.., k k0..) of operand
// `op`: load() issues the global reads (zero-filled out of range), store()
// converts and writes them to LDS in the operand's SliceLayout.  Splitting
// the two lets the main loop fetch the next slice while the MFMAs consume
// the current one.
template <typename T, int ROWS, int BK, int NT, typename TG, bool KC>
struct TileStage {
  static constexpr bool LKC = LdsKC<T, KC>::value;
  typedef SliceLayout<T, ROWS, BK, LKC> L;
  // elements per vector: 16 bytes of the wider of the global and LDS types,
  // so each lane's LDS store is one contiguous 16-byte (or narrower) write
  static constexpr int V = 16 / (sizeof(TG) > sizeof(T) ? sizeof(TG) : sizeof(T));
  static constexpr int NV = KC ? ROWS * (BK / V) : BK * (ROWS / V);
  static constexpr int PER = (NV + NT - 1) / NT;
  static_assert(KC ? (BK % V == 0) : (ROWS % V == 0), "tile shape vs vector width");
  typedef TG vt __attribute__((ext_vector_type(V)));
  typedef T st __attribute__((ext_vector_type(V)));
  vt buf[PER];

  __device__ inline void coords(int vid, int& row, int& kk) const {
    if constexpr (KC) {
      row = vid / (BK / V);
      kk = (vid % (BK / V)) * V;
    } else {
      kk = vid / (ROWS / V);
      row = (vid % (ROWS / V)) * V;
    }
  }

  __device__ inline void load(const GOperand<TG, KC>& op, int64_t r0, int64_t k0, int tid) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * NT;
      if (NV % NT != 0 && vid >= NV) break;
      int row, kk;
      coords(vid, row, kk);
      const int64_t gr = r0 + row, gk = k0 + kk;
      if constexpr (KC) {
        if (gr < op.rows && gk + V <= op.K && op.vec) {
          buf[p] = *reinterpret_cast<const vt*>(op.p + gr * op.ld + gk);
        } else {
#pragma unroll
          for (int j = 0; j < V; ++j)
            buf[p][j] = (gr < op.rows && gk + j < op.K) ? op.p[gr * op.ld + gk + j] : (TG)0;
        }
      } else {
        if (gk < op.K && gr + V <= op.rows && op.vec) {
          buf[p] = *reinterpret_cast<const vt*>(op.p + gr + gk * op.ld);
        } else {
#pragma unroll
          for (int j = 0; j < V; ++j)
            buf[p][j] = (gr + j < op.rows && gk < op.K) ? op.p[gr + j + gk * op.ld] : (TG)0;
        }
      }
    }
  }

  __device__ inline void store(T* __restrict__ s, const GOperand<TG, KC>& op, int64_t k0,
                               int tid) const {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int vid = tid + p * NT;
      if (NV % NT != 0 && vid >= NV) break;
      int row, kk;
      coords(vid, row, kk);
      if constexpr (LKC != KC) {
        // row-contiguous vector (rows row..row+V-1 at k = kk) into a
        // k-contiguous slice: one element per row
#pragma unroll
        for (int j = 0; j < V; ++j) s[L::at(row + j, kk)] = scale_cvt<T>(buf[p][j], op.kscale, k0 + kk);
        continue;
      }
      T* dst = s + L::at(row, kk);  // the V elements run along the contiguous index
      st v;
      if (op.kscale == nullptr && sizeof(T) == sizeof(TG)) {
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = (T)buf[p][j];
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = scale_cvt<T>(buf[p][j], op.kscale, k0 + (KC ? kk + j : kk));
      }
      *reinterpret_cast<st*>(dst) = v;
    }
  }
};

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

template <class Cfg, int ROWS, bool KC>
__device__ inline typename Cfg::MM::frag load_frag(const typename Cfg::T* s, int row, int kk,
                                                   int lane) {
  typedef typename Cfg::MM MM;
  typedef SliceLayout<typename Cfg::T, ROWS, Cfg::BK, LdsKC<typename Cfg::T, KC>::value> L;
  if constexpr (MM::EPL == 1) {
    return s[L::at(row, kk + (lane >> 4))];
  } else {
    return *reinterpret_cast<const typename MM::frag*>(s + L::at(row, kk + (lane >> 4) * MM::EPL));
  }
}

// acc += A(m0.., kb..ke) * B(n0.., kb..ke)^T over the k range [kb, ke).
// smem must hold TileSmem<Cfg, KCA, KCB>::bytes.
template <class Cfg, typename TGA, bool KCA, typename TGB, bool KCB>
__device__ inline void tile_mainloop(TileAcc<Cfg>& acc, const GOperand<TGA, KCA>& A,
                                     const GOperand<TGB, KCB>& B, int64_t m0, int64_t n0,
                                     int64_t kb, int64_t ke, typename Cfg::T* smem) {
  typedef typename Cfg::T T;
  typedef typename Cfg::MM MM;
  typedef TileSmem<Cfg, KCA, KCB> SM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  GOperand<TGA, KCA> a = A;
  GOperand<TGB, KCB> b = B;
  a.K = ke < A.K ? ke : A.K;
  b.K = ke < B.K ? ke : B.K;
  TileStage<T, Cfg::BM, Cfg::BK, Cfg::NT, TGA, KCA> sa;
  TileStage<T, Cfg::BN, Cfg::BK, Cfg::NT, TGB, KCB> sb;
  if (kb >= ke) return;
  sa.load(a, m0, kb, tid);
  sb.load(b, n0, kb, tid);
  sa.store(smem, a, kb, tid);
  sb.store(smem + SM::LA::ELEMS, b, kb, tid);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += Cfg::BK) {
    const bool more = k0 + Cfg::BK < ke;
    if (more) {
      sa.load(a, m0, k0 + Cfg::BK, tid);
      sb.load(b, n0, k0 + Cfg::BK, tid);
    }
    const T* As = smem + buf * SM::STAGE;
    const T* Bs = As + SM::LA::ELEMS;
#pragma unroll
    for (int kk = 0; kk < Cfg::BK; kk += MM::KS) {
      typename MM::frag fa[Cfg::MI], fb[Cfg::NI];
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
        fa[i] = load_frag<Cfg, Cfg::BM, KCA>(As, wm * Cfg::WTM + i * 16 + (lane & 15), kk, lane);
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
        fb[j] = load_frag<Cfg, Cfg::BN, KCB>(Bs, wn * Cfg::WTN + j * 16 + (lane & 15), kk, lane);
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) acc.a[i][j] = MM::mma(fa[i], fb[j], acc.a[i][j]);
    }
    if (more) {
      T* nA = smem + (buf ^ 1) * SM::STAGE;
      sa.store(nA, a, k0 + Cfg::BK, tid);
      sb.store(nA + SM::LA::ELEMS, b, k0 + Cfg::BK, tid);
    }
    __syncthreads();
    buf ^= 1;
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
