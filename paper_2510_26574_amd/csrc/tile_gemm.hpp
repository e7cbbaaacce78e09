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
// contiguous index).  A k-contiguous slice of a 2-byte type with 128-byte rows
// (BK = 64, read as 16-byte MFMA fragments) is instead stored unpadded with
// its 16-byte chunks permuted per row by lds_swz8, which keeps the fragment
// reads free of bank conflicts (the padded rows cost two passes per read).
template <typename T, int ROWS, int BK, bool KC>
struct SliceLayout {
  static constexpr bool SWZ = KC && sizeof(T) == 2 && BK * sizeof(T) == 128;
  static constexpr int LDK = SWZ ? BK : BK + 16 / (int)sizeof(T);
  static constexpr int LDR = ROWS + 16;
  static constexpr int ELEMS = KC ? ROWS * LDK : BK * LDR;
  __device__ static inline int at(int row, int k) {
    if constexpr (SWZ) return row * LDK + ((((k >> 3) ^ lds_swz8(row)) << 3) | (k & 7));
    return KC ? row * LDK + k : k * LDR + row;
  }
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
// LOWER_B: B(n, k) = 0 for k > n (a lower-triangular right factor, as in a
// product with an inverse Cholesky factor): an MFMA whose k-step lies wholly
// above its 16 columns, or whose columns are all past B's valid rows, is
// skipped (a wave-uniform branch).
template <class Cfg, typename TGA, bool KCA, typename TGB, bool KCB, bool LOWER_B = false>
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
      for (int j = 0; j < Cfg::NI; ++j) {
        if constexpr (LOWER_B) {
          const int64_t c0 = n0 + wn * Cfg::WTN + j * 16;
          if (k0 + kk >= c0 + 16 || c0 >= b.rows) continue;
        }
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i) acc.a[i][j] = MM::mma(fa[i], fb[j], acc.a[i][j]);
      }
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

// ------------------------------------------------- direct global->LDS staging
// On gfx950 global_load_lds_dwordx4 copies 16 bytes per lane from any global
// address straight into LDS: lane l of one wave instruction writes bytes
// [16 l, 16 l + 16) after the instruction's wave-uniform LDS base.  A padded
// slice (SliceLayout) is therefore filled chunk by chunk, line by line; the
// pad chunk at the end of each line is filled from the line's first chunk.
// In a swizzled slice LDS chunk j of a line holds the line's global chunk
// j ^ lds_swz8(line), which is what the lane of that chunk fetches.
// No registers hold data in flight, so several stages can be outstanding at
// once (the register-staged main loop above has one).
#define RPC_GPTR(p) ((const void __attribute__((address_space(1)))*)(p))
#define RPC_LPTR(p) ((void __attribute__((address_space(3)))*)(p))

// s_waitcnt vmcnt(N) only (expcnt and lgkmcnt left at their no-wait maxima).
template <int N>
__device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
__device__ inline void wait_vmcnt_dyn(int n) {
  switch (n) {
#define RPC_VMCASE(i) \
  case i:             \
    wait_vmcnt<i>();  \
    break;
    RPC_VMCASE(1) RPC_VMCASE(2) RPC_VMCASE(3) RPC_VMCASE(4) RPC_VMCASE(5) RPC_VMCASE(6)
    RPC_VMCASE(7) RPC_VMCASE(8) RPC_VMCASE(9) RPC_VMCASE(10) RPC_VMCASE(11) RPC_VMCASE(12)
    RPC_VMCASE(13) RPC_VMCASE(14) RPC_VMCASE(15) RPC_VMCASE(16) RPC_VMCASE(17) RPC_VMCASE(18)
    RPC_VMCASE(19) RPC_VMCASE(20) RPC_VMCASE(21) RPC_VMCASE(22) RPC_VMCASE(23) RPC_VMCASE(24)
    RPC_VMCASE(25) RPC_VMCASE(26) RPC_VMCASE(27) RPC_VMCASE(28) RPC_VMCASE(29) RPC_VMCASE(30)
    RPC_VMCASE(31) RPC_VMCASE(32)
#undef RPC_VMCASE
    default:
      wait_vmcnt<0>();  // anything else: wait for everything (always safe)
  }
}

// Barrier between waves of the workgroup without the memory fence of
// __syncthreads (which would wait for every outstanding global load); the
// empty asm statements keep the compiler from moving memory accesses across.
__device__ inline void lds_barrier() {
  // lgkmcnt(0) only (vmcnt 63, expcnt 7): this wave's LDS reads are done
  __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <typename T, int ROWS, int BK, bool KC, int NW>
struct DirectSlice {
  typedef SliceLayout<T, ROWS, BK, KC> L;
  static constexpr int E = 16 / (int)sizeof(T);          // elements per chunk
  static constexpr int PITCH = KC ? L::LDK : L::LDR;      // elements per LDS line
  static constexpr int LINES = KC ? ROWS : BK;
  static constexpr int CPL = PITCH / E;                   // chunks per line, pad included
  static constexpr int DCPL = (KC ? BK : ROWS) / E;       // data chunks per line
  static constexpr int WINST = LINES * CPL / 64;          // wave instructions per slice
  static_assert(PITCH % E == 0 && (LINES * CPL) % 64 == 0 && (L::SWZ ? DCPL == CPL : DCPL < CPL),
                "direct slice shape");
  __device__ static inline int count(int wave) { return wave < WINST ? (WINST - wave + NW - 1) / NW : 0; }
  // rows r0 .. r0 + ROWS - 1 and k0 .. k0 + BK - 1 must be readable
  __device__ static inline void issue(T* slice, const T* p, int64_t ld, int64_t r0, int64_t k0,
                                      int wave, int lane) {
    for (int q = wave; q < WINST; q += NW) {
      const int c = q * 64 + lane;
      const int line = c / CPL;
      int j = c % CPL;
      if constexpr (L::SWZ) j ^= lds_swz8(line);
      else if (j >= DCPL) j = 0;
      const T* g = KC ? p + (r0 + line) * ld + k0 + (int64_t)j * E
                      : p + (r0 + (int64_t)j * E) + (k0 + line) * ld;
      __builtin_amdgcn_global_load_lds(RPC_GPTR(g), RPC_LPTR(slice + q * 64 * E), 16, 0, 0);
    }
  }
};

// LDS bytes of the NS-stage direct pipeline.
template <class Cfg, int NS, bool KCA, bool KCB>
struct DirectSmem {
  static constexpr size_t bytes = (size_t)NS * TileSmem<Cfg, KCA, KCB>::STAGE * sizeof(typename Cfg::T);
};

// acc += A(m0.., kb..ke) * B(n0.., kb..ke)^T like tile_mainloop, with NS-stage
// direct staging (NS - 1 stages in flight).  Operands are read in their LDS
// type (no conversion or scaling).  a_avail / b_avail: rows of A / B that may
// be read (>= the valid rows; rows past the valid count feed only outputs
// that the caller discards).  Tiles that would read past them, and a final
// partial k-stage, go through the register-staged path with zero fill.
// smem holds DirectSmem<Cfg, NS, KCA, KCB>::bytes.
//
// n_active: output columns n0 .. n0 + n_active - 1 are wanted; a wave whose
// whole column slice lies beyond them skips its MFMAs (it still loads and
// synchronises with the workgroup) and leaves its accumulators unchanged.
// rot: the full k-stages are visited starting at stage rot mod (their count)
// and wrapping around, so workgroups that share an operand (all of them read
// the same pivot rows) do not all hit the same L2 lines at the same time.
template <class Cfg, int NS, bool KCA, bool KCB>
__device__ inline void tile_mainloop_direct(TileAcc<Cfg>& acc,
                                            const GOperand<typename Cfg::T, KCA>& A,
                                            const GOperand<typename Cfg::T, KCB>& B, int64_t m0,
                                            int64_t n0, int64_t kb, int64_t ke, int64_t a_avail,
                                            int64_t b_avail, typename Cfg::T* smem,
                                            int n_active = 1 << 30, int rot = 0) {
  typedef typename Cfg::T T;
  typedef typename Cfg::MM MM;
  typedef TileSmem<Cfg, KCA, KCB> SM;
  constexpr int NW = Cfg::NT / 64;
  typedef DirectSlice<T, Cfg::BM, Cfg::BK, KCA, NW> DA;
  typedef DirectSlice<T, Cfg::BN, Cfg::BK, KCB, NW> DB;
  static_assert(NS >= 2, "pipeline depth");
  static_assert(LdsKC<T, KCA>::value == KCA && LdsKC<T, KCB>::value == KCB,
                "direct staging keeps the global orientation in LDS");
  if (kb >= ke) return;
  const int64_t kend = ke < A.K ? (ke < B.K ? ke : B.K) : (A.K < B.K ? A.K : B.K);
  const bool full_tile = m0 + Cfg::BM <= a_avail && n0 + Cfg::BN <= b_avail && A.vec && B.vec;
  const int nfull = full_tile && kend > kb ? (int)((kend - kb) / Cfg::BK) : 0;
  if (nfull == 0) {
    tile_mainloop<Cfg>(acc, A, B, m0, n0, kb, ke, smem);
    return;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  const int per = DA::count(wave) + DB::count(wave);
  const bool idle = wn * Cfg::WTN >= n_active;
  const int r0s = rot % nfull;
  auto issue = [&](int s) {
    T* base = smem + (s % NS) * SM::STAGE;
    const int ps = s + r0s < nfull ? s + r0s : s + r0s - nfull;  // stage in k order
    const int64_t k0 = kb + (int64_t)ps * Cfg::BK;
    DA::issue(base, A.p, A.ld, m0, k0, wave, lane);
    DB::issue(base + SM::LA::ELEMS, B.p, B.ld, n0, k0, wave, lane);
  };
  auto compute = [&](const T* As) {
    if (idle) return;
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
  };
  // the caller's LDS may still be read by other waves (a previous product)
  lds_barrier();
  for (int s = 0; s < NS - 1 && s < nfull; ++s) issue(s);
  for (int s = 0; s < nfull; ++s) {
    const int ahead = (nfull - 1 - s) < (NS - 2) ? (nfull - 1 - s) : (NS - 2);
    wait_vmcnt_dyn(ahead * per);  // this wave's chunks of stage s have landed
    lds_barrier();                // ... and every other wave's; stage s - 1 is consumed
    if (s + NS - 1 < nfull) issue(s + NS - 1);
    compute(smem + (s % NS) * SM::STAGE);
  }
  const int64_t kt = kb + (int64_t)nfull * Cfg::BK;
  if (kt < ke) {
    // partial last stage: register-staged with zero fill, into a free buffer
    TileStage<T, Cfg::BM, Cfg::BK, Cfg::NT, T, KCA> sa;
    TileStage<T, Cfg::BN, Cfg::BK, Cfg::NT, T, KCB> sb;
    GOperand<T, KCA> a = A;
    GOperand<T, KCB> b = B;
    a.K = ke < A.K ? ke : A.K;
    b.K = ke < B.K ? ke : B.K;
    sa.load(a, m0, kt, tid);
    sb.load(b, n0, kt, tid);
    T* buf = smem + (nfull % NS) * SM::STAGE;
    lds_barrier();  // every wave is done with the buffer being overwritten
    sa.store(buf, a, kt, tid);
    sb.store(buf + SM::LA::ELEMS, b, kt, tid);
    __syncthreads();
    compute(buf);
  }
  lds_barrier();  // the caller may reuse smem
}

// ----------------------------------------------- coalesced column-major store
// The MFMA accumulator layout spreads one store instruction over 16 columns,
// a few scattered rows each.  Column-major outputs are therefore staged per
// wave through LDS ([col][row], odd pitch) and written back one column
// segment per instruction, WTM consecutive rows at a time.  `val(row, col,
// v)` gives the value for tile-local (row, col); entries outside [0, M) x
// [0, N) (global) are not written.  smem must be free (no other wave still
// reading it) and hold ColStoreSmem<Cfg, TO>::bytes.
template <class Cfg, typename TO>
struct ColStoreSmem {
  static constexpr int LDP = Cfg::WTM + 1;
  static constexpr size_t bytes = (size_t)(Cfg::NT / 64) * Cfg::WTN * LDP * sizeof(TO);
};

template <class Cfg, typename TO, typename Fn>
__device__ inline void store_colmajor(TileAcc<Cfg>& acc, void* smem, TO* __restrict__ out,
                                      int64_t ld, int64_t m0, int64_t n0, int64_t M, int64_t N,
                                      Fn&& val) {
  constexpr int LDP = ColStoreSmem<Cfg, TO>::LDP;
  static_assert(64 % Cfg::WTM == 0 || Cfg::WTM % 64 == 0, "wave tile rows vs wave width");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
  TO* s = reinterpret_cast<TO*>(smem) + (size_t)wave * Cfg::WTN * LDP;
  for_each_acc<Cfg>(acc, [&](int row, int col, typename Cfg::MM::acc_t v) {
    s[(col - wn * Cfg::WTN) * LDP + (row - wm * Cfg::WTM)] = val(row, col, v);
  });
  // the wave reads back what its own lanes wrote: LDS operations of one wave
  // complete in order; the asm statements keep the compiler from reordering
  asm volatile("" ::: "memory");
  const int64_t mb = m0 + wm * Cfg::WTM, nb = n0 + wn * Cfg::WTN;
  if constexpr (Cfg::WTM >= 64) {
#pragma unroll 4
    for (int c = 0; c < Cfg::WTN; ++c) {
      const int64_t n = nb + c;
#pragma unroll
      for (int rr = 0; rr < Cfg::WTM; rr += 64) {
        const int64_t m = mb + rr + lane;
        if (m < M && n < N) out[m + n * ld] = s[c * LDP + rr + lane];
      }
    }
  } else {
    constexpr int CPI = 64 / Cfg::WTM;  // columns per store instruction
    const int r = lane % Cfg::WTM, cq = lane / Cfg::WTM;
#pragma unroll 4
    for (int c = 0; c < Cfg::WTN; c += CPI) {
      const int64_t m = mb + r, n = nb + c + cq;
      if (m < M && n < N) out[m + n * ld] = s[(c + cq) * LDP + r];
    }
  }
  asm volatile("" ::: "memory");
}
