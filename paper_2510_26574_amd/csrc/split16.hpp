// Float32 products on the fp16 MFMA pipe as split pairs, for gfx950.
//
// Each operand element x is scaled by a power of two (exact) and split into
// hi = fp16(x) and lo = fp16(x - hi), so x = hi + lo to 22 bits; a product x y
// is taken as hi_x hi_y + hi_x lo_y + lo_x hi_y (the dropped lo_x lo_y is below
// 2^-22 |x y|), each term an exact fp16 product accumulated in float32 by
// v_mfma_f32_16x16x32_f16.  This is the three-product float32 emulation of
// Ootomo and Yokota (2022): three fp16 MFMAs per float32 product against one
// float32 MFMA of a fifth of the rate.
#pragma once
#include "common.hpp"
#include "tile_gemm.hpp"

// acc += 2^24 F(m0:m0+128, :k) FSa(:nt, :k)^T on the fp16 MFMA pipe, for a
// float32 factor.  Each operand element x is scaled by 2^12 (exact; |x| <= 1
// because the rows of F have norm at most 1) and split into hi = fp16(x) and
// lo = fp16(x - hi); a product is taken as hi hi + hi lo + lo hi (unit
// roundoff 2^-22, the three-product float32 emulation of Ootomo and Yokota,
// 2022), at three fp16 MFMAs per product against one float32 MFMA of a fifth
// of the rate.  The 16x16x32 fp16 MFMA shares its accumulator layout with the
// bf16 one of the kernel-column product.
//
// Staging through registers, double buffered, 64 k per stage:
//   A (F, column-major): thread t holds row t % 128 at k groups t / 128 and
//     t / 128 + 4 (8 consecutive k each; every load is a 256-byte row run
//     across the wave);
//   B (FSa, k-contiguous rows): thread t holds row t / 4 at k groups t % 4
//     and t % 4 + 4;
// both land in LDS as [row][k] fp16 pairs (hi and lo arrays, 128-byte rows
// with their 16-byte chunks permuted by lds_swz8 against bank conflicts), so
// every MFMA operand is one 16-byte read.
struct SchurSplit {
  static constexpr int BK = 64;
  static constexpr int LDK = BK;
  static constexpr int ELEMS = 128 * LDK;
  // half offset of 16-byte chunk c (k = 8 c .. 8 c + 7) of a staged row
  __device__ static inline int at(int row, int c) { return row * LDK + 8 * (c ^ lds_swz8(row)); }
  static constexpr size_t bytes = 2 * 4 * (size_t)ELEMS * sizeof(_Float16);
  static constexpr float SC = 4096.0f;  // 2^12 per operand
};
typedef _Float16 v8h_t __attribute__((ext_vector_type(8)));

__device__ inline void split8(const float (&x)[8], v8h_t& hi, v8h_t& lo,
                              float sc = SchurSplit::SC) {
  // x sc is exact (sc a power of two); hi = fp16(x sc), lo = fp16(x sc - hi)
  uint32_t hw[4], lw[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) split_pair_f16(x[e] * sc, x[e + 1] * sc, hw[e >> 1], lw[e >> 1]);
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const v4u h4 = {hw[0], hw[1], hw[2], hw[3]}, l4 = {lw[0], lw[1], lw[2], lw[3]};
  hi = __builtin_bit_cast(v8h_t, h4);
  lo = __builtin_bit_cast(v8h_t, l4);
}

// Register ring of two stages: the global reads of stage s + 2 are issued
// while the MFMAs consume stage s, and stage s + 1 is converted into LDS after
// them.  begin() issues the reads of the first two stages, so a caller can
// overlap their latency with other work before run().
// A_ROWS: A is k-contiguous too (A[m * ldf + l], the points of a distance
// product), loaded like B: thread t holds row t / 4 at k groups t % 4 and
// t % 4 + 4.
// Two shapes: eight waves on a 128 x 128 tile, or (A column-major only) four
// waves on 128 x 64, where a thread holds row t % 128 of A at k groups t / 128
// + 2 h (h < 4); B always takes four threads per row.
template <class Cfg, bool A_ROWS = false>
struct SchurSplitPipe {
  static_assert(Cfg::BM == 128 && ((Cfg::NT == 512 && Cfg::BN == 128) ||
                                   (Cfg::NT == 256 && Cfg::BN == 64 && !A_ROWS)),
                "eight waves on 128 x 128, or four on 128 x 64");
  static constexpr int BK = SchurSplit::BK, LDK = SchurSplit::LDK;
  static constexpr int ELA = 128 * LDK, ELB = Cfg::BN * LDK;  // halfs per hi or lo slice
  static constexpr int GA = A_ROWS ? 2 : 8 * 128 / Cfg::NT;  // A k-groups per thread
  static constexpr int GS = A_ROWS ? 4 : Cfg::NT / 128;      // and their stride
  static constexpr int STAGE = 2 * ELA + 2 * ELB;             // halfs per LDS buffer
  static constexpr size_t single_bytes = (size_t)STAGE * sizeof(_Float16);
  const float* __restrict__ F;
  int64_t ldf, N;
  const float* __restrict__ FSa;
  int r, nt, k;
  int64_t m0;
  float bsc = SchurSplit::SC;  // power-of-two scale of the B operand
  float asc = SchurSplit::SC;  // and of the A operand
  float a0[GA][8], b0[2][8], a1[GA][8], b1[2][8];

  // rows [row of this thread] of a k-contiguous operand (stride ld, `rows`
  // rows), 8 consecutive k at k groups g and g + 4 of the stage at kb
  __device__ inline void load_rows(float (&x)[2][8], const float* __restrict__ P, int64_t ld,
                                   int64_t row, int64_t rows, int kb, int g) const {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k0 = kb + 8 * (g + 4 * h);
      const float* p = P + row * ld + k0;
      if (row < rows && k0 + 8 <= k && (ld % 4) == 0) {
        const v4f u = *reinterpret_cast<const v4f*>(p);
        const v4f w = *reinterpret_cast<const v4f*>(p + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          x[h][e] = u[e];
          x[h][4 + e] = w[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[h][e] = (row < rows && k0 + e < k) ? p[e] : 0.0f;
      }
    }
  }

  __device__ inline void load_a(float (&a)[GA][8], int kb) const {
    const int tid = threadIdx.x;
    if constexpr (A_ROWS) {
      load_rows(a, F, ldf, m0 + (tid >> 2), N, kb, tid & 3);
    } else {
      const int arow = tid & 127, ag = tid >> 7;
      const int64_t am = m0 + arow;
#pragma unroll
      for (int h = 0; h < GA; ++h) {
        const int k0 = kb + 8 * (ag + GS * h);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          a[h][e] = (am < N && k0 + e < k) ? F[am + (int64_t)(k0 + e) * ldf] : 0.0f;
      }
    }
  }
  __device__ inline void load_b(float (&b)[2][8], int kb) const {
    const int tid = threadIdx.x;
    load_rows(b, FSa, r, tid >> 2, nt, kb, tid & 3);
  }
  __device__ inline void load(float (&a)[GA][8], float (&b)[2][8], int kb) const {
    load_a(a, kb);
    load_b(b, kb);
  }

  __device__ inline void store(const float (&a)[GA][8], const float (&b)[2][8], _Float16* sm,
                               int buf) const {
    const int tid = threadIdx.x;
    const int arow = A_ROWS ? tid >> 2 : tid & 127, ag = A_ROWS ? tid & 3 : tid >> 7;
    const int brow = tid >> 2, bg = tid & 3;
    _Float16* base = sm + (size_t)buf * STAGE;
#pragma unroll
    for (int h = 0; h < GA; ++h) {
      v8h_t hi, lo;
      split8(a[h], hi, lo, asc);
      const int o = SchurSplit::at(arow, ag + GS * h);
      *reinterpret_cast<v8h_t*>(base + o) = hi;
      *reinterpret_cast<v8h_t*>(base + ELA + o) = lo;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v8h_t hi, lo;
      split8(b[h], hi, lo, bsc);
      const int o = SchurSplit::at(brow, bg + 4 * h);
      *reinterpret_cast<v8h_t*>(base + 2 * ELA + o) = hi;
      *reinterpret_cast<v8h_t*>(base + 2 * ELA + ELB + o) = lo;
    }
  }

  __device__ inline void compute(TileAcc<Cfg>& acc, const _Float16* sm, int buf) const {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % Cfg::WAVES_M, wn = wave / Cfg::WAVES_M;
    if (wn * Cfg::WTN >= nt) return;  // this wave's columns are all beyond the block
    const _Float16* base = sm + (size_t)buf * STAGE;
#pragma unroll
    for (int kq = 0; kq < BK; kq += 32) {
      // B fragments for the whole k-step, A fragments one row block at a time
      // (fewer live registers)
      v8h_t bh[Cfg::NI], bl[Cfg::NI];
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        const int o = SchurSplit::at(wn * Cfg::WTN + j * 16 + (lane & 15), kq / 8 + (lane >> 4));
        bh[j] = *reinterpret_cast<const v8h_t*>(base + 2 * ELA + o);
        bl[j] = *reinterpret_cast<const v8h_t*>(base + 2 * ELA + ELB + o);
      }
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i) {
        const int o = SchurSplit::at(wm * Cfg::WTM + i * 16 + (lane & 15), kq / 8 + (lane >> 4));
        const v8h_t ah = *reinterpret_cast<const v8h_t*>(base + o);
        const v8h_t al = *reinterpret_cast<const v8h_t*>(base + ELA + o);
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) {
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc.a[i][j], 0, 0, 0);
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc.a[i][j], 0, 0, 0);
          acc.a[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc.a[i][j], 0, 0, 0);
        }
      }
    }
  }

  __device__ inline void begin() {
    load(a0, b0, 0);
    if (BK < k) load(a1, b1, BK);
  }

  // Single-buffer form (half the LDS, so two workgroups share a CU): one
  // stage of register prefetch, stage s + 1 converted after stage s's MFMAs.
  __device__ inline void begin1() { load(a0, b0, 0); }
  __device__ inline void run1(TileAcc<Cfg>& acc, char* smem_raw) {
    _Float16* sm = reinterpret_cast<_Float16*>(smem_raw);
    const int ns = (k + BK - 1) / BK;
    __syncthreads();  // the LDS may still be read by the preceding product
    store(a0, b0, sm, 0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
      if (s + 1 < ns) load(a0, b0, (s + 1) * BK);
      compute(acc, sm, 0);
      __syncthreads();  // every wave is done with the buffer (the caller reuses it too)
      if (s + 1 < ns) {
        store(a0, b0, sm, 0);
        __syncthreads();
      }
    }
  }

  // Single-buffer form with only A in the register ring: B (a few hundred KB
  // shared by every workgroup, so served from L2) is read after the stage's
  // MFMAs, which keeps its 16 registers out of the loop's live set (the
  // fused column kernels then fit 128 VGPRs without spilling).
  __device__ inline void begin1a() { load_a(a0, 0); }
  __device__ inline void run1b(TileAcc<Cfg>& acc, char* smem_raw) {
    _Float16* sm = reinterpret_cast<_Float16*>(smem_raw);
    const int ns = (k + BK - 1) / BK;
    __syncthreads();  // the LDS may still be read by the preceding product
    load_b(b0, 0);
    store(a0, b0, sm, 0);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
      if (s + 1 < ns) load_a(a0, (s + 1) * BK);
      compute(acc, sm, 0);
      __syncthreads();  // every wave is done with the buffer (the caller reuses it too)
      if (s + 1 < ns) {
        load_b(b0, (s + 1) * BK);
        store(a0, b0, sm, 0);
        __syncthreads();
      }
    }
  }

  // acc += 2^24 F(m0.., :k) FSa(:nt, :k)^T; begin() must have been called.
  __device__ inline void run(TileAcc<Cfg>& acc, char* smem_raw) {
    _Float16* sm = reinterpret_cast<_Float16*>(smem_raw);
    const int ns = (k + BK - 1) / BK;
    __syncthreads();  // the LDS may still be read by the preceding product
    store(a0, b0, sm, 0);
    __syncthreads();
    // stage s sits in LDS buffer s & 1; even stages pass through (a0, b0),
    // odd ones through (a1, b1)
    for (int s = 0; s < ns; s += 2) {
      if (s + 2 < ns) load(a0, b0, (s + 2) * BK);
      compute(acc, sm, 0);
      if (s + 1 < ns) store(a1, b1, sm, 1);
      __syncthreads();
      if (s + 1 >= ns) break;
      if (s + 3 < ns) load(a1, b1, (s + 3) * BK);
      compute(acc, sm, 1);
      if (s + 2 < ns) store(a0, b0, sm, 0);
      __syncthreads();
    }
  }
};

