// Shared device helpers for the gfx950 kernels: vector types, MFMA wrappers
// with their lane layouts, wave reductions, and the error plumbing of the
// C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rpchol.h"

typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

#define RPC_WAVE 64

// ---------------------------------------------------------------- MFMA
// Layouts measured on gfx950 (16 x 16 output tile, 64 lanes):
//   A[m][k] operand: lane l holds m = l % 16 and the k-slot l / 16 (one
//     element for f32/f64, eight consecutive k for bf16);
//   B[k][n] operand: lane l holds n = l % 16 and the same k-slot;
//   f32 / bf16 accumulators: element i of lane l is D[4 (l/16) + i][l % 16];
//   f64 accumulators:        element i of lane l is D[(l/16) + 4 i][l % 16].
// Only the pairing of A and B k-slots matters for the product, so loaders
// may permute k freely as long as A and B agree.
template <typename T>
struct Mma;

template <>
struct Mma<double> {
  typedef double frag;
  typedef v4d acc;
  typedef double acc_t;
  static constexpr int KS = 4;   // k per instruction
  static constexpr int EPL = 1;  // k elements per lane per instruction
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Mma<float> {
  typedef float frag;
  typedef v4f acc;
  typedef float acc_t;
  static constexpr int KS = 4;
  static constexpr int EPL = 1;
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <>
struct Mma<__bf16> {
  typedef v8bf frag;
  typedef v4f acc;
  typedef float acc_t;
  static constexpr int KS = 32;
  static constexpr int EPL = 8;
  __device__ static inline acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// --------------------------------------------------------- conversions
template <typename T>
__device__ inline T cvt(float x);
template <>
__device__ inline float cvt<float>(float x) { return x; }
template <>
__device__ inline double cvt<double>(float x) { return (double)x; }
template <>
__device__ inline __bf16 cvt<__bf16>(float x) { return (__bf16)x; }

template <typename T>
__device__ inline T cvtd(double x);
template <>
__device__ inline float cvtd<float>(double x) { return (float)x; }
template <>
__device__ inline double cvtd<double>(double x) { return x; }
template <>
__device__ inline __bf16 cvtd<__bf16>(double x) { return (__bf16)(float)x; }

template <typename T>
__device__ inline double to_d(T x) { return (double)x; }
template <>
__device__ inline double to_d<__bf16>(__bf16 x) { return (double)(float)x; }

// element i of a points row of element type TX, as float64 (exact)
template <typename TX>
__device__ inline double ld_point(const TX* __restrict__ p, int64_t i) {
  return to_d(p[i]);
}

// Split of two float32 values into fp16 pairs: hi = fp16(v) (round to
// nearest, one packed conversion for both), lo = fp16(v - hi) by one
// mixed-precision fma per value (v - hi is exact in float32, so hi + lo
// carries v to 22 bits).  Returns the two hi halves packed in *hb (v0 in bits
// 15:0) and the two lo halves in *lb.  The caller scales v into fp16 range.
typedef _Float16 v2h_t __attribute__((ext_vector_type(2)));
__device__ inline void split_pair_f16(float v0, float v1, uint32_t& hb, uint32_t& lb) {
  v2h_t hp;
  hp[0] = (_Float16)v0;
  hp[1] = (_Float16)v1;
  hb = __builtin_bit_cast(uint32_t, hp);
  // mixlo writes bits 15:0 and mixhi bits 31:16 of the same register
  asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(lb) : "v"(v0), "v"(hb));
  asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "+v"(lb) : "v"(v1), "v"(hb));
}

// ------------------------------------------------------------ LDS layout
// Bank behaviour of the gfx950 LDS, as counted (SQ_LDS_BANK_CONFLICT):
//   ds_read_b128:  64 banks of 4 bytes; a wave is served in four passes of 16
//     lanes, a pass being the four-lane groups g = lane / 4 of one half-wave
//     whose three low bits have equal parity (lanes 0-3, 12-15, 20-23, 24-27);
//   ds_write_b128: 32 banks, 8 consecutive lanes per pass;
//   ds_write_b64:  32 banks, 16 consecutive lanes per pass.
// A 16 x 32 fp16/bf16 MFMA fragment (lane: row lane % 16, 16-byte k-chunk
// lane / 16) read from rows padded to 144 bytes therefore takes two passes per
// pass-group.  Rows of 128 bytes (eight chunks, no pad) whose chunk index is
// XORed with lds_swz8(row) serve it in one, and keep conflict-free both the
// row-major chunk writes (eight lanes on one row) and the writes of four lanes
// per row at a fixed chunk group: the three bits of lds_swz8 over rows
// 8 m .. 8 m + 7 are a permutation, rows 2 m and 2 m + 1 differ in bit 2, and
// bit 3 of the row separates rows r and r + 8 of one pass.
__device__ inline int lds_swz8(int row) {
  return (((row & 1) << 2) | ((row >> 1) & 3)) ^ ((row & 8) >> 1);
}

// Broadcast lane `src` (wave-uniform) of a double held in a VGPR pair.
__device__ inline double bcast_lane(double v, int src) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// ------------------------------------------------------ wave reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RPC_WAVE);
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RPC_WAVE);
  return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RPC_WAVE);
  return v;
}

// Status words written from the device (first error wins).
__device__ inline void set_status(int32_t* st, int32_t code) {
  if (st) atomicCAS(st, 0, code);
}

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Host-side bump allocator over a caller-provided workspace.
struct WsCursor {
  char* base;
  size_t used;
  size_t cap;
  bool ok;
  template <typename T>
  T* take(size_t count) {
    size_t off = align_up(used, 256);
    size_t need = off + align_up(count * sizeof(T), 256);
    if (base == nullptr || need > cap) {
      ok = false;
      used = need;
      return nullptr;
    }
    used = need;
    return reinterpret_cast<T*>(base + off);
  }
};

// Calls f((TX*)nullptr) with TX the element type of points of rpc_dtype
// `dt` (float, double or __bf16); RPC_EINVAL for any other type.
template <typename Fn>
inline int with_points_type(int32_t dt, Fn&& f) {
  if (dt == RPC_F32) return f((const float*)nullptr);
  if (dt == RPC_F64) return f((const double*)nullptr);
  if (dt == RPC_BF16) return f((const __bf16*)nullptr);
  return RPC_EINVAL;
}

// A captured and instantiated HIP graph (rpc_graph of the C-ABI).
struct rpc_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace rpc_internal {
// The batched form issues many jobs from one host thread and must never block
// it: while set on the calling thread, bistoch_eig issues the fallback
// launches of its eigensolver unconditionally instead of reading the
// convergence flag back to the host.
void set_host_gate_off(bool off);
}  // namespace rpc_internal

#define RPC_HIP_CHECK(expr)                    \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return RPC_EHIP;     \
  } while (0)

#define RPC_LAUNCH_CHECK()                           \
  do {                                               \
    hipError_t _e = hipGetLastError();               \
    if (_e != hipSuccess) return RPC_EHIP;           \
  } while (0)
