// Learned surrogate of the Nystrom extension on gfx950.
//
// A two-hidden-layer perceptron (exact GELU) maps a standardised state to
// approximate eigenfunction values; a scalar residual head on the last hidden
// layer predicts the log10 RMS error of those values so that callers can fall
// back to the exact extension (nystrom_extend) point by point.
//
// Every product is a bf16 MFMA tile product with fp32 accumulation (the tile
// engine of tile_gemm.hpp, 64 x 64 x 64 tiles, four waves of 32 x 32).  The
// epilogues fuse the bias, the GELU and its derivative, the loss and the
// output error, so each layer costs one pass over its activations:
//   forward   z = A W^T + b  -> z (fp32) and gelu(z) (bf16)
//   output    y = A W3^T + b3 -> dY = 2 (y - t) / (B n_out) (bf16) + loss partials
//   backward  dA = dY W -> dZ = dA * gelu'(z) (bf16)
//   gradients G_s = dY^T A over batch split s (fp32 partials, bias sums too)
// and one elementwise kernel sums the split partials in a fixed order and
// applies AdamW to the fp32 parameters, refreshing their bf16 copy.
#include <math.h>

#include "common.hpp"
#include "profile.hpp"
#include "tile_gemm.hpp"

namespace {

constexpr int64_t SEG = 64;       // alignment of each parameter segment (elements)
constexpr int64_t MAXB = 65536;   // batch limit and inference chunk (rows)
constexpr int64_t FB_CHUNK = 65536;  // fallback points per Nystrom call
typedef TileCfg<__bf16, 64, 64, 64, 2, 2> Cfg;
constexpr int TB = 64;  // tile edge (rows and columns)

struct Lay {
  int64_t W1, b1, W2, b2, W3, b3, total;
  int d, h, nout, n3;
};

bool make_layout(const sur_shape* s, Lay& L) {
  if (!s || s->d < 8 || s->d > 4096 || s->d % 8 != 0 || s->h < 64 || s->h > 4096 || s->h % 64 != 0 ||
      s->n_out < 1 || s->n_out > 255)
    return false;
  const int64_t d = s->d, h = s->h;
  const int n3 = (s->n_out + 1 + 15) / 16 * 16;
  int64_t o = 0;
  auto seg = [&](int64_t n) {
    const int64_t a = o;
    o += (int64_t)align_up((size_t)n, (size_t)SEG);
    return a;
  };
  L.W1 = seg(h * d);
  L.b1 = seg(h);
  L.W2 = seg(h * h);
  L.b2 = seg(h);
  L.W3 = seg((int64_t)n3 * h);
  L.b3 = seg(n3);
  L.total = o;
  L.d = s->d;
  L.h = s->h;
  L.nout = s->n_out;
  L.n3 = n3;
  return true;
}

// 0: pad entry (never trained, kept zero), 1: trained in phase 0 (W1..b3
// except the residual head), 2: residual head (phase 1).
__device__ inline int entry_class(const Lay& L, int64_t i) {
  if (i >= L.W1 && i < L.W1 + (int64_t)L.h * L.d) return 1;
  if (i >= L.b1 && i < L.b1 + L.h) return 1;
  if (i >= L.W2 && i < L.W2 + (int64_t)L.h * L.h) return 1;
  if (i >= L.b2 && i < L.b2 + L.h) return 1;
  if (i >= L.W3 && i < L.W3 + (int64_t)L.n3 * L.h) {
    const int row = (int)((i - L.W3) / L.h);
    return row < L.nout ? 1 : (row == L.nout ? 2 : 0);
  }
  if (i >= L.b3 && i < L.b3 + L.n3) {
    const int j = (int)(i - L.b3);
    return j < L.nout ? 1 : (j == L.nout ? 2 : 0);
  }
  return 0;
}

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Index of parameter entry i in the initialisation stream (order W1, b1, W2,
// b2, W3, b3, wr, br; row-major within a matrix) and its fan-in; -1 for pad.
__device__ inline int64_t init_index(const Lay& L, int64_t i, int& fan) {
  const int64_t d = L.d, h = L.h, no = L.nout;
  const int64_t o2 = h * d + h, o3 = o2 + h * h + h;
  if (i >= L.W1 && i < L.W1 + h * d) { fan = L.d; return i - L.W1; }
  if (i >= L.b1 && i < L.b1 + h) { fan = L.d; return h * d + (i - L.b1); }
  if (i >= L.W2 && i < L.W2 + h * h) { fan = L.h; return o2 + (i - L.W2); }
  if (i >= L.b2 && i < L.b2 + h) { fan = L.h; return o2 + h * h + (i - L.b2); }
  fan = L.h;
  if (i >= L.W3 && i < L.W3 + (int64_t)L.n3 * h) {
    const int64_t row = (i - L.W3) / h, col = (i - L.W3) % h;
    if (row < no) return o3 + row * h + col;
    if (row == no) return o3 + no * h + no + col;
    return -1;
  }
  if (i >= L.b3 && i < L.b3 + L.n3) {
    const int64_t j = i - L.b3;
    if (j < no) return o3 + no * h + j;
    if (j == no) return o3 + no * h + no + h;
  }
  return -1;
}

// Parameters from the uniform stream u (if given): (2 u - 1) / sqrt(fan_in);
// pad entries zero; moments zero; bf16 copy.
__global__ void k_sur_init(Lay L, const double* __restrict__ u, float* __restrict__ p,
                           float* __restrict__ m, float* __restrict__ v,
                           __bf16* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= L.total) return;
  int fan = 1;
  const int64_t j = init_index(L, i, fan);
  float x;
  if (j < 0)
    x = 0.0f;
  else if (u)
    x = (float)((2.0 * u[j] - 1.0) * (1.0 / sqrt((double)fan)));
  else
    x = p[i];
  p[i] = x;
  m[i] = 0.0f;
  v[i] = 0.0f;
  wb[i] = (__bf16)x;
}

// Batch assembly: Xh[b][c] = bf16((X[row][c] - mean[c]) rstd[c]) (c < d; zero
// up to ldxh), row = idx[b] (or r0 + b when idx is null); targets gathered
// into Tb (phase 0: tscale T[row + j ldt], j < nout; phase 1: T[row]).
template <typename TT>
__global__ __launch_bounds__(256) void k_sur_gather(const float* __restrict__ X, int64_t ldx,
                                                    int64_t N, int d,
                                                    const double* __restrict__ mean,
                                                    const double* __restrict__ rstd,
                                                    const int64_t* __restrict__ idx, int64_t r0,
                                                    __bf16* __restrict__ Xh, int ldxh,
                                                    const TT* __restrict__ T, int64_t ldt,
                                                    double tscale, int phase, int nout,
                                                    float* __restrict__ Tb,
                                                    int32_t* status) {
  const int64_t b = blockIdx.x;
  int64_t row = idx ? idx[b] : r0 + b;
  const bool ok = row >= 0 && row < N;
  if (!ok) {
    if (threadIdx.x == 0) set_status(status, RPC_EINVAL);
    row = 0;
  }
  for (int c = threadIdx.x; c < ldxh; c += 256) {
    float v = 0.0f;
    if (ok && c < d) v = (float)(((double)X[row * ldx + c] - mean[c]) * rstd[c]);
    Xh[b * ldxh + c] = (__bf16)v;
  }
  if (T) {
    if (phase == 0) {
      for (int j = threadIdx.x; j < nout; j += 256)
        Tb[b * nout + j] = ok ? (float)(tscale * (double)T[row + (int64_t)j * ldt]) : 0.0f;
    } else if (threadIdx.x == 0) {
      Tb[b] = ok ? (float)T[row] : 0.0f;
    }
  }
}

// Hidden layer: z = A W^T + bias (A: M x K bf16, W: N x K bf16, both
// k-contiguous); z (fp32, optional) and gelu(z) (bf16) row-major, ld ldo.
__global__ __launch_bounds__(256) void k_sur_hidden(const __bf16* __restrict__ A, int64_t lda,
                                                    int64_t M, int K,
                                                    const __bf16* __restrict__ W,
                                                    const float* __restrict__ bias, int N,
                                                    float* __restrict__ z,
                                                    __bf16* __restrict__ act, int64_t ldo) {
  extern __shared__ __align__(16) char smem_raw[];
  __bf16* smem = reinterpret_cast<__bf16*>(smem_raw);
  const int64_t n0 = (int64_t)blockIdx.x * TB, m0 = (int64_t)blockIdx.y * TB;
  GOperand<__bf16, true> a{A, lda, M, K, nullptr, true};
  GOperand<__bf16, true> w{W, K, N, K, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, w, m0, n0, 0, K, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, float v) {
    const int64_t m = m0 + row, n = n0 + col;
    if (m < M && n < N) {
      v += bias[n];
      if (z) z[m * ldo + n] = v;
      act[m * ldo + n] = (__bf16)gelu_f(v);
    }
  });
}

// Output layer y = A W3^T + b3 over the n3 rows of W3.
//   mode 0 (training, phase 0): dY = 2 (y - t) / (M n_out) for columns < n_out,
//          zero elsewhere; loss partial sum (y - t)^2;
//   mode 1 (training, phase 1): column n_out only, dY = 2 (res - t) / M;
//   mode 2 (inference): Phi(m, j) = y (column-major), res(m) = column n_out.
__global__ __launch_bounds__(256) void k_sur_output(const __bf16* __restrict__ A, int64_t lda,
                                                    int64_t M, int K,
                                                    const __bf16* __restrict__ W,
                                                    const float* __restrict__ bias, int n3,
                                                    int nout, int mode,
                                                    const float* __restrict__ Tb, float gscale,
                                                    __bf16* __restrict__ dY,
                                                    float* __restrict__ lpart,
                                                    float* __restrict__ Phi, int64_t ldphi,
                                                    float* __restrict__ res) {
  extern __shared__ __align__(16) char smem_raw[];
  __bf16* smem = reinterpret_cast<__bf16*>(smem_raw);
  __shared__ float red[4];
  const int64_t n0 = (int64_t)blockIdx.x * TB, m0 = (int64_t)blockIdx.y * TB;
  GOperand<__bf16, true> a{A, lda, M, K, nullptr, true};
  GOperand<__bf16, true> w{W, K, n3, K, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, w, m0, n0, 0, K, smem);
  float sq = 0.0f;
  for_each_acc<Cfg>(acc, [&](int row, int col, float v) {
    const int64_t m = m0 + row;
    const int n = (int)(n0 + col);
    if (m >= M || n >= n3) return;
    v += bias[n];
    if (mode == 2) {
      if (n < nout) Phi[m + (int64_t)n * ldphi] = v;
      if (n == nout && res) res[m] = v;
      return;
    }
    float g = 0.0f;
    if (mode == 0 && n < nout) {
      const float e = v - Tb[m * nout + n];
      sq += e * e;
      g = 2.0f * e * gscale;
    } else if (mode == 1 && n == nout) {
      const float e = v - Tb[m];
      sq += e * e;
      g = 2.0f * e * gscale;
    }
    dY[m * n3 + n] = (__bf16)g;
  });
  if (mode == 2) return;
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Back-propagation through a hidden layer: dA = dY W (dY: M x Nw bf16
// k-contiguous; W: Nw x Kin bf16, read as the Kin x Nw operand, row-
// contiguous), dZ = dA * gelu'(z) (bf16, row-major ld ldo).
__global__ __launch_bounds__(256) void k_sur_dx(const __bf16* __restrict__ dY, int64_t ldy,
                                                int64_t M, int Nw,
                                                const __bf16* __restrict__ W, int Kin,
                                                const float* __restrict__ z,
                                                __bf16* __restrict__ dZ, int64_t ldo) {
  extern __shared__ __align__(16) char smem_raw[];
  __bf16* smem = reinterpret_cast<__bf16*>(smem_raw);
  const int64_t k0 = (int64_t)blockIdx.x * TB, m0 = (int64_t)blockIdx.y * TB;
  GOperand<__bf16, true> a{dY, ldy, M, Nw, nullptr, true};
  GOperand<__bf16, false> w{W, Kin, Kin, Nw, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, a, w, m0, k0, 0, Nw, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, float v) {
    const int64_t m = m0 + row, k = k0 + col;
    if (m < M && k < Kin) dZ[m * ldo + k] = (__bf16)(v * gelu_grad_f(z[m * ldo + k]));
  });
}

// Weight and bias gradient partials of one layer over batch split s:
//   part[s][offW + n K + k] = sum_{m in split} dY[m][n] A[m][k]
//   part[s][offb + n]       = sum_{m in split} dY[m][n]   (blocks with blockIdx.x == 0)
// Both operands are read row-contiguous (the batch index is the reduction).
__global__ __launch_bounds__(256) void k_sur_wgrad(const __bf16* __restrict__ dY, int64_t ldy,
                                                   int N, const __bf16* __restrict__ A,
                                                   int64_t lda, int K, int64_t M,
                                                   int64_t mchunk, float* __restrict__ part,
                                                   int64_t total, int64_t offW, int64_t offb) {
  extern __shared__ __align__(16) char smem_raw[];
  __bf16* smem = reinterpret_cast<__bf16*>(smem_raw);
  __shared__ float bred[4][TB];
  const int64_t k0 = (int64_t)blockIdx.x * TB, n0 = (int64_t)blockIdx.y * TB;
  const int s = blockIdx.z;
  const int64_t kb = (int64_t)s * mchunk;
  const int64_t ke = kb + mchunk < M ? kb + mchunk : M;
  float* P = part + (int64_t)s * total;
  GOperand<__bf16, false> g{dY, ldy, N, M, nullptr, true};
  GOperand<__bf16, false> x{A, lda, K, M, nullptr, true};
  TileAcc<Cfg> acc;
  acc.zero();
  tile_mainloop<Cfg>(acc, g, x, n0, k0, kb, ke, smem);
  for_each_acc<Cfg>(acc, [&](int row, int col, float v) {
    const int64_t n = n0 + row, k = k0 + col;
    if (n < N && k < K) P[offW + n * K + k] = v;
  });
  if (blockIdx.x == 0) {
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    float sum = 0.0f;
    if (n0 + c < N)
      for (int64_t m = kb + ph; m < ke; m += 4) sum += (float)dY[m * ldy + n0 + c];
    bred[ph][c] = sum;
    __syncthreads();
    if (ph == 0 && n0 + c < N) P[offb + n0 + c] = ((bred[0][c] + bred[1][c]) + bred[2][c]) + bred[3][c];
  }
}

// Sum the split partials (fixed order) and apply AdamW to the entries the
// phase trains; c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
// tdev (optional): the step number is tdev[0] + 1 and c1, c2 follow from it
// here (a captured epoch replays with the counter kept in device memory).
__global__ void k_sur_adamw(Lay L, int phase, int S, const float* __restrict__ part,
                            float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            __bf16* __restrict__ wb, float* __restrict__ grad, double lr,
                            double b1, double b2, double eps, double wd, double c1, double c2,
                            const int64_t* __restrict__ tdev) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= L.total) return;
  if (tdev) {
    const double t = (double)(tdev[0] + 1);
    c1 = 1.0 / (1.0 - pow(b1, t));
    c2 = 1.0 / (1.0 - pow(b2, t));
  }
  const int cls = entry_class(L, i);
  const bool tr = (phase == 0 && cls == 1) || (phase == 1 && cls == 2);
  if (!tr) {
    if (grad) grad[i] = 0.0f;
    return;
  }
  float gs = 0.0f;
  for (int s = 0; s < S; ++s) gs += part[(int64_t)s * L.total + i];
  if (grad) grad[i] = gs;
  const double g = gs;
  const double mm = b1 * (double)m[i] + (1.0 - b1) * g;
  const double vv = b2 * (double)v[i] + (1.0 - b2) * g * g;
  const double pp = (double)p[i];
  const double pn = pp - lr * wd * pp - lr * (mm * c1) / (sqrt(vv * c2) + eps);
  m[i] = (float)mm;
  v[i] = (float)vv;
  p[i] = (float)pn;
  wb[i] = (__bf16)(float)pn;
}

__global__ void k_sur_step_inc(int64_t* t) { t[0] += 1; }

// loss = scale * sum(part[0..n)) in float64, one workgroup.
__global__ __launch_bounds__(256) void k_sur_loss(const float* __restrict__ part, int n,
                                                  double scale, double* __restrict__ loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += (double)part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = scale * (((red[0] + red[1]) + red[2]) + red[3]);
}

// Per-feature column sums over row chunks: sum x (mean == null) or
// sum (x - mean)^2.  part[ch][c], float64.
__global__ __launch_bounds__(256) void k_col_stats(const float* __restrict__ X, int64_t ldx,
                                                   int64_t N, int64_t d, int64_t rows,
                                                   const double* __restrict__ mean,
                                                   double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ch = blockIdx.y;
  if (c >= d) return;
  const int64_t r0 = ch * rows, r1 = r0 + rows < N ? r0 + rows : N;
  double s = 0.0;
  if (mean) {
    const double mu = mean[c];
    for (int64_t r = r0; r < r1; ++r) {
      const double t = (double)X[r * ldx + c] - mu;
      s += t * t;
    }
  } else {
    for (int64_t r = r0; r < r1; ++r) s += (double)X[r * ldx + c];
  }
  part[ch * d + c] = s;
}

// mode 0: out[c] = sum / N (mean); mode 1: out[c] = 1/sqrt(sum / N), 1 if zero.
__global__ void k_col_finish(const double* __restrict__ part, int64_t nch, int64_t d, int64_t N,
                             int mode, double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= d) return;
  double s = 0.0;
  for (int64_t ch = 0; ch < nch; ++ch) s += part[ch * d + c];
  s /= (double)N;
  if (mode == 0)
    out[c] = s;
  else
    out[c] = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
}

__global__ void k_res_target(const float* __restrict__ Ps, int64_t lds,
                             const double* __restrict__ Pn, int64_t ldn, double scale, int64_t M,
                             int nout, double* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  double s = 0.0;
  for (int j = 0; j < nout; ++j) {
    const double t = (double)Ps[m + (int64_t)j * lds] - scale * Pn[m + (int64_t)j * ldn];
    s += t * t;
  }
  s = sqrt(s / nout);
  out[m] = s > 0.0 ? log10(s) : -307.6526555685888;  // log10 of the smallest normal double
}

// Fallback selection: per block of 1024 rows, count res > thr.
__global__ __launch_bounds__(1024) void k_fb_count(const float* __restrict__ res, int64_t M,
                                                   float thr, int32_t* __restrict__ cnt) {
  __shared__ int32_t wc[16];
  const int64_t m = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const bool f = m < M && res[m] > thr;
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < 16; ++w) s += wc[w];
    cnt[blockIdx.x] = s;
  }
}

// Exclusive prefix of the block counts (one workgroup, serial per thread
// chunk then across chunks); offs[nb] = total.
__global__ __launch_bounds__(256) void k_fb_scan(const int32_t* __restrict__ cnt, int64_t nb,
                                                 int64_t* __restrict__ offs) {
  __shared__ int64_t part[256];
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += cnt[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int64_t v = part[t];
      part[t] = acc;
      acc += v;
    }
    offs[nb] = acc;
  }
  __syncthreads();
  int64_t acc = part[threadIdx.x];
  for (int64_t b = b0; b < b1; ++b) {
    offs[b] = acc;
    acc += cnt[b];
  }
}

// Ascending list of the fallback rows.
__global__ __launch_bounds__(1024) void k_fb_list(const float* __restrict__ res, int64_t M,
                                                  float thr, const int64_t* __restrict__ offs,
                                                  int64_t* __restrict__ list) {
  __shared__ int32_t wc[16];
  const int64_t m = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const bool f = m < M && res[m] > thr;
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wc[w] = __popcll(bal);
  __syncthreads();
  if (f) {
    int64_t o = offs[blockIdx.x];
    for (int i = 0; i < w; ++i) o += wc[i];
    o += __popcll(bal & ((1ull << lane) - 1ull));
    list[o] = m;
  }
}

__global__ void k_gather_rows(const float* __restrict__ Y, int64_t ldy, int64_t d,
                              const int64_t* __restrict__ list, int64_t n,
                              float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * d) return;
  const int64_t i = e / d, c = e % d;
  out[e] = Y[list[i] * ldy + c];
}

__global__ void k_scatter_phi(const double* __restrict__ Pn, int64_t ldn,
                              const int64_t* __restrict__ list, int64_t n, int nout, double scale,
                              float* __restrict__ Phi, int64_t ldphi) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nout) return;
  const int64_t i = e % n, j = e / n;
  Phi[list[i] + j * ldphi] = (float)(scale * Pn[i + j * ldn]);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }
inline unsigned ntile(int64_t n) { return (unsigned)((n + TB - 1) / TB); }
constexpr size_t SMEM_KK = TileSmem<Cfg, true, true>::bytes;
constexpr size_t SMEM_KR = TileSmem<Cfg, true, false>::bytes;
constexpr size_t SMEM_RR = TileSmem<Cfg, false, false>::bytes;

inline int64_t dpad_of(const Lay& L) { return (int64_t)align_up((size_t)L.d, 32); }

struct TrainWs {
  __bf16 *Xh, *a1, *a2, *dY, *d2, *d1;
  float *Tb, *z1, *z2, *lpart, *part;
  int nlp;
};

size_t carve_train(WsCursor& c, TrainWs& w, const Lay& L, int64_t B, int S) {
  const int64_t dp = dpad_of(L);
  w.Xh = c.take<__bf16>((size_t)B * dp);
  w.Tb = c.take<float>((size_t)B * L.nout);
  w.z1 = c.take<float>((size_t)B * L.h);
  w.a1 = c.take<__bf16>((size_t)B * L.h);
  w.z2 = c.take<float>((size_t)B * L.h);
  w.a2 = c.take<__bf16>((size_t)B * L.h);
  w.dY = c.take<__bf16>((size_t)B * L.n3);
  w.d2 = c.take<__bf16>((size_t)B * L.h);
  w.d1 = c.take<__bf16>((size_t)B * L.h);
  w.nlp = (int)(ntile(B) * ntile(L.n3));
  w.lpart = c.take<float>((size_t)w.nlp);
  w.part = c.take<float>((size_t)S * L.total);
  return c.used;
}

struct InferWs {
  __bf16 *Xh, *a1, *a2;
};

size_t carve_infer(WsCursor& c, InferWs& w, const Lay& L, int64_t M) {
  const int64_t R = M < MAXB ? (M > 0 ? M : 1) : MAXB;
  w.Xh = c.take<__bf16>((size_t)R * dpad_of(L));
  w.a1 = c.take<__bf16>((size_t)R * L.h);
  w.a2 = c.take<__bf16>((size_t)R * L.h);
  return c.used;
}

int run_infer(const Lay& L, const float* params, const __bf16* wb, const float* Y, int64_t ldy,
              int64_t M, const double* mean, const double* rstd, float* Phi, int64_t ldphi,
              float* res, InferWs& w, int32_t* status, hipStream_t st) {
  const int64_t dp = dpad_of(L);
  for (int64_t r0 = 0; r0 < M; r0 += MAXB) {
    const int64_t R = M - r0 < MAXB ? M - r0 : MAXB;
    hipLaunchKernelGGL((k_sur_gather<float>), dim3((unsigned)R), dim3(256), 0, st, Y, ldy, M, L.d,
                       mean, rstd, (const int64_t*)nullptr, r0, w.Xh, (int)dp,
                       (const float*)nullptr, (int64_t)0, 0.0, 0, L.nout, (float*)nullptr, status);
    hipLaunchKernelGGL(k_sur_hidden, dim3(ntile(L.h), ntile(R)), dim3(256), SMEM_KK, st,
                       (const __bf16*)w.Xh, dp, R, L.d, wb + L.W1, params + L.b1, L.h,
                       (float*)nullptr, w.a1, (int64_t)L.h);
    hipLaunchKernelGGL(k_sur_hidden, dim3(ntile(L.h), ntile(R)), dim3(256), SMEM_KK, st,
                       (const __bf16*)w.a1, (int64_t)L.h, R, L.h, wb + L.W2, params + L.b2, L.h,
                       (float*)nullptr, w.a2, (int64_t)L.h);
    hipLaunchKernelGGL(k_sur_output, dim3(ntile(L.n3), ntile(R)), dim3(256), SMEM_KK, st,
                       (const __bf16*)w.a2, (int64_t)L.h, R, L.h, wb + L.W3, params + L.b3, L.n3,
                       L.nout, 2, (const float*)nullptr, 0.0f, (__bf16*)nullptr, (float*)nullptr,
                       Phi + r0, ldphi, res ? res + r0 : nullptr);
    RPC_LAUNCH_CHECK();
  }
  return RPC_OK;
}

}  // namespace

extern "C" {

int surrogate_layout(const sur_shape* shape, sur_layout* out) {
  Lay L;
  if (!out || !make_layout(shape, L)) return RPC_EINVAL;
  out->W1 = L.W1;
  out->b1 = L.b1;
  out->W2 = L.W2;
  out->b2 = L.b2;
  out->W3 = L.W3;
  out->b3 = L.b3;
  out->total = L.total;
  out->n3 = L.n3;
  return RPC_OK;
}

int surrogate_init_uniforms(const sur_shape* shape, int64_t* count) {
  Lay L;
  if (!count || !make_layout(shape, L)) return RPC_EINVAL;
  const int64_t d = L.d, h = L.h, no = L.nout;
  *count = h * d + h + h * h + h + no * h + no + h + 1;
  return RPC_OK;
}

int surrogate_init(const sur_shape* shape, const double* uniforms, int64_t n_uniforms,
                   float* params, float* adam_m, float* adam_v, uint16_t* wbf16,
                   rpc_stream_t stream) {
  Lay L;
  int64_t need = 0;
  if (!make_layout(shape, L) || !params || !adam_m || !adam_v || !wbf16) return RPC_EINVAL;
  surrogate_init_uniforms(shape, &need);
  if (uniforms && n_uniforms < need) return RPC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_sur_init, dim3(nblk(L.total)), dim3(256), 0, st, L, uniforms, params, adam_m,
                     adam_v, reinterpret_cast<__bf16*>(wbf16));
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

static int64_t stats_chunks(int64_t N) {
  const int64_t c = (N + 4095) / 4096;
  return c < 1 ? 1 : (c > 512 ? 512 : c);
}

int surrogate_standardize_workspace_size(int64_t N, int64_t d, size_t* bytes) {
  if (!bytes || N < 1 || d < 1) return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  c.take<double>((size_t)stats_chunks(N) * d);
  *bytes = c.used;
  return RPC_OK;
}

int surrogate_standardize(const float* X, int64_t N, int64_t d, int64_t ldx, double* mean,
                          double* rstd, void* workspace, size_t workspace_bytes,
                          rpc_stream_t stream) {
  if (!X || !mean || !rstd || N < 1 || d < 1 || ldx < d) return RPC_EINVAL;
  WsCursor c{(char*)workspace, 0, workspace_bytes, true};
  const int64_t nch = stats_chunks(N);
  double* part = c.take<double>((size_t)nch * d);
  if (!c.ok) return RPC_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const int64_t rows = (N + nch - 1) / nch;
  const dim3 g((unsigned)((d + 255) / 256), (unsigned)nch);
  hipLaunchKernelGGL(k_col_stats, g, dim3(256), 0, st, X, ldx, N, d, rows, (const double*)nullptr,
                     part);
  hipLaunchKernelGGL(k_col_finish, dim3(nblk(d)), dim3(256), 0, st, (const double*)part, nch, d, N,
                     0, mean);
  hipLaunchKernelGGL(k_col_stats, g, dim3(256), 0, st, X, ldx, N, d, rows, (const double*)mean,
                     part);
  hipLaunchKernelGGL(k_col_finish, dim3(nblk(d)), dim3(256), 0, st, (const double*)part, nch, d, N,
                     1, rstd);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

static int norm_splits(int32_t s) { return s == 0 ? 8 : s; }

int surrogate_train_workspace_size(const sur_shape* shape, int64_t batch, int32_t splits,
                                   size_t* bytes) {
  Lay L;
  const int S = norm_splits(splits);
  if (!bytes || !make_layout(shape, L) || batch < 1 || batch > MAXB || S < 1 || S > 64)
    return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  TrainWs w;
  *bytes = carve_train(c, w, L, batch, S);
  return RPC_OK;
}

static int train_step_impl(const sur_shape* shape, const sur_train_opts* o, const float* X,
                           int64_t ldx, int64_t N, const double* mean, const double* rstd,
                           const int64_t* idx, int64_t batch, const void* T, int32_t t_dtype,
                           int64_t ldt, double tscale, float* params, float* adam_m,
                           float* adam_v, uint16_t* wbf16, float* grad, double* loss,
                           void* workspace, size_t workspace_bytes, int32_t* dev_status,
                           rpc_stream_t stream, int64_t* tdev);

int surrogate_train_step(const sur_shape* shape, const sur_train_opts* o, const float* X,
                         int64_t ldx, int64_t N, const double* mean, const double* rstd,
                         const int64_t* idx, int64_t batch, const void* T, int32_t t_dtype,
                         int64_t ldt, double tscale, float* params, float* adam_m,
                         float* adam_v, uint16_t* wbf16, float* grad, double* loss,
                         void* workspace, size_t workspace_bytes, int32_t* dev_status,
                         rpc_stream_t stream) {
  return train_step_impl(shape, o, X, ldx, N, mean, rstd, idx, batch, T, t_dtype, ldt, tscale,
                         params, adam_m, adam_v, wbf16, grad, loss, workspace, workspace_bytes,
                         dev_status, stream, nullptr);
}

static int train_step_impl(const sur_shape* shape, const sur_train_opts* o, const float* X,
                           int64_t ldx, int64_t N, const double* mean, const double* rstd,
                           const int64_t* idx, int64_t batch, const void* T, int32_t t_dtype,
                           int64_t ldt, double tscale, float* params, float* adam_m,
                           float* adam_v, uint16_t* wbf16, float* grad, double* loss,
                           void* workspace, size_t workspace_bytes, int32_t* dev_status,
                           rpc_stream_t stream, int64_t* tdev) {
  Lay L;
  if (!o || !make_layout(shape, L)) return RPC_EINVAL;
  const int S = norm_splits(o->splits);
  if (!X || !mean || !rstd || !idx || !T || !params || !adam_m || !adam_v || !wbf16 || N < 1 ||
      ldx < L.d || batch < 1 || batch > MAXB || S < 1 || S > 64 || o->step < 1 ||
      (o->phase != 0 && o->phase != 1) || (t_dtype != RPC_F32 && t_dtype != RPC_F64) ||
      (o->phase == 0 && ldt < N) || !(o->lr >= 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
      !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps > 0.0) || !(o->weight_decay >= 0.0))
    return RPC_EINVAL;
  WsCursor c{(char*)workspace, 0, workspace_bytes, true};
  TrainWs w;
  carve_train(c, w, L, batch, S);
  if (!c.ok) return RPC_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  __bf16* wb = reinterpret_cast<__bf16*>(wbf16);
  const int64_t B = batch, dp = dpad_of(L), h = L.h;
  const int ph = o->phase;
  prof::begin(prof::SUR_TRAIN, st);
  if (t_dtype == RPC_F64)
    hipLaunchKernelGGL((k_sur_gather<double>), dim3((unsigned)B), dim3(256), 0, st, X, ldx, N, L.d,
                       mean, rstd, idx, (int64_t)0, w.Xh, (int)dp, (const double*)T, ldt, tscale,
                       ph, L.nout, w.Tb, dev_status);
  else
    hipLaunchKernelGGL((k_sur_gather<float>), dim3((unsigned)B), dim3(256), 0, st, X, ldx, N, L.d,
                       mean, rstd, idx, (int64_t)0, w.Xh, (int)dp, (const float*)T, ldt, tscale,
                       ph, L.nout, w.Tb, dev_status);
  hipLaunchKernelGGL(k_sur_hidden, dim3(ntile(h), ntile(B)), dim3(256), SMEM_KK, st,
                     (const __bf16*)w.Xh, dp, B, L.d, (const __bf16*)(wb + L.W1),
                     (const float*)(params + L.b1), L.h, w.z1, w.a1, h);
  hipLaunchKernelGGL(k_sur_hidden, dim3(ntile(h), ntile(B)), dim3(256), SMEM_KK, st,
                     (const __bf16*)w.a1, h, B, L.h, (const __bf16*)(wb + L.W2),
                     (const float*)(params + L.b2), L.h, w.z2, w.a2, h);
  const float gscale = ph == 0 ? (float)(1.0 / ((double)B * L.nout)) : (float)(1.0 / (double)B);
  hipLaunchKernelGGL(k_sur_output, dim3(ntile(L.n3), ntile(B)), dim3(256), SMEM_KK, st,
                     (const __bf16*)w.a2, h, B, L.h, (const __bf16*)(wb + L.W3),
                     (const float*)(params + L.b3), L.n3, L.nout, ph, (const float*)w.Tb, gscale,
                     w.dY, w.lpart, (float*)nullptr, (int64_t)0, (float*)nullptr);
  const int64_t mchunk = (B + S - 1) / S;
  hipLaunchKernelGGL(k_sur_wgrad, dim3(ntile(h), ntile(L.n3), (unsigned)S), dim3(256), SMEM_RR, st,
                     (const __bf16*)w.dY, (int64_t)L.n3, L.n3, (const __bf16*)w.a2, h, L.h, B,
                     mchunk, w.part, L.total, L.W3, L.b3);
  if (ph == 0) {
    hipLaunchKernelGGL(k_sur_dx, dim3(ntile(h), ntile(B)), dim3(256), SMEM_KR, st,
                       (const __bf16*)w.dY, (int64_t)L.n3, B, L.n3, (const __bf16*)(wb + L.W3),
                       L.h, (const float*)w.z2, w.d2, h);
    hipLaunchKernelGGL(k_sur_wgrad, dim3(ntile(h), ntile(h), (unsigned)S), dim3(256), SMEM_RR, st,
                       (const __bf16*)w.d2, h, L.h, (const __bf16*)w.a1, h, L.h, B, mchunk, w.part,
                       L.total, L.W2, L.b2);
    hipLaunchKernelGGL(k_sur_dx, dim3(ntile(h), ntile(B)), dim3(256), SMEM_KR, st,
                       (const __bf16*)w.d2, h, B, L.h, (const __bf16*)(wb + L.W2), L.h,
                       (const float*)w.z1, w.d1, h);
    hipLaunchKernelGGL(k_sur_wgrad, dim3(ntile(L.d), ntile(h), (unsigned)S), dim3(256), SMEM_RR, st,
                       (const __bf16*)w.d1, h, L.h, (const __bf16*)w.Xh, dp, L.d, B, mchunk,
                       w.part, L.total, L.W1, L.b1);
  }
  const double t = (double)o->step;
  const double c1 = 1.0 / (1.0 - pow(o->beta1, t)), c2 = 1.0 / (1.0 - pow(o->beta2, t));
  hipLaunchKernelGGL(k_sur_adamw, dim3(nblk(L.total)), dim3(256), 0, st, L, ph, S,
                     (const float*)w.part, params, adam_m, adam_v, wb, grad, o->lr, o->beta1,
                     o->beta2, o->eps, o->weight_decay, c1, c2, (const int64_t*)tdev);
  if (tdev) hipLaunchKernelGGL(k_sur_step_inc, dim3(1), dim3(1), 0, st, tdev);
  if (loss) {
    const double ls = ph == 0 ? 1.0 / ((double)B * L.nout) : 1.0 / (double)B;
    hipLaunchKernelGGL(k_sur_loss, dim3(1), dim3(256), 0, st, (const float*)w.lpart, w.nlp, ls,
                       loss);
  }
  RPC_LAUNCH_CHECK();
  prof::end(prof::SUR_TRAIN, st);
  return RPC_OK;
}

int surrogate_train_epoch(const sur_shape* shape, const sur_train_opts* o, const float* X,
                          int64_t ldx, int64_t N, const double* mean, const double* rstd,
                          const int64_t* idx, int64_t n_idx, int64_t batch, const void* T,
                          int32_t t_dtype, int64_t ldt, double tscale, float* params,
                          float* adam_m, float* adam_v, uint16_t* wbf16, double* loss,
                          void* workspace, size_t workspace_bytes, int32_t* dev_status,
                          rpc_stream_t stream) {
  if (!o || !idx || n_idx < 1 || batch < 1) return RPC_EINVAL;
  sur_train_opts so = *o;
  int64_t s = 0;
  for (int64_t b0 = 0; b0 < n_idx; b0 += batch, ++s) {
    const int64_t nb = n_idx - b0 < batch ? n_idx - b0 : batch;
    so.step = o->step + s;
    const int rc = surrogate_train_step(shape, &so, X, ldx, N, mean, rstd, idx + b0, nb, T, t_dtype,
                                        ldt, tscale, params, adam_m, adam_v, wbf16, nullptr,
                                        loss ? loss + s : nullptr, workspace, workspace_bytes,
                                        dev_status, stream);
    if (rc != RPC_OK) return rc;
  }
  return RPC_OK;
}

int surrogate_train_graph_create(const sur_shape* shape, const sur_train_opts* o, const float* X,
                                 int64_t ldx, int64_t N, const double* mean, const double* rstd,
                                 const int64_t* idx, int64_t n_idx, int64_t batch, const void* T,
                                 int32_t t_dtype, int64_t ldt, double tscale, float* params,
                                 float* adam_m, float* adam_v, uint16_t* wbf16, double* loss,
                                 int64_t* step_counter, void* workspace, size_t workspace_bytes,
                                 int32_t* dev_status, rpc_stream_t stream, rpc_graph* out) {
  if (!out || !stream || !o || !idx || !step_counter || n_idx < 1 || batch < 1 || prof::enabled())
    return RPC_EINVAL;
  *out = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  RPC_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  sur_train_opts so = *o;
  so.step = 1;  // checked only; the step number comes from step_counter
  int rc = RPC_OK;
  int64_t s = 0;
  for (int64_t b0 = 0; b0 < n_idx && rc == RPC_OK; b0 += batch, ++s) {
    const int64_t nb = n_idx - b0 < batch ? n_idx - b0 : batch;
    rc = train_step_impl(shape, &so, X, ldx, N, mean, rstd, idx + b0, nb, T, t_dtype, ldt, tscale,
                         params, adam_m, adam_v, wbf16, nullptr, loss ? loss + s : nullptr,
                         workspace, workspace_bytes, dev_status, stream, step_counter);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != RPC_OK || e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return rc != RPC_OK ? rc : RPC_EHIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return RPC_EHIP;
  }
  *out = new rpc_graph_s{g, x};
  return RPC_OK;
}

int surrogate_infer_workspace_size(const sur_shape* shape, int64_t M, size_t* bytes) {
  Lay L;
  if (!bytes || !make_layout(shape, L) || M < 0) return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  InferWs w;
  *bytes = carve_infer(c, w, L, M);
  return RPC_OK;
}

int surrogate_infer(const sur_shape* shape, const float* params, const uint16_t* wbf16,
                    const float* Y, int64_t ldy, int64_t M, const double* mean,
                    const double* rstd, float* Phi, int64_t ldphi, float* res, void* workspace,
                    size_t workspace_bytes, int32_t* dev_status, rpc_stream_t stream) {
  Lay L;
  if (!make_layout(shape, L) || !params || !wbf16 || !Y || !mean || !rstd || !Phi || M < 0 ||
      ldy < L.d || ldphi < M)
    return RPC_EINVAL;
  if (M == 0) return RPC_OK;
  WsCursor c{(char*)workspace, 0, workspace_bytes, true};
  InferWs w;
  carve_infer(c, w, L, M);
  if (!c.ok) return RPC_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  prof::begin(prof::SUR_INFER, st);
  const int rc = run_infer(L, params, reinterpret_cast<const __bf16*>(wbf16), Y, ldy, M, mean, rstd,
                           Phi, ldphi, res, w, dev_status, st);
  prof::end(prof::SUR_INFER, st);
  return rc;
}

int surrogate_residual_target(const float* Phi_s, int64_t lds, const double* Phi_n,
                              int64_t ldn, double scale, int64_t M, int32_t n_out, double* out,
                              rpc_stream_t stream) {
  if (!Phi_s || !Phi_n || !out || M < 0 || n_out < 1 || lds < M || ldn < M) return RPC_EINVAL;
  if (M == 0) return RPC_OK;
  hipLaunchKernelGGL(k_res_target, dim3(nblk(M)), dim3(256), 0, (hipStream_t)stream, Phi_s, lds,
                     Phi_n, ldn, scale, M, n_out, out);
  RPC_LAUNCH_CHECK();
  return RPC_OK;
}

struct ExtWs {
  InferWs inf;
  float* res;
  int32_t* cnt;
  int64_t* offs;
  int64_t* list;
  float* Yf;
  double* Pn;
  void* nws;
  size_t nws_bytes;
};

static int carve_ext(WsCursor& c, ExtWs& w, const Lay& L, int64_t M, int64_t d, int r, int nev) {
  carve_infer(c, w.inf, L, M);
  const int64_t Mx = M > 0 ? M : 1;
  const int64_t nb = (Mx + 1023) / 1024;
  const int64_t FC = Mx < FB_CHUNK ? Mx : FB_CHUNK;
  w.res = c.take<float>((size_t)Mx);
  w.cnt = c.take<int32_t>((size_t)nb);
  w.offs = c.take<int64_t>((size_t)nb + 1);
  w.list = c.take<int64_t>((size_t)Mx);
  w.Yf = c.take<float>((size_t)FC * d);
  w.Pn = c.take<double>((size_t)FC * nev);
  size_t nb_bytes = 0;
  const int rc = nystrom_extend_workspace_size(FC, d, r, nev, &nb_bytes);
  if (rc != RPC_OK) return rc;
  w.nws = c.take<char>(nb_bytes);
  w.nws_bytes = nb_bytes;
  return RPC_OK;
}

int surrogate_extend_workspace_size(const sur_shape* shape, int64_t M, int64_t d, int32_t r,
                                    int32_t nev, size_t* bytes) {
  Lay L;
  if (!bytes || !make_layout(shape, L) || M < 0 || d != L.d || r < 1 || nev < L.nout)
    return RPC_EINVAL;
  WsCursor c{nullptr, 0, 0, true};
  ExtWs w;
  const int rc = carve_ext(c, w, L, M, d, r, nev);
  if (rc != RPC_OK) return rc;
  *bytes = c.used;
  return RPC_OK;
}

int surrogate_extend(const sur_shape* shape, const float* params, const uint16_t* wbf16,
                     const double* mean, const double* rstd, double log10_threshold,
                     const rpc_points* Y, const rpc_points* X, const int64_t* pivots,
                     const int32_t* k, const void* F, int32_t f_dtype, int64_t ldf, int32_t r,
                     const double* c, const double* ext_E, int32_t nev, double scale,
                     float* Phi, int64_t ldphi, float* res, int64_t* n_fallback,
                     void* workspace, size_t workspace_bytes, int32_t* dev_status,
                     rpc_stream_t stream) {
  Lay L;
  if (!make_layout(shape, L) || !Y || !X || !Y->X || !n_fallback || !Phi || Y->d != L.d ||
      X->d != L.d || nev < L.nout || Y->N < 0 || ldphi < Y->N || Y->dtype != RPC_F32)
    return RPC_EINVAL;
  const float* Yx = static_cast<const float*>(Y->X);
  const int64_t M = Y->N;
  *n_fallback = 0;
  if (M == 0) return RPC_OK;
  WsCursor cur{(char*)workspace, 0, workspace_bytes, true};
  ExtWs w;
  int rc = carve_ext(cur, w, L, M, L.d, r, nev);
  if (rc != RPC_OK) return rc;
  if (!cur.ok) return RPC_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  float* rs = res ? res : w.res;
  rc = run_infer(L, params, reinterpret_cast<const __bf16*>(wbf16), Yx, Y->ldx, M, mean, rstd,
                 Phi, ldphi, rs, w.inf, dev_status, st);
  if (rc != RPC_OK) return rc;
  const int64_t nb = (M + 1023) / 1024;
  const float thr = (float)log10_threshold;
  hipLaunchKernelGGL(k_fb_count, dim3((unsigned)nb), dim3(1024), 0, st, (const float*)rs, M, thr,
                     w.cnt);
  hipLaunchKernelGGL(k_fb_scan, dim3(1), dim3(256), 0, st, (const int32_t*)w.cnt, nb, w.offs);
  hipLaunchKernelGGL(k_fb_list, dim3((unsigned)nb), dim3(1024), 0, st, (const float*)rs, M, thr,
                     (const int64_t*)w.offs, w.list);
  RPC_LAUNCH_CHECK();
  int64_t nf = 0;
  RPC_HIP_CHECK(hipMemcpyAsync(&nf, w.offs + nb, sizeof(nf), hipMemcpyDeviceToHost, st));
  RPC_HIP_CHECK(hipStreamSynchronize(st));
  *n_fallback = nf;
  for (int64_t f0 = 0; f0 < nf; f0 += FB_CHUNK) {
    const int64_t n = nf - f0 < FB_CHUNK ? nf - f0 : FB_CHUNK;
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n * L.d)), dim3(256), 0, st, Yx, Y->ldx,
                       (int64_t)L.d, (const int64_t*)(w.list + f0), n, w.Yf);
    RPC_LAUNCH_CHECK();
    rpc_points Yc{n, (int64_t)L.d, (int64_t)L.d, w.Yf, Y->eps, RPC_F32};
    rc = nystrom_extend(&Yc, X, pivots, k, F, f_dtype, ldf, r, c, ext_E, nev, w.Pn, n, w.nws,
                        w.nws_bytes, dev_status, stream);
    if (rc != RPC_OK) return rc;
    hipLaunchKernelGGL(k_scatter_phi, dim3(nblk(n * L.nout)), dim3(256), 0, st,
                       (const double*)w.Pn, n, (const int64_t*)(w.list + f0), n, L.nout, scale,
                       Phi, ldphi);
    RPC_LAUNCH_CHECK();
  }
  return RPC_OK;
}

}  // extern "C"
