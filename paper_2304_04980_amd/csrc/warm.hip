// Learned warm start: a convolutional network over the K x N grid maps each
// node's initial state and parameters (x0, A_ii, B_ii) to the coefficients
// of a Chebyshev-in-time expansion of its multipliers delta~; the expansion
// is the initial iterate of Algorithm 1 (which allows any delta^(0)).  The
// network is trained on solves of the method itself.  This file holds its
// forward, backward and optimiser kernels and their C entry points.
//
// Network.  `layers` 3 x 3 convolutions with zero padding, ReLU after all
// but the last; 64 channels throughout; the input has 32 channels (x0, A_ii
// row-major, B_ii row-major, zero padded); output channel 16 s + c is
// Chebyshev coefficient c of state component s (n = 4).  Weights are kept in
// FP32 (master copy, Adam moments) and used as BF16; every product runs on
// the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation); activations and back-propagated gradients are stored as
// BF16, the network output and the loss in FP32/FP64.
//
// Convolution as a matrix product.  For one layer, output (channel o,
// pixel p) = sum over taps (di, dj) and input channels c of
// W[o][tap][c] x[p + (di, dj)][c].  A workgroup of 4 wavefronts covers 64
// pixels of one sample; each wavefront holds 16 pixels x 64 output channels
// as four 16 x 16 MFMA accumulators (M = output channels, N = pixels), and
// steps K over (tap, 32-channel chunk): per step one 16-byte load of 8 input
// channels per lane (pixel-major, channels contiguous) and four 16-byte
// weight loads.  The input gradient is the same product with the weights
// transposed and the taps flipped, W'[c][8 - tap][o] = W[o][tap][c], and the
// ReLU mask applied in the epilogue.  The weight gradient
// dW[o][tap][c] = sum_p dy[p][o] x[p + tap][c] contracts over pixels: it
// reads channel-major copies of dy and x (8 consecutive pixels of one
// channel per lane), one wavefront per tap, and writes per-workgroup partial
// sums that a second kernel adds in a fixed order.
//
// Pixel order.  Pixel p = j K + i (column j, row i), the node order of the
// problem arrays, so features and outputs need no transposition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "api_common.h"

using namespace lqg;

namespace {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWidth = 64;   // channels of every layer output
constexpr int kCin0 = 32;    // padded input channels
constexpr int kCheb = 16;    // Chebyshev coefficients per state component
constexpr int kTaps = 9;
constexpr int kMaxLayers = 8;
constexpr int kDwChunk = 256;  // pixels per weight-gradient workgroup

__device__ __forceinline__ bf16x8 zero8() {
  return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
}

enum ConvMode { kFwdRelu = 0, kFwdLinear = 1, kBwdData = 2 };

struct ConvArgs {
  int K, N, P;
  const bf16* in;        // sample s at in + s * in_stride, [P][CIN]
  long long in_stride;
  const int* idx;        // sample of batch entry b (NULL: b)
  const bf16* w;         // [64][9][CIN]
  const float* bias;     // [64] (forward only)
  bf16* out_nhwc;        // [B][P][64]
  bf16* out_chw;         // [B][64][P]
  float* out_f32;        // [B][P][64] (linear layer)
  const bf16* mask;      // [B][P][64] input activation of the layer (backward)
};

template <int CIN, int MODE>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n16 = lane & 15, g = lane >> 4;
  const int pw = blockIdx.x * 64 + wv * 16 + n16;  // this lane's pixel
  const bool pin = pw < a.P;
  const int i = pw % a.K, j = pw / a.K;
  const long long smp = a.idx ? a.idx[b] : b;
  const bf16* in = a.in + smp * a.in_stride;
  f32x4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < kTaps; ++tap) {
    const int ii = i + tap / 3 - 1, jj = j + tap % 3 - 1;
    const bool valid = pin && ii >= 0 && ii < a.K && jj >= 0 && jj < a.N;
    const bf16* src = in + (long long)(jj * a.K + ii) * CIN + 8 * g;
#pragma unroll
    for (int c0 = 0; c0 < CIN; c0 += 32) {
      bf16x8 bv = zero8();
      if (valid) bv = *reinterpret_cast<const bf16x8*>(src + c0);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(
            a.w + ((16 * ct + n16) * kTaps + tap) * CIN + c0 + 8 * g);
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ct], 0, 0, 0);
      }
    }
  }
  if (!pin) return;
  const long long row = ((long long)b * a.P + pw) * kWidth;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int co0 = 16 * ct + 4 * g;  // this lane holds channels co0 .. co0 + 3
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = acc[ct][r];
    if (MODE == kFwdLinear) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] += a.bias[co0 + r];
      *reinterpret_cast<f32x4*>(a.out_f32 + row + co0) = f32x4{v[0], v[1], v[2], v[3]};
      continue;
    }
    if (MODE == kFwdRelu) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r] + a.bias[co0 + r], 0.f);
    } else {
      const bf16x4 mk = *reinterpret_cast<const bf16x4*>(a.mask + row + co0);
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = (float)mk[r] > 0.f ? v[r] : 0.f;
    }
    bf16x4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = (bf16)v[r];
    *reinterpret_cast<bf16x4*>(a.out_nhwc + row + co0) = o;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      a.out_chw[((long long)b * kWidth + co0 + r) * a.P + pw] = o[r];
  }
}

// Per-workgroup partial weight gradient of one layer: workgroup = (batch
// entry, chunk of kDwChunk pixels), wavefront = tap.
template <int CIN>
__global__ __launch_bounds__(576) void k_conv_dw(int K, int N, int P,
                                                 const bf16* __restrict__ dy_chw,
                                                 const bf16* __restrict__ x_base,
                                                 long long x_stride,
                                                 const int* __restrict__ idx,
                                                 float* __restrict__ part) {
  const int nchunk = P / kDwChunk;
  const int b = blockIdx.x / nchunk, ch = blockIdx.x % nchunk;
  const int tap = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n16 = lane & 15, g = lane >> 4;
  const int di = tap / 3 - 1, dj = tap % 3 - 1;
  const long long smp = idx ? idx[b] : b;
  const bf16* x = x_base + smp * x_stride;  // channel-major [CIN][P]
  const bf16* dy = dy_chw + (long long)b * kWidth * P;
  constexpr int NT = CIN / 16;
  f32x4 acc[4][NT];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int cs = 0; cs < NT; ++cs) acc[ct][cs] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int p0 = ch * kDwChunk; p0 < (ch + 1) * kDwChunk; p0 += 32) {
    const int pg = p0 + 8 * g;  // this lane's 8 pixels: rows i0..i0+7 of column j0
    const int i0 = pg % K, j0 = pg / K;
    const int jj = j0 + dj;
    const bool colv = jj >= 0 && jj < N;
    const int q0 = jj * K + i0;
    bf16x8 av[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      av[ct] = *reinterpret_cast<const bf16x8*>(dy + (long long)(16 * ct + n16) * P + pg);
#pragma unroll
    for (int cs = 0; cs < NT; ++cs) {
      const bf16* xr = x + (long long)(16 * cs + n16) * P;
      bf16x8 bv = zero8();
      if (colv) {
        if (di == 0) {
          bv = *reinterpret_cast<const bf16x8*>(xr + q0);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int ii = i0 + e + di;
            if (ii >= 0 && ii < K) bv[e] = xr[q0 + e + di];
          }
        }
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        acc[ct][cs] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[ct], bv, acc[ct][cs], 0, 0, 0);
    }
  }
  float* out = part + (long long)blockIdx.x * kWidth * kTaps * CIN;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int cs = 0; cs < NT; ++cs)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[((16 * ct + 4 * g + r) * kTaps + tap) * CIN + 16 * cs + n16] = acc[ct][cs][r];
}

// grad[e] = sum over the nwg partials (fixed order).
__global__ void k_dw_reduce(const float* __restrict__ part, int nwg, int count,
                            float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.f;
  for (int w = 0; w < nwg; ++w) s += part[(long long)w * count + e];
  grad[e] = s;
}

// Bias gradient: db[o] = sum over batch and pixels of dy[o][p]; one
// workgroup per channel.
__global__ __launch_bounds__(256) void k_db(const bf16* __restrict__ dy_chw,
                                            int B, int P, float* __restrict__ db) {
  const int o = blockIdx.x;
  double s = 0.0;
  for (int b = 0; b < B; ++b) {
    const bf16* r = dy_chw + ((long long)b * kWidth + o) * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) s += (double)(float)r[p];
  }
  s = block_sum<256>(s);
  if (threadIdx.x == 0) db[o] = (float)s;
}

// Chebyshev values T_c(tau_t), tau_t = 2 t / T - 1, c < kCheb, by the
// three-term recurrence.
__device__ __forceinline__ void cheb_at(int t, int T, double (&v)[kCheb]) {
  const double tau = 2.0 * t / T - 1.0;
  v[0] = 1.0;
  v[1] = tau;
#pragma unroll
  for (int c = 2; c < kCheb; ++c) v[c] = 2.0 * tau * v[c - 1] - v[c - 2];
}

// Gram matrix G[c][d] = sum_t T_c(tau_t) T_d(tau_t) of the expansion basis.
__global__ __launch_bounds__(256) void k_gram(int T, float* __restrict__ gram) {
  const int c = threadIdx.x / kCheb, d = threadIdx.x % kCheb;
  double s = 0.0;
  for (int t = 0; t <= T; ++t) {
    double v[kCheb];
    cheb_at(t, T, v);
    s += v[c] * v[d];
  }
  gram[threadIdx.x] = (float)s;
}

// Loss of the expansion against the target trajectory, through the
// projections tgt[p][16 s + c] = sum_t T_c(tau_t) delta*_t[p][s]:
//   sum_t (sum_c a_c T_c - delta*_t)^2 = a'Ga - 2 a'tgt + |delta*|^2.
// One thread per (batch entry, pixel, state component): writes the
// gradient 2 (G a - tgt) / (|delta*|^2 B) as BF16 in both layouts and its
// share of sum (a'Ga - 2 a'tgt) / |delta*|^2.
__global__ __launch_bounds__(256) void k_loss(int P, int B, const float* __restrict__ out,
                                              const float* __restrict__ tgt_base,
                                              long long tgt_stride,
                                              const int* __restrict__ idx,
                                              const float* __restrict__ gram,
                                              bf16* __restrict__ dy_nhwc,
                                              bf16* __restrict__ dy_chw,
                                              double* __restrict__ part) {
  __shared__ float G[kCheb * kCheb];
  G[threadIdx.x] = gram[threadIdx.x];
  __syncthreads();
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lp = 0.0;
  if (gid < (long long)B * P * 4) {
    const int s4 = (int)(gid & 3);
    const long long bp = gid >> 2;
    const int b = (int)(bp / P), p = (int)(bp % P);
    const long long smp = idx ? idx[b] : b;
    const float* tg = tgt_base + smp * tgt_stride;
    const float dd = tg[(long long)P * kWidth];
    const float* av = out + bp * kWidth + s4 * kCheb;
    const float* tv = tg + (long long)p * kWidth + s4 * kCheb;
    float a[kCheb], t[kCheb];
#pragma unroll
    for (int c = 0; c < kCheb; ++c) {
      a[c] = av[c];
      t[c] = tv[c];
    }
    const float sc = 2.0f / (dd * (float)B);
    double q = 0.0;
#pragma unroll
    for (int c = 0; c < kCheb; ++c) {
      float ga = 0.f;
#pragma unroll
      for (int d = 0; d < kCheb; ++d) ga = fmaf(G[c * kCheb + d], a[d], ga);
      q += (double)a[c] * ((double)ga - 2.0 * (double)t[c]);
      const bf16 gv = (bf16)(sc * (ga - t[c]));
      dy_nhwc[bp * kWidth + s4 * kCheb + c] = gv;
      dy_chw[((long long)b * kWidth + s4 * kCheb + c) * P + p] = gv;
    }
    lp = q / (double)dd;
  }
  lp = block_sum<256>(lp);
  if (threadIdx.x == 0) part[blockIdx.x] = lp;
}

// A given output gradient dout (FP32 [B][P][64]) rounded to BF16 (nearest
// even) into both layouts of the first gradient buffer.
__global__ __launch_bounds__(256) void k_dout_bf16(int P, int B, const float* __restrict__ dout,
                                                   bf16* __restrict__ dy_nhwc,
                                                   bf16* __restrict__ dy_chw) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)B * P * kWidth) return;
  const int ch = (int)(g % kWidth);
  const long long bp = g / kWidth;
  const int b = (int)(bp / P), p = (int)(bp % P);
  const bf16 v = (bf16)dout[g];
  dy_nhwc[g] = v;
  dy_chw[((long long)b * kWidth + ch) * P + p] = v;
}

// out[0] = sum of n partials (fixed order).
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ part, int n,
                                             double* __restrict__ out) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += part[k];
  s = block_sum<256>(s);
  if (threadIdx.x == 0) out[0] = s;
}

// Projections of a solved trajectory delta* ([T+1][N][K][n], FP64) onto the
// Chebyshev basis: tgt[p][16 s + c] (FP32), and per-workgroup partial sums of
// |delta*|^2.  One thread per (pixel, state component).
__global__ __launch_bounds__(256) void k_targets(int P, int T, int n,
                                                 const double* __restrict__ delta,
                                                 float* __restrict__ tgt,
                                                 double* __restrict__ part) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  double dd = 0.0;
  if (gid < P * n) {
    const int p = gid / n, s = gid % n;
    double acc[kCheb];
#pragma unroll
    for (int c = 0; c < kCheb; ++c) acc[c] = 0.0;
    for (int t = 0; t <= T; ++t) {
      const double v = delta[((long long)t * P + p) * n + s];
      double tc[kCheb];
      cheb_at(t, T, tc);
#pragma unroll
      for (int c = 0; c < kCheb; ++c) acc[c] = fma(tc[c], v, acc[c]);
      dd = fma(v, v, dd);
    }
#pragma unroll
    for (int c = 0; c < kCheb; ++c) tgt[(long long)p * kWidth + s * kCheb + c] = (float)acc[c];
  }
  dd = block_sum<256>(dd);
  if (threadIdx.x == 0) part[blockIdx.x] = dd;
}
__global__ __launch_bounds__(256) void k_targets_dd(const double* __restrict__ part,
                                                    int n, float* __restrict__ dd) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += part[k];
  s = block_sum<256>(s);
  if (threadIdx.x == 0) dd[0] = (float)s;
}

// delta^(0)[t][p][s] = sum_c out[p][16 s + c] T_c(tau_t) (FP64, interface
// layout [T+1][N][K][n] = [T+1][P][n]).
__global__ __launch_bounds__(256) void k_expand(int P, int T, int n,
                                                const float* __restrict__ out,
                                                double* __restrict__ delta) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)(T + 1) * P * n) return;
  const int t = (int)(gid / ((long long)P * n));
  const int ps = (int)(gid - (long long)t * P * n);
  const int p = ps / n, s = ps % n;
  double tc[kCheb];
  cheb_at(t, T, tc);
  double v = 0.0;
#pragma unroll
  for (int c = 0; c < kCheb; ++c)
    v = fma((double)out[(long long)p * kWidth + s * kCheb + c], tc[c], v);
  delta[gid] = v;
}

// Input features of one problem, pixel p = j K + i: channels x0 (n), A_ii
// (n^2), B_ii (n m), zeros; written pixel-major [P][32] and channel-major
// [32][P].
__global__ void k_features(int P, int n, int m, const double* __restrict__ A,
                           const double* __restrict__ Bm, const double* __restrict__ x0,
                           bf16* __restrict__ feat) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float f[kCin0];
#pragma unroll
  for (int c = 0; c < kCin0; ++c) f[c] = 0.f;
  for (int c = 0; c < n; ++c) f[c] = (float)x0[(long long)p * n + c];
  for (int c = 0; c < n * n; ++c) f[n + c] = (float)A[(long long)p * n * n + c];
  for (int c = 0; c < n * m; ++c) f[n + n * n + c] = (float)Bm[(long long)p * n * m + c];
  bf16* row = feat + (long long)p * kCin0;
  bf16* col = feat + (long long)P * kCin0;
#pragma unroll
  for (int c = 0; c < kCin0; ++c) {
    const bf16 v = (bf16)f[c];
    row[c] = v;
    col[(long long)c * P + p] = v;
  }
}

// BF16 copies of one layer's weights: wq[o][tap][c] and, for the input
// gradient, wt[c][8 - tap][o].
__global__ void k_prep_w(int cin, const float* __restrict__ W, bf16* __restrict__ wq,
                         bf16* __restrict__ wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kWidth * kTaps * cin) return;
  const int o = e / (kTaps * cin), tap = (e / cin) % kTaps, c = e % cin;
  const bf16 v = (bf16)W[e];
  wq[e] = v;
  if (wt) wt[((long long)c * kTaps + (kTaps - 1 - tap)) * kWidth + o] = v;
}

// Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(long long count, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float c1,
                       float c2) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  constexpr float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gv = g[e];
  const float mv = b1 * m[e] + (1.f - b1) * gv;
  const float vv = b2 * v[e] + (1.f - b2) * gv * gv;
  m[e] = mv;
  v[e] = vv;
  w[e] -= lr * (mv / c1) / (sqrtf(vv / c2) + eps);
}

// ---------------------------------------------------------------- host side
struct NetShape {
  int K, N, n, m, T, L, P;
  int cin[kMaxLayers];
  size_t woff[kMaxLayers], boff[kMaxLayers], count;
};

bool make_shape(const lqgrid_wsnet_desc* d, NetShape* s) {
  if (!d || d->K < 1 || d->N < 1 || d->T < 1 || d->layers < 2 || d->layers > kMaxLayers)
    return false;
  if (d->n * kCheb != kWidth) return false;                 // output channels
  if (d->n + d->n * d->n + d->n * d->m > kCin0 || d->m < 1) return false;
  if (d->K % 8 != 0 || ((long long)d->K * d->N) % kDwChunk != 0) return false;
  s->K = d->K;
  s->N = d->N;
  s->n = d->n;
  s->m = d->m;
  s->T = d->T;
  s->L = d->layers;
  s->P = d->K * d->N;
  size_t off = 0;
  for (int l = 0; l < s->L; ++l) {
    s->cin[l] = l == 0 ? kCin0 : kWidth;
    s->woff[l] = off;
    off += (size_t)kWidth * kTaps * s->cin[l];
    s->boff[l] = off;
    off += kWidth;
  }
  s->count = off;
  return true;
}

size_t feat_elems(const NetShape& s) { return (size_t)2 * s.P * kCin0; }          // bf16
size_t tgt_elems(const NetShape& s) { return (size_t)s.P * kWidth + 16; }          // fp32

struct WsLayout {
  size_t wq[kMaxLayers], wt[kMaxLayers];
  size_t act_nhwc[kMaxLayers], act_chw[kMaxLayers];
  size_t out, dy_nhwc[2], dy_chw[2], part, loss_part, scal, gram, total;
  int nwg, nloss;
};

WsLayout make_ws(const NetShape& s, int B) {
  WsLayout w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t act = (size_t)B * s.P * kWidth;
  for (int l = 0; l < s.L; ++l) {
    w.wq[l] = take((size_t)kWidth * kTaps * s.cin[l] * 2);
    w.wt[l] = take((size_t)kWidth * kTaps * s.cin[l] * 2);
  }
  for (int l = 0; l + 1 < s.L; ++l) {
    w.act_nhwc[l] = take(act * 2);
    w.act_chw[l] = take(act * 2);
  }
  w.out = take(act * 4);
  for (int k = 0; k < 2; ++k) {
    w.dy_nhwc[k] = take(act * 2);
    w.dy_chw[k] = take(act * 2);
  }
  w.nwg = B * (s.P / kDwChunk);
  w.part = take((size_t)w.nwg * kWidth * kTaps * kWidth * 4);
  w.nloss = (int)(((long long)B * s.P * 4 + 255) / 256);
  w.loss_part = take((size_t)std::max(w.nloss, (s.P * s.n + 255) / 256) * 8);
  w.scal = take(64);
  w.gram = take(kCheb * kCheb * 4);
  w.total = off;
  return w;
}

struct Net {
  NetShape s;
  WsLayout w;
  char* ws;
  hipStream_t st;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

int check_ws(const Net& net, size_t ws_bytes) {
  if (!net.ws || (reinterpret_cast<uintptr_t>(net.ws) % kAlign) != 0 ||
      ws_bytes < net.w.total)
    return LQGRID_EWORKSPACE;
  return LQGRID_OK;
}

void prep_weights(const Net& net, const float* params) {
  for (int l = 0; l < net.s.L; ++l) {
    const int cnt = kWidth * kTaps * net.s.cin[l];
    hipLaunchKernelGGL(k_prep_w, dim3((cnt + 255) / 256), dim3(256), 0, net.st,
                       net.s.cin[l], params + net.s.woff[l], net.at<bf16>(net.w.wq[l]),
                       l > 0 ? net.at<bf16>(net.w.wt[l]) : nullptr);
  }
}

void launch_conv(const Net& net, int B, int cin, int mode, const ConvArgs& a) {
  const dim3 g((net.s.P + 63) / 64, B);
  if (cin == kCin0) {
    if (mode == kFwdRelu) hipLaunchKernelGGL((k_conv<kCin0, kFwdRelu>), g, dim3(256), 0, net.st, a);
    else hipLaunchKernelGGL((k_conv<kCin0, kFwdLinear>), g, dim3(256), 0, net.st, a);
  } else {
    if (mode == kFwdRelu) hipLaunchKernelGGL((k_conv<kWidth, kFwdRelu>), g, dim3(256), 0, net.st, a);
    else if (mode == kFwdLinear) hipLaunchKernelGGL((k_conv<kWidth, kFwdLinear>), g, dim3(256), 0, net.st, a);
    else hipLaunchKernelGGL((k_conv<kWidth, kBwdData>), g, dim3(256), 0, net.st, a);
  }
}

// Forward pass of B samples (features of sample idx[b]); the output lands in
// the workspace's FP32 buffer.
void backward_layers(Net& net, int batch, const bf16* fb, const int* index, float* grad);

void forward(const Net& net, int B, const bf16* feats, const int* idx,
             const float* params) {
  prep_weights(net, params);
  const NetShape& s = net.s;
  for (int l = 0; l < s.L; ++l) {
    ConvArgs a{};
    a.K = s.K;
    a.N = s.N;
    a.P = s.P;
    if (l == 0) {
      a.in = feats;
      a.in_stride = (long long)feat_elems(s);
      a.idx = idx;
    } else {
      a.in = net.at<bf16>(net.w.act_nhwc[l - 1]);
      a.in_stride = (long long)s.P * kWidth;
      a.idx = nullptr;
    }
    a.w = net.at<bf16>(net.w.wq[l]);
    a.bias = params + s.boff[l];
    const bool last = l == s.L - 1;
    if (last) {
      a.out_f32 = net.at<float>(net.w.out);
    } else {
      a.out_nhwc = net.at<bf16>(net.w.act_nhwc[l]);
      a.out_chw = net.at<bf16>(net.w.act_chw[l]);
    }
    launch_conv(net, B, s.cin[l], last ? kFwdLinear : kFwdRelu, a);
  }
}

}  // namespace

extern "C" {

size_t lqgrid_wsnet_param_count(const lqgrid_wsnet_desc* d) {
  NetShape s;
  return make_shape(d, &s) ? s.count : 0;
}

size_t lqgrid_wsnet_sample_bytes(const lqgrid_wsnet_desc* d, int which) {
  NetShape s;
  if (!make_shape(d, &s)) return 0;
  return which == 0 ? feat_elems(s) * 2 : tgt_elems(s) * 4;
}

size_t lqgrid_wsnet_workspace_bytes(const lqgrid_wsnet_desc* d, int batch) {
  NetShape s;
  if (!make_shape(d, &s) || batch < 1) return 0;
  return make_ws(s, batch).total;
}

int lqgrid_wsnet_features(const lqgrid_wsnet_desc* d, const lqgrid_problem_desc* prob,
                          const double* x0, void* feat, void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || !prob || !x0 || !feat || !prob->A || !prob->B)
    return LQGRID_EINVAL;
  if (prob->K != s.K || prob->N != s.N || prob->n != s.n || prob->m != s.m)
    return LQGRID_EINVAL;
  if (prob->time_varying || prob->n_node || prob->m_node) return LQGRID_EUNSUPPORTED;
  clear_stale_error();
  hipLaunchKernelGGL(k_features, dim3((s.P + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), s.P, s.n, s.m, prob->A,
                     prob->B, x0, static_cast<bf16*>(feat));
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

int lqgrid_wsnet_targets(const lqgrid_wsnet_desc* d, const double* delta, float* target,
                         void* workspace, size_t ws_bytes, void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || !delta || !target) return LQGRID_EINVAL;
  Net net{s, make_ws(s, 1), static_cast<char*>(workspace),
          reinterpret_cast<hipStream_t>(stream)};
  int st = check_ws(net, ws_bytes);
  if (st != LQGRID_OK) return st;
  clear_stale_error();
  const int nb = (s.P * s.n + 255) / 256;
  double* part = net.at<double>(net.w.loss_part);
  hipLaunchKernelGGL(k_targets, dim3(nb), dim3(256), 0, net.st, s.P, s.T, s.n, delta,
                     target, part);
  hipLaunchKernelGGL(k_targets_dd, dim3(1), dim3(256), 0, net.st, part, nb,
                     target + (size_t)s.P * kWidth);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

int lqgrid_wsnet_forward(const lqgrid_wsnet_desc* d, int batch, const void* feats,
                         const int* index, const float* params, float* out,
                         void* workspace, size_t ws_bytes, void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || batch < 1 || !feats || !params || !out) return LQGRID_EINVAL;
  Net net{s, make_ws(s, batch), static_cast<char*>(workspace),
          reinterpret_cast<hipStream_t>(stream)};
  int st = check_ws(net, ws_bytes);
  if (st != LQGRID_OK) return st;
  clear_stale_error();
  forward(net, batch, static_cast<const bf16*>(feats), index, params);
  HIPCHECK(hipMemcpyAsync(out, net.at<float>(net.w.out),
                          (size_t)batch * s.P * kWidth * 4, hipMemcpyDeviceToDevice,
                          net.st));
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

int lqgrid_wsnet_gradient(const lqgrid_wsnet_desc* d, int batch, const void* feats,
                          const float* targets, const int* index, const float* params,
                          float* grad, double* loss, void* workspace, size_t ws_bytes,
                          void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || batch < 1 || !feats || !targets || !params || !grad)
    return LQGRID_EINVAL;
  Net net{s, make_ws(s, batch), static_cast<char*>(workspace),
          reinterpret_cast<hipStream_t>(stream)};
  int st = check_ws(net, ws_bytes);
  if (st != LQGRID_OK) return st;
  clear_stale_error();
  const bf16* fb = static_cast<const bf16*>(feats);
  forward(net, batch, fb, index, params);
  // loss and its gradient w.r.t. the output (slot 0)
  float* gram = net.at<float>(net.w.gram);
  hipLaunchKernelGGL(k_gram, dim3(1), dim3(256), 0, net.st, s.T, gram);
  double* lpart = net.at<double>(net.w.loss_part);
  hipLaunchKernelGGL(k_loss, dim3(net.w.nloss), dim3(256), 0, net.st, s.P, batch,
                     net.at<float>(net.w.out), targets, (long long)tgt_elems(s), index,
                     gram, net.at<bf16>(net.w.dy_nhwc[0]), net.at<bf16>(net.w.dy_chw[0]),
                     lpart);
  double* lsum = net.at<double>(net.w.scal);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, net.st, lpart, net.w.nloss, lsum);
  backward_layers(net, batch, fb, index, grad);
  HIPCHECK(hipGetLastError());
  if (loss) {
    double h = 0.0;
    HIPCHECK(hipMemcpyAsync(&h, lsum, sizeof(double), hipMemcpyDeviceToHost, net.st));
    HIPCHECK(hipStreamSynchronize(net.st));
    *loss = h / batch + 1.0;  // + |delta*|^2 / |delta*|^2 per sample
  }
  return LQGRID_OK;
}

int lqgrid_wsnet_backward(const lqgrid_wsnet_desc* d, int batch, const void* feats,
                          const int* index, const float* params, const float* dout,
                          float* grad, void* workspace, size_t ws_bytes, void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || batch < 1 || !feats || !params || !dout || !grad)
    return LQGRID_EINVAL;
  Net net{s, make_ws(s, batch), static_cast<char*>(workspace),
          reinterpret_cast<hipStream_t>(stream)};
  int st = check_ws(net, ws_bytes);
  if (st != LQGRID_OK) return st;
  clear_stale_error();
  const bf16* fb = static_cast<const bf16*>(feats);
  forward(net, batch, fb, index, params);
  const long long cnt = (long long)batch * s.P * kWidth;
  hipLaunchKernelGGL(k_dout_bf16, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, net.st,
                     s.P, batch, dout, net.at<bf16>(net.w.dy_nhwc[0]),
                     net.at<bf16>(net.w.dy_chw[0]));
  backward_layers(net, batch, fb, index, grad);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

}  // extern "C"

namespace {

// Gradients of every layer's weights and biases from the output gradient in
// slot 0 of the gradient buffers (BF16, both layouts), into grad.
void backward_layers(Net& net, int batch, const bf16* fb, const int* index, float* grad) {
  const NetShape& s = net.s;
  int cur = 0;
  for (int l = s.L - 1; l >= 0; --l) {
    const int cin = s.cin[l];
    const bf16* xin;
    long long xstride;
    const int* xidx;
    if (l == 0) {
      xin = fb + (size_t)s.P * kCin0;  // channel-major half of each feature sample
      xstride = (long long)feat_elems(s);
      xidx = index;
    } else {
      xin = net.at<bf16>(net.w.act_chw[l - 1]);
      xstride = (long long)s.P * kWidth;
      xidx = nullptr;
    }
    const bf16* dyc = net.at<bf16>(net.w.dy_chw[cur]);
    float* part = net.at<float>(net.w.part);
    if (cin == kCin0)
      hipLaunchKernelGGL(k_conv_dw<kCin0>, dim3(net.w.nwg), dim3(576), 0, net.st, s.K, s.N,
                         s.P, dyc, xin, xstride, xidx, part);
    else
      hipLaunchKernelGGL(k_conv_dw<kWidth>, dim3(net.w.nwg), dim3(576), 0, net.st, s.K, s.N,
                         s.P, dyc, xin, xstride, xidx, part);
    const int cnt = kWidth * kTaps * cin;
    hipLaunchKernelGGL(k_dw_reduce, dim3((cnt + 255) / 256), dim3(256), 0, net.st, part,
                       net.w.nwg, cnt, grad + s.woff[l]);
    hipLaunchKernelGGL(k_db, dim3(kWidth), dim3(256), 0, net.st, dyc, batch, s.P,
                       grad + s.boff[l]);
    if (l > 0) {
      ConvArgs a{};
      a.K = s.K;
      a.N = s.N;
      a.P = s.P;
      a.in = net.at<bf16>(net.w.dy_nhwc[cur]);
      a.in_stride = (long long)s.P * kWidth;
      a.w = net.at<bf16>(net.w.wt[l]);
      a.out_nhwc = net.at<bf16>(net.w.dy_nhwc[1 - cur]);
      a.out_chw = net.at<bf16>(net.w.dy_chw[1 - cur]);
      a.mask = net.at<bf16>(net.w.act_nhwc[l - 1]);
      launch_conv(net, batch, kWidth, kBwdData, a);
      cur = 1 - cur;
    }
  }
}

}  // namespace

extern "C" {

int lqgrid_wsnet_adam(const lqgrid_wsnet_desc* d, float* params, const float* grad,
                      float* moments, int step, float lr, void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || !params || !grad || !moments || step < 1 || !(lr >= 0.f))
    return LQGRID_EINVAL;
  clear_stale_error();
  const float c1 = 1.f - std::pow(0.9f, (float)step);
  const float c2 = 1.f - std::pow(0.999f, (float)step);
  const long long cnt = (long long)s.count;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), cnt, params, grad, moments,
                     moments + cnt, lr, c1, c2);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

int lqgrid_wsnet_predict(const lqgrid_wsnet_desc* d, const void* feat, const float* params,
                         double* delta_init, void* workspace, size_t ws_bytes,
                         void* stream) {
  NetShape s;
  if (!make_shape(d, &s) || !feat || !params || !delta_init) return LQGRID_EINVAL;
  Net net{s, make_ws(s, 1), static_cast<char*>(workspace),
          reinterpret_cast<hipStream_t>(stream)};
  int st = check_ws(net, ws_bytes);
  if (st != LQGRID_OK) return st;
  clear_stale_error();
  forward(net, 1, static_cast<const bf16*>(feat), nullptr, params);
  const long long tot = (long long)(s.T + 1) * s.P * s.n;
  hipLaunchKernelGGL(k_expand, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, net.st,
                     s.P, s.T, s.n, net.at<float>(net.w.out), delta_init);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

}  // extern "C"
