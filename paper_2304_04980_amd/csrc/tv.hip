// Time-varying data (Sec. II: A_{i,j,t}, B_{i,j,t}, E..H_{i,j,t}, Q_{i,j,t},
// R_{i,j,t}).  Every block of the operators carries its time index:
//
//   Psi_hat_t = Q_t^-1 + [A_hat Q^-1 A_hat' + B R^-1 B']_{t-1}  (t >= 1),
//   Psi_hat_0 = Q_0^-1,  Delta_{t+1,t} = -A_hat_t Q_t^-1,
//   Xi~ = Psi~ - Delta,  Omega~ = Phi~ - Psi~,
//   one Phi_bar_{v,t} per super-column v and time t (eq. "decomposed_problem")
//
// so no coefficient is shared by the lanes of a wavefront: each lane (time
// step) reads its own.  Layouts put t fastest (leading dimension ldt), so a
// wavefront's coefficient reads are coalesced like its vector reads:
//
//   TG13 [p][13][n*n][ldt]  13-point blocks of [A_hat Q^-1 A_hat' + B R^-1 B']_{t-1}
//                           at t >= 1 (zero at t = 0)
//   TQi  [p][n*n][ldt]      Q_t^-1 (Q_T^-1 at t = T)
//   TCdn [p][5][n*n][ldt]   A_hat_t[p,q] Q_{t,q}^-1       (t < T)
//   TCup [p][5][n*n][ldt]   Q_{t,p}^-1 A_hat_t[q,p]'      (t < T)
//   TAT5 [p][5][n*n][ldt]   A_hat_t[q,p]'                 (recovery)
//   TRiBT[p][m*n][ldt]      R_t^-1 B_t'                   (recovery)
//   TA5  [p][5][n*n][ldt]   A_hat_t[p,q]                  (t < T; factored Delta)
//   TBRB [p][n*n][ldt]      B_{t-1} R_{t-1}^-1 B_{t-1}'   (t >= 1; factored Delta)
//   TFw  [v][row][32][ldt][8], TBw [v][row][16][ldt][8]: the one-chain
//        factor products of every Phi_bar_{v,t} (see bodies_setup.h fw_at),
//        row r of the eight rows of a block row (2n <= 8) fastest.
//
// The operator kernels run one thread per (node, t); they are bound by the
// coefficient reads.  Delta is applied in the factored form of Sec. II-B,
// Delta = A~ Q~^-1 A~' + B~ R~^-1 B~', in two passes (12 n^2 coefficients
// per node and step instead of the 24 n^2 of the 13-point form); the
// 13-point blocks serve the Omega~ right-hand side and the factorisation.  The block
// solve runs eight threads per (v, t) system, one per row of a 2n-row block
// row, exchanging the block row's values by cross-lane reads.
#include "bodies_setup.h"
#include "tv.h"

namespace lqg {
namespace {
using namespace dev;

__device__ __forceinline__ bool cross_pair(int j, int jq) { return (j >> 1) != (jq >> 1); }

// rho = r + Xi~ x (MODE 1) or tau = r + Omega~ x (MODE 2); r nullable.
//   Xi~ = Psi~ - Delta: the time couplings of Delta with the sign flipped,
//   Omega~ = Phi~ - Psi~: the 13-point blocks between different super-columns
//   with the sign flipped.
template <typename T, int NS, int MODE>
__global__ __launch_bounds__(256) void k_tv_stencil(Dims D, TvCoef<T> C,
                                                    const T* __restrict__ x,
                                                    const T* __restrict__ r,
                                                    T* __restrict__ y, const Scalars* sc,
                                                    int check) {
  static_assert(MODE == 1 || MODE == 2, "right-hand sides only");
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ldt = D.ldt, K = D.K;
  const int t = (int)(g % ldt), p = (int)(g / ldt);
  constexpr int nn = NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = p / K, i = p - j * K;
  T acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = r ? r[((size_t)p * NS + a) * ldt + t] : T(0);
  auto term = [&](const T* blk, int q, int tq) {
    T xv[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) xv[b] = x[((size_t)q * NS + b) * ldt + tq];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
      for (int b = 0; b < NS; ++b)
        acc[a] = fma(MODE == 2 ? -blk[(size_t)(a * NS + b) * ldt] : blk[(size_t)(a * NS + b) * ldt],
                     xv[b], acc[a]);
  };
  if (MODE == 2) {
    for (int k = 0; k < 13; ++k) {
      const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= D.N || !cross_pair(j, jq)) continue;
      term(C.G13 + ((size_t)p * 13 + k) * nn * ldt + t, jq * K + iq, t);
    }
  } else {
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= D.N) continue;
      const int q = jq * K + iq;
      if (t >= 1) term(C.Cdn + ((size_t)p * 5 + k) * nn * ldt + (t - 1), q, t - 1);
      if (t < D.T) term(C.Cup + ((size_t)p * 5 + k) * nn * ldt + t, q, t + 1);
    }
  }
#pragma unroll
  for (int a = 0; a < NS; ++a) y[((size_t)p * NS + a) * ldt + t] = acc[a];
}

// First pass of the factored Delta apply, w = -Q~^-1 A~' d:
//   w_t = -Q_t^-1 d_t + sum_k Q_{t,p}^-1 A_hat_t[q_k,p]' d_{t+1}(q_k)  (t < T),
//   w_T = -Q_T^-1 d_T,
// over the 5-point neighbours q_k of node p inside the grid.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_tv_delta_w(Dims D, TvCoef<T> C,
                                                    const T* __restrict__ d,
                                                    T* __restrict__ w, const Scalars* sc,
                                                    int check) {
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ldt = D.ldt, K = D.K;
  const int t = (int)(g % ldt), p = (int)(g / ldt);
  constexpr int nn = NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = p / K, i = p - j * K;
  T acc[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) acc[a] = T(0);
  auto term = [&](const T* blk, int q, int tq, T sign) {
    T xv[NS];
#pragma unroll
    for (int b = 0; b < NS; ++b) xv[b] = d[((size_t)q * NS + b) * ldt + tq];
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
      for (int b = 0; b < NS; ++b)
        acc[a] = fma(sign * blk[(size_t)(a * NS + b) * ldt], xv[b], acc[a]);
  };
  term(C.Qi + (size_t)p * nn * ldt + t, p, t, T(-1));
  if (t < D.T) {
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= D.N) continue;
      term(C.Cup + ((size_t)p * 5 + k) * nn * ldt + t, jq * K + iq, t + 1, T(1));
    }
  }
#pragma unroll
  for (int a = 0; a < NS; ++a) w[((size_t)p * NS + a) * ldt + t] = acc[a];
}

// Second pass, y = Delta d = -A~ w + B~ R~^-1 B~' d:
//   y_t = sum_k A_hat_{t-1}[p,q_k] w_{t-1}(q_k) + B_{t-1} R_{t-1}^-1 B_{t-1}' d_t
//         - w_t  (t >= 1),   y_0 = -w_0,
// and one FP64 partial of d'y per workgroup.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_tv_delta_y(Dims D, TvCoef<T> C,
                                                    const T* __restrict__ d,
                                                    const T* __restrict__ w,
                                                    T* __restrict__ y,
                                                    double* __restrict__ partial,
                                                    const Scalars* sc, int check) {
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ldt = D.ldt, K = D.K;
  const int t = (int)(g % ldt), p = (int)(g / ldt);
  constexpr int nn = NS * NS;
  double dot = 0.0;
  if (p < D.real_nodes && t < D.Tt) {
    const int j = p / K, i = p - j * K;
    T acc[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = -w[((size_t)p * NS + a) * ldt + t];
    auto term = [&](const T* blk, const T* x, int q, int tq) {
      T xv[NS];
#pragma unroll
      for (int b = 0; b < NS; ++b) xv[b] = x[((size_t)q * NS + b) * ldt + tq];
#pragma unroll
      for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b < NS; ++b) acc[a] = fma(blk[(size_t)(a * NS + b) * ldt], xv[b], acc[a]);
    };
    if (t >= 1) {
      for (int k = 0; k < 5; ++k) {
        const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
        if (iq < 0 || iq >= K || jq < 0 || jq >= D.N) continue;
        term(C.A5 + ((size_t)p * 5 + k) * nn * ldt + (t - 1), w, jq * K + iq, t - 1);
      }
      term(C.BRB + (size_t)p * nn * ldt + t, d, p, t);
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      y[((size_t)p * NS + a) * ldt + t] = acc[a];
      dot += (double)acc[a] * (double)d[((size_t)p * NS + a) * ldt + t];
    }
  }
  if (partial) {
    const double s = block_sum<256>(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Value of lane `src` of the wavefront.
template <typename T>
__device__ __forceinline__ T lane_read(T v, int src) {
  return __shfl(v, src, kWave);
}

// theta = Phi~^-1 tau for time-varying data: eight threads per (v, t), thread
// r of a system owning row r of every 2n-row block row (rows past 2n idle),
// forward then backward substitution over the K block rows with the one-chain
// products (bodies_setup.h factor):
//   z_i = Linv_i tau_i - M1_i z_{i-1} - M2_i z_{i-2},  w_{i-1} = Linv_{i-1}' z_{i-1}
//   theta_i = w_i - N1_i theta_{i+1} - N2_i theta_{i+2}.
// w is parked in `wpark` (vector layout).  A workgroup of 256 threads holds
// 32 time steps of one super-column.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_tv_phi_solve(Dims D, TvCoef<T> C,
                                                      const T* __restrict__ tau,
                                                      T* __restrict__ out,
                                                      T* __restrict__ wpark,
                                                      const Scalars* sc, int check) {
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  constexpr int NB = 2 * NS;
  const int tiles = (D.Tt + 31) / 32;
  const int v = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  if (v >= D.V) return;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int r = lane & 7, sys0 = lane & ~7;
  const int t = tile * 32 + wv * 8 + (lane >> 3);
  const bool act = r < NB && t < D.Tt;
  const int tl = t < D.Tt ? t : D.Tt - 1;  // clamped time for loads
  const int h = r < NB ? r / NS : 0, c = r < NB ? r % NS : 0;
  const int j = 2 * v + h;
  const int K = D.K, ldt = D.ldt;
  const size_t ld8 = (size_t)ldt * 8;
  auto vec_at = [&](int i) { return ((size_t)(j * K + i) * NS + c) * ldt + tl; };
  const T* Fw = C.Fw + (size_t)v * fw_rows(K) * kFwRow * ld8 + (size_t)tl * 8 + r;
  const T* Bw = C.Bw + (size_t)v * K * kBwRow * ld8 + (size_t)tl * 8 + r;
  auto fw = [&](int row, int k) { return Fw[((size_t)row * kFwRow + k) * ld8]; };
  auto bw = [&](int row, int k) { return Bw[((size_t)row * kBwRow + k) * ld8]; };
  T z1 = T(0), z2 = T(0);  // z_{i-1}, z_{i-2} of this row
  for (int i = 0; i < K; ++i) {
    const T tr = act ? tau[vec_at(i)] : T(0);
    T z = T(0), w = T(0);
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      const T tc = lane_read(tr, sys0 + cc);
      const T y1 = lane_read(z1, sys0 + cc);
      const T y2 = lane_read(z2, sys0 + cc);
      z = fma(fw(i, 16 + cc), tc, z);
      z = fma(-fw(i, cc), y1, z);
      z = fma(-fw(i, 8 + cc), y2, z);
      w = fma(fw(i, 24 + cc), y1, w);  // w_{i-1} = Linv_{i-1}' z_{i-1}
    }
    if (i >= 1 && act) wpark[vec_at(i - 1)] = w;
    z2 = z1;
    z1 = z;
  }
  {  // w_{K-1}: table row K holds Linv_{K-1}'
    T w = T(0);
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) w = fma(fw(K, 24 + cc), lane_read(z1, sys0 + cc), w);
    if (act) wpark[vec_at(K - 1)] = w;
  }
  T th1 = T(0), th2 = T(0);  // theta_{i+1}, theta_{i+2}
  for (int i = K - 1; i >= 0; --i) {
    T th = act ? wpark[vec_at(i)] : T(0);
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      th = fma(-bw(i, cc), lane_read(th1, sys0 + cc), th);
      th = fma(-bw(i, 8 + cc), lane_read(th2, sys0 + cc), th);
    }
    if (act) out[vec_at(i)] = th;
    th2 = th1;
    th1 = th;
  }
}

// x_t = Q_t^-1 (-dl_t + [t < T] sum_k A_hat_t[q_k,p]' dl_{t+1}(q_k)),
// u_t = R_t^-1 B_t' dl_{t+1}  (Sec. II-B), in the interface layout.
template <int NS>
__global__ __launch_bounds__(256) void k_tv_recover(Dims D, TvCoef<double> C,
                                                    const double* __restrict__ dl,
                                                    double* __restrict__ x,
                                                    double* __restrict__ u) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ldt = D.ldt, K = D.K, m = D.m;
  const int t = (int)(g % ldt), p = (int)(g / ldt);
  if (p >= D.real_nodes || t >= D.Tt) return;
  constexpr int nn = NS * NS;
  const int j = p / K, i = p - j * K;
  double a[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) a[e] = -dl[((size_t)p * NS + e) * ldt + t];
  if (t < D.T) {
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= D.N) continue;
      const int q = jq * K + iq;
      const double* blk = C.AT5 + ((size_t)p * 5 + k) * nn * ldt + t;
#pragma unroll
      for (int r = 0; r < NS; ++r)
#pragma unroll
        for (int b = 0; b < NS; ++b)
          a[r] = fma(blk[(size_t)(r * NS + b) * ldt], dl[((size_t)q * NS + b) * ldt + t + 1], a[r]);
    }
  }
  if (x) {
    double* xp = x + ((size_t)t * D.real_nodes + p) * NS;
    const double* Qi = C.Qi + (size_t)p * nn * ldt + t;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < NS; ++b) s = fma(Qi[(size_t)(r * NS + b) * ldt], a[b], s);
      xp[r] = s;
    }
  }
  if (u && t < D.T) {
    double* up = u + ((size_t)t * D.real_nodes + p) * m;
    const double* RB = C.RiBT + (size_t)p * m * NS * ldt + t;
    for (int e = 0; e < m; ++e) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < NS; ++b)
        s = fma(RB[(size_t)(e * NS + b) * ldt], dl[((size_t)p * NS + b) * ldt + t + 1], s);
      up[e] = s;
    }
  }
}

// Scatter of one block array that the time-invariant assembly wrote for
// nsl consecutive time slices s0 .. s0 + nsl - 1 (slice b at src + b * stride,
// row r = (node, coefficient) at [r]) into its time-fastest array dst[r][t]
// at t = s + toff.  A workgroup transposes 64 rows x kTvBatch slices through
// LDS, so that both the reads (64 consecutive rows of one slice) and the
// writes (kTvBatch consecutive times of one row) are contiguous.
__global__ __launch_bounds__(256) void k_tv_scatter(const double* __restrict__ src,
                                                    long long stride, long long rows,
                                                    double* __restrict__ dst, int ldt, int s0,
                                                    int nsl, int toff) {
  __shared__ double tile[64][kTvBatch + 1];
  const long long r0 = (long long)blockIdx.x * 64;
  for (int k = threadIdx.x; k < 64 * kTvBatch; k += 256) {
    const int b = k / 64, rl = k % 64;  // row fastest: coalesced reads
    const long long r = r0 + rl;
    if (b < nsl && r < rows) tile[rl][b] = src[(long long)b * stride + r];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 64 * kTvBatch; k += 256) {
    const int rl = k / kTvBatch, b = k % kTvBatch;  // time fastest: contiguous writes
    const long long r = r0 + rl;
    if (b < nsl && r < rows) dst[r * ldt + s0 + b + toff] = tile[rl][b];
  }
}

__global__ __launch_bounds__(64) void k_tv_factor(Dims D, Coef C, Scalars* sc) {
  factor(D, C, sc, blockIdx.x, blockIdx.y);
}

}  // namespace

#define LQG_TV_DISPATCH(n, CALL) \
  switch (n) {                   \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    default: break;              \
  }

inline int tv_blocks(const Dims& D) {
  return (int)(((long long)D.real_nodes * D.ldt + 255) / 256);
}

template <typename T>
int tv_delta_apply(const Dims& D, const TvCoef<T>& C, const T* d, T* y, double* partial,
                   const Scalars* sc, int check, hipStream_t s) {
  const int nb = tv_blocks(D);
#define CALL(NS)                                                                            \
  hipLaunchKernelGGL((k_tv_delta_w<T, NS>), dim3(nb), dim3(256), 0, s, D, C, d, C.dw, sc,     \
                     check);                                                                \
  hipLaunchKernelGGL((k_tv_delta_y<T, NS>), dim3(nb), dim3(256), 0, s, D, C, d,             \
                     (const T*)C.dw, y, partial, sc, check)
  LQG_TV_DISPATCH(D.n, CALL)
#undef CALL
  return nb;
}

template <typename T>
void tv_xi_rhs(const Dims& D, const TvCoef<T>& C, const T* r, const T* dl, T* rho,
               const Scalars* sc, int check, hipStream_t s) {
#define CALL(NS)                                                                        \
  hipLaunchKernelGGL((k_tv_stencil<T, NS, 1>), dim3(tv_blocks(D)), dim3(256), 0, s, D, C, \
                     dl, r, rho, sc, check)
  LQG_TV_DISPATCH(D.n, CALL)
#undef CALL
}

template <typename T>
void tv_omega_rhs(const Dims& D, const TvCoef<T>& C, const T* rho, const T* th, T* tau,
                  const Scalars* sc, int check, hipStream_t s) {
#define CALL(NS)                                                                        \
  hipLaunchKernelGGL((k_tv_stencil<T, NS, 2>), dim3(tv_blocks(D)), dim3(256), 0, s, D, C, \
                     th, rho, tau, sc, check)
  LQG_TV_DISPATCH(D.n, CALL)
#undef CALL
}

template <typename T>
void tv_phi_solve(const Dims& D, const TvCoef<T>& C, const T* tau, T* out,
                  const Scalars* sc, int check, hipStream_t s) {
  const int g = D.V * ((D.Tt + 31) / 32);
#define CALL(NS)                                                                    \
  hipLaunchKernelGGL((k_tv_phi_solve<T, NS>), dim3(g), dim3(256), 0, s, D, C, tau, out, \
                     C.w, sc, check)
  LQG_TV_DISPATCH(D.n, CALL)
#undef CALL
}

void tv_recover(const Dims& D, const TvCoef<double>& C, const double* dl, double* x,
                double* u, hipStream_t s) {
#define CALL(NS) \
  hipLaunchKernelGGL(k_tv_recover<NS>, dim3(tv_blocks(D)), dim3(256), 0, s, D, C, dl, x, u)
  LQG_TV_DISPATCH(D.n, CALL)
#undef CALL
}

void tv_scatter_batch(const Dims& D, const Coef& S, const TvCoef<double>& C, int s0, int nsl,
                      hipStream_t s) {
  const long long nodes = D.nodes, nn = (long long)D.n * D.n, mn = (long long)D.m * D.n;
  const int nfull = s0 + nsl - 1 == D.T ? nsl - 1 : nsl;  // slice T: Q_T^-1 only
  auto one = [&](const double* src, long long per, double* dst, int n, int toff) {
    if (n <= 0 || !src || !dst) return;
    const long long rows = nodes * per;
    hipLaunchKernelGGL(k_tv_scatter, dim3((unsigned)((rows + 63) / 64)), dim3(256), 0, s, src,
                       rows, rows, dst, D.ldt, s0, n, toff);
  };
  one(S.G13, 13 * nn, const_cast<double*>(C.G13), nfull, 1);
  one(S.Qi, nn, const_cast<double*>(C.Qi), nsl, 0);
  one(S.Cdn, 5 * nn, const_cast<double*>(C.Cdn), nfull, 0);
  one(S.Cup, 5 * nn, const_cast<double*>(C.Cup), nfull, 0);
  one(S.AT5, 5 * nn, const_cast<double*>(C.AT5), nfull, 0);
  one(S.RiBT, mn, const_cast<double*>(C.RiBT), nfull, 0);
  one(S.A5, 5 * nn, const_cast<double*>(C.A5), nfull, 0);
  one(S.BRB, nn, const_cast<double*>(C.BRB), nfull, 1);
}

void tv_factor(const Dims& D, const Coef& C, Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_tv_factor, dim3(D.V, D.Tt), dim3(64), 0, s, D, C, sc);
}

template int tv_delta_apply<double>(const Dims&, const TvCoef<double>&, const double*,
                                    double*, double*, const Scalars*, int, hipStream_t);
template int tv_delta_apply<float>(const Dims&, const TvCoef<float>&, const float*, float*,
                                   double*, const Scalars*, int, hipStream_t);
template void tv_xi_rhs<double>(const Dims&, const TvCoef<double>&, const double*,
                                const double*, double*, const Scalars*, int, hipStream_t);
template void tv_xi_rhs<float>(const Dims&, const TvCoef<float>&, const float*, const float*,
                               float*, const Scalars*, int, hipStream_t);
template void tv_omega_rhs<double>(const Dims&, const TvCoef<double>&, const double*,
                                   const double*, double*, const Scalars*, int, hipStream_t);
template void tv_omega_rhs<float>(const Dims&, const TvCoef<float>&, const float*,
                                  const float*, float*, const Scalars*, int, hipStream_t);
template void tv_phi_solve<double>(const Dims&, const TvCoef<double>&, const double*, double*,
                                   const Scalars*, int, hipStream_t);
template void tv_phi_solve<float>(const Dims&, const TvCoef<float>&, const float*, float*,
                                  const Scalars*, int, hipStream_t);

}  // namespace lqg
