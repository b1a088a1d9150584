// Hot-path kernels of one PCG iteration (Algorithm 1) and of the NBJM
// preconditioner (Algorithm 2), generic over the vector element type T
// (double for the FP64 path, float for the FP32 sweeps of the precision
// form; partial sums are always accumulated in FP64).
//
// Work mapping: a wavefront owns one grid node (or one row of a super-column
// block row for the block solve) and 64 consecutive time steps, one per lane.
// The operator blocks are time invariant, so every coefficient address is
// wave-uniform; the vectors are time-fastest, so each lane's accesses form
// one contiguous segment per (node, component).  The t = 0 and t = T special
// cases of Delta (Psi_hat_0 = Q^-1, no t-1 / t+1 neighbour) are lane
// predicates.
#include "launch.h"

namespace lqg {
namespace {

template <int NS, typename T>
__device__ __forceinline__ void load_node(const T* __restrict__ v, int p, int t,
                                          int ldt, T (&x)[NS]) {
  const T* b = v + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) x[c] = b[(size_t)c * ldt];
}
template <int NS, typename T>
__device__ __forceinline__ void store_node(T* __restrict__ v, int p, int t,
                                           int ldt, const T (&x)[NS]) {
  T* b = v + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) b[(size_t)c * ldt] = x[c];
}
// acc += M x   (M: NS x NS row-major, wave-uniform)
template <int NS, typename T>
__device__ __forceinline__ void mv_add(const T* __restrict__ M, const T (&x)[NS],
                                       T (&acc)[NS]) {
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(M[a * NS + b], x[b], acc[a]);
}
template <int NS, typename T>
__device__ __forceinline__ void mv_sub(const T* __restrict__ M, const T (&x)[NS],
                                       T (&acc)[NS]) {
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(-M[a * NS + b], x[b], acc[a]);
}

__device__ __forceinline__ bool is_done(const Scalars* sc, int check) {
  return check && __builtin_nontemporal_load(&sc->done) != 0;
}

// Logical block of the node-tile kernels: chunk-major, node group (4 nodes,
// one per wavefront) fastest, remapped per XCD.  Returns false for padding.
__device__ __forceinline__ bool node_tile(const Dims& D, int* lb, int* p, int* t) {
  const int ngroups = (D.real_nodes + 3) / 4;
  *lb = xcd_block();
  if (*lb >= ngroups * ((D.Tt + kWave - 1) / kWave)) return false;
  *p = uniform((*lb % ngroups) * 4 + (threadIdx.x >> 6));
  *t = (*lb / ngroups) * kWave + (threadIdx.x & (kWave - 1));
  return true;
}

// ---------------------------------------------------------------------------
// y = Delta d, fused partial sums of y'd (FP64).
//   y_t(p) = Q_t^-1 d_t(p)
//          + [t>=1] ( sum_13 G[p][k] d_t(p+o_k) - sum_5 Cdn[p][k] d_{t-1}(p+o_k) )
//          - [t<T]  sum_5 Cup[p][k] d_{t+1}(p+o_k)
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_delta(Dims D, OpCoef<T> C,
                                               const T* __restrict__ d,
                                               T* __restrict__ y,
                                               double* __restrict__ partial,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  int lb, p, t;
  if (!node_tile(D, &lb, &p, &t)) return;
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  double dot = 0.0;
  if (p < D.real_nodes && t < D.Tt) {
    const int j = uniform(p / K), i = uniform(p - (p / K) * K);
    T self[NS], acc[NS], nb[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = T(0);
    load_node<NS>(d, p, t, ldt, self);
    mv_add<NS>(C.Qi + p * nn, self, acc);
    if (t == T_) mv_add<NS>(C.QTd + p * nn, self, acc);
    if (t >= 1) {
#pragma unroll
      for (int k = 0; k < 13; ++k) {
        const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
        if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
        load_node<NS>(d, jq * K + iq, t, ldt, nb);
        mv_add<NS>(C.G13 + ((size_t)p * 13 + k) * nn, nb, acc);
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
        if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
        load_node<NS>(d, jq * K + iq, t - 1, ldt, nb);
        mv_sub<NS>(C.Cdn + ((size_t)p * 5 + k) * nn, nb, acc);
      }
    }
    if (t < T_) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
        if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
        load_node<NS>(d, jq * K + iq, t + 1, ldt, nb);
        mv_sub<NS>(C.Cup + ((size_t)p * 5 + k) * nn, nb, acc);
      }
    }
    store_node<NS>(y, p, t, ldt, acc);
#pragma unroll
    for (int a = 0; a < NS; ++a) dot = fma((double)acc[a], (double)self[a], dot);
  }
  dot = block_sum<256>(dot);
  if (partial && threadIdx.x == 0) partial[lb] = dot;
}

// tau = rho + Omega~ theta, Omega~ = Phi~ - Psi~: minus the blocks of
// Psi_hat_t (t >= 1) that couple different super-columns; Omega_hat_0 = 0.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_omega(Dims D, OpCoef<T> C,
                                               const T* __restrict__ rho,
                                               const T* __restrict__ th,
                                               T* __restrict__ tau,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  int lb, p, t;
  if (!node_tile(D, &lb, &p, &t)) return;
  const int ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  T acc[NS], nb[NS];
  if (rho) load_node<NS>(rho, p, t, ldt, acc);
  else
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = T(0);
  if (t >= 1) {
#pragma unroll
    for (int k = 0; k < 13; ++k) {
      const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
      if ((jq >> 1) == (j >> 1)) continue;  // same super-column: inside Phi~
      load_node<NS>(th, jq * K + iq, t, ldt, nb);
      mv_sub<NS>(C.G13 + ((size_t)p * 13 + k) * nn, nb, acc);
    }
  }
  store_node<NS>(tau, p, t, ldt, acc);
}

// rho = r + Xi~ dl, Xi~ = Psi~ - Delta:
//   (Xi~ dl)_t(p) = [t>=1] sum_5 Cdn[p][k] dl_{t-1}(q) + [t<T] sum_5 Cup[p][k] dl_{t+1}(q)
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_xi(Dims D, OpCoef<T> C,
                                            const T* __restrict__ r,
                                            const T* __restrict__ dl,
                                            T* __restrict__ rho,
                                            const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  int lb, p, t;
  if (!node_tile(D, &lb, &p, &t)) return;
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  T acc[NS], nb[NS];
  if (r) load_node<NS>(r, p, t, ldt, acc);
  else
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = T(0);
  if (t >= 1) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
      load_node<NS>(dl, jq * K + iq, t - 1, ldt, nb);
      mv_add<NS>(C.Cdn + ((size_t)p * 5 + k) * nn, nb, acc);
    }
  }
  if (t < T_) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
      load_node<NS>(dl, jq * K + iq, t + 1, ldt, nb);
      mv_add<NS>(C.Cup + ((size_t)p * 5 + k) * nn, nb, acc);
    }
  }
  store_node<NS>(rho, p, t, ldt, acc);
}

// ---------------------------------------------------------------------------
// Buffer-resource access for the block solve: a lane outside the current
// factor class uses an out-of-range offset, whose loads return 0 and whose
// stores are dropped, so the sweeps have no divergent branches.
constexpr int kPre = 4;
constexpr unsigned kOob = 0x80000000u;     // beyond every vector (< 2 GiB)
constexpr int kRsrcWord3 = 0x00020000;     // raw buffer, 32-bit dwords

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p,
                                                            long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)bytes, kRsrcWord3);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r,
                                                 unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r,
                                               unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off,
                                       double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off,
                                       float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
// Coefficient j of a factor row whose dwords are spread one per lane.
template <typename T>
__device__ __forceinline__ T coef(unsigned reg, int j);
template <>
__device__ __forceinline__ double coef<double>(unsigned reg, int j) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)reg, 2 * j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)reg, 2 * j + 1);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <>
__device__ __forceinline__ float coef<float>(unsigned reg, int j) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane((int)reg, j));
}

// Forward/backward substitution with the banded block Cholesky factor of
// Phi_bar_{v,cls} (eq. "decomposed_problem") for the 64 time steps of this
// workgroup.  The 2n rows of each block row are split over 2n wavefronts,
// one row per wavefront (R selects it at compile time), one time step per
// lane.  Per block row the wavefronts exchange their row of z_i (theta_i)
// through LDS with one barrier:
//   z_i     = Linv_i tau_i - M1_i z_{i-1} - M2_i z_{i-2}
//   w_i     = Linv_i' z_i                  (parked in `out`)
//   theta_i = w_i - N1_i theta_{i+1} - N2_i theta_{i+2}
// Latency hiding: a row's 32 (16) factor coefficients of a block row are one
// coalesced vector load, lane k holding dword k; they are prefetched kPre
// block rows ahead in a register ring and moved to scalar registers with
// v_readlane when used, so no scalar-memory wait is tied to the LDS
// exchange.  tau and w are prefetched the same way.
template <typename T, int NS, int R>
__device__ __forceinline__ void sweep_row(const Dims& D, const OpCoef<T>& C,
                                          int cls, int v, int lane, int t,
                                          bool act, __amdgpu_buffer_rsrc_t rtau,
                                          __amdgpu_buffer_rsrc_t rout,
                                          T (*zb)[2 * NS][kWave]) {
  constexpr int NB = 2 * NS;
  constexpr int NT = R + 1;  // rows of tau that row R of z needs
  constexpr int ES = sizeof(T);
  constexpr int FD = kFwRow * ES / 4, BD = kBwRow * ES / 4;  // dwords per row
  const int K = D.K;
  const unsigned istride = (unsigned)(NS * D.ldt * ES);  // bytes per block row
  unsigned rb[NT];  // byte offset of row c of block row 0 (node (0, 2v + c/NS))
#pragma unroll
  for (int c = 0; c < NT; ++c)
    rb[c] = act ? (unsigned)((((size_t)(2 * v + c / NS) * K * NS + (c % NS)) * D.ldt + t) * ES)
                : kOob;
  const unsigned ro = act ? (unsigned)((((size_t)(2 * v + R / NS) * K * NS + (R % NS)) * D.ldt + t) * ES)
                          : kOob;
  // this row's factor coefficients: block row i at fw + i * fstep dwords
  const size_t rows0 = ((size_t)cls * D.V + v) * K;
  const size_t frows0 = ((size_t)cls * D.V + v) * (K + 1);
  const unsigned* fw = reinterpret_cast<const unsigned*>(C.Fw + (frows0 * NB + R) * kFwRow) + (lane % FD);
  const unsigned* bw = reinterpret_cast<const unsigned*>(C.Bw + (rows0 * NB + R) * kBwRow) + (lane % BD);
  const size_t fstep = (size_t)NB * FD, bstep = (size_t)NB * BD;

  // ---------------------------------------------------------- forward
  // Block row i uses ring slot i % kPre; loads for row i + kPre (clamped)
  // go into the slot just consumed.  The main loop covers whole chunks of
  // kPre rows with straight-line code, so every wait on a prefetched slot
  // is an exact in-order vmcnt count.
  T z1[NB], z2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) z1[b] = z2[b] = T(0);
  unsigned cring[kPre];
  T tring[kPre][NT];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    cring[u] = fw[(size_t)min(u, K) * fstep];
#pragma unroll
    for (int c = 0; c < NT; ++c)
      tring[u][c] = buf_ld<T>(rtau, rb[c] + (unsigned)min(u, K - 1) * istride);
  }
  auto fstep_body = [&](int i, int s, bool has_prev) {
    const unsigned cf = cring[s];
    T ti[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) ti[c] = tring[s][c];
    const int in = min(i + kPre, K);
    cring[s] = fw[(size_t)in * fstep];
    const int it = min(in, K - 1);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[s][c] = buf_ld<T>(rtau, rb[c] + (unsigned)it * istride);
    if (has_prev) {  // w_{i-1} = row R of Linv_{i-1}' times z_{i-1}
      T acc = T(0);
#pragma unroll
      for (int c = R; c < NB; ++c) acc = fma(coef<T>(cf, 24 + c), z1[c], acc);
      buf_st(rout, ro + (unsigned)(i - 1) * istride, acc);
    }
    T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c <= R) a0 = fma(coef<T>(cf, 16 + c), ti[c], a0);
      a1 = fma(coef<T>(cf, c), z1[c], a1);
      a2 = fma(coef<T>(cf, 8 + c), z2[c], a2);
    }
    zb[i & 1][R][lane] = a0 - a1 - a2;
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      z2[b] = z1[b];
      z1[b] = zb[i & 1][b][lane];
    }
  };
  fstep_body(0, 0, false);
  int i = 1;
  for (; i + kPre <= K; i += kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) fstep_body(i + u, (1 + u) % kPre, true);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (i + u < K) fstep_body(i + u, (1 + u) % kPre, true);
  {  // w_{K-1}: block row K of Fw carries Linv_{K-1}'
    const unsigned cf = fw[(size_t)K * fstep];
    T acc = T(0);
#pragma unroll
    for (int c = R; c < NB; ++c) acc = fma(coef<T>(cf, 24 + c), z1[c], acc);
    buf_st(rout, ro + (unsigned)(K - 1) * istride, acc);
  }
  lds_barrier();  // every wavefront is done reading zb before it is reused

  // ---------------------------------------------------------- backward
  T t1[NB], t2[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) t1[b] = t2[b] = T(0);
  unsigned bring[kPre];
  T wring[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int iu = K - 1 - u >= 0 ? K - 1 - u : 0;
    bring[u] = bw[(size_t)iu * bstep];
    wring[u] = buf_ld<T>(rout, ro + (unsigned)iu * istride);
  }
  auto bstep_body = [&](int i, int s) {
    const unsigned cb = bring[s];
    const T wi = wring[s];
    const int in = max(i - kPre, 0);
    bring[s] = bw[(size_t)in * bstep];
    wring[s] = buf_ld<T>(rout, ro + (unsigned)in * istride);
    T a1 = T(0), a2 = T(0);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      a1 = fma(coef<T>(cb, c), t1[c], a1);
      a2 = fma(coef<T>(cb, 8 + c), t2[c], a2);
    }
    const T th = wi - a1 - a2;
    buf_st(rout, ro + (unsigned)i * istride, th);
    zb[i & 1][R][lane] = th;
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      t2[b] = t1[b];
      t1[b] = zb[i & 1][b][lane];
    }
  };
  int j = K - 1;  // block row K-1-u uses slot u % kPre
  for (; j - kPre + 1 >= 0; j -= kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) bstep_body(j - u, u);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (j - u >= 0) bstep_body(j - u, u);
  lds_barrier();
}

template <typename T, int NS, int R = 0>
__device__ __forceinline__ void sweep_dispatch(int w, const Dims& D,
                                               const OpCoef<T>& C, int cls,
                                               int v, int lane, int t, bool act,
                                               __amdgpu_buffer_rsrc_t rtau,
                                               __amdgpu_buffer_rsrc_t rout,
                                               T (*zb)[2 * NS][kWave]) {
  if constexpr (R < 2 * NS) {
    if (w == R) sweep_row<T, NS, R>(D, C, cls, v, lane, t, act, rtau, rout, zb);
    else sweep_dispatch<T, NS, R + 1>(w, D, C, cls, v, lane, t, act, rtau, rout, zb);
  }
}

// out = Phi~^-1 tau.  One workgroup of 2n wavefronts per (super-column v,
// 64 time steps).  t = 0: Phi_bar_{v,0} = blkdiag(Q^-1), so theta = Q tau
// per node.  t = T uses the second factor class when Q_T != Q.
template <typename T, int NS>
__global__ __launch_bounds__(2 * NS * kWave) void k_phi_solve(
    Dims D, OpCoef<T> C, const T* __restrict__ tau, T* __restrict__ out,
    const Scalars* sc, int check, int qt_distinct) {
  if (is_done(sc, check)) return;
  __shared__ T zb[2][2 * NS][kWave];
  const int nchunks = (D.Tt + kWave - 1) / kWave;
  const int lb = xcd_block();  // super-column major: a v's chunks share an XCD
  if (lb >= D.V * nchunks) return;
  const int v = lb / nchunks, chunk = lb % nchunks;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x >> 6);
  const int t0 = chunk * kWave;
  const int t = t0 + lane;
  const int T_ = D.T;
  const bool valid = t < D.Tt;
  const long long bytes = D.vlen * (long long)sizeof(T);
  const __amdgpu_buffer_rsrc_t rtau = make_rsrc(tau, bytes);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out, bytes);
  sweep_dispatch<T, NS>(w, D, C, 0, v, lane, t,
                        valid && t >= 1 && !(qt_distinct && t == T_), rtau, rout, zb);
  if (qt_distinct && t0 <= T_ && T_ < t0 + kWave)
    sweep_dispatch<T, NS>(w, D, C, 1, v, lane, t, valid && t == T_, rtau, rout, zb);
  if (chunk == 0) {
    // t = 0 for every block row: independent n x n products, one block row
    // per lane; wavefront w computes row w of the pair
    const size_t nn = (size_t)NS * NS;
    const int h = w / NS, a = w % NS;
    for (int i = lane; i < D.K; i += kWave) {
      const int p = (2 * v + h) * D.K + i;
      const T* Qp = C.Qm + p * nn + a * NS;
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NS; ++b)
        acc = fma(Qp[b], tau[((size_t)p * NS + b) * D.ldt], acc);
      out[((size_t)p * NS + a) * D.ldt] = acc;
    }
  }
}

// x_t = Q_t^-1 (-dl_t + [t<T] A_hat' dl_{t+1}),  u_t = R^-1 B' dl_{t+1}
// (Sec. II-B: x~ = Q~^-1 A~' delta~, u~ = R~^-1 B~' delta~), written in the
// interface layout.
template <int NS>
__global__ __launch_bounds__(256) void k_recover(Dims D, Coef C,
                                                 const double* __restrict__ dl,
                                                 double* __restrict__ x,
                                                 double* __restrict__ u) {
  int lb, p, t;
  if (!node_tile(D, &lb, &p, &t)) return;
  const int T = D.T, ldt = D.ldt, K = D.K, N = D.N, m = D.m;
  const size_t nn = (size_t)NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  double a[NS], nb[NS], xo[NS];
  load_node<NS>(dl, p, t, ldt, a);
#pragma unroll
  for (int c = 0; c < NS; ++c) a[c] = -a[c];
  if (t < T) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
      load_node<NS>(dl, jq * K + iq, t + 1, ldt, nb);
      mv_add<NS>(C.AT5 + ((size_t)p * 5 + k) * nn, nb, a);
    }
  }
#pragma unroll
  for (int c = 0; c < NS; ++c) xo[c] = 0.0;
  mv_add<NS>((t == T ? C.QTi : C.Qi) + p * nn, a, xo);
  if (x) {
    double* xp = x + ((size_t)t * D.real_nodes + p) * NS;
#pragma unroll
    for (int c = 0; c < NS; ++c) xp[c] = xo[c];
  }
  if (u && t < T) {
    load_node<NS>(dl, p, t + 1, ldt, nb);
    double* up = u + ((size_t)t * D.real_nodes + p) * m;
    const double* RB = C.RiBT + (size_t)p * m * NS;
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < NS; ++b) s = fma(RB[c * NS + b], nb[b], s);
      up[c] = s;
    }
  }
}

inline int node_blocks(const Dims& D) {
  return ((D.real_nodes + 3) / 4) * ((D.Tt + kWave - 1) / kWave);
}
inline dim3 node_grid(const Dims& D) { return dim3(padded_grid(node_blocks(D))); }

}  // namespace

#define LQG_DISPATCH_N(n, CALL) \
  switch (n) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    case 4: CALL(4); break;     \
    default: break;             \
  }

template <typename T>
int delta_apply(const Dims& D, const OpCoef<T>& C, const T* d, T* y,
                double* partial, const Scalars* sc, int check_done,
                hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS)                                                              \
  hipLaunchKernelGGL((k_delta<T, NS>), g, dim3(256), 0, s, D, C, d, y, partial, \
                     sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
  return node_blocks(D);
}

template <typename T>
void omega_rhs(const Dims& D, const OpCoef<T>& C, const T* rho, const T* th,
               T* tau, const Scalars* sc, int check_done, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS)                                                               \
  hipLaunchKernelGGL((k_omega<T, NS>), g, dim3(256), 0, s, D, C, rho, th, tau, \
                     sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

template <typename T>
void xi_rhs(const Dims& D, const OpCoef<T>& C, const T* r, const T* dl, T* rho,
            const Scalars* sc, int check_done, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS)                                                                 \
  hipLaunchKernelGGL((k_xi<T, NS>), g, dim3(256), 0, s, D, C, r, dl, rho, sc, \
                     check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

template <typename T>
void phi_solve(const Dims& D, const OpCoef<T>& C, const T* tau, T* out,
               const Scalars* sc, int check_done, int qt_distinct,
               hipStream_t s) {
  const dim3 g(padded_grid(D.V * ((D.Tt + kWave - 1) / kWave)));
#define CALL(NS)                                                                   \
  hipLaunchKernelGGL((k_phi_solve<T, NS>), g, dim3(2 * NS * kWave), 0, s, D, C, \
                     tau, out, sc, check_done, qt_distinct)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

template int delta_apply<double>(const Dims&, const OpCoef<double>&, const double*,
                                 double*, double*, const Scalars*, int, hipStream_t);
template int delta_apply<float>(const Dims&, const OpCoef<float>&, const float*,
                                float*, double*, const Scalars*, int, hipStream_t);
template void omega_rhs<double>(const Dims&, const OpCoef<double>&, const double*,
                                const double*, double*, const Scalars*, int, hipStream_t);
template void omega_rhs<float>(const Dims&, const OpCoef<float>&, const float*,
                               const float*, float*, const Scalars*, int, hipStream_t);
template void xi_rhs<double>(const Dims&, const OpCoef<double>&, const double*,
                             const double*, double*, const Scalars*, int, hipStream_t);
template void xi_rhs<float>(const Dims&, const OpCoef<float>&, const float*,
                            const float*, float*, const Scalars*, int, hipStream_t);
template void phi_solve<double>(const Dims&, const OpCoef<double>&, const double*,
                                double*, const Scalars*, int, int, hipStream_t);
template void phi_solve<float>(const Dims&, const OpCoef<float>&, const float*,
                               float*, const Scalars*, int, int, hipStream_t);

void recover(const Dims& D, const Coef& C, const double* dl, double* x,
             double* u, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS) hipLaunchKernelGGL(k_recover<NS>, g, dim3(256), 0, s, D, C, dl, x, u)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

}  // namespace lqg
