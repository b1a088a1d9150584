// Per-tile bodies of the hot-path kernels of one PCG iteration (Algorithm 1)
// and of the NBJM preconditioner (Algorithm 2), generic over the vector
// element type T (double for FP64, float for the FP32 sweeps of the
// precision form; partial sums are always accumulated in FP64).  The
// single-problem kernels (ops.hip) and the batched kernels (batch.hip) call
// the same bodies; they differ only in how a workgroup finds its problem
// and tile.
//
// Work mapping: a wavefront owns one grid node (or one row of a super-column
// block row for the block solve) and 64 consecutive time steps, one per lane.
// The operator blocks are time invariant, so every coefficient address is
// wave-uniform; the vectors are time-fastest, so each lane's accesses form
// one contiguous segment per (node, component).  The t = 0 and t = T special
// cases of Delta (Psi_hat_0 = Q^-1, no t-1 / t+1 neighbour) are lane
// predicates.
#pragma once
#include <type_traits>

#include "launch.h"

namespace lqg {
namespace dev {

// Address spaces.  Vectors live in global memory; the operator blocks and
// factors are time invariant and no kernel writes them while it runs, so
// they are read through the constant address space, which lets every
// wave-uniform coefficient load be a scalar load.  Stating both explicitly
// keeps the code generation the same whether a pointer is a kernel argument
// (single problem) or was read from a per-problem record (batched form),
// where the compiler could otherwise prove neither and fall back to flat
// vector loads.
template <typename T>
using gptr = T __attribute__((address_space(1)))*;
template <typename T>
using kptr = const T __attribute__((address_space(4)))*;
template <typename T>
__device__ __forceinline__ gptr<T> glob(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ gptr<const T> glob(const T* p) {
  return (gptr<const T>)p;
}
template <typename T>
__device__ __forceinline__ kptr<T> invariant(const T* p) {
  return (kptr<T>)p;
}

template <int NS, typename T>
__device__ __forceinline__ void load_node(const T* __restrict__ v, int p, int t,
                                          int ldt, T (&x)[NS]) {
  gptr<const T> b = glob(v) + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) x[c] = b[(size_t)c * ldt];
}
template <int NS, typename T>
__device__ __forceinline__ void store_node(T* __restrict__ v, int p, int t,
                                           int ldt, const T (&x)[NS]) {
  gptr<T> b = glob(v) + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) b[(size_t)c * ldt] = x[c];
}
// acc += M x   (M: NS x NS row-major, wave-uniform)
template <int NS, typename T>
__device__ __forceinline__ void mv_add(const T* Mg, const T (&x)[NS],
                                       T (&acc)[NS]) {
  kptr<T> M = invariant(Mg);
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(M[a * NS + b], x[b], acc[a]);
}
template <int NS, typename T>
__device__ __forceinline__ void mv_sub(const T* Mg, const T (&x)[NS],
                                       T (&acc)[NS]) {
  kptr<T> M = invariant(Mg);
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(-M[a * NS + b], x[b], acc[a]);
}

__device__ __forceinline__ bool is_done(const Scalars* sc, int check) {
  return check && __builtin_nontemporal_load(&sc->done) != 0;
}

// Node tiles: 4 nodes (one per wavefront of a 256-thread workgroup) x 64
// consecutive time steps (one per lane).  Tile (group, chunk) covers nodes
// 4 group .. 4 group + 3 and t = 64 chunk .. 64 chunk + 63.
__host__ __device__ inline int node_groups(const Dims& D) {
  return (D.real_nodes + 3) / 4;
}
__host__ __device__ inline int time_chunks(const Dims& D) {
  return (D.Tt + kWave - 1) / kWave;
}
__device__ __forceinline__ void node_coords(int group, int chunk, int* p, int* t) {
  *p = uniform(group * 4 + (threadIdx.x >> 6));
  *t = chunk * kWave + (threadIdx.x & (kWave - 1));
}

// ---------------------------------------------------------------------------
// y = Delta d on one node tile; the tile's FP64 partial sum of y'd is written
// to *partial (when non-null) by thread 0.  Every thread of the workgroup
// must call this (it contains a workgroup reduction).
//   y_t(p) = Q_t^-1 d_t(p)
//          + [t>=1] ( sum_13 G[p][k] d_t(p+o_k) - sum_5 Cdn[p][k] d_{t-1}(p+o_k) )
//          - [t<T]  sum_5 Cup[p][k] d_{t+1}(p+o_k)
template <typename T, int NS>
__device__ __forceinline__ void delta_tile(const Dims& D, const OpCoef<T>& C,
                                           const T* __restrict__ d,
                                           T* __restrict__ y,
                                           double* __restrict__ partial,
                                           int group, int chunk) {
  int p, t;
  node_coords(group, chunk, &p, &t);
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
  if (partial && threadIdx.x == 0) *partial = dot;
}

// tau = rho + Omega~ theta on one node tile, Omega~ = Phi~ - Psi~: minus the
// blocks of Psi_hat_t (t >= 1) that couple different super-columns;
// Omega_hat_0 = 0.  rho may be null (zero).
template <typename T, int NS>
__device__ __forceinline__ void omega_tile(const Dims& D, const OpCoef<T>& C,
                                           const T* __restrict__ rho,
                                           const T* __restrict__ th,
                                           T* __restrict__ tau, int group,
                                           int chunk) {
  int p, t;
  node_coords(group, chunk, &p, &t);
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

// rho = r + Xi~ dl on one node tile, Xi~ = Psi~ - Delta:
//   (Xi~ dl)_t(p) = [t>=1] sum_5 Cdn[p][k] dl_{t-1}(q) + [t<T] sum_5 Cup[p][k] dl_{t+1}(q)
// r may be null (zero).
template <typename T, int NS>
__device__ __forceinline__ void xi_tile(const Dims& D, const OpCoef<T>& C,
                                        const T* __restrict__ r,
                                        const T* __restrict__ dl,
                                        T* __restrict__ rho, int group,
                                        int chunk) {
  int p, t;
  node_coords(group, chunk, &p, &t);
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

// Compile-time loop: f(std::integral_constant<int, k>) for k = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// One row of NW factor coefficients of a block row, as the sweeps read it.
//   FP64: lane k holds dword k of the row (one coalesced load); coefficient j
//         is moved to scalar registers with two v_readlane when used.
//   FP32: lane l holds coefficient 16 g + (l mod 16) in register g, i.e. every
//         16-lane row of the wavefront holds the same 16 coefficients; the
//         product with coefficient j takes it from lane j mod 16 of the
//         lane's own row by a DPP row broadcast (row_newbcast) that folds into
//         the FMA, so no instruction is spent on moving coefficients.
template <typename T, int NW>
struct CoefRow;
template <int NW>
struct CoefRow<double, NW> {
  unsigned r;
  __device__ __forceinline__ void load(gptr<const unsigned> row, int lane) {
    r = row[lane % (2 * NW)];
  }
  template <int J>
  __device__ __forceinline__ double get() const {
    return coef<double>(r, J);
  }
};
template <int NW>
struct CoefRow<float, NW> {
  unsigned g[NW / 16];
  __device__ __forceinline__ void load(gptr<const unsigned> row, int lane) {
#pragma unroll
    for (int k = 0; k < NW / 16; ++k) g[k] = row[16 * k + (lane & 15)];
  }
  template <int J>
  __device__ __forceinline__ float get() const {
    constexpr int kRowNewBcast = 0x150;  // DPP row_newbcast:0
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, (int)g[J >> 4], kRowNewBcast + (J & 15),
                                           0xF, 0xF, true));
  }
};

// Forward/backward substitution with the banded block Cholesky factor of
// Phi_bar_{v,cls} (eq. "decomposed_problem") for the 64 time steps of this
// workgroup.  The 2n rows of each block row are split over 2n wavefronts,
// one row per wavefront (R selects it at compile time), one time step per
// lane.  Per block row the wavefronts exchange their row of z_i (theta_i)
// through LDS with one barrier:
//   z_i     = Linv_i tau_i - M1_i z_{i-1} - M2_i z_{i-2}
//   w_i     = Linv_i' z_i                  (parked in `out`)
//   theta_i = w_i - N1_i theta_{i+1} - N2_i theta_{i+2}
// Latency hiding: a row's 32 (16) factor coefficients of a block row are
// fetched by coalesced vector loads kPre block rows ahead into a register
// ring (CoefRow: FP64 through v_readlane, FP32 through DPP row broadcasts),
// so no scalar-memory wait is tied to the LDS exchange.  tau and w are
// prefetched the same way.
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
  const size_t frows0 = ((size_t)cls * D.V + v) * fw_rows(K);
  gptr<const unsigned> fw =
      glob(reinterpret_cast<const unsigned*>(C.Fw + (frows0 * NB + R) * kFwRow));
  gptr<const unsigned> bw =
      glob(reinterpret_cast<const unsigned*>(C.Bw + (rows0 * NB + R) * kBwRow));
  const size_t fstep = (size_t)NB * FD, bstep = (size_t)NB * BD;

  // ---------------------------------------------------------- forward
  // Ring slots: block row r of the factor in cring[r % kPre], tau row r in
  // tring[r % kPre]; each is refilled kPre rows ahead right after its last
  // use.  The main loop covers whole chunks of kPre rows with straight-line
  // code, so every wait on a prefetched slot is an exact in-order vmcnt
  // count.  Only  z_i = p_i - M1_i z_{i-1}  waits for the exchange of
  // z_{i-1}; the partial p_{i+1} = Linv_{i+1} tau_{i+1} - M2_{i+1} z_{i-1}
  // and w_{i-1} are computed while the other wavefronts reach the barrier.
  T z1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) z1[b] = T(0);
  CoefRow<T, kFwRow> cring[kPre];
  T tring[kPre][NT];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    cring[u].load(fw + (size_t)min(u, K) * fstep, lane);
#pragma unroll
    for (int c = 0; c < NT; ++c)
      tring[u][c] = buf_ld<T>(rtau, rb[c] + (unsigned)min(u, K - 1) * istride);
  }
  T pre = T(0);  // p_0 = Linv_0 tau_0
  sfor<0, R + 1>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    pre = fma(cring[0].template get<16 + c>(), tring[0][c], pre);
  });
#pragma unroll
  for (int c = 0; c < NT; ++c)
    tring[0][c] = buf_ld<T>(rtau, rb[c] + (unsigned)min(kPre, K - 1) * istride);
  auto fstep_body = [&](int i, int s, int sn, bool has_prev) {
    const CoefRow<T, kFwRow> cf = cring[s];
    T zi = pre;
    if (has_prev) {  // z_i = p_i - M1_i z_{i-1}, two interleaved chains
      T e0 = T(0), e1 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c % 2 == 0) e0 = fma(cf.template get<c>(), z1[c], e0);
        else e1 = fma(cf.template get<c>(), z1[c], e1);
      });
      zi = pre - (e0 + e1);
    }
    zb[i & 1][R][lane] = zi;
    if (has_prev) {  // w_{i-1} = row R of Linv_{i-1}' z_{i-1} (parked in out)
      T acc = T(0);
      sfor<R, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        acc = fma(cf.template get<24 + c>(), z1[c], acc);
      });
      buf_st(rout, ro + (unsigned)(i - 1) * istride, acc);
    }
    {  // p_{i+1} = Linv_{i+1} tau_{i+1} - M2_{i+1} z_{i-1}
      const CoefRow<T, kFwRow>& cn = cring[sn];
      T a0 = T(0), a2 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c <= R) a0 = fma(cn.template get<16 + c>(), tring[sn][c], a0);
        a2 = fma(cn.template get<8 + c>(), z1[c], a2);
      });
      pre = a0 - a2;
    }
    cring[s].load(fw + (size_t)min(i + kPre, K) * fstep, lane);
    const int it = min(i + 1 + kPre, K - 1);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[sn][c] = buf_ld<T>(rtau, rb[c] + (unsigned)it * istride);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) z1[b] = zb[i & 1][b][lane];
  };
  fstep_body(0, 0, 1, false);
  int i = 1;
  for (; i + kPre <= K; i += kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) fstep_body(i + u, (1 + u) % kPre, (2 + u) % kPre, true);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (i + u < K) fstep_body(i + u, (1 + u) % kPre, (2 + u) % kPre, true);
  {  // w_{K-1}: block row K of Fw carries Linv_{K-1}'
    CoefRow<T, kFwRow> cf;
    cf.load(fw + (size_t)K * fstep, lane);
    T acc = T(0);
    sfor<R, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      acc = fma(cf.template get<24 + c>(), z1[c], acc);
    });
    buf_st(rout, ro + (unsigned)(K - 1) * istride, acc);
  }
  lds_barrier();  // every wavefront is done reading zb before it is reused

  // ---------------------------------------------------------- backward
  // Step k handles block row j = K-1-k: theta_j = q_j - N1_j theta_{j+1},
  // with q_j = w_j - N2_j theta_{j+2} computed one step earlier.  Block row
  // r of the backward factor and w_r live in bring / wring slot
  // (K-1-r) % kPre.
  T t1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) t1[b] = T(0);
  CoefRow<T, kBwRow> bring[kPre];
  T wring[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int iu = K - 1 - u >= 0 ? K - 1 - u : 0;
    bring[u].load(bw + (size_t)iu * bstep, lane);
    wring[u] = buf_ld<T>(rout, ro + (unsigned)iu * istride);
  }
  T q = wring[0];  // q_{K-1} = w_{K-1}
  wring[0] = buf_ld<T>(rout, ro + (unsigned)max(K - 1 - kPre, 0) * istride);
  auto bstep_body = [&](int j, int s, int sn, bool has_next) {
    const CoefRow<T, kBwRow> cb = bring[s];
    T th = q;
    if (has_next) {  // theta_j = q_j - N1_j theta_{j+1}
      T e0 = T(0), e1 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c % 2 == 0) e0 = fma(cb.template get<c>(), t1[c], e0);
        else e1 = fma(cb.template get<c>(), t1[c], e1);
      });
      th = q - (e0 + e1);
    }
    zb[j & 1][R][lane] = th;
    buf_st(rout, ro + (unsigned)j * istride, th);
    {  // q_{j-1} = w_{j-1} - N2_{j-1} theta_{j+1}
      const CoefRow<T, kBwRow>& cn = bring[sn];
      T a2 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        a2 = fma(cn.template get<8 + c>(), t1[c], a2);
      });
      q = wring[sn] - a2;
    }
    bring[s].load(bw + (size_t)max(j - kPre, 0) * bstep, lane);
    wring[sn] = buf_ld<T>(rout, ro + (unsigned)max(j - 1 - kPre, 0) * istride);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) t1[b] = zb[j & 1][b][lane];
  };
  bstep_body(K - 1, 0, 1 % kPre, false);
  int j = K - 2;  // step k = K-1-j uses slots k % kPre and (k+1) % kPre
  for (; j - kPre + 1 >= 0; j -= kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) bstep_body(j - u, (1 + u) % kPre, (2 + u) % kPre, true);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (j - u >= 0) bstep_body(j - u, (1 + u) % kPre, (2 + u) % kPre, true);
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

// Forward/backward substitution with the twisted factor of Phi_bar_{v,cls}
// (factor_twisted: block rows ordered [0 .. m-1 | K-1 .. m+2 | m, m+1],
// m = (K-2)/2, |B| = K-2-m bottom rows).  4n wavefronts: the top chain on
// wavefronts 0 .. 2n-1, the bottom chain on 2n .. 4n-1, one row R each, so
// the two chains run side by side and each wavefront passes about K/2
// exchange barriers per direction instead of K.  Each half exchanges its z
// (theta) rows through its own LDS buffer `zo`; the two middle block rows
// read the other half's buffer `zx`.  The work between barriers b-1 and b is
// step b, and step b writes slot b & 1, so a slot is rewritten only after
// every reader has passed the next barrier.  Steps (both halves pass the
// same 2 |B| + 5 barriers):
//   0 .. |B|-1     top positions 0 .. m-1 (after |B| - m idle steps),
//                  bottom positions 0 .. |B|-1 (rows K-1 .. m+2)
//   |B|            top: z_m = p_m - M1_m z_{m-1} - X_t z_{m+2};
//                  bottom: p_{m+1} -= M1 z_{m+2} + X_b1 z_{m-1}
//   |B|+1          top: w_m;  bottom: z_{m+1} = p_{m+1} - X_b2 z_m
//   |B|+2          bottom: theta_{m+1} = Linv_{m+1}' z_{m+1}
//   |B|+3 ..       top: theta_m, theta_{m-1}, .., theta_0;  bottom (one step
//                  later, once theta_m is known): theta_{m+2} .. theta_{K-1}
// Coefficients, tau and w are prefetched kPre positions ahead as in
// sweep_row; the middle rows' coefficients sit in registers from the start.
template <typename T, int NS, int R>
__device__ __forceinline__ void sweep_twisted(const Dims& D, const OpCoef<T>& C,
                                              int cls, int v, int lane, int t,
                                              bool act, bool top,
                                              __amdgpu_buffer_rsrc_t rtau,
                                              __amdgpu_buffer_rsrc_t rout,
                                              T (*zo)[2 * NS][kWave],
                                              T (*zx)[2 * NS][kWave]) {
  constexpr int NB = 2 * NS;
  constexpr int NT = R + 1;
  constexpr int ES = sizeof(T);
  constexpr int FD = kFwRow * ES / 4, BD = kBwRow * ES / 4;
  const int K = D.K;
  const int m = (K - 2) / 2, nbot = K - 2 - m, pad = nbot - m;
  const int len = top ? m + 1 : nbot + 1;  // chain positions, middle row last
  const int rbase = top ? 0 : K - 1, rdir = top ? 1 : -1;
  const unsigned istride = (unsigned)(NS * D.ldt * ES);
  auto roff = [&](int k) { return (unsigned)(rbase + rdir * k) * istride; };
  unsigned rb[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c)
    rb[c] = act ? (unsigned)((((size_t)(2 * v + c / NS) * K * NS + (c % NS)) * D.ldt + t) * ES)
                : kOob;
  const unsigned ro = act ? (unsigned)((((size_t)(2 * v + R / NS) * K * NS + (R % NS)) * D.ldt + t) * ES)
                          : kOob;
  const size_t cv = (size_t)cls * D.V + v;
  gptr<const unsigned> fw = glob(reinterpret_cast<const unsigned*>(
      C.Fw + ((cv * fw_rows(K) + (top ? 0 : m + 2)) * NB + R) * kFwRow));
  gptr<const unsigned> bw = glob(reinterpret_cast<const unsigned*>(
      C.Bw + ((cv * K + (top ? 0 : m + 1)) * NB + R) * kBwRow));
  const size_t fstep = (size_t)NB * FD, bstep = (size_t)NB * BD;
  CoefRow<T, kFwRow> cx, cmid, clast;
  cx.load(glob(reinterpret_cast<const unsigned*>(C.Xw + (cv * NB + R) * kFwRow)), lane);
  cmid.load(fw + (size_t)(len - 1) * fstep, lane);
  clast.load(fw + (size_t)len * fstep, lane);

  // ---------------------------------------------------------- forward
  const int fso = top ? pad : 0;  // step of position 0
  for (int u = 0; u < fso; ++u) lds_barrier();
  T z1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) z1[b] = T(0);
  CoefRow<T, kFwRow> cring[kPre];
  T tring[kPre][NT];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    cring[u].load(fw + (size_t)min(u, len) * fstep, lane);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[u][c] = buf_ld<T>(rtau, rb[c] + roff(min(u, len - 1)));
  }
  T pre = T(0);
  sfor<0, R + 1>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    pre = fma(cring[0].template get<16 + c>(), tring[0][c], pre);
  });
#pragma unroll
  for (int c = 0; c < NT; ++c) tring[0][c] = buf_ld<T>(rtau, rb[c] + roff(min(kPre, len - 1)));
  auto w_of = [&](const CoefRow<T, kFwRow>& cf, const T* z) {  // row R of Linv' z
    T acc = T(0);
    sfor<R, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      acc = fma(cf.template get<24 + c>(), z[c], acc);
    });
    return acc;
  };
  auto fstep_body = [&](int i, int s, int sn, bool has_prev) {
    const CoefRow<T, kFwRow> cf = cring[s];
    T zi = pre;
    if (has_prev) {
      T e0 = T(0), e1 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c % 2 == 0) e0 = fma(cf.template get<c>(), z1[c], e0);
        else e1 = fma(cf.template get<c>(), z1[c], e1);
      });
      zi = pre - (e0 + e1);
    }
    zo[(i + fso) & 1][R][lane] = zi;
    if (has_prev) buf_st(rout, ro + roff(i - 1), w_of(cf, z1));
    {
      const CoefRow<T, kFwRow>& cn = cring[sn];
      T a0 = T(0), a2 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c <= R) a0 = fma(cn.template get<16 + c>(), tring[sn][c], a0);
        a2 = fma(cn.template get<8 + c>(), z1[c], a2);
      });
      pre = a0 - a2;
    }
    cring[s].load(fw + (size_t)min(i + kPre, len) * fstep, lane);
    const int it = min(i + 1 + kPre, len - 1);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[sn][c] = buf_ld<T>(rtau, rb[c] + roff(it));
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) z1[b] = zo[(i + fso) & 1][b][lane];
  };
  fstep_body(0, 0, 1, false);
  int i = 1;
  for (; i + kPre <= len - 1; i += kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) fstep_body(i + u, (1 + u) % kPre, (2 + u) % kPre, true);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (i + u < len - 1) fstep_body(i + u, (1 + u) % kPre, (2 + u) % kPre, true);

  // ---------------------------------------------------------- middle rows
  const int sm = nbot;  // step of z_m
  T zy[NB];
  if (top) {
#pragma unroll
    for (int b = 0; b < NB; ++b) zy[b] = zx[(sm - 1) & 1][b][lane];  // z_{m+2}
    T e0 = T(0), e1 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      e0 = fma(cmid.template get<c>(), z1[c], e0);
      e1 = fma(cx.template get<c>(), zy[c], e1);
    });
    zo[sm & 1][R][lane] = pre - (e0 + e1);
    buf_st(rout, ro + roff(len - 2), w_of(cmid, z1));  // w_{m-1}
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) z1[b] = zo[sm & 1][b][lane];
    buf_st(rout, ro + roff(len - 1), w_of(clast, z1));  // w_m
    lds_barrier();
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) zy[b] = zx[(sm - 1) & 1][b][lane];  // z_{m-1}
    T e0 = T(0), e1 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      e0 = fma(cmid.template get<c>(), z1[c], e0);
      e1 = fma(cx.template get<8 + c>(), zy[c], e1);
    });
    pre -= e0 + e1;
    buf_st(rout, ro + roff(len - 2), w_of(cmid, z1));  // w_{m+2}
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) zy[b] = zx[sm & 1][b][lane];  // z_m
    T e2 = T(0), e3 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c % 2 == 0) e2 = fma(cx.template get<16 + c>(), zy[c], e2);
      else e3 = fma(cx.template get<16 + c>(), zy[c], e3);
    });
    zo[(sm + 1) & 1][R][lane] = pre - (e2 + e3);
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) z1[b] = zo[(sm + 1) & 1][b][lane];  // z_{m+1}
    const T th = w_of(clast, z1);  // theta_{m+1}
    zo[(sm + 2) & 1][R][lane] = th;
    buf_st(rout, ro + roff(len - 1), th);
  }
  lds_barrier();  // step sm + 2

  // ---------------------------------------------------------- backward
  // Backward step kk handles position bs - kk: theta = q - N1 theta_next,
  // with q = w - N2 theta_next_next prepared one step earlier.
  T t1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) t1[b] = (top ? zx : zo)[(sm + 2) & 1][b][lane];  // theta_{m+1}
  const int bs = top ? len - 1 : len - 2, cnt = bs + 1;
  const int bso = top ? sm + 3 : sm + 4;  // step of backward step 0
  CoefRow<T, kBwRow> bring[kPre];
  T wring[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int iu = max(bs - u, 0);
    bring[u].load(bw + (size_t)iu * bstep, lane);
    wring[u] = buf_ld<T>(rout, ro + roff(iu));
  }
  T q = wring[0];
  wring[0] = buf_ld<T>(rout, ro + roff(max(bs - kPre, 0)));
  auto bstep_body = [&](int kk, int s, int sn) {
    const int p = bs - kk;
    const CoefRow<T, kBwRow> cb = bring[s];
    T e0 = T(0), e1 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c % 2 == 0) e0 = fma(cb.template get<c>(), t1[c], e0);
      else e1 = fma(cb.template get<c>(), t1[c], e1);
    });
    const T th = q - (e0 + e1);
    zo[(kk + bso) & 1][R][lane] = th;
    buf_st(rout, ro + roff(p), th);
    {
      const CoefRow<T, kBwRow>& cn = bring[sn];
      T a2 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        a2 = fma(cn.template get<8 + c>(), t1[c], a2);
      });
      q = wring[sn] - a2;
    }
    bring[s].load(bw + (size_t)max(p - kPre, 0) * bstep, lane);
    wring[sn] = buf_ld<T>(rout, ro + roff(max(p - 1 - kPre, 0)));
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) t1[b] = zo[(kk + bso) & 1][b][lane];
  };
  if (!top) {  // step sm + 3: wait for theta_m, then fold N2 theta_m into q
    lds_barrier();
#pragma unroll
    for (int b = 0; b < NB; ++b) zy[b] = zx[(sm + 3) & 1][b][lane];
    T a2 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      a2 = fma(bring[0].template get<8 + c>(), zy[c], a2);
    });
    q -= a2;
  }
  bstep_body(0, 0, 1);
  int kk = 1;
  for (; kk + kPre <= cnt; kk += kPre) {
#pragma unroll
    for (int u = 0; u < kPre; ++u) bstep_body(kk + u, (1 + u) % kPre, (2 + u) % kPre);
  }
#pragma unroll
  for (int u = 0; u < kPre - 1; ++u)
    if (kk + u < cnt) bstep_body(kk + u, (1 + u) % kPre, (2 + u) % kPre);
  for (int u = 0; u < (top ? pad : 0); ++u) lds_barrier();
  lds_barrier();  // every wavefront is done reading the buffers
}

template <typename T, int NS, int R = 0>
__device__ __forceinline__ void twisted_dispatch(int w, const Dims& D,
                                                 const OpCoef<T>& C, int cls,
                                                 int v, int lane, int t, bool act,
                                                 bool top,
                                                 __amdgpu_buffer_rsrc_t rtau,
                                                 __amdgpu_buffer_rsrc_t rout,
                                                 T (*zo)[2 * NS][kWave],
                                                 T (*zx)[2 * NS][kWave]) {
  if constexpr (R < 2 * NS) {
    if (w == R)
      sweep_twisted<T, NS, R>(D, C, cls, v, lane, t, act, top, rtau, rout, zo, zx);
    else
      twisted_dispatch<T, NS, R + 1>(w, D, C, cls, v, lane, t, act, top, rtau, rout, zo, zx);
  }
}

// out = Phi~^-1 tau for super-column v and time steps 64 chunk .. 64 chunk
// + 63, by one workgroup of 2n wavefronts (zb: the workgroup's LDS exchange
// buffer).  t = 0: Phi_bar_{v,0} = blkdiag(Q^-1), so theta = Q tau per node.
// t = T uses the second factor class when Q_T != Q.
template <typename T, int NS>
__device__ __forceinline__ void phi_tile(const Dims& D, const OpCoef<T>& C,
                                         const T* __restrict__ tau,
                                         T* __restrict__ out, int qt_distinct,
                                         int v, int chunk,
                                         T (*zb)[2 * NS][kWave]) {
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
    gptr<const T> tg = glob(tau);
    gptr<T> og = glob(out);
    for (int i = lane; i < D.K; i += kWave) {
      const int p = (2 * v + h) * D.K + i;
      gptr<const T> Qp = glob(C.Qm) + p * nn + a * NS;  // per-lane rows
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NS; ++b)
        acc = fma(Qp[b], tg[((size_t)p * NS + b) * D.ldt], acc);
      og[((size_t)p * NS + a) * D.ldt] = acc;
    }
  }
}

// phi_tile with the twisted factor: 4n wavefronts per workgroup, zb holds
// the two halves' exchange buffers.
template <typename T, int NS>
__device__ __forceinline__ void phi_tile_twisted(const Dims& D, const OpCoef<T>& C,
                                                 const T* __restrict__ tau,
                                                 T* __restrict__ out, int qt_distinct,
                                                 int v, int chunk,
                                                 T (*zb)[2][2 * NS][kWave]) {
  constexpr int NB = 2 * NS;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x >> 6);
  const bool top = w < NB;
  const int R = top ? w : w - NB;
  const int t0 = chunk * kWave;
  const int t = t0 + lane;
  const int T_ = D.T;
  const bool valid = t < D.Tt;
  const long long bytes = D.vlen * (long long)sizeof(T);
  const __amdgpu_buffer_rsrc_t rtau = make_rsrc(tau, bytes);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out, bytes);
  T(*zo)[NB][kWave] = zb[top ? 0 : 1];
  T(*zx)[NB][kWave] = zb[top ? 1 : 0];
  twisted_dispatch<T, NS>(R, D, C, 0, v, lane, t,
                          valid && t >= 1 && !(qt_distinct && t == T_), top, rtau, rout,
                          zo, zx);
  if (qt_distinct && t0 <= T_ && T_ < t0 + kWave)
    twisted_dispatch<T, NS>(R, D, C, 1, v, lane, t, valid && t == T_, top, rtau, rout, zo,
                            zx);
  if (chunk == 0) {  // t = 0: theta = Q tau per node, block rows split over the halves
    const size_t nn = (size_t)NS * NS;
    const int h = R / NS, a = R % NS;
    gptr<const T> tg = glob(tau);
    gptr<T> og = glob(out);
    for (int i = lane + (top ? 0 : kWave); i < D.K; i += 2 * kWave) {
      const int p = (2 * v + h) * D.K + i;
      gptr<const T> Qp = glob(C.Qm) + p * nn + a * NS;
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < NS; ++b)
        acc = fma(Qp[b], tg[((size_t)p * NS + b) * D.ldt], acc);
      og[((size_t)p * NS + a) * D.ldt] = acc;
    }
  }
}

}  // namespace dev
}  // namespace lqg
