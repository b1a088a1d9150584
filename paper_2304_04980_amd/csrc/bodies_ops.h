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
// The same with a wave-uniform byte offset in the instruction's scalar
// offset field (no per-lane address arithmetic).
template <typename T>
__device__ __forceinline__ T buf_lds(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double buf_lds<double>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                  unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_lds<float>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_sts(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                        double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_sts(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                        float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
// Compile-time loop: f(std::integral_constant<int, k>) for k = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// acc + (or -) c * z where c is lane L of the lane's own 16-lane row of
// register c (DPP row_newbcast folded into the FMA).  The compiler emits a
// separate v_mov_b32_dpp for the broadcast and has no 64-bit form, so these
// are inline assembly; the registers read through DPP are only ever written
// by vector-memory loads (no VALU write within the DPP wait states), which a
// check over the generated code (check_dpp.py) confirms.
template <int L, bool NEG>
__device__ __forceinline__ float dpp_fmac(float acc, float c, float z) {
  if constexpr (NEG)
    asm("v_fmac_f32_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc) : "v"(c), "v"(z), "n"(L));
  else
    asm("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc) : "v"(c), "v"(z), "n"(L));
  return acc;
}
template <int L, bool NEG>
__device__ __forceinline__ double dpp_fmac(double acc, double c, double z) {
  if constexpr (NEG)
    asm("v_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc) : "v"(c), "v"(z), "n"(L));
  else
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(acc) : "v"(c), "v"(z), "n"(L));
  return acc;
}

// NW wave-uniform coefficients (a node's operator blocks), held 16 per
// register: lane l of register k holds coefficient 16 k + l mod 16.  Loaded
// by one vector load per 16 coefficients, all issued together (the scalar
// loads they replace are L2 misses that a wavefront otherwise waits for one
// block at a time).  Coefficients past NW read whatever follows (or zero out
// of range) and are never used.
template <typename T, int NW>
struct NodeBlocks {
  static constexpr int kRegs = (NW + 15) / 16;
  T g[kRegs];
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, unsigned base, int lane) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k)
      g[k] = buf_lds<T>(rs, (unsigned)((16 * k + (lane & 15)) * sizeof(T)), base);
  }
  // acc +=/-= M x, M the NS x NS row-major block starting at coefficient J0
  template <int J0, bool NEG, int NS>
  __device__ __forceinline__ void mv(const T (&x)[NS], T (&acc)[NS]) const {
    sfor<0, NS>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      sfor<0, NS>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        constexpr int J = J0 + a * NS + b;
        acc[a] = dpp_fmac<J & 15, NEG>(acc[a], g[J >> 4], x[b]);
      });
    });
  }
};
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const T* base, long long count) {
  return make_rsrc(base, count * (long long)sizeof(T));
}

// A node's operator blocks as the stencil tiles apply them: in registers
// through DPP-broadcast FMAs for FP32 (NodeBlocks), through the scalar cache
// for FP64 (whose register copy costs more occupancy than it saves latency).
// count: number of T in the whole array; base: first coefficient of node p.
template <typename T, int NW>
struct TileBlocks;
template <int NW>
struct TileBlocks<float, NW> {
  NodeBlocks<float, NW> b;
  __device__ __forceinline__ void load(const float* arr, long long count, long long first,
                                       int lane) {
    b.load(block_rsrc(arr, count), (unsigned)(first * sizeof(float)), lane);
  }
  template <int J0, bool NEG, int NS>
  __device__ __forceinline__ void mv(const float (&x)[NS], float (&acc)[NS]) const {
    b.template mv<J0, NEG>(x, acc);
  }
};
template <int NW>
struct TileBlocks<double, NW> {
  const double* m;
  __device__ __forceinline__ void load(const double* arr, long long, long long first, int) {
    m = arr + first;
  }
  template <int J0, bool NEG, int NS>
  __device__ __forceinline__ void mv(const double (&x)[NS], double (&acc)[NS]) const {
    if constexpr (NEG) mv_sub<NS>(m + J0, x, acc);
    else mv_add<NS>(m + J0, x, acc);
  }
};

// Node tiles: 4 nodes (one per wavefront of a 256-thread workgroup) x time
// chunks c0 .. c1-1 of 64 consecutive steps (one per lane).  Group g covers
// nodes 4 g .. 4 g + 3 and t = 64 c .. 64 c + 63 for each chunk c.  A
// wavefront that runs several chunks of its node reloads the node's operator
// blocks from the scalar cache rather than from L2.
__host__ __device__ inline int node_groups(const Dims& D) {
  return (D.real_nodes + 3) / 4;
}
__host__ __device__ inline int time_chunks(const Dims& D) {
  return (D.Tt + kWave - 1) / kWave;
}
__device__ __forceinline__ int tile_node(int group) {
  return uniform(group * 4 + (threadIdx.x >> 6));
}

// The NS components of node q at the lane's time offset toff (bytes), by
// buffer loads whose node offset is wave-uniform (scalar offset field).
template <int NS, typename T>
__device__ __forceinline__ void load_nb(__amdgpu_buffer_rsrc_t r, unsigned toff, int q,
                                        int ldt, T (&x)[NS]) {
  const unsigned base = (unsigned)q * (unsigned)(NS * ldt * sizeof(T));
#pragma unroll
  for (int c = 0; c < NS; ++c)
    x[c] = buf_lds<T>(r, toff, base + (unsigned)(c * ldt * sizeof(T)));
}
template <int NS, typename T>
__device__ __forceinline__ void store_nb(__amdgpu_buffer_rsrc_t r, unsigned toff, int q,
                                         int ldt, const T (&x)[NS]) {
  const unsigned base = (unsigned)q * (unsigned)(NS * ldt * sizeof(T));
#pragma unroll
  for (int c = 0; c < NS; ++c) buf_sts(r, toff, base + (unsigned)(c * ldt * sizeof(T)), x[c]);
}
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const Dims& D, const T* v) {
  return make_rsrc(v, D.vlen * (long long)sizeof(T));
}

// Per-lane time offsets of a tile row: every lane (also those past the last
// step) stays active so that the DPP-broadcast FMAs read valid source lanes;
// loads use time indices clamped into [0, Tt), so every access lies inside
// its row (finite data), terms outside their time range are masked by
// selects, and results of lanes past Tt are discarded by the stores.
struct TileTime {
  int t;               // this lane's time step
  bool valid;          // t < Tt
  unsigned off, prev, next;  // byte offsets of min(t, Tt-1) and its clamped neighbours
};
template <typename T>
__device__ __forceinline__ TileTime tile_time(const Dims& D, int chunk) {
  TileTime r;
  r.t = chunk * kWave + (threadIdx.x & (kWave - 1));
  r.valid = r.t < D.Tt;
  const int tl = min(r.t, D.Tt - 1);
  r.off = (unsigned)tl * sizeof(T);
  r.prev = (unsigned)max(tl - 1, 0) * sizeof(T);
  r.next = (unsigned)min(tl + 1, D.Tt - 1) * sizeof(T);
  return r;
}
template <int NS, typename T>
__device__ __forceinline__ void zero_unless(bool keep, T (&x)[NS]) {
#pragma unroll
  for (int c = 0; c < NS; ++c) x[c] = keep ? x[c] : T(0);
}

// ---------------------------------------------------------------------------
// y = Delta d on one node tile (one time chunk); the tile's FP64 partial sum
// of y'd is written to *partial (when non-null) by thread 0.  Every thread of
// the workgroup must call this (it contains a workgroup reduction).
//   y_t(p) = Q_t^-1 d_t(p)
//          + [t>=1] ( sum_13 G[p][k] d_t(p+o_k) - sum_5 Cdn[p][k] d_{t-1}(p+o_k) )
//          - [t<T]  sum_5 Cup[p][k] d_{t+1}(p+o_k)
// The node's 25 operator blocks are applied through TileBlocks.
template <typename T, int NS>
__device__ __forceinline__ void delta_tile(const Dims& D, const OpCoef<T>& C,
                                           const T* __restrict__ d,
                                           T* __restrict__ y,
                                           double* __restrict__ partial,
                                           int group, int chunk) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  double dot = 0.0;
  if (p < D.real_nodes) {  // wave-uniform
    const int j = uniform(p / K), i = uniform(p - (p / K) * K);
    const long long nodes = D.nodes;
    TileBlocks<T, 13 * nn> G;
    TileBlocks<T, 5 * nn> Cd, Cu;
    TileBlocks<T, nn> Qi, Qd;
    G.load(C.G13, nodes * 13 * nn, (long long)p * 13 * nn, lane);
    Cd.load(C.Cdn, nodes * 5 * nn, (long long)p * 5 * nn, lane);
    Cu.load(C.Cup, nodes * 5 * nn, (long long)p * 5 * nn, lane);
    Qi.load(C.Qi, nodes * nn, (long long)p * nn, lane);
    Qd.load(C.QTd, nodes * nn, (long long)p * nn, lane);
    const __amdgpu_buffer_rsrc_t rd = vec_rsrc(D, d), ry = vec_rsrc(D, y);
    const TileTime tt = tile_time<T>(D, chunk);
    T self[NS], acc[NS], nb[NS], sq[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = T(0);
    load_nb<NS>(rd, tt.off, p, ldt, self);
    Qi.template mv<0, false>(self, acc);
#pragma unroll
    for (int c = 0; c < NS; ++c) sq[c] = self[c];
    zero_unless<NS>(tt.t == T_, sq);
    Qd.template mv<0, false>(sq, acc);
    sfor<0, 13>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) return;
      load_nb<NS>(rd, tt.off, jq * K + iq, ldt, nb);
      zero_unless<NS>(tt.t >= 1, nb);
      G.template mv<k * nn, false>(nb, acc);
    });
    sfor<0, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) return;
      load_nb<NS>(rd, tt.prev, jq * K + iq, ldt, nb);
      zero_unless<NS>(tt.t >= 1, nb);
      Cd.template mv<k * nn, true>(nb, acc);
      load_nb<NS>(rd, tt.next, jq * K + iq, ldt, nb);
      zero_unless<NS>(tt.t < T_, nb);
      Cu.template mv<k * nn, true>(nb, acc);
    });
    store_nb<NS>(ry, tt.valid ? tt.off : kOob, p, ldt, acc);
    if (tt.valid) {
#pragma unroll
      for (int a = 0; a < NS; ++a) dot = fma((double)acc[a], (double)self[a], dot);
    }
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
                                           T* __restrict__ tau, int group, int c0,
                                           int c1) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  if (p >= D.real_nodes) return;  // wave-uniform
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  TileBlocks<T, 13 * nn> G;
  G.load(C.G13, (long long)D.nodes * 13 * nn, (long long)p * 13 * nn, lane);
  const __amdgpu_buffer_rsrc_t rth = vec_rsrc(D, th), rtau = vec_rsrc(D, tau);
  const __amdgpu_buffer_rsrc_t rrho = vec_rsrc(D, rho ? rho : th);
  // the five 13-point offsets that leave the super-column: (0, -2) and
  // (0, +2) always, and the three of dj = -1 (left column of its pair) or
  // dj = +1 (right column)
  const bool left = (j & 1) == 0;
  for (int chunk = c0; chunk < c1; ++chunk) {
    const TileTime tt = tile_time<T>(D, chunk);
    T acc[NS], a1[NS];
    if (rho) load_nb<NS>(rrho, tt.off, p, ldt, acc);
    else
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[a] = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a) a1[a] = T(0);
    auto apply = [&](auto side) {
      constexpr int sgn = decltype(side)::value;  // -1: left column, +1: right
      constexpr int ks[5] = {off13_index(0, -2), off13_index(0, 2), off13_index(-1, sgn),
                             off13_index(0, sgn), off13_index(1, sgn)};
      T nb[5][NS];
      sfor<0, 5>([&](auto uc) {  // every neighbour's loads first
        constexpr int k = ks[decltype(uc)::value];
        const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
        const bool in = iq >= 0 && iq < K && jq >= 0 && jq < N;
        load_nb<NS>(rth, in ? tt.off : kOob, in ? jq * K + iq : 0, ldt, nb[decltype(uc)::value]);
      });
      sfor<0, 5>([&](auto uc) {
        constexpr int k = ks[decltype(uc)::value];
        G.template mv<k * nn, true>(nb[decltype(uc)::value], a1);
      });
    };
    if (left) apply(std::integral_constant<int, -1>{});
    else apply(std::integral_constant<int, 1>{});
    zero_unless<NS>(tt.t >= 1, a1);
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] += a1[a];
    store_nb<NS>(rtau, tt.valid ? tt.off : kOob, p, ldt, acc);
  }
}

// rho = r + Xi~ dl on one node tile, Xi~ = Psi~ - Delta:
//   (Xi~ dl)_t(p) = [t>=1] sum_5 Cdn[p][k] dl_{t-1}(q) + [t<T] sum_5 Cup[p][k] dl_{t+1}(q)
// r may be null (zero).
template <typename T, int NS>
__device__ __forceinline__ void xi_tile(const Dims& D, const OpCoef<T>& C,
                                        const T* __restrict__ r,
                                        const T* __restrict__ dl,
                                        T* __restrict__ rho, int group, int c0,
                                        int c1) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  if (p >= D.real_nodes) return;  // wave-uniform
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  TileBlocks<T, 5 * nn> Cd, Cu;
  Cd.load(C.Cdn, (long long)D.nodes * 5 * nn, (long long)p * 5 * nn, lane);
  Cu.load(C.Cup, (long long)D.nodes * 5 * nn, (long long)p * 5 * nn, lane);
  const __amdgpu_buffer_rsrc_t rdl = vec_rsrc(D, dl), rrho = vec_rsrc(D, rho);
  const __amdgpu_buffer_rsrc_t rr = vec_rsrc(D, r ? r : dl);
  for (int chunk = c0; chunk < c1; ++chunk) {
    const TileTime tt = tile_time<T>(D, chunk);
    T acc[NS], a1[NS], a2[NS], nb[NS];
    if (r) load_nb<NS>(rr, tt.off, p, ldt, acc);
    else
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[a] = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a) a1[a] = a2[a] = T(0);
    sfor<0, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) return;
      load_nb<NS>(rdl, tt.prev, jq * K + iq, ldt, nb);
      Cd.template mv<k * nn, false>(nb, a1);
      load_nb<NS>(rdl, tt.next, jq * K + iq, ldt, nb);
      Cu.template mv<k * nn, false>(nb, a2);
    });
    zero_unless<NS>(tt.t >= 1, a1);
    zero_unless<NS>(tt.t < T_, a2);
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] += a1[a] + a2[a];
    store_nb<NS>(rrho, tt.valid ? tt.off : kOob, p, ldt, acc);
  }
}

// Whole-wavefront lane moves (DPP wave_shr / wave_shl / wave_ror /
// wave_rol by one lane); a 64-bit value moves as two 32-bit halves.  A lane
// whose source lies outside the wavefront keeps `old`.
constexpr int kWaveShl1 = 0x130, kWaveRol1 = 0x134, kWaveShr1 = 0x138, kWaveRor1 = 0x13C;
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float old, float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double old, double x) {
  const long long o = __double_as_longlong(old), v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, 0xf, 0xf, false);
  const int hi =
      __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// lane l <- x[l-1]; lane 0 <- prev[63]
template <typename T>
__device__ __forceinline__ T from_prev_lane(T x, T prev) {
  return dpp_mov<kWaveShr1>(dpp_mov<kWaveRor1>(prev, prev), x);
}
// lane l <- x[l+1]; lane 63 <- next[0]
template <typename T>
__device__ __forceinline__ T from_next_lane(T x, T next) {
  return dpp_mov<kWaveShl1>(dpp_mov<kWaveRol1>(next, next), x);
}

// rho = r + Xi~ dl for one node over all its time chunks.  The 5-point
// blocks do not depend on t, so with W_t = sum_5 Cdn[p][k] dl_t(q) and
// V_t = sum_5 Cup[p][k] dl_t(q) the right-hand side is
// [t>=1] W_{t-1} + [t<T] V_{t+1}: one aligned read of each neighbour per
// chunk forms W and V, which reach the lanes of t+1 and t-1 by lane moves; the
// chunk boundaries take lane 63 of the previous chunk's W and lane 0 of the
// next chunk's V, computed one chunk ahead.  Same terms and order as
// xi_tile, so the same sums.
template <typename T, int NS>
__device__ __forceinline__ void xi_rows(const Dims& D, const OpCoef<T>& C,
                                        const T* __restrict__ r,
                                        const T* __restrict__ dl,
                                        T* __restrict__ rho, int group) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  if (p >= D.real_nodes) return;  // wave-uniform
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  TileBlocks<T, 5 * nn> Cd, Cu;
  Cd.load(C.Cdn, (long long)D.nodes * 5 * nn, (long long)p * 5 * nn, lane);
  Cu.load(C.Cup, (long long)D.nodes * 5 * nn, (long long)p * 5 * nn, lane);
  const __amdgpu_buffer_rsrc_t rdl = vec_rsrc(D, dl), rrho = vec_rsrc(D, rho);
  const __amdgpu_buffer_rsrc_t rr = vec_rsrc(D, r ? r : dl);
  const int nc = time_chunks(D);
  auto prod = [&](int c, T(&W)[NS], T(&V)[NS]) {
    const unsigned off = (unsigned)min(c * kWave + lane, D.Tt - 1) * sizeof(T);
#pragma unroll
    for (int a = 0; a < NS; ++a) W[a] = V[a] = T(0);
    // every neighbour's loads first (out-of-grid ones read as zero through an
    // out-of-range offset; their blocks are zero), then the products
    T nb[5][NS];
    sfor<0, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      const bool in = iq >= 0 && iq < K && jq >= 0 && jq < N;
      load_nb<NS>(rdl, in ? off : kOob, in ? jq * K + iq : 0, ldt, nb[k]);
    });
    sfor<0, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      Cd.template mv<k * nn, false>(nb[k], W);
      Cu.template mv<k * nn, false>(nb[k], V);
    });
  };
  T Wp[NS], W[NS], V[NS], Wn[NS], Vn[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) Wp[a] = T(0);
  prod(0, W, V);
  for (int c = 0; c < nc; ++c) {
    if (c + 1 < nc) {
      prod(c + 1, Wn, Vn);
    } else {
#pragma unroll
      for (int a = 0; a < NS; ++a) Wn[a] = Vn[a] = T(0);
    }
    const TileTime tt = tile_time<T>(D, c);
    T acc[NS], a1[NS], a2[NS];
    if (r) load_nb<NS>(rr, tt.off, p, ldt, acc);
    else
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[a] = T(0);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      a1[a] = from_prev_lane(W[a], Wp[a]);
      a2[a] = from_next_lane(V[a], Vn[a]);
    }
    zero_unless<NS>(tt.t >= 1, a1);
    zero_unless<NS>(tt.t < T_, a2);
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] += a1[a] + a2[a];
    store_nb<NS>(rrho, tt.valid ? tt.off : kOob, p, ldt, acc);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      Wp[a] = W[a];
      W[a] = Wn[a];
      V[a] = Vn[a];
    }
  }
}

constexpr bool five_point_leads_thirteen() {
  for (int k = 0; k < 5; ++k)
    if (kOff5[k][0] != kOff13[k][0] || kOff5[k][1] != kOff13[k][1]) return false;
  return true;
}
static_assert(five_point_leads_thirteen(), "the 5-point offsets lead the 13-point list");

// y = Delta d for one node over all its time chunks (the sum as in
// delta_tile), with the Cdn / Cup terms formed as in xi_rows: the 13 aligned
// neighbour reads of a chunk give sum_13 G d_t(q), W_t = sum_5 Cdn d_t(q) and
// V_t = sum_5 Cup d_t(q), and W_{t-1}, V_{t+1} reach their lanes by lane
// moves, the chunk boundaries from the neighbouring chunks (one chunk ahead).
// The workgroup's FP64 partial of y'd goes to *partial.  Every thread of the
// workgroup must call this.
template <typename T, int NS>
__device__ __forceinline__ void delta_rows(const Dims& D, const OpCoef<T>& C,
                                           const T* __restrict__ d,
                                           T* __restrict__ y,
                                           double* __restrict__ partial, int group) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  double dot = 0.0;
  if (p < D.real_nodes) {  // wave-uniform
    const int j = uniform(p / K), i = uniform(p - (p / K) * K);
    const long long nodes = D.nodes;
    TileBlocks<T, 13 * nn> G;
    TileBlocks<T, 5 * nn> Cd, Cu;
    TileBlocks<T, nn> Qi, Qd;
    G.load(C.G13, nodes * 13 * nn, (long long)p * 13 * nn, lane);
    Cd.load(C.Cdn, nodes * 5 * nn, (long long)p * 5 * nn, lane);
    Cu.load(C.Cup, nodes * 5 * nn, (long long)p * 5 * nn, lane);
    Qi.load(C.Qi, nodes * nn, (long long)p * nn, lane);
    Qd.load(C.QTd, nodes * nn, (long long)p * nn, lane);
    const __amdgpu_buffer_rsrc_t rd = vec_rsrc(D, d), ry = vec_rsrc(D, y);
    const int nc = time_chunks(D);
    struct Prod {
      T self[NS], g[NS], w[NS], v[NS];
    };
    auto prod = [&](int c, Prod& P) {
      const unsigned off = (unsigned)min(c * kWave + lane, D.Tt - 1) * sizeof(T);
#pragma unroll
      for (int a = 0; a < NS; ++a) P.g[a] = P.w[a] = P.v[a] = T(0);
      load_nb<NS>(rd, off, p, ldt, P.self);
      sfor<0, 13>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
        if (iq < 0 || iq >= K || jq < 0 || jq >= N) return;
        T nb[NS];
        if constexpr (k == 0) {
#pragma unroll
          for (int a = 0; a < NS; ++a) nb[a] = P.self[a];
        } else {
          load_nb<NS>(rd, off, jq * K + iq, ldt, nb);
        }
        G.template mv<k * nn, false>(nb, P.g);
        if constexpr (k < 5) {  // the 5-point offsets lead the 13-point list
          Cd.template mv<k * nn, false>(nb, P.w);
          Cu.template mv<k * nn, false>(nb, P.v);
        }
      });
    };
    Prod cur, nxt;
    T wp[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) wp[a] = T(0);
    prod(0, cur);
    for (int c = 0; c < nc; ++c) {
      if (c + 1 < nc) {
        prod(c + 1, nxt);
      } else {
#pragma unroll
        for (int a = 0; a < NS; ++a) nxt.self[a] = nxt.g[a] = nxt.w[a] = nxt.v[a] = T(0);
      }
      const TileTime tt = tile_time<T>(D, c);
      T acc[NS], sq[NS], a1[NS], a2[NS];
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[a] = T(0);
      Qi.template mv<0, false>(cur.self, acc);
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        sq[a] = cur.self[a];
        a1[a] = from_prev_lane(cur.w[a], wp[a]);
        a2[a] = from_next_lane(cur.v[a], nxt.v[a]);
      }
      zero_unless<NS>(tt.t == T_, sq);
      Qd.template mv<0, false>(sq, acc);
      T g[NS];
#pragma unroll
      for (int a = 0; a < NS; ++a) g[a] = cur.g[a] - a1[a];
      zero_unless<NS>(tt.t >= 1, g);
      zero_unless<NS>(tt.t < T_, a2);
#pragma unroll
      for (int a = 0; a < NS; ++a) acc[a] += g[a] - a2[a];
      store_nb<NS>(ry, tt.valid ? tt.off : kOob, p, ldt, acc);
      if (tt.valid) {
#pragma unroll
        for (int a = 0; a < NS; ++a) dot = fma((double)acc[a], (double)cur.self[a], dot);
      }
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        wp[a] = cur.w[a];
        cur.self[a] = nxt.self[a];
        cur.g[a] = nxt.g[a];
        cur.w[a] = nxt.w[a];
        cur.v[a] = nxt.v[a];
      }
    }
  }
  dot = block_sum<256>(dot);
  if (partial && threadIdx.x == 0) *partial = dot;
}

// The factored Delta apply, Delta = A~ Q~^-1 A~' + B~ R~^-1 B~' (Sec. II-B),
// as two passes over the nodes (12 block products per node and step instead
// of the 25 of the assembled 13-point form):
//   w_t(p) = Q_t^-1 (A~'d)_t(p) = -Q_t^-1 d_t(p) + [t<T] sum_5 Cup[p][k] d_{t+1}(q_k)
//   y_t(p) = -w_t(p) + [t>=1] ( sum_5 A5[p][k] w_{t-1}(q_k) + BRB[p] d_t(p) )
// with Cup[p][k] = Q_p^-1 A_hat[q_k,p]' and A5[p][k] = A_hat[p,q_k]; the
// t+1 / t-1 terms are formed at t from aligned reads and moved one lane
// (the chunk boundaries from the neighbouring chunks), as in delta_rows.
// One wavefront per node over all its time chunks.
template <typename T, int NS>
__device__ __forceinline__ void delta_w_rows(const Dims& D, const OpCoef<T>& C,
                                             const T* __restrict__ d, T* __restrict__ w,
                                             int group) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  if (p >= D.real_nodes) return;  // wave-uniform
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  const long long nodes = D.nodes;
  TileBlocks<T, 5 * nn> Cu;
  TileBlocks<T, nn> Qi, Qd;
  Cu.load(C.Cup, nodes * 5 * nn, (long long)p * 5 * nn, lane);
  Qi.load(C.Qi, nodes * nn, (long long)p * nn, lane);
  Qd.load(C.QTd, nodes * nn, (long long)p * nn, lane);
  const __amdgpu_buffer_rsrc_t rd = vec_rsrc(D, d), rw = vec_rsrc(D, w);
  const int nc = time_chunks(D);
  // One chunk's reads: d at the node (nb[0]) and at its four neighbours
  // (out-of-grid neighbours read as zero through an out-of-range offset).
  struct Ld {
    T nb[5][NS];
  };
  auto issue = [&](int c, Ld& L) {
    const unsigned off = (unsigned)min(c * kWave + lane, D.Tt - 1) * sizeof(T);
    load_nb<NS>(rd, off, p, ldt, L.nb[0]);
    sfor<1, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      const bool in = iq >= 0 && iq < K && jq >= 0 && jq < N;
      load_nb<NS>(rd, in ? off : kOob, in ? jq * K + iq : 0, ldt, L.nb[k]);
    });
  };
  struct Prod {
    T self[NS], v[NS];
  };
  auto cup = [&](const Ld& L, Prod& P) {  // V_t = sum_k Cup_k d_t(q_k)
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      P.v[a] = T(0);
      P.self[a] = L.nb[0][a];
    }
    sfor<0, 5>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      Cu.template mv<k * nn, false>(L.nb[k], P.v);
    });
  };
  // w_t = -Q^-1 d_t (- Q_T^-1 d_T at t = T) + V_{t+1}; V_{t+1} of lane 63
  // comes from the next chunk's products (lane move)
  auto finish = [&](int c, const Prod& cur, const Prod& nxt) {
    const TileTime tt = tile_time<T>(D, c);
    T acc[NS], a2[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      acc[a] = T(0);
      a2[a] = from_next_lane(cur.v[a], nxt.v[a]);
    }
    Qi.template mv<0, true>(cur.self, acc);
    if (c == nc - 1) {  // wave-uniform: the chunk holding t = T
      T sq[NS];
#pragma unroll
      for (int a = 0; a < NS; ++a) sq[a] = cur.self[a];
      zero_unless<NS>(tt.t == T_, sq);
      Qd.template mv<0, true>(sq, acc);
    }
    zero_unless<NS>(tt.t < T_, a2);
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] += a2[a];
    store_nb<NS>(rw, tt.valid ? tt.off : kOob, p, ldt, acc);
  };
  Prod zero;
#pragma unroll
  for (int a = 0; a < NS; ++a) zero.self[a] = zero.v[a] = T(0);
  if constexpr (sizeof(T) == 4) {
    // software pipeline over chunks: the reads of chunk c + 2 are issued
    // before the products of chunk c + 1 (whose reads were issued one chunk
    // earlier) and the output of chunk c; two read buffers alternate
    Ld LA, LB;
    Prod P0, P1;
    issue(0, LA);
    if (nc > 1) issue(1, LB);
    cup(LA, P0);
    // on entry Pc holds chunk c's products and X chunk c + 1's reads; Y is free
    auto step = [&](int c, Ld& X, Ld& Y, Prod& Pc, Prod& Pn) {
      if (c + 2 < nc) issue(c + 2, Y);
      if (c + 1 < nc) cup(X, Pn);
      finish(c, Pc, c + 1 < nc ? Pn : zero);
    };
    for (int c = 0; c < nc; c += 2) {
      step(c, LB, LA, P0, P1);
      if (c + 1 >= nc) break;
      step(c + 1, LA, LB, P1, P0);
    }
  } else {
    Ld L;
    Prod cur, nxt;
    issue(0, L);
    cup(L, cur);
    for (int c = 0; c < nc; ++c) {
      if (c + 1 < nc) {
        issue(c + 1, L);
        cup(L, nxt);
      } else {
        nxt = zero;
      }
      finish(c, cur, nxt);
      cur = nxt;
    }
  }
}

// Second pass: y from w and d; the workgroup's FP64 partial of y'd to
// *partial.  Every thread of the workgroup must call this.
template <typename T, int NS>
__device__ __forceinline__ void delta_y_rows(const Dims& D, const OpCoef<T>& C,
                                             const T* __restrict__ d,
                                             const T* __restrict__ w, T* __restrict__ y,
                                             double* __restrict__ partial, int group) {
  constexpr int nn = NS * NS;
  const int p = tile_node(group);
  const int T_ = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const int lane = threadIdx.x & (kWave - 1);
  double dot = 0.0;
  if (p < D.real_nodes) {  // wave-uniform
    const int j = uniform(p / K), i = uniform(p - (p / K) * K);
    const long long nodes = D.nodes;
    TileBlocks<T, 5 * nn> A5;
    TileBlocks<T, nn> Bb;
    A5.load(C.A5, nodes * 5 * nn, (long long)p * 5 * nn, lane);
    Bb.load(C.BRB, nodes * nn, (long long)p * nn, lane);
    const __amdgpu_buffer_rsrc_t rd = vec_rsrc(D, d), rw = vec_rsrc(D, w),
                                 ry = vec_rsrc(D, y);
    const int nc = time_chunks(D);
    // One chunk's reads: d at the node, w at the node (nb[0]) and at its four
    // neighbours (out-of-grid neighbours read as zero).
    struct Ld {
      T self[NS], nb[5][NS];
    };
    auto issue = [&](int c, Ld& L) {
      const TileTime tt = tile_time<T>(D, c);
      load_nb<NS>(rd, tt.off, p, ldt, L.self);
      load_nb<NS>(rw, tt.off, p, ldt, L.nb[0]);
      sfor<1, 5>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
        const bool in = iq >= 0 && iq < K && jq >= 0 && jq < N;
        load_nb<NS>(rw, in ? tt.off : kOob, in ? jq * K + iq : 0, ldt, L.nb[k]);
      });
    };
    T xp[NS];  // the previous chunk's sum_5 A5 w
#pragma unroll
    for (int a = 0; a < NS; ++a) xp[a] = T(0);
    // y_t = (sum_5 A5 w)_{t-1} + B R^-1 B' d_t - w_t  (t >= 1), y_0 = -w_0
    auto body = [&](int c, const Ld& L) {
      const TileTime tt = tile_time<T>(D, c);
      T x[NS], acc[NS], a1[NS];
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        x[a] = T(0);
        acc[a] = T(0);
      }
      sfor<0, 5>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        A5.template mv<k * nn, false>(L.nb[k], x);
      });
      Bb.template mv<0, false>(L.self, acc);
#pragma unroll
      for (int a = 0; a < NS; ++a) a1[a] = from_prev_lane(x[a], xp[a]) + acc[a];
      zero_unless<NS>(tt.t >= 1, a1);
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        acc[a] = a1[a] - L.nb[0][a];
        xp[a] = x[a];
      }
      store_nb<NS>(ry, tt.valid ? tt.off : kOob, p, ldt, acc);
      if (tt.valid) {
#pragma unroll
        for (int a = 0; a < NS; ++a) dot = fma((double)acc[a], (double)L.self[a], dot);
      }
    };
    if constexpr (sizeof(T) == 4) {
      // the reads of chunk c + 1 are issued before the products of chunk c;
      // two read buffers alternate
      Ld LA, LB;
      issue(0, LA);
      for (int c = 0; c < nc; c += 2) {
        if (c + 1 < nc) issue(c + 1, LB);
        body(c, LA);
        if (c + 1 >= nc) break;
        if (c + 2 < nc) issue(c + 2, LA);
        body(c + 1, LB);
      }
    } else {
      Ld L;
      for (int c = 0; c < nc; ++c) {
        issue(c, L);
        body(c, L);
      }
    }
  }
  dot = block_sum<256>(dot);
  if (partial && threadIdx.x == 0) *partial = dot;
}

// One row of NW factor coefficients of a block row, as the sweeps read it:
// lane l holds coefficient 16 g + (l mod 16) in register g, i.e. every 16-lane
// row of the wavefront holds the same 16 coefficients.  The product with
// coefficient j takes it from lane j mod 16 of the lane's own row by a DPP
// row broadcast (row_newbcast) in the FMA itself (v_fmac_f32_dpp,
// v_fmac_f64_dpp through dpp_fmac), so no instruction is spent on moving
// coefficients.
template <typename T, int NW>
struct CoefRow;
template <int NW>
struct CoefRow<double, NW> {
  double g[NW / 16];
  __device__ __forceinline__ void load(gptr<const unsigned> row, int lane) {
    gptr<const double> rd = reinterpret_cast<gptr<const double>>(row);
#pragma unroll
    for (int k = 0; k < NW / 16; ++k) g[k] = rd[16 * k + (lane & 15)];
  }
  template <int J>
  __device__ __forceinline__ double fmac(double acc, double z) const {
    return dpp_fmac<J & 15, false>(acc, g[J >> 4], z);
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
  template <int J>
  __device__ __forceinline__ float fmac(float acc, float z) const {
    return dpp_fmac<J & 15, false>(acc, __builtin_bit_cast(float, g[J >> 4]), z);
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
    pre = cring[0].template fmac<16 + c>(pre, tring[0][c]);
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
        if constexpr (c % 2 == 0) e0 = cf.template fmac<c>(e0, z1[c]);
        else e1 = cf.template fmac<c>(e1, z1[c]);
      });
      zi = pre - (e0 + e1);
    }
    zb[i & 1][R][lane] = zi;
    if (has_prev) {  // w_{i-1} = row R of Linv_{i-1}' z_{i-1} (parked in out)
      T acc = T(0);
      sfor<R, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        acc = cf.template fmac<24 + c>(acc, z1[c]);
      });
      buf_st(rout, ro + (unsigned)(i - 1) * istride, acc);
    }
    {  // p_{i+1} = Linv_{i+1} tau_{i+1} - M2_{i+1} z_{i-1}
      const CoefRow<T, kFwRow>& cn = cring[sn];
      T a0 = T(0), a2 = T(0);
      sfor<0, NB>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c <= R) a0 = cn.template fmac<16 + c>(a0, tring[sn][c]);
        a2 = cn.template fmac<8 + c>(a2, z1[c]);
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
      acc = cf.template fmac<24 + c>(acc, z1[c]);
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
        if constexpr (c % 2 == 0) e0 = cb.template fmac<c>(e0, t1[c]);
        else e1 = cb.template fmac<c>(e1, t1[c]);
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
        a2 = cn.template fmac<8 + c>(a2, t1[c]);
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

// Rows of a block row that one wavefront of the twisted solve handles.
template <int NS>
constexpr int kRowsPerWave = 2;
template <int NS>
constexpr int kWavesPerHalf = 2 * NS / kRowsPerWave<NS>;
// LDS of the twisted solve: the two halves' exchange buffers, and, for FP64,
// in the rest of the 160 KiB of a CU, the last kWKeep<T, NS> positions of
// each chain's parked w (so only the earlier ones make the round trip to
// HBM).  For FP32 the solve is not bound by that traffic and measured faster
// without it (the full-size allocation also limits a CU to one workgroup).
constexpr int kLdsBytes = 160 * 1024;
template <typename T, int NS>
constexpr int kWKeep = sizeof(T) == 4 ? 0
                                      : (kLdsBytes - 2 * 2 * 2 * NS * kWave * (int)sizeof(T)) /
                                                (2 * 2 * NS * kWave * (int)sizeof(T)) -
                                            1;
template <typename T, int NS>
constexpr int kWKeepAlloc = kWKeep<T, NS> + 1;  // + a spare slot

// Forward/backward substitution with the twisted factor of Phi_bar_{v,cls}
// (factor_twisted: block rows ordered [0 .. m-1 | K-1 .. m+2 | m, m+1],
// m = (K-2)/2, |B| = K-2-m bottom rows).  The top chain runs on one half of
// the workgroup's wavefronts, the bottom chain on the other, so the two
// chains proceed side by side and each wavefront passes about K/2 exchange
// barriers per direction instead of K.  A wavefront handles rows R0 ..
// R0+NR-1 of every block row for 64 time steps (one per lane); NR = 4 (n =
// 2, 4) keeps the all-to-all exchange of z through LDS small against the
// arithmetic.  Each half exchanges its z (theta) rows through its own LDS
// buffer `zo`; the two middle block rows read the other half's buffer `zx`.
// The work between barriers b-1 and b is step b, and step b writes slot
// b & 1, so a slot is rewritten only after every reader has passed the next
// barrier.  Steps (both halves pass the same 2 |B| + 5 barriers):
//   0 .. |B|-1     top positions 0 .. m-1 (after |B| - m idle steps),
//                  bottom positions 0 .. |B|-1 (rows K-1 .. m+2)
//   |B|            top: z_m = p_m - M1_m z_{m-1} - X_t z_{m+2};
//                  bottom: p_{m+1} -= M1 z_{m+2} + X_b1 z_{m-1}
//   |B|+1          top: w_m;  bottom: z_{m+1} = p_{m+1} - X_b2 z_m
//   |B|+2          bottom: theta_{m+1} = Linv_{m+1}' z_{m+1}
//   |B|+3 ..       top: theta_m, theta_{m-1}, .., theta_0;  bottom (one step
//                  later, once theta_m is known): theta_{m+2} .. theta_{K-1}
// Software pipelining across the barriers: a step first issues the LDS read
// of the previous position's z (theta), then does the work that does not
// need it -- M2_i z_{i-2}, Linv_{i+1} tau_{i+1}, w_{i-2} = Linv_{i-2}'
// z_{i-2} (backward: w_p - N2_p theta_{p+2}) -- while the read is in flight,
// and only then the product with M1 (N1) that the exchange feeds.
// Coefficient rows and tau are prefetched into register rings (slot =
// position mod ring depth), w into a ring in the backward sweep; the rows
// around the middle sit in registers from the start.  Row offsets go into the
// buffer instructions' scalar offset.
template <typename T, int NS, int R0, int NR>
__device__ __forceinline__ void sweep_twisted(const Dims& D, const OpCoef<T>& C,
                                              int cls, int v, int lane, int t,
                                              bool act, bool top,
                                              __amdgpu_buffer_rsrc_t rtau,
                                              __amdgpu_buffer_rsrc_t rout,
                                              T (*zo)[2 * NS][kWave],
                                              T (*zx)[2 * NS][kWave],
                                              T (*wl)[2 * NS][kWave]) {
  constexpr int NB = 2 * NS;
  constexpr int NT = R0 + NR;  // tau rows that rows R0 .. R0+NR-1 of z need
  // ring depth: coefficient rows are fetched kP - 2 steps before first use
  constexpr int kP = sizeof(T) == 4 ? 6 : 4;
  constexpr int ES = sizeof(T);
  constexpr int FD = kFwRow * ES / 4, BD = kBwRow * ES / 4;
  using Row = CoefRow<T, kFwRow>;
  using BRow = CoefRow<T, kBwRow>;
  using I0 = std::integral_constant<int, 0>;
  using I8 = std::integral_constant<int, 8>;
  const int K = D.K;
  const int m = (K - 2) / 2, nbot = K - 2 - m, pad = nbot - m;
  const int len = top ? m + 1 : nbot + 1;  // chain positions, middle row last
  const int rbase = top ? 0 : K - 1, rdir = top ? 1 : -1;
  const unsigned istride = (unsigned)(NS * D.ldt * ES);
  auto roff = [&](int k) { return (unsigned)(rbase + rdir * k) * istride; };
  auto row_off = [&](int c) {  // byte offset of row c of block row 0 at lane t
    return act ? (unsigned)((((size_t)(2 * v + c / NS) * K * NS + (c % NS)) * D.ldt + t) * ES)
               : kOob;
  };
  unsigned rb[NT], ro[NR];
#pragma unroll
  for (int c = 0; c < NT; ++c) rb[c] = row_off(c);
#pragma unroll
  for (int j = 0; j < NR; ++j) ro[j] = row_off(R0 + j);
  const size_t cv = (size_t)cls * D.V + v;
  gptr<const unsigned> fw = glob(reinterpret_cast<const unsigned*>(
      C.Fw + ((cv * fw_rows(K) + (top ? 0 : m + 2)) * NB + R0) * kFwRow));
  gptr<const unsigned> bw = glob(reinterpret_cast<const unsigned*>(
      C.Bw + ((cv * K + (top ? 0 : m + 1)) * NB + R0) * kBwRow));
  const size_t fstep = (size_t)NB * FD, bstep = (size_t)NB * BD;
  auto load_f = [&](Row* dst, gptr<const unsigned> base) {
#pragma unroll
    for (int j = 0; j < NR; ++j) dst[j].load(base + (size_t)j * FD, lane);
  };
  auto load_b = [&](BRow* dst, gptr<const unsigned> base) {
#pragma unroll
    for (int j = 0; j < NR; ++j) dst[j].load(base + (size_t)j * BD, lane);
  };
  Row cx[NR], cpm[NR], cmid[NR], clast[NR];
  load_f(cx, glob(reinterpret_cast<const unsigned*>(C.Xw + (cv * NB + R0) * kFwRow)));
  load_f(cpm, fw + (size_t)(len - 2) * fstep);
  load_f(cmid, fw + (size_t)(len - 1) * fstep);
  load_f(clast, fw + (size_t)len * fstep);

  auto dot8 = [&](const auto& cf, auto base, const T* z, T acc) {
    constexpr int B0 = decltype(base)::value;
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      acc = cf.template fmac<B0 + c>(acc, z[c]);
    });
    return acc;
  };
  auto dot8x2 = [&](const auto& cf, auto base, const T* z) {  // two chains
    constexpr int B0 = decltype(base)::value;
    T e0 = T(0), e1 = T(0);
    sfor<0, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c % 2 == 0) e0 = cf.template fmac<B0 + c>(e0, z[c]);
      else e1 = cf.template fmac<B0 + c>(e1, z[c]);
    });
    return e0 + e1;
  };
  // row R0+J of Linv' z (upper triangle) and of Linv tau (lower triangle)
  auto w_of = [&](auto jc, const Row& cf, const T* z) {
    constexpr int J = decltype(jc)::value;
    T acc = T(0);
    sfor<R0 + J, NB>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      acc = cf.template fmac<24 + c>(acc, z[c]);
    });
    return acc;
  };
  auto linv_tau = [&](auto jc, const Row& cf, const T* tv) {
    constexpr int J = decltype(jc)::value;
    T acc = T(0);
    sfor<0, R0 + J + 1>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      acc = cf.template fmac<16 + c>(acc, tv[c]);
    });
    return acc;
  };
  auto read_all = [&](T* dst, T (*buf)[kWave]) {
#pragma unroll
    for (int b = 0; b < NB; ++b) dst[b] = buf[b][lane];
  };
  // Parked w of position k, row R0+j: LDS for the last kWKeep positions,
  // else HBM.  Without branches, which would split the pipelined steps: both
  // accesses are issued, the HBM one with an out-of-range offset when the
  // value lives in LDS (store dropped, load returns 0), the LDS one at the
  // spare slot kWKeep when it lives in HBM, and a select picks the result.
  constexpr int kKeep = kWKeep<T, NS>;
  const int kl = max(0, len - kKeep);
  auto put_w = [&](int k, int j, T val) {
    if constexpr (kKeep == 0) {
      buf_sts(rout, ro[j], roff(k), val);
    } else {
      const bool in_lds = k >= kl;
      wl[in_lds ? k - kl : kKeep][R0 + j][lane] = val;
      buf_sts(rout, in_lds ? kOob : ro[j], roff(k), val);
    }
  };
  // The backward sweep's ring of parked w: slot s holds the HBM read (whead)
  // and, with LDS parking, the LDS read (wlds) of its position; the two are
  // selected where the value is used, not where it is fetched, so the select
  // does not wait for the HBM read at once.
  constexpr int kWL = kKeep > 0 ? kP : 1;
  T whead[kP][NR], wlds[kWL][NR];
  auto fetch_w = [&](int s, int k) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if constexpr (kKeep == 0) {
        whead[s][j] = buf_lds<T>(rout, ro[j], roff(k));
      } else {
        const bool in_lds = k >= kl;
        wlds[s][j] = wl[in_lds ? k - kl : kKeep][R0 + j][lane];
        whead[s][j] = buf_lds<T>(rout, in_lds ? kOob : ro[j], roff(k));
      }
    }
  };
  auto wval = [&](int s, int k, int j) {  // parked w of position k, row R0+j, from slot s
    if constexpr (kKeep == 0) return whead[s][j];
    else return k >= kl ? wlds[s][j] : whead[s][j];
  };

  // ---------------------------------------------------------- forward
  const int fso = top ? pad : 0;  // step of position 0
  for (int u = 0; u < fso; ++u) lds_barrier();
  T z2[NB], zn[NB], a[NR];
#pragma unroll
  for (int b = 0; b < NB; ++b) z2[b] = T(0);
  Row cring[kP][NR];
  T tring[kP][NT];
#pragma unroll
  for (int u = 0; u < kP; ++u) {
    load_f(cring[u], fw + (size_t)min(u, len) * fstep);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[u][c] = buf_lds<T>(rtau, rb[c], roff(min(u, len - 1)));
  }
  // position 0: z_0 = Linv_0 tau_0; then a = Linv_1 tau_1
  sfor<0, NR>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    zo[fso & 1][R0 + j][lane] = linv_tau(jc, cring[0][j], tring[0]);
    a[j] = linv_tau(jc, cring[1][j], tring[1]);
  });
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    tring[0][c] = buf_lds<T>(rtau, rb[c], roff(min(kP, len - 1)));
    tring[1][c] = buf_lds<T>(rtau, rb[c], roff(min(kP + 1, len - 1)));
  }
  lds_barrier();
  // Standard position i >= 1 (sp, s, sn: ring slots of rows i-1, i, i+1).
  // park: i >= 2 (w_{i-2} exists), a compile-time flag so that the steps of
  // the unrolled loop have no branch (a branch would make the compiler's
  // wait counts on the prefetched loads conservative).
  auto fstep_body = [&](int i, int sp, int s, int sn, auto park) {
    read_all(zn, zo[(i - 1 + fso) & 1]);  // z_{i-1}
    T pre[NR], an[NR];
    sfor<0, NR>([&](auto jc) {  // independent of z_{i-1}
      constexpr int j = decltype(jc)::value;
      pre[j] = a[j] - dot8(cring[s][j], I8{}, z2, T(0));
      if constexpr (decltype(park)::value) put_w(i - 2, j, w_of(jc, cring[sp][j], z2));
      an[j] = linv_tau(jc, cring[sn][j], tring[sn]);
    });
    sfor<0, NR>([&](auto jc) {  // z_i = Linv_i tau_i - M2_i z_{i-2} - M1_i z_{i-1}
      constexpr int j = decltype(jc)::value;
      zo[(i + fso) & 1][R0 + j][lane] = pre[j] - dot8x2(cring[s][j], I0{}, zn);
      a[j] = an[j];
    });
#pragma unroll
    for (int b = 0; b < NB; ++b) z2[b] = zn[b];
    load_f(cring[sp], fw + (size_t)min(i - 1 + kP, len) * fstep);
    const int it = min(i + 1 + kP, len - 1);
#pragma unroll
    for (int c = 0; c < NT; ++c) tring[sn][c] = buf_lds<T>(rtau, rb[c], roff(it));
    lds_barrier();
  };
  using Park = std::true_type;
  // position 1 (len - 1 >= 3 with the twisted order, K >= 8), then positions
  // 2 .. len - 2 in groups of kP (slots of position i: (i - 1) mod kP ...)
  fstep_body(1, 0, 1 % kP, 2 % kP, std::false_type{});
  int i = 2;
  for (; i + kP <= len - 1; i += kP) {
#pragma unroll
    for (int u = 0; u < kP; ++u)
      fstep_body(i + u, (1 + u) % kP, (2 + u) % kP, (3 + u) % kP, Park{});
  }
#pragma unroll
  for (int u = 0; u < kP - 1; ++u)
    if (i + u < len - 1) fstep_body(i + u, (1 + u) % kP, (2 + u) % kP, (3 + u) % kP, Park{});

  // the backward sweep's first coefficient rows, fetched a few steps early
  const int bs = top ? len - 1 : len - 2, cnt = bs + 1;
  BRow bring[kP][NR];
#pragma unroll
  for (int u = 0; u < kP; ++u) load_b(bring[u], bw + (size_t)max(bs - u, 0) * bstep);

  // ---------------------------------------------------------- middle rows
  // Here: z2 = z of position len-3, a = Linv tau of position len-1, and
  // z of position len-2 in zo.
  const int sm = nbot;  // step of z_m
  T zy[NB], pre[NR];
  read_all(zn, zo[(sm - 1) & 1]);  // top: z_{m-1}; bottom: z_{m+2}
  read_all(zy, zx[(sm - 1) & 1]);  // top: z_{m+2}; bottom: z_{m-1}
  sfor<0, NR>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    pre[j] = a[j] - dot8(cmid[j], I8{}, z2, T(0));
    put_w(len - 3, j, w_of(jc, cpm[j], z2));
    put_w(len - 2, j, w_of(jc, cmid[j], zn));
  });
  if (top) {
    sfor<0, NR>([&](auto jc) {  // z_m
      constexpr int j = decltype(jc)::value;
      zo[sm & 1][R0 + j][lane] = pre[j] - (dot8x2(cmid[j], I0{}, zn) + dot8x2(cx[j], I0{}, zy));
    });
    lds_barrier();
    read_all(zn, zo[sm & 1]);
    sfor<0, NR>([&](auto jc) {  // w_m
      constexpr int j = decltype(jc)::value;
      put_w(len - 1, j, w_of(jc, clast[j], zn));
    });
    lds_barrier();
  } else {
    sfor<0, NR>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      pre[j] -= dot8x2(cmid[j], I0{}, zn) + dot8x2(cx[j], I8{}, zy);
    });
    lds_barrier();
    read_all(zy, zx[sm & 1]);  // z_m
    sfor<0, NR>([&](auto jc) {  // z_{m+1}
      constexpr int j = decltype(jc)::value;
      zo[(sm + 1) & 1][R0 + j][lane] =
          pre[j] - dot8x2(cx[j], std::integral_constant<int, 16>{}, zy);
    });
    lds_barrier();
    read_all(zn, zo[(sm + 1) & 1]);
    sfor<0, NR>([&](auto jc) {  // theta_{m+1}
      constexpr int j = decltype(jc)::value;
      const T th = w_of(jc, clast[j], zn);
      zo[(sm + 2) & 1][R0 + j][lane] = th;
      buf_sts(rout, ro[j], roff(len - 1), th);
    });
  }
  lds_barrier();  // step sm + 2

  // ---------------------------------------------------------- backward
  // Backward step kk handles position p = bs - kk:
  //   theta_p = (w_p - N2_p theta_{p+2}) - N1_p theta_{p+1}
  // with theta_{p+1} from the exchange and theta_{p+2} in registers (t2).
  T t2[NB], tn[NB];
  const int bso = top ? sm + 3 : sm + 4;  // step of backward step 0
#pragma unroll
  for (int u = 0; u < kP; ++u) fetch_w(u, max(bs - u, 0));
  // theta_p = q - N1_p theta_{p+1} for the rows of this wavefront; refill
  auto bfinish = [&](int kk, int p, int s, const T* q) {
    sfor<0, NR>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const T th = q[j] - dot8x2(bring[s][j], I0{}, tn);
      zo[(kk + bso) & 1][R0 + j][lane] = th;
      buf_sts(rout, ro[j], roff(p), th);
    });
    load_b(bring[s], bw + (size_t)max(p - kP, 0) * bstep);
    fetch_w(s, max(p - kP, 0));
    lds_barrier();
  };
  if (top) {  // step sm + 3: theta_m = w_m - N1_m theta_{m+1}
    read_all(tn, zx[(sm + 2) & 1]);
    T q[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) q[j] = wval(0, bs, j);
    bfinish(0, bs, 0, q);
#pragma unroll
    for (int b = 0; b < NB; ++b) t2[b] = tn[b];
  } else {  // step sm + 3 idle; step sm + 4: theta_{m+2}, once theta_m is known
    read_all(t2, zo[(sm + 2) & 1]);  // theta_{m+1}
    lds_barrier();
    read_all(tn, zx[(sm + 3) & 1]);  // theta_m
    // roles swapped for this row: N1 pairs with theta_{m+1}, N2 with theta_m
    T q[NR];
    sfor<0, NR>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      q[j] = wval(0, bs, j) - dot8x2(bring[0][j], I0{}, t2);
      const T th = q[j] - dot8x2(bring[0][j], I8{}, tn);
      zo[bso & 1][R0 + j][lane] = th;
      buf_sts(rout, ro[j], roff(bs), th);
    });
    load_b(bring[0], bw + (size_t)max(bs - kP, 0) * bstep);
    fetch_w(0, max(bs - kP, 0));
    lds_barrier();
  }
  auto bstep_body = [&](int kk, int s) {
    read_all(tn, zo[(kk - 1 + bso) & 1]);  // theta_{p+1}
    T q[NR];
    sfor<0, NR>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      q[j] = wval(s, bs - kk, j) - dot8(bring[s][j], I8{}, t2, T(0));
    });
    bfinish(kk, bs - kk, s, q);
#pragma unroll
    for (int b = 0; b < NB; ++b) t2[b] = tn[b];
  };
  // One explicit drain of the vector-memory counter before the loop: the two
  // middle-row paths above join here, and without it the compiler's wait at
  // the loop head (valid for both paths and for every iteration) is far more
  // conservative than the ring's prefetch distance.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt untouched
  int kk = 1;
  for (; kk + kP <= cnt; kk += kP) {
#pragma unroll
    for (int u = 0; u < kP; ++u) bstep_body(kk + u, (1 + u) % kP);
  }
#pragma unroll
  for (int u = 0; u < kP - 1; ++u)
    if (kk + u < cnt) bstep_body(kk + u, (1 + u) % kP);
  for (int u = 0; u < (top ? pad : 0); ++u) lds_barrier();
  lds_barrier();  // every wavefront is done reading the buffers
}

template <typename T, int NS, int W = 0>
__device__ __forceinline__ void twisted_dispatch(int w, const Dims& D,
                                                 const OpCoef<T>& C, int cls,
                                                 int v, int lane, int t, bool act,
                                                 bool top,
                                                 __amdgpu_buffer_rsrc_t rtau,
                                                 __amdgpu_buffer_rsrc_t rout,
                                                 T (*zo)[2 * NS][kWave],
                                                 T (*zx)[2 * NS][kWave],
                                                 T (*wl)[2 * NS][kWave]) {
  constexpr int NR = kRowsPerWave<NS>;
  if constexpr (W < kWavesPerHalf<NS>) {
    if (w == W)
      sweep_twisted<T, NS, W * NR, NR>(D, C, cls, v, lane, t, act, top, rtau, rout, zo, zx,
                                       wl);
    else
      twisted_dispatch<T, NS, W + 1>(w, D, C, cls, v, lane, t, act, top, rtau, rout, zo, zx,
                                     wl);
  }
}

// phi_tile with the twisted factor: 2 kWavesPerHalf wavefronts per
// workgroup, zb holds the two halves' exchange buffers, wb their parked w.
template <typename T, int NS>
__device__ __forceinline__ void phi_tile_twisted(const Dims& D, const OpCoef<T>& C,
                                                 const T* __restrict__ tau,
                                                 T* __restrict__ out, int qt_distinct,
                                                 int v, int chunk,
                                                 T (*zb)[2][2 * NS][kWave],
                                                 T (*wb)[kWKeepAlloc<T, NS>][2 * NS][kWave]) {
  constexpr int NB = 2 * NS, WH = kWavesPerHalf<NS>;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = uniform(threadIdx.x >> 6);
  const bool top = w < WH;
  const int wi = top ? w : w - WH;
  const int t0 = chunk * kWave;
  const int t = t0 + lane;
  const int T_ = D.T;
  const bool valid = t < D.Tt;
  const long long bytes = D.vlen * (long long)sizeof(T);
  const __amdgpu_buffer_rsrc_t rtau = make_rsrc(tau, bytes);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(out, bytes);
  T(*zo)[NB][kWave] = zb[top ? 0 : 1];
  T(*zx)[NB][kWave] = zb[top ? 1 : 0];
  T(*wl)[NB][kWave] = wb[top ? 0 : 1];
  twisted_dispatch<T, NS>(wi, D, C, 0, v, lane, t,
                          valid && t >= 1 && !(qt_distinct && t == T_), top, rtau, rout,
                          zo, zx, wl);
  if (qt_distinct && t0 <= T_ && T_ < t0 + kWave)
    twisted_dispatch<T, NS>(wi, D, C, 1, v, lane, t, valid && t == T_, top, rtau, rout, zo,
                            zx, wl);
  {  // t = 0: theta = Q tau per node, item = (block row i, row R), spread over
     // the time-chunk workgroups of this super-column so none runs long
    const size_t nn = (size_t)NS * NS;
    gptr<const T> tg = glob(tau);
    gptr<T> og = glob(out);
    const int nthr = 2 * WH * kWave;
    for (int item = chunk * nthr + threadIdx.x; item < D.K * NB;
         item += time_chunks(D) * nthr) {
      const int i = item / NB, R = item - (item / NB) * NB;
      const int h = R / NS, a = R % NS;
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
