// Node-temporal block Jacobi preconditioner (the alternative nesting of the
// preconditioner: time kept whole, space split into nodes).
//
// D_node, the part of Delta that couples each grid node only to itself, is
// for node p the block-tridiagonal matrix over t = 0..T with diagonal blocks
// Psi_hat_t[p,p] (Q_0^-1 at t = 0; Q_t^-1 + [A_hat Q^-1 A_hat' + B R^-1 B']
// [p,p] of time t - 1 for t >= 1) and off-diagonal blocks
// E_t = Delta_{t+1,t}[p,p] = -A_hat_t[p,p] Q_{t,p}^-1 (eq. "structure_of_Delta").
// It is a principal block part of the positive definite Delta, hence
// positive definite, and P = D_node is a valid PCG preconditioner.
//
// Factorisation (one thread per node, sequential in t): block Cholesky
//   L_tt = chol(D_t - S_t S_t'),  S_t = E_{t-1} L_{t-1,t-1}^-T,
// stored as the products the solve uses, Linv_t = L_tt^-1, M_t = Linv_t S_t,
// N_t = Linv_t' S_{t+1}' and Linv_t' (for the backward sweep), in a table
// [t][node group of 16][4][16][n][n]: the coefficients one wavefront (16
// nodes) needs for one step of either sweep are two contiguous runs, and
// each lane's row of a block is contiguous.
// Solve:  z_t = Linv_t tau_t - M_t z_{t-1},  theta_t = Linv_t' z_t - N_t theta_{t+1}.
#include "bodies_setup.h"
#include "nt.h"

namespace lqg {
namespace {

constexpr int kNtGroup = 16;  // nodes per table group (the nodes of one wavefront)
constexpr int kNtBlocks = 4;  // Linv_t, M_t, N_t, Linv_t'

__host__ __device__ inline size_t nt_index(const Dims& D, int t, int k, int p, int e,
                                           int nn) {
  const size_t G = ((size_t)D.nodes + kNtGroup - 1) / kNtGroup;
  return ((((size_t)t * G + p / kNtGroup) * kNtBlocks + k) * kNtGroup + p % kNtGroup) * nn +
         e;
}

// One thread per node (dummy nodes: identity blocks).  tv: the time-fastest
// arrays of time-varying data, else the time-invariant blocks of C.
template <int NS>
__global__ __launch_bounds__(64) void k_nt_factor(Dims D, Coef C, TvCoef<double> V, int tv,
                                                  double* __restrict__ tab, Scalars* sc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D.nodes) return;
  constexpr int nn = NS * NS;
  const bool dummy = p >= D.real_nodes;
  const size_t ldt = D.ldt;
  auto put = [&](int t, int k, int e, double v) { tab[nt_index(D, t, k, p, e, nn)] = v; };
  double Lp[nn], S[nn], A[nn], Li[nn];
  for (int e = 0; e < nn; ++e) Lp[e] = 0.0;
  bool bad = false;
  for (int t = 0; t <= D.T; ++t) {
    // diagonal block D_t
    for (int e = 0; e < nn; ++e) {
      double d;
      if (dummy) {
        d = (e / NS == e % NS) ? 1.0 : 0.0;
      } else if (tv) {
        d = V.G13[(((size_t)p * 13) * nn + e) * ldt + t] + V.Qi[((size_t)p * nn + e) * ldt + t];
      } else {
        d = (t == D.T ? C.QTi : C.Qi)[(size_t)p * nn + e];
        if (t >= 1) d += C.G13[(size_t)p * 13 * nn + e];
      }
      A[e] = d;
    }
    for (int e = 0; e < nn; ++e) S[e] = 0.0;
    if (t >= 1 && !dummy) {
      // E = Delta_{t,t-1}[p,p] = -Cdn_{t-1}[p][self];  S = E Linv_{t-1}'
      double E[nn];
      for (int e = 0; e < nn; ++e)
        E[e] = -(tv ? V.Cdn[((size_t)p * 5 * nn + e) * ldt + (t - 1)]
                    : C.Cdn[(size_t)p * 5 * nn + e]);
      for (int a = 0; a < NS; ++a)
        for (int b = 0; b < NS; ++b) {
          double s = 0.0;
          for (int c = 0; c < NS; ++c) s += E[a * NS + c] * Lp[b * NS + c];
          S[a * NS + b] = s;
        }
      for (int a = 0; a < NS; ++a)  // A -= S S'
        for (int b = 0; b < NS; ++b) {
          double s = 0.0;
          for (int c = 0; c < NS; ++c) s += S[a * NS + c] * S[b * NS + c];
          A[a * NS + b] -= s;
        }
      // N_{t-1} = Linv_{t-1}' S'
      for (int a = 0; a < NS; ++a)
        for (int b = 0; b < NS; ++b) {
          double s = 0.0;
          for (int c = 0; c < NS; ++c) s += Lp[c * NS + a] * S[b * NS + c];
          put(t - 1, 2, a * NS + b, s);
        }
    } else if (t >= 1) {
      for (int e = 0; e < nn; ++e) put(t - 1, 2, e, 0.0);
    }
    // Cholesky A = L L' (lower), then Li = L^-1
    double L[nn];
    for (int e = 0; e < nn; ++e) L[e] = 0.0;
    for (int cc = 0; cc < NS; ++cc) {
      double s = A[cc * NS + cc];
      for (int k = 0; k < cc; ++k) s -= L[cc * NS + k] * L[cc * NS + k];
      if (!(s > 0.0) || !isfinite(s)) {
        bad = true;
        s = 1.0;
      }
      const double dg = sqrt(s);
      L[cc * NS + cc] = dg;
      for (int r = cc + 1; r < NS; ++r) {
        double v = A[r * NS + cc];
        for (int k = 0; k < cc; ++k) v -= L[r * NS + k] * L[cc * NS + k];
        L[r * NS + cc] = v / dg;
      }
    }
    for (int e = 0; e < nn; ++e) Li[e] = 0.0;
    for (int cc = 0; cc < NS; ++cc) {  // column cc of L^-1 by forward substitution
      for (int r = cc; r < NS; ++r) {
        double v = (r == cc) ? 1.0 : 0.0;
        for (int k = cc; k < r; ++k) v -= L[r * NS + k] * Li[k * NS + cc];
        Li[r * NS + cc] = v / L[r * NS + r];
      }
    }
    for (int a = 0; a < NS; ++a)
      for (int b = 0; b < NS; ++b) {
        double m = 0.0;
        for (int c = 0; c < NS; ++c) m += Li[a * NS + c] * S[c * NS + b];
        put(t, 0, a * NS + b, Li[a * NS + b]);
        put(t, 1, a * NS + b, m);  // M_t = Linv_t S_t
        put(t, 3, a * NS + b, Li[b * NS + a]);
      }
    for (int e = 0; e < nn; ++e) Lp[e] = Li[e];
  }
  for (int e = 0; e < nn; ++e) put(D.T, 2, e, 0.0);
  if (bad) atomicOr(&sc->flag_notspd, 1);
}

// Compile-time loop: f(std::integral_constant<int, k>) for k = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void nt_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    nt_for<B + 1, E>(f);
  }
}

// Lane c of the lane's quad (DPP quad_perm broadcast; every lane active).
template <int C>
__device__ __forceinline__ float quad_bcast(float v) {
  constexpr int ctrl = C | (C << 2) | (C << 4) | (C << 6);
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xf, 0xf, false));
}
template <int C>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = C | (C << 2) | (C << 4) | (C << 6);
  struct P {
    int lo, hi;
  };
  P x = __builtin_bit_cast(P, v);
  x.lo = __builtin_amdgcn_mov_dpp(x.lo, ctrl, 0xf, 0xf, false);
  x.hi = __builtin_amdgcn_mov_dpp(x.hi, ctrl, 0xf, 0xf, false);
  return __builtin_bit_cast(double, x);
}

template <typename T>
struct Vec16;  // 16-byte vector of T
template <>
struct Vec16<float> {
  using type = float4;
};
template <>
struct Vec16<double> {
  using type = double2;
};

// theta = D_node^-1 tau: four lanes per node (lane r of a quad owns state
// component r; components past n idle), sixteen nodes per wavefront.  The
// recurrence is sequential in t.  The forward sweep writes z to zbuf, the
// backward sweep reads it back from there and writes theta to out (separate
// buffers, so the reads of z need not wait for the stores of theta).  A
// lane's row of tau (z, theta) is read and
// written in tiles of TB consecutive steps by 16-byte accesses; the other
// components of the node come from the quad by DPP broadcasts; the
// coefficient rows of step t are fetched RING steps ahead into a register
// ring (slot t mod RING).  Tile entries past the last step are written as
// zero, which keeps the row padding zero.
template <typename T, int NS, int TB>
__global__ __launch_bounds__(256) void k_nt_solve(Dims D, const T* __restrict__ tab,
                                                  const T* __restrict__ tau,
                                                  T* __restrict__ zbuf, T* __restrict__ out,
                                                  const Scalars* sc, int check) {
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  constexpr int nn = NS * NS;
  constexpr int RING = sizeof(T) == 4 ? 8 : 4;  // steps of coefficient prefetch
  constexpr int VW = 16 / (int)sizeof(T);  // elements per 16-byte access
  constexpr int NV = TB / VW;
  static_assert(TB % RING == 0 && TB % VW == 0, "tile shape");
  using VT = typename Vec16<T>::type;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane & 3;
  const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  const bool node_ok = p < D.nodes;
  const bool act = node_ok && r < NS;
  const int pc = node_ok ? p : 0;
  const int rc = r < NS ? r : 0;
  const size_t ldt = D.ldt;
  const int Tt = D.Tt;
  const int nbt = (Tt + TB - 1) / TB;  // nbt * TB <= ldt (ldt is a multiple of 16)
  const T* trow = tau + ((size_t)pc * NS + rc) * ldt;
  const T* zrow = zbuf + ((size_t)pc * NS + rc) * ldt;
  // row rc of coefficient block k of step t
  auto row_ld = [&](int t, int k, T (&x)[NS]) {
    const T* src = tab + nt_index(D, t, k, pc, rc * NS, nn);
    if constexpr (NS * sizeof(T) % 16 == 0) {
#pragma unroll
      for (int v = 0; v < NS / VW; ++v) {
        const VT q = reinterpret_cast<const VT*>(src)[v];
        const T* e = reinterpret_cast<const T*>(&q);
#pragma unroll
        for (int k2 = 0; k2 < VW; ++k2) x[v * VW + k2] = e[k2];
      }
    } else {
#pragma unroll
      for (int c = 0; c < NS; ++c) x[c] = src[c];
    }
  };
  auto ld_tile = [&](const T* row, int b, T (&x)[TB]) {
    const VT* src = reinterpret_cast<const VT*>(row + (size_t)b * TB);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const VT q = src[v];
      const T* e = reinterpret_cast<const T*>(&q);
#pragma unroll
      for (int k = 0; k < VW; ++k) x[v * VW + k] = e[k];
    }
  };
  // stores through a buffer resource: lanes without a row of their own
  // (components past n, nodes past the grid) and tiles past the end use an
  // out-of-range offset and their stores are dropped, so no branch splits the
  // sweep
  const __amdgpu_buffer_rsrc_t rout = __builtin_amdgcn_make_buffer_rsrc(
      out, (short)0, (int)(D.vlen * (long long)sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(
      zbuf, (short)0, (int)(D.vlen * (long long)sizeof(T)), 0x00020000);
  const unsigned obase = (unsigned)(((size_t)pc * NS + rc) * ldt * sizeof(T));
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  auto st_tile = [&](__amdgpu_buffer_rsrc_t rdst, int b, const T (&x)[TB]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      VT q;
      T* e = reinterpret_cast<T*>(&q);
#pragma unroll
      for (int k = 0; k < VW; ++k) e[k] = x[v * VW + k];
      const unsigned off = obase + (unsigned)((b * TB + v * VW) * sizeof(T));
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, q), rdst,
                                             act && b < nbt ? off : 0x80000000u, 0, 0);
    }
  };
  // sum_c m[c] x_c over the quad's components x_c of v (two partial sums)
  auto qdot = [&](const T (&m)[NS], T v) {
    T e0 = T(0), e1 = T(0);
    nt_for<0, NS>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c % 2 == 0) e0 = fma(m[c], quad_bcast<c>(v), e0);
      else e1 = fma(m[c], quad_bcast<c>(v), e1);
    });
    return e0 + e1;
  };
  T ca[RING][NS], cb[RING][NS];
  T zt[TB];

  // forward: z_t = Linv_t tau_t - M_t z_{t-1}
  auto ld_f = [&](int t, int slot) {
    t = min(max(t, 0), Tt - 1);
    row_ld(t, 0, ca[slot]);  // Linv_t row rc
    row_ld(t, 1, cb[slot]);  // M_t row rc
  };
#pragma unroll
  for (int u = 0; u < RING; ++u) ld_f(u, u);
  // Every step runs on every lane and tile: steps past the last one compute on
  // clamped indices and their results are discarded, so the sweep has no
  // branch and the prefetched loads stay in flight across steps.  Tiles are
  // handled in pairs with two tau (z) buffers, the next tile's read issued
  // before the current tile's steps.
  T tA[TB], tB[TB];
  T zp = T(0);
  auto ftile = [&](int b, const T (&cur)[TB]) {
#pragma unroll
    for (int s = 0; s < TB; ++s) {
      const int t = b * TB + s;
      const int slot = s % RING;
      const bool live = t < Tt;  // wave-uniform
      const T z = qdot(ca[slot], cur[s]) - qdot(cb[slot], zp);
      zt[s] = live ? z : T(0);
      zp = live ? z : zp;
      ld_f(t + RING, slot);
    }
    st_tile(rz, b, zt);
  };
  ld_tile(trow, 0, tA);
  int b = 0;
  for (; b + 1 < nbt; b += 2) {
    ld_tile(trow, b + 1, tB);
    ftile(b, tA);
    ld_tile(trow, min(b + 2, nbt - 1), tA);
    ftile(b + 1, tB);
  }
  // the last tile when nbt is odd, else a tile past the end whose stores are
  // dropped (no branch, so the backward sweep starts from one code path)
  ftile(b, tA);

  // backward: theta_t = Linv_t' z_t - N_t theta_{t+1}; z_t is this lane's
  // own forward result, read back from zbuf
  auto ld_b = [&](int t, int slot) {
    // clamped at both ends: on the steps past the last one of the last tile
    // t - RING can still be >= Tt (up to TB - 1 such steps)
    t = min(max(t, 0), Tt - 1);
    row_ld(t, 3, ca[slot]);  // Linv_t' row rc
    row_ld(t, 2, cb[slot]);  // N_t row rc
  };
#pragma unroll
  for (int q = 0; q < RING; ++q) {  // slot q: the step t in [Tt - RING, Tt) with t = q mod RING
    const int t = Tt - 1 - (((Tt - 1 - q) % RING) + RING) % RING;
    ld_b(t, q);
  }
  T th = T(0);
  auto btile = [&](int b, const T (&cur)[TB]) {
#pragma unroll
    for (int s = TB - 1; s >= 0; --s) {
      const int t = b * TB + s;
      const int slot = s % RING;
      const bool live = t < Tt;  // wave-uniform
      const T v = qdot(ca[slot], cur[s]) - qdot(cb[slot], th);
      zt[s] = live ? v : T(0);
      th = live ? v : th;
      ld_b(t - RING, slot);
    }
    st_tile(rout, b, zt);
  };
  ld_tile(zrow, nbt - 1, tA);
  b = nbt - 1;
  for (; b >= 1; b -= 2) {  // tiles b and b - 1; z of tile b - 2 read ahead
    ld_tile(zrow, b - 1, tB);
    btile(b, tA);
    ld_tile(zrow, max(b - 2, 0), tA);
    btile(b - 1, tB);
  }
  if (b >= 0) btile(b, tA);
}

}  // namespace

#define LQG_NT_DISPATCH(n, CALL) \
  switch (n) {                   \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    default: break;              \
  }

size_t nt_table_doubles(const Dims& D) {
  const size_t G = ((size_t)D.nodes + kNtGroup - 1) / kNtGroup;
  return (size_t)D.Tt * G * kNtBlocks * kNtGroup * D.n * D.n;
}

void nt_factor(const Dims& D, const Coef& C, const TvCoef<double>& V, int tv, double* tab,
               Scalars* sc, hipStream_t s) {
#define CALL(NS) \
  hipLaunchKernelGGL(k_nt_factor<NS>, dim3((D.nodes + 63) / 64), dim3(64), 0, s, D, C, V, tv, tab, sc)
  LQG_NT_DISPATCH(D.n, CALL)
#undef CALL
}

template <typename T>
void nt_solve(const Dims& D, const T* tab, const T* tau, T* zbuf, T* out, const Scalars* sc,
              int check, hipStream_t s) {
  const int blocks = (int)(((long long)D.nodes * 4 + 255) / 256);
  constexpr int TB = sizeof(T) == 4 ? 16 : 8;
#define CALL(NS)                                                                             \
  hipLaunchKernelGGL((k_nt_solve<T, NS, TB>), dim3(blocks), dim3(256), 0, s, D, tab, tau, zbuf, \
                     out, sc, check)
  LQG_NT_DISPATCH(D.n, CALL)
#undef CALL
}

template void nt_solve<double>(const Dims&, const double*, const double*, double*, double*,
                               const Scalars*, int, hipStream_t);
template void nt_solve<float>(const Dims&, const float*, const float*, float*, float*,
                              const Scalars*, int, hipStream_t);

}  // namespace lqg
