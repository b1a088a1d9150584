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
// N_t = Linv_t' S_{t+1}', in a node-fastest table [t][3][n*n][nodes] so that
// the lanes of a wavefront (consecutive nodes) read one coalesced segment.
// Solve:  z_t = Linv_t tau_t - M_t z_{t-1},  theta_t = Linv_t' z_t - N_t theta_{t+1}.
#include "bodies_setup.h"
#include "nt.h"

namespace lqg {
namespace {

constexpr int kNtBatch = 8;  // time steps whose loads are issued together

// One thread per node (dummy nodes: identity blocks).  tv: the time-fastest
// arrays of time-varying data, else the time-invariant blocks of C.
template <int NS>
__global__ __launch_bounds__(64) void k_nt_factor(Dims D, Coef C, TvCoef<double> V, int tv,
                                                  double* __restrict__ tab, Scalars* sc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D.nodes) return;
  constexpr int nn = NS * NS;
  const bool dummy = p >= D.real_nodes;
  const size_t nodes = D.nodes, ldt = D.ldt;
  auto put = [&](int t, int k, int e, double v) {
    tab[(((size_t)t * 3 + k) * nn + e) * nodes + p] = v;
  };
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
      }
    for (int e = 0; e < nn; ++e) Lp[e] = Li[e];
  }
  for (int e = 0; e < nn; ++e) put(D.T, 2, e, 0.0);
  if (bad) atomicOr(&sc->flag_notspd, 1);
}

template <typename T>
__device__ __forceinline__ T quad_read(T v, int src) {
  return __shfl(v, src, kWave);
}

// theta = D_node^-1 tau: four lanes per node (lane r of a quad owns state
// component r; components past n idle), sixteen nodes per wavefront.  The
// recurrence is sequential in t, so the loads are software-pipelined: the
// coefficients and right-hand sides of the next kNtBatch steps are issued
// before the products of the current ones (two register buffers).
template <typename T, int NS>
struct NtBuf {
  T v[kNtBatch];             // tau_t (forward) or z_t (backward)
  T a[kNtBatch][NS];         // Linv_t row (forward) / Linv_t' row (backward)
  T b[kNtBatch][NS];         // M_t row (forward) / N_t row (backward)
};

template <typename T, int NS>
__global__ __launch_bounds__(256) void k_nt_solve(Dims D, const T* __restrict__ tab,
                                                  const T* __restrict__ tau,
                                                  T* __restrict__ out, const Scalars* sc,
                                                  int check) {
  if (check && __builtin_nontemporal_load(&sc->done) != 0) return;
  constexpr int nn = NS * NS;
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane & 3, q0 = lane & ~3;
  const int p = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  const bool node_ok = p < D.nodes;
  const bool act = node_ok && r < NS;
  const int pc = node_ok ? p : 0;
  const int rc = r < NS ? r : 0;
  const size_t nodes = D.nodes, ldt = D.ldt;
  const size_t vrow = ((size_t)pc * NS + rc) * ldt;
  const int Tt = D.Tt;
  const int nb = (Tt + kNtBatch - 1) / kNtBatch;
  auto coef = [&](int t, int k, int row, int col) {
    return tab[(((size_t)t * 3 + k) * nn + row * NS + col) * nodes + pc];
  };
  // forward: batch i covers t = i kNtBatch + b
  auto fload = [&](int i, NtBuf<T, NS>& B) {
#pragma unroll
    for (int b = 0; b < kNtBatch; ++b) {
      const int t = min(i * kNtBatch + b, Tt - 1);
      B.v[b] = tau[vrow + t];
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        B.a[b][c] = coef(t, 0, rc, c);
        B.b[b][c] = coef(t, 1, rc, c);
      }
    }
  };
  T zp = T(0);
  auto fcomp = [&](int i, const NtBuf<T, NS>& B) {
#pragma unroll
    for (int b = 0; b < kNtBatch; ++b) {
      const int t = i * kNtBatch + b;
      if (t >= Tt) break;
      T z = T(0);
#pragma unroll
      for (int c = 0; c < NS; ++c) z = fma(B.a[b][c], quad_read(B.v[b], q0 + c), z);
#pragma unroll
      for (int c = 0; c < NS; ++c) z = fma(-B.b[b][c], quad_read(zp, q0 + c), z);
      if (act) out[vrow + t] = z;
      zp = z;
    }
  };
  NtBuf<T, NS> B0, B1;
  fload(0, B0);
  for (int i = 0; i < nb; i += 2) {
    if (i + 1 < nb) fload(i + 1, B1);
    fcomp(i, B0);
    if (i + 1 >= nb) break;
    if (i + 2 < nb) fload(i + 2, B0);
    fcomp(i + 1, B1);
  }
  // backward: batch i covers t = Tt - 1 - (i kNtBatch + b); z_t is read back
  // from `out` (this thread's own forward stores)
  auto bload = [&](int i, NtBuf<T, NS>& B) {
#pragma unroll
    for (int b = 0; b < kNtBatch; ++b) {
      const int t = max(Tt - 1 - (i * kNtBatch + b), 0);
      B.v[b] = act ? out[vrow + t] : T(0);
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        B.a[b][c] = coef(t, 0, c, rc);  // Linv_t' row r
        B.b[b][c] = coef(t, 2, rc, c);
      }
    }
  };
  T th = T(0);
  auto bcomp = [&](int i, const NtBuf<T, NS>& B) {
#pragma unroll
    for (int b = 0; b < kNtBatch; ++b) {
      const int t = Tt - 1 - (i * kNtBatch + b);
      if (t < 0) break;
      T v = T(0);
#pragma unroll
      for (int c = 0; c < NS; ++c) v = fma(B.a[b][c], quad_read(B.v[b], q0 + c), v);
#pragma unroll
      for (int c = 0; c < NS; ++c) v = fma(-B.b[b][c], quad_read(th, q0 + c), v);
      if (act) out[vrow + t] = v;
      th = v;
    }
  };
  bload(0, B0);
  for (int i = 0; i < nb; i += 2) {
    if (i + 1 < nb) bload(i + 1, B1);
    bcomp(i, B0);
    if (i + 1 >= nb) break;
    if (i + 2 < nb) bload(i + 2, B0);
    bcomp(i + 1, B1);
  }
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
  return (size_t)D.Tt * 3 * D.n * D.n * D.nodes;
}

void nt_factor(const Dims& D, const Coef& C, const TvCoef<double>& V, int tv, double* tab,
               Scalars* sc, hipStream_t s) {
#define CALL(NS) \
  hipLaunchKernelGGL(k_nt_factor<NS>, dim3((D.nodes + 63) / 64), dim3(64), 0, s, D, C, V, tv, tab, sc)
  LQG_NT_DISPATCH(D.n, CALL)
#undef CALL
}

template <typename T>
void nt_solve(const Dims& D, const T* tab, const T* tau, T* out, const Scalars* sc, int check,
              hipStream_t s) {
  const int blocks = (int)(((long long)D.nodes * 4 + 255) / 256);
#define CALL(NS)                                                                         \
  hipLaunchKernelGGL((k_nt_solve<T, NS>), dim3(blocks), dim3(256), 0, s, D, tab, tau, out, \
                     sc, check)
  LQG_NT_DISPATCH(D.n, CALL)
#undef CALL
}

template void nt_solve<double>(const Dims&, const double*, const double*, double*,
                               const Scalars*, int, hipStream_t);
template void nt_solve<float>(const Dims&, const float*, const float*, float*,
                              const Scalars*, int, hipStream_t);

}  // namespace lqg
