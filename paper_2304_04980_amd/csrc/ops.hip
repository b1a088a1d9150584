// Single-problem kernels of one PCG iteration and of the NBJM preconditioner:
// each workgroup finds its tile from its (XCD-remapped) block index and runs
// the shared tile body.  check != 0 makes a kernel return at once when the
// device flag sc->done is set (converged iterations become no-ops).
#include "bodies_ops.h"

namespace lqg {
namespace {
using namespace dev;

// Logical block of the one-chunk node tiles (k_recover): chunk-major, node
// group fastest, remapped per XCD.  Returns false for padding blocks.
__device__ __forceinline__ bool node_tile(const Dims& D, int* lb, int* p, int* t) {
  const int ngroups = node_groups(D);
  *lb = xcd_block();
  if (*lb >= ngroups * time_chunks(D)) return false;
  *p = tile_node(*lb % ngroups);
  *t = (*lb / ngroups) * kWave + (threadIdx.x & (kWave - 1));
  return true;
}

// The stencil kernels of the iteration: one workgroup per group of 4 nodes,
// each wavefront one node over all its time chunks, so that the node's
// operator blocks are read once and a chunk's t-1 / t+1 terms come from the
// neighbouring chunks by lane moves.  Blocks are XCD-remapped, so an XCD
// holds neighbouring nodes.

template <typename T, int NS>
__global__ __launch_bounds__(256) void k_delta(Dims D, OpCoef<T> C,
                                               const T* __restrict__ d,
                                               T* __restrict__ y,
                                               double* __restrict__ partial,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lb = xcd_block();
  if (lb >= node_groups(D)) return;
  delta_rows<T, NS>(D, C, d, y, partial ? partial + lb : nullptr, lb);
}

// The factored Delta apply (delta_w_rows / delta_y_rows): two passes.
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_delta_w(Dims D, OpCoef<T> C,
                                                 const T* __restrict__ d,
                                                 const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lb = xcd_block();
  if (lb >= node_groups(D)) return;
  delta_w_rows<T, NS>(D, C, d, C.W, lb);
}
template <typename T, int NS>
__global__ __launch_bounds__(256) void k_delta_y(Dims D, OpCoef<T> C,
                                                 const T* __restrict__ d,
                                                 T* __restrict__ y,
                                                 double* __restrict__ partial,
                                                 const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lb = xcd_block();
  if (lb >= node_groups(D)) return;
  delta_y_rows<T, NS>(D, C, d, C.W, y, partial ? partial + lb : nullptr, lb);
}

template <typename T, int NS>
__global__ __launch_bounds__(256) void k_omega(Dims D, OpCoef<T> C,
                                               const T* __restrict__ rho,
                                               const T* __restrict__ th,
                                               T* __restrict__ tau,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lb = xcd_block();
  if (lb >= node_groups(D)) return;
  omega_tile<T, NS>(D, C, rho, th, tau, lb, 0, time_chunks(D));
}

template <typename T, int NS>
__global__ __launch_bounds__(256) void k_xi(Dims D, OpCoef<T> C,
                                            const T* __restrict__ r,
                                            const T* __restrict__ dl,
                                            T* __restrict__ rho,
                                            const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lb = xcd_block();
  if (lb >= node_groups(D)) return;
  xi_rows<T, NS>(D, C, r, dl, rho, lb);
}

// One workgroup of 2n wavefronts per (super-column v, 64 time steps),
// super-column major so that a v's chunks share an XCD.
template <typename T, int NS>
__global__ __launch_bounds__(2 * NS * kWave) void k_phi_solve(
    Dims D, OpCoef<T> C, const T* __restrict__ tau, T* __restrict__ out,
    const Scalars* sc, int check, int qt_distinct) {
  if (is_done(sc, check)) return;
  __shared__ T zb[2][2 * NS][kWave];
  const int nchunks = time_chunks(D);
  const int lb = xcd_block();
  if (lb >= D.V * nchunks) return;
  phi_tile<T, NS>(D, C, tau, out, qt_distinct, lb / nchunks, lb % nchunks, zb);
}

template <typename T, int NS>
__global__ __launch_bounds__(2 * kWavesPerHalf<NS> * kWave) void k_phi_solve_twisted(
    Dims D, OpCoef<T> C, const T* __restrict__ tau, T* __restrict__ out,
    const Scalars* sc, int check, int qt_distinct) {
  if (is_done(sc, check)) return;
  __shared__ T zb[2][2][2 * NS][kWave];
  __shared__ T wb[2][kWKeepAlloc<T, NS>][2 * NS][kWave];
  const int nchunks = time_chunks(D);
  const int lb = xcd_block();
  if (lb >= D.V * nchunks) return;
  phi_tile_twisted<T, NS>(D, C, tau, out, qt_distinct, lb / nchunks, lb % nchunks, zb, wb);
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
inline dim3 group_grid(const Dims& D) { return dim3(padded_grid(node_groups(D))); }

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
  const int nb = node_groups(D);  // one partial of y'd per workgroup
  const dim3 g(padded_grid(nb));
  if (C.A5 && C.BRB && C.W) {  // the factored form, two passes
#define CALL(NS)                                                                     \
  hipLaunchKernelGGL((k_delta_w<T, NS>), g, dim3(256), 0, s, D, C, d, sc, check_done); \
  hipLaunchKernelGGL((k_delta_y<T, NS>), g, dim3(256), 0, s, D, C, d, y, partial, sc,  \
                     check_done)
    LQG_DISPATCH_N(D.n, CALL)
#undef CALL
    return nb;
  }
#define CALL(NS)                                                              \
  hipLaunchKernelGGL((k_delta<T, NS>), g, dim3(256), 0, s, D, C, d, y, partial, \
                     sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
  return nb;
}

template <typename T>
void omega_rhs(const Dims& D, const OpCoef<T>& C, const T* rho, const T* th,
               T* tau, const Scalars* sc, int check_done, hipStream_t s) {
  const dim3 g = group_grid(D);
#define CALL(NS)                                                               \
  hipLaunchKernelGGL((k_omega<T, NS>), g, dim3(256), 0, s, D, C, rho, th, tau, \
                     sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

template <typename T>
void xi_rhs(const Dims& D, const OpCoef<T>& C, const T* r, const T* dl, T* rho,
            const Scalars* sc, int check_done, hipStream_t s) {
  const dim3 g = group_grid(D);
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
#define CALL_TW(NS)                                                            \
  hipLaunchKernelGGL((k_phi_solve_twisted<T, NS>), g, dim3(2 * kWavesPerHalf<NS> * kWave), 0, s, \
                     D, C, tau, out, sc, check_done, qt_distinct)
  if (twisted(D)) {
    LQG_DISPATCH_N(D.n, CALL_TW)
  } else {
    LQG_DISPATCH_N(D.n, CALL)
  }
#undef CALL_TW
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
