// Hot-path kernels of one PCG iteration (Algorithm 1) and of the NBJM
// preconditioner (Algorithm 2).
//
// Work mapping: a wavefront owns one grid node (or one super-column for the
// block solve) and 64 consecutive time steps, one per lane.  The operator
// blocks are time invariant, so every coefficient address is wave-uniform and
// is read through the scalar cache into SGPRs; the vectors are time-fastest,
// so each lane's accesses form one contiguous 512-byte segment per
// (node, component).  The t = 0 and t = T special cases of Delta
// (Psi_hat_0 = Q^-1, no t-1 / t+1 neighbour) are lane predicates.
#include "launch.h"

namespace lqg {
namespace {

template <int NS>
__device__ __forceinline__ void load_node(const double* __restrict__ v,
                                          int p, int t, int ldt,
                                          double (&x)[NS]) {
  const double* b = v + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) x[c] = b[(size_t)c * ldt];
}
template <int NS>
__device__ __forceinline__ void store_node(double* __restrict__ v, int p, int t,
                                           int ldt, const double (&x)[NS]) {
  double* b = v + (size_t)p * NS * ldt + t;
#pragma unroll
  for (int c = 0; c < NS; ++c) b[(size_t)c * ldt] = x[c];
}
// acc += M x   (M: NS x NS row-major, wave-uniform)
template <int NS>
__device__ __forceinline__ void mv_add(const double* __restrict__ M,
                                       const double (&x)[NS],
                                       double (&acc)[NS]) {
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(M[a * NS + b], x[b], acc[a]);
}
template <int NS>
__device__ __forceinline__ void mv_sub(const double* __restrict__ M,
                                       const double (&x)[NS],
                                       double (&acc)[NS]) {
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int b = 0; b < NS; ++b) acc[a] = fma(-M[a * NS + b], x[b], acc[a]);
}

__device__ __forceinline__ bool is_done(const Scalars* sc, int check) {
  return check && __builtin_nontemporal_load(&sc->done) != 0;
}

// ---------------------------------------------------------------------------
// y = Delta d, fused partial sums of y'd.
//   y_t(p) = Q_t^-1 d_t(p)
//          + [t>=1] ( sum_13 G[p][k] d_t(p+o_k) - sum_5 Cdn[p][k] d_{t-1}(p+o_k) )
//          - [t<T]  sum_5 Cup[p][k] d_{t+1}(p+o_k)
template <int NS>
__global__ __launch_bounds__(256) void k_delta(Dims D, Coef C,
                                               const double* __restrict__ d,
                                               double* __restrict__ y,
                                               double* __restrict__ partial,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int p = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int t = blockIdx.y * kWave + lane;
  const int T = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  double dot = 0.0;
  if (p < D.real_nodes && t < D.Tt) {
    const int j = uniform(p / K), i = uniform(p - (p / K) * K);
    double self[NS], acc[NS], nb[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = 0.0;
    load_node<NS>(d, p, t, ldt, self);
    mv_add<NS>(C.Qi + p * nn, self, acc);
    if (t == T) mv_add<NS>(C.QTd + p * nn, self, acc);
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
    if (t < T) {
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
    for (int a = 0; a < NS; ++a) dot = fma(acc[a], self[a], dot);
  }
  dot = block_sum<256>(dot);
  if (partial && threadIdx.x == 0)
    partial[blockIdx.y * gridDim.x + blockIdx.x] = dot;
}

// tau = rho + Omega~ theta, Omega~ = Phi~ - Psi~: minus the blocks of
// Psi_hat_t (t >= 1) that couple different super-columns; Omega_hat_0 = 0.
template <int NS>
__global__ __launch_bounds__(256) void k_omega(Dims D, Coef C,
                                               const double* __restrict__ rho,
                                               const double* __restrict__ th,
                                               double* __restrict__ tau,
                                               const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int p = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int t = blockIdx.y * kWave + lane;
  const int ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  double acc[NS], nb[NS];
  if (rho) load_node<NS>(rho, p, t, ldt, acc);
  else
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = 0.0;
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
template <int NS>
__global__ __launch_bounds__(256) void k_xi(Dims D, Coef C,
                                            const double* __restrict__ r,
                                            const double* __restrict__ dl,
                                            double* __restrict__ rho,
                                            const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int p = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int t = blockIdx.y * kWave + lane;
  const int T = D.T, ldt = D.ldt, K = D.K, N = D.N;
  const size_t nn = (size_t)NS * NS;
  if (p >= D.real_nodes || t >= D.Tt) return;
  const int j = uniform(p / K), i = uniform(p - (p / K) * K);
  double acc[NS], nb[NS];
  if (r) load_node<NS>(r, p, t, ldt, acc);
  else
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = 0.0;
  if (t >= 1) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int iq = i + kOff5[k][0], jq = j + kOff5[k][1];
      if (iq < 0 || iq >= K || jq < 0 || jq >= N) continue;
      load_node<NS>(dl, jq * K + iq, t - 1, ldt, nb);
      mv_add<NS>(C.Cdn + ((size_t)p * 5 + k) * nn, nb, acc);
    }
  }
  if (t < T) {
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

// Forward/backward substitution with the banded block Cholesky factor of
// Phi_bar_{v,cls} for this lane's time step.  z (the forward result) is
// parked in `out` and overwritten by theta in the backward sweep.
template <int NS>
__device__ __forceinline__ void sweep(const Dims& D, const Coef& C, int cls,
                                      int v, int t, const double* __restrict__ tau,
                                      double* __restrict__ out) {
  constexpr int NB = 2 * NS, NB2 = NB * NB;
  const int K = D.K, ldt = D.ldt;
  const int p0 = (2 * v) * K, p1 = (2 * v + 1) * K;  // column starts
  const double* F0 = C.Lf + (((size_t)cls * D.V + v) * K) * 3 * NB2;
  double zm1[NB], zm2[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) zm1[a] = zm2[a] = 0.0;
  for (int i = 0; i < K; ++i) {
    const double* F = F0 + (size_t)i * 3 * NB2;
    double s[NB], h0[NS], h1[NS];
    load_node<NS>(tau, p0 + i, t, ldt, h0);
    load_node<NS>(tau, p1 + i, t, ldt, h1);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      s[a] = h0[a];
      s[NS + a] = h1[a];
    }
    if (i >= 1) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) s[a] = fma(-F[NB2 + a * NB + b], zm1[b], s[a]);
    }
    if (i >= 2) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          s[a] = fma(-F[2 * NB2 + a * NB + b], zm2[b], s[a]);
    }
    double z[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b <= a; ++b) acc = fma(F[a * NB + b], s[b], acc);
      z[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      h0[a] = z[a];
      h1[a] = z[NS + a];
    }
    store_node<NS>(out, p0 + i, t, ldt, h0);
    store_node<NS>(out, p1 + i, t, ldt, h1);
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      zm2[a] = zm1[a];
      zm1[a] = z[a];
    }
  }
  // backward: theta_i = Linv_i' (z_i - L_{i+1,i}' theta_{i+1} - L_{i+2,i}' theta_{i+2})
#pragma unroll
  for (int a = 0; a < NB; ++a) zm1[a] = zm2[a] = 0.0;
  for (int i = K - 1; i >= 0; --i) {
    const double* F = F0 + (size_t)i * 3 * NB2;
    double s[NB], h0[NS], h1[NS];
    load_node<NS>(out, p0 + i, t, ldt, h0);
    load_node<NS>(out, p1 + i, t, ldt, h1);
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      s[a] = h0[a];
      s[NS + a] = h1[a];
    }
    if (i + 1 < K) {
      const double* F1 = F0 + (size_t)(i + 1) * 3 * NB2 + NB2;  // L_{i+1,i}
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) s[a] = fma(-F1[b * NB + a], zm1[b], s[a]);
    }
    if (i + 2 < K) {
      const double* F2 = F0 + (size_t)(i + 2) * 3 * NB2 + 2 * NB2;  // L_{i+2,i}
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) s[a] = fma(-F2[b * NB + a], zm2[b], s[a]);
    }
    double th[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = a; b < NB; ++b) acc = fma(F[b * NB + a], s[b], acc);
      th[a] = acc;
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      h0[a] = th[a];
      h1[a] = th[NS + a];
    }
    store_node<NS>(out, p0 + i, t, ldt, h0);
    store_node<NS>(out, p1 + i, t, ldt, h1);
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      zm2[a] = zm1[a];
      zm1[a] = th[a];
    }
  }
}

// out = Phi~^-1 tau.  One wavefront per (super-column v, 64 time steps).
// t = 0: Phi_bar_{v,0} = blkdiag(Q^-1), so theta = Q tau per node.
template <int NS>
__global__ __launch_bounds__(64) void k_phi_solve(Dims D, Coef C,
                                                  const double* __restrict__ tau,
                                                  double* __restrict__ out,
                                                  const Scalars* sc, int check,
                                                  int qt_distinct) {
  if (is_done(sc, check)) return;
  const int v = blockIdx.x;
  const int t = blockIdx.y * kWave + (threadIdx.x & (kWave - 1));
  const int T = D.T;
  const bool valid = t < D.Tt;
  const bool cls0 = valid && t >= 1 && !(qt_distinct && t == T);
  if (cls0) sweep<NS>(D, C, 0, v, t, tau, out);
  if (qt_distinct && valid && t == T) sweep<NS>(D, C, 1, v, t, tau, out);
  if (valid && t == 0) {
    const size_t nn = (size_t)NS * NS;
    for (int h = 0; h < 2; ++h)
      for (int i = 0; i < D.K; ++i) {
        const int p = (2 * v + h) * D.K + i;
        double x[NS], acc[NS];
        load_node<NS>(tau, p, 0, D.ldt, x);
#pragma unroll
        for (int a = 0; a < NS; ++a) acc[a] = 0.0;
        mv_add<NS>(C.Qm + p * nn, x, acc);
        store_node<NS>(out, p, 0, D.ldt, acc);
      }
  }
}

// ------------------------------------------------------------ flat vectors
__global__ __launch_bounds__(256) void k_dir(long long n,
                                             const double* __restrict__ q,
                                             double* __restrict__ d,
                                             const Scalars* sc) {
  if (sc->done) return;
  const double beta = sc->beta;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x)
    d[g] = fma(beta, d[g], q[g]);
}

__global__ __launch_bounds__(256) void k_update(long long n,
                                                const double* __restrict__ d,
                                                const double* __restrict__ y,
                                                double* __restrict__ dl,
                                                double* __restrict__ r,
                                                double* __restrict__ partial,
                                                const Scalars* sc) {
  if (sc->done) return;
  const double th = sc->theta;
  double acc = 0.0;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x) {
    dl[g] = fma(th, d[g], dl[g]);
    const double rn = fma(-th, y[g], r[g]);
    r[g] = rn;
    acc = fma(rn, rn, acc);
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_dot(long long n,
                                             const double* __restrict__ a,
                                             const double* __restrict__ b,
                                             double* __restrict__ partial,
                                             const Scalars* sc, int check) {
  if (is_done(sc, check)) return;
  double acc = 0.0;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x)
    acc = fma(a[g], b[g], acc);
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_sub_norm(long long n,
                                                  const double* __restrict__ rd,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ r,
                                                  double* __restrict__ psum,
                                                  double* __restrict__ pmax) {
  double acc = 0.0, mx = 0.0;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x) {
    const double v = rd[g] - y[g];
    r[g] = v;
    acc = fma(v, v, acc);
    mx = fmax(mx, fabs(v));
  }
  acc = block_sum<256>(acc);
  mx = block_max<256>(mx);
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = acc;
    pmax[blockIdx.x] = mx;
  }
}

__global__ __launch_bounds__(256) void k_norms(long long n,
                                               const double* __restrict__ a,
                                               double* __restrict__ psum,
                                               double* __restrict__ pmax) {
  double acc = 0.0, mx = 0.0;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x) {
    acc = fma(a[g], a[g], acc);
    mx = fmax(mx, fabs(a[g]));
  }
  acc = block_sum<256>(acc);
  mx = block_max<256>(mx);
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = acc;
    pmax[blockIdx.x] = mx;
  }
}

__global__ __launch_bounds__(256) void k_copy(long long n,
                                              const double* __restrict__ a,
                                              double* __restrict__ b) {
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x)
    b[g] = a[g];
}

__global__ __launch_bounds__(256) void k_zero(long long n, double* __restrict__ a) {
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x)
    a[g] = 0.0;
}

// Deterministic fixed-order reduction of np partials, then the scalar update
// of Algorithm 1 selected by mode.
__global__ __launch_bounds__(256) void k_scalar(int mode,
                                                const double* __restrict__ psum,
                                                const double* __restrict__ pmax,
                                                int np, Scalars* sc, double tol) {
  const bool gated = (mode == kModeYd || mode == kModeRr || mode == kModeMu);
  if (gated && sc->done) return;
  double s = 0.0, m = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    s += psum[k];
    if (pmax) m = fmax(m, pmax[k]);
  }
  s = block_sum<256>(s);
  if (pmax) m = block_max<256>(m);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case kModeRd2:
      sc->rd2 = s;
      sc->rdinf = m;
      sc->rr = s;     // residual of the zero start
      sc->rinf = m;
      sc->tol2 = tol * tol * s;
      sc->done = kRunning;
      break;
    case kModeYd:
      sc->yd = s;
      if (!(s > 0.0) || !isfinite(s) || !isfinite(sc->mu)) sc->done = kBreakdown;
      else sc->theta = sc->mu / s;
      break;
    case kModeRr:
      sc->rr = s;
      sc->iter += 1;
      if (!isfinite(s)) sc->done = kBreakdown;
      else if (s <= sc->tol2) sc->done = kConverged;
      else if (sc->iter >= sc->max_iter) sc->done = kMaxIter;
      break;
    case kModeMu:
      if (!(s > 0.0) || !isfinite(s)) {
        sc->done = kBreakdown;
      } else {
        sc->beta = s / sc->mu;
        sc->mu = s;
      }
      break;
    case kModeMuInit:
      sc->mu = s;
      sc->beta = 0.0;
      sc->done = (s > 0.0 && isfinite(s)) ? kRunning : kBreakdown;
      break;
    case kModeTrue:
      sc->rr = s;
      sc->rinf = m;
      break;
  }
}

// interface [T+1][N][K][n] -> internal [p][c][t]
__global__ void k_to_internal(Dims D, const double* __restrict__ abi,
                              double* __restrict__ in) {
  const long long total = (long long)D.real_nodes * D.n * D.Tt;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       g < total; g += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(g % D.Tt);
    const long long pc = g / D.Tt;  // p*n + c
    in[pc * D.ldt + t] = abi[(long long)t * D.real_nodes * D.n + pc];
  }
}
__global__ void k_to_abi(Dims D, const double* __restrict__ in,
                         double* __restrict__ abi) {
  const long long per_t = (long long)D.real_nodes * D.n;
  const long long total = per_t * D.Tt;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       g < total; g += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(g / per_t);
    const long long pc = g - (long long)t * per_t;
    abi[g] = in[pc * D.ldt + t];
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
  const int lane = threadIdx.x & (kWave - 1);
  const int p = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int t = blockIdx.y * kWave + lane;
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

inline dim3 node_grid(const Dims& D) {
  return dim3((D.real_nodes + 3) / 4, (D.Tt + kWave - 1) / kWave);
}

}  // namespace

#define LQG_DISPATCH_N(n, CALL) \
  switch (n) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    case 4: CALL(4); break;     \
    default: break;             \
  }

int delta_apply(const Dims& D, const Coef& C, const double* d, double* y,
                double* partial, const Scalars* sc, int check_done,
                hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS) \
  hipLaunchKernelGGL(k_delta<NS>, g, dim3(256), 0, s, D, C, d, y, partial, sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
  return (int)(g.x * g.y);
}

void omega_rhs(const Dims& D, const Coef& C, const double* rho,
               const double* th, double* tau, const Scalars* sc,
               int check_done, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS) \
  hipLaunchKernelGGL(k_omega<NS>, g, dim3(256), 0, s, D, C, rho, th, tau, sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

void xi_rhs(const Dims& D, const Coef& C, const double* r, const double* dl,
            double* rho, const Scalars* sc, int check_done, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS) \
  hipLaunchKernelGGL(k_xi<NS>, g, dim3(256), 0, s, D, C, r, dl, rho, sc, check_done)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

void phi_solve(const Dims& D, const Coef& C, const double* tau, double* out,
               const Scalars* sc, int check_done, int qt_distinct,
               hipStream_t s) {
  const dim3 g(D.V, (D.Tt + kWave - 1) / kWave);
#define CALL(NS)                                                            \
  hipLaunchKernelGGL(k_phi_solve<NS>, g, dim3(64), 0, s, D, C, tau, out, sc, \
                     check_done, qt_distinct)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

void recover(const Dims& D, const Coef& C, const double* dl, double* x,
             double* u, hipStream_t s) {
  const dim3 g = node_grid(D);
#define CALL(NS) hipLaunchKernelGGL(k_recover<NS>, g, dim3(256), 0, s, D, C, dl, x, u)
  LQG_DISPATCH_N(D.n, CALL)
#undef CALL
}

void vec_dir(const Dims& D, const double* q, double* d, const Scalars* sc,
             hipStream_t s) {
  hipLaunchKernelGGL(k_dir, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, q, d, sc);
}
int vec_update(const Dims& D, const double* d, const double* y, double* dl,
               double* r, double* partial, const Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, d, y,
                     dl, r, partial, sc);
  return kFlatBlocks;
}
int vec_dot(const Dims& D, const double* a, const double* b, double* partial,
            const Scalars* sc, int check_done, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, a, b,
                     partial, sc, check_done);
  return kFlatBlocks;
}
int vec_sub_norm(const Dims& D, const double* rd, const double* y, double* r,
                 double* psum, double* pmax, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_norm, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, rd,
                     y, r, psum, pmax);
  return kFlatBlocks;
}
int vec_norms(const Dims& D, const double* a, double* psum, double* pmax,
              hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, a,
                     psum, pmax);
  return kFlatBlocks;
}
void vec_copy(const Dims& D, const double* a, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, a, b);
}
void vec_zero(double* a, long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(kFlatBlocks), dim3(256), 0, s, len, a);
}
void scalar_step(int mode, const double* psum, const double* pmax, int np,
                 Scalars* sc, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(256), 0, s, mode, psum, pmax, np,
                     sc, tol);
}
void to_internal(const Dims& D, const double* abi, double* internal,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_to_internal, dim3(kFlatBlocks), dim3(256), 0, s, D, abi,
                     internal);
}
void to_abi(const Dims& D, const double* internal, double* abi, hipStream_t s) {
  hipLaunchKernelGGL(k_to_abi, dim3(kFlatBlocks), dim3(256), 0, s, D, internal,
                     abi);
}

}  // namespace lqg
