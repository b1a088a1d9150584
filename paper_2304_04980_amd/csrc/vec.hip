// Flat vector kernels of Algorithm 1 (direction, update, dot products,
// norms), the device-side scalar step, the layout conversions between the
// interface order [T+1][N][K][n] and the internal time-fastest order, and the
// FP64 <-> FP32 conversions of the iterative refinement.  Vectors of element
// type T are processed as flat arrays of D.vlen entries (padding entries are
// zero and stay zero); every partial sum is accumulated in FP64 with a
// fixed-order reduction, so results are bitwise reproducible.
#include "launch.h"

namespace lqg {
namespace {

#define GRID_STRIDE(g, n)                                                   \
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n; \
       g += (long long)gridDim.x * blockDim.x)

// In FP32, k_dir and k_dot stream 16-byte units (4 floats), two per thread
// and loop pass, so that each wavefront keeps more bytes in flight; a vector
// length that is not a multiple of the unit ends in a scalar tail (D.vlen
// always is one).  FP64 and k_update (four streams) keep the plain loop,
// which measured faster there.
template <typename T>
struct alignas(16) Unit16 {
  static constexpr int kLanes = 16 / sizeof(T);
  T e[kLanes];
};

template <typename T>
__global__ __launch_bounds__(256) void k_dir(long long n, const T* __restrict__ q,
                                             T* __restrict__ d,
                                             const Scalars* sc) {
  if (sc->done) return;
  const T beta = (T)sc->beta;
  if constexpr (sizeof(T) == 8) {
    GRID_STRIDE(g, n) d[g] = fma(beta, d[g], q[g]);
    return;
  }
  using V = Unit16<T>;
  constexpr int W = V::kLanes;
  const long long nu = n / W, stride = (long long)gridDim.x * blockDim.x;
  const V* __restrict__ qv = reinterpret_cast<const V*>(q);
  V* __restrict__ dv = reinterpret_cast<V*>(d);
  long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; g + stride < nu; g += 2 * stride) {
    V a = dv[g], b = dv[g + stride];
    const V qa = qv[g], qb = qv[g + stride];
#pragma unroll
    for (int e = 0; e < W; ++e) {
      a.e[e] = fma(beta, a.e[e], qa.e[e]);
      b.e[e] = fma(beta, b.e[e], qb.e[e]);
    }
    dv[g] = a;
    dv[g + stride] = b;
  }
  if (g < nu) {
    V a = dv[g];
    const V qa = qv[g];
#pragma unroll
    for (int e = 0; e < W; ++e) a.e[e] = fma(beta, a.e[e], qa.e[e]);
    dv[g] = a;
  }
  for (long long t = nu * W + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += stride)
    d[t] = fma(beta, d[t], q[t]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_update(long long n,
                                                const T* __restrict__ d,
                                                const T* __restrict__ y,
                                                T* __restrict__ x,
                                                T* __restrict__ r,
                                                double* __restrict__ partial,
                                                const Scalars* sc) {
  if (sc->done) return;
  const T th = (T)sc->theta;
  double acc = 0.0;
  GRID_STRIDE(g, n) {
    x[g] = fma(th, d[g], x[g]);
    const T rn = fma(-th, y[g], r[g]);
    r[g] = rn;
    acc = fma((double)rn, (double)rn, acc);
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot(long long n, const T* __restrict__ a,
                                             const T* __restrict__ b,
                                             double* __restrict__ partial,
                                             const Scalars* sc, int check) {
  if (check && sc->done) return;
  double acc = 0.0;
  if constexpr (sizeof(T) == 8) {
    GRID_STRIDE(g, n) acc = fma((double)a[g], (double)b[g], acc);
    acc = block_sum<256>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
    return;
  }
  using V = Unit16<T>;
  constexpr int W = V::kLanes;
  const long long nu = n / W, stride = (long long)gridDim.x * blockDim.x;
  const V* __restrict__ av = reinterpret_cast<const V*>(a);
  const V* __restrict__ bv = reinterpret_cast<const V*>(b);
  long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; g + stride < nu; g += 2 * stride) {
    const V a0 = av[g], b0 = bv[g], a1 = av[g + stride], b1 = bv[g + stride];
#pragma unroll
    for (int e = 0; e < W; ++e) acc = fma((double)a0.e[e], (double)b0.e[e], acc);
#pragma unroll
    for (int e = 0; e < W; ++e) acc = fma((double)a1.e[e], (double)b1.e[e], acc);
  }
  if (g < nu) {
    const V a0 = av[g], b0 = bv[g];
#pragma unroll
    for (int e = 0; e < W; ++e) acc = fma((double)a0.e[e], (double)b0.e[e], acc);
  }
  for (long long t = nu * W + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += stride)
    acc = fma((double)a[t], (double)b[t], acc);
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_norms(long long n, const T* __restrict__ a,
                                               double* __restrict__ psum,
                                               double* __restrict__ pmax) {
  double acc = 0.0, mx = 0.0;
  GRID_STRIDE(g, n) {
    const double v = (double)a[g];
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

__global__ __launch_bounds__(256) void k_sub_norm(long long n,
                                                  const double* __restrict__ rd,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ r,
                                                  double* __restrict__ psum,
                                                  double* __restrict__ pmax) {
  double acc = 0.0, mx = 0.0;
  GRID_STRIDE(g, n) {
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

// out = (T)(s * a)
template <typename T>
__global__ __launch_bounds__(256) void k_scale_to(long long n,
                                                  const double* __restrict__ a,
                                                  double s, T* __restrict__ out) {
  GRID_STRIDE(g, n) out[g] = (T)(s * a[g]);
}

// x += s * (double)e
template <typename T>
__global__ __launch_bounds__(256) void k_axpy_from(long long n, double s,
                                                   const T* __restrict__ e,
                                                   double* __restrict__ x) {
  GRID_STRIDE(g, n) x[g] = fma(s, (double)e[g], x[g]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(long long n, T* __restrict__ a) {
  GRID_STRIDE(g, n) a[g] = T(0);
}

__global__ __launch_bounds__(256) void k_to_float(long long n,
                                                  const double* __restrict__ a,
                                                  float* __restrict__ b) {
  GRID_STRIDE(g, n) b[g] = (float)a[g];
}

// Deterministic fixed-order reduction of np partials, then the scalar update
// of Algorithm 1 selected by mode.  Four independent accumulators per thread
// keep several loads in flight.
constexpr int kScalarThreads = 1024;
__global__ __launch_bounds__(kScalarThreads) void k_scalar(int mode,
                                                           const double* __restrict__ psum,
                                                           const double* __restrict__ pmax,
                                                           int np, Scalars* sc, double tol) {
  if (scalar_mode_gated(mode) && sc->done) return;
  constexpr int B = kScalarThreads;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, m = 0.0;
  int k = threadIdx.x;
  for (; k + 3 * B < np; k += 4 * B) {
    s0 += psum[k];
    s1 += psum[k + B];
    s2 += psum[k + 2 * B];
    s3 += psum[k + 3 * B];
    if (pmax)
      m = fmax(fmax(m, fmax(pmax[k], pmax[k + B])), fmax(pmax[k + 2 * B], pmax[k + 3 * B]));
  }
  for (; k < np; k += B) {
    s0 += psum[k];
    if (pmax) m = fmax(m, pmax[k]);
  }
  double s = block_sum<B>((s0 + s1) + (s2 + s3));
  if (pmax) m = block_max<B>(m);
  if (threadIdx.x != 0) return;
  scalar_apply(mode, s, m, sc, nullptr, tol);
}

// interface [T+1][N][K][n] -> internal [p][c][t]
__global__ void k_to_internal(Dims D, const double* __restrict__ abi,
                              double* __restrict__ in) {
  const long long total = (long long)D.real_nodes * D.n * D.Tt;
  GRID_STRIDE(g, total) {
    const int t = (int)(g % D.Tt);
    const long long pc = g / D.Tt;  // p*n + c
    in[pc * D.ldt + t] = abi[(long long)t * D.real_nodes * D.n + pc];
  }
}
__global__ void k_to_abi(Dims D, const double* __restrict__ in,
                         double* __restrict__ abi) {
  const long long per_t = (long long)D.real_nodes * D.n;
  const long long total = per_t * D.Tt;
  GRID_STRIDE(g, total) {
    const int t = (int)(g / per_t);
    const long long pc = g - (long long)t * per_t;
    abi[g] = in[pc * D.ldt + t];
  }
}

}  // namespace

template <typename T>
void vec_dir(const Dims& D, const T* q, T* d, const Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_dir<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, q, d, sc);
}
template <typename T>
int vec_update(const Dims& D, const T* d, const T* y, T* x, T* r,
               double* partial, const Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, d,
                     y, x, r, partial, sc);
  return kFlatBlocks;
}
template <typename T>
int vec_dot(const Dims& D, const T* a, const T* b, double* partial,
            const Scalars* sc, int check_done, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, a, b,
                     partial, sc, check_done);
  return kFlatBlocks;
}
template <typename T>
int vec_norms(const Dims& D, const T* a, double* psum, double* pmax,
              hipStream_t s) {
  hipLaunchKernelGGL(k_norms<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, a,
                     psum, pmax);
  return kFlatBlocks;
}
template <typename T>
void vec_zero(T* a, long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_zero<T>, dim3(kFlatBlocks), dim3(256), 0, s, len, a);
}
template <typename T>
void vec_scale_to(const Dims& D, const double* a, double scale, T* out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen,
                     a, scale, out);
}
template <typename T>
void vec_axpy_from(const Dims& D, double scale, const T* e, double* x,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_from<T>, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen,
                     scale, e, x);
}

#define LQG_INSTANTIATE(T)                                                        \
  template void vec_dir<T>(const Dims&, const T*, T*, const Scalars*, hipStream_t); \
  template int vec_update<T>(const Dims&, const T*, const T*, T*, T*, double*,    \
                             const Scalars*, hipStream_t);                        \
  template int vec_dot<T>(const Dims&, const T*, const T*, double*,               \
                          const Scalars*, int, hipStream_t);                      \
  template int vec_norms<T>(const Dims&, const T*, double*, double*, hipStream_t); \
  template void vec_zero<T>(T*, long long, hipStream_t);                          \
  template void vec_scale_to<T>(const Dims&, const double*, double, T*,           \
                                hipStream_t);                                     \
  template void vec_axpy_from<T>(const Dims&, double, const T*, double*,          \
                                 hipStream_t);
LQG_INSTANTIATE(double)
LQG_INSTANTIATE(float)
#undef LQG_INSTANTIATE

int vec_sub_norm(const Dims& D, const double* rd, const double* y, double* r,
                 double* psum, double* pmax, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_norm, dim3(kFlatBlocks), dim3(256), 0, s, D.vlen, rd,
                     y, r, psum, pmax);
  return kFlatBlocks;
}
void copy_to_float(const double* a, float* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(kFlatBlocks), dim3(256), 0, s, n, a, b);
}
void scalar_step(int mode, const double* psum, const double* pmax, int np,
                 Scalars* sc, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kScalarThreads), 0, s, mode, psum, pmax, np,
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
