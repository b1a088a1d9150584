// Single-problem setup kernels (the bodies are shared with the batched
// form): ingest and assembly, the banded block Cholesky factorisation of
// every distinct Phi_bar_{v,t}, and the right-hand side r_delta.
#include "bodies_setup.h"

namespace lqg {
namespace {
using namespace dev;

__global__ void k_node_prep(Dims D, ProblemIn P, Coef C, Scalars* sc) {
  node_prep(D, P, C, sc, blockIdx.x * blockDim.x + threadIdx.x);
}
template <int NS>
__global__ void k_stencil(Dims D, ProblemIn P, Coef C) {
  stencil<NS>(D, P, C, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}
// one 64-thread workgroup per (v, cls)
__global__ __launch_bounds__(64) void k_factor(Dims D, Coef C, Scalars* sc) {
  factor(D, C, sc, blockIdx.x, blockIdx.y);
}
__global__ __launch_bounds__(128) void k_factor_twisted(Dims D, Coef C, Scalars* sc) {
  factor_twisted(D, C, sc, blockIdx.x, blockIdx.y);
}
__global__ void k_rhs_init(Dims D, const double* __restrict__ x0,
                           const int* __restrict__ nsz, double* __restrict__ rd) {
  rhs_init(D, x0, nsz, rd, blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void k_rhs_boundary(Dims D, const double* __restrict__ Anbr, Boundary bc,
                               double* __restrict__ rd) {
  rhs_boundary(D, Anbr, bc.alo, bc.ahi, bc.blo, bc.bhi, rd,
               (long long)blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void k_ingest_mask(Dims D, ProblemIn P, const int* nsz, const int* msz,
                              ProblemIn out, int* nsz_out, Scalars* sc) {
  ingest_mask(D, P, nsz, msz, out, nsz_out, sc, blockIdx.x * blockDim.x + threadIdx.x);
}

// Slice b of a time-varying batch (launch.h TvSlices).
__device__ inline ProblemIn user_slice(const ProblemIn& P, const TvSlices& S, int b) {
  const int s = S.s0 + b, sl = s < S.T ? s : S.T - 1;
  ProblemIn r = P;
  r.A = P.A + sl * S.sA;
  r.A_nbr = P.A_nbr + sl * S.sN;
  r.B = P.B + sl * S.sB;
  r.R = P.R + sl * S.sR;
  r.Q = (s == S.T && S.QT) ? S.QT : P.Q + sl * S.sA;
  r.QT = r.Q;
  return r;
}
__device__ inline ProblemIn in_slice(const ProblemIn& P, const TvSlices& S, int b) {
  ProblemIn r = P;
  r.A = P.A + b * S.iA;
  r.A_nbr = P.A_nbr + b * S.iN;
  r.B = P.B + b * S.iB;
  r.Q = P.Q + b * S.iA;
  r.R = P.R + b * S.iR;
  r.QT = r.Q;
  return r;
}
__device__ inline Coef coef_slice(const Coef& C, const TvSlices& S, int b) {
  Coef r = C;
  r.G13 = C.G13 + b * S.cG13;
  r.Qi = C.Qi + b * S.cQi;
  r.Cdn = C.Cdn + b * S.c5;
  r.Cup = C.Cup + b * S.c5;
  r.AT5 = C.AT5 + b * S.c5;
  r.A5 = C.A5 + b * S.c5;
  r.RiBT = C.RiBT + b * S.cRiBT;
  r.BRB = C.BRB + b * S.cBRB;
  return r;
}
__global__ void k_ingest_tv(Dims D, ProblemIn P, TvSlices S, const int* nsz, const int* msz,
                            ProblemIn in, int* nsz_out, Scalars* sc) {
  const int b = blockIdx.y;
  ingest_mask(D, user_slice(P, S, b), nsz, msz, in_slice(in, S, b), nsz_out, sc,
              blockIdx.x * blockDim.x + threadIdx.x);
}
__global__ void k_node_prep_tv(Dims D, ProblemIn in, TvSlices S, Coef C, Scalars* sc) {
  const int b = blockIdx.y;
  node_prep(D, in_slice(in, S, b), coef_slice(C, S, b), sc,
            blockIdx.x * blockDim.x + threadIdx.x);
}
template <int NS>
__global__ void k_stencil_tv(Dims D, ProblemIn in, TvSlices S, Coef C) {
  const int b = blockIdx.y;
  stencil<NS>(D, in_slice(in, S, b), coef_slice(C, S, b),
              (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

}  // namespace

void launch_setup(const Dims& D, const ProblemIn& P, const Coef& C,
                  Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_node_prep, dim3((D.nodes + 127) / 128), dim3(128), 0, s,
                     D, P, C, sc);
  const long long work = (long long)D.nodes * 18;
  const dim3 g((unsigned)((work + 127) / 128));
  switch (D.n) {
    case 1: hipLaunchKernelGGL(k_stencil<1>, g, dim3(128), 0, s, D, P, C); break;
    case 2: hipLaunchKernelGGL(k_stencil<2>, g, dim3(128), 0, s, D, P, C); break;
    case 3: hipLaunchKernelGGL(k_stencil<3>, g, dim3(128), 0, s, D, P, C); break;
    case 4: hipLaunchKernelGGL(k_stencil<4>, g, dim3(128), 0, s, D, P, C); break;
    default: break;
  }
}

void launch_factor(const Dims& D, const Coef& C, Scalars* sc, hipStream_t s) {
  if (twisted(D))
    hipLaunchKernelGGL(k_factor_twisted, dim3(D.V, 2), dim3(128), 0, s, D, C, sc);
  else
    hipLaunchKernelGGL(k_factor, dim3(D.V, 2), dim3(64), 0, s, D, C, sc);
}

void launch_rhs_init(const Dims& D, const double* x0, double* rd,
                     hipStream_t s, const int* nsz) {
  const int work = D.real_nodes * D.n;
  hipLaunchKernelGGL(k_rhs_init, dim3((work + 255) / 256), dim3(256), 0, s, D,
                     x0, nsz, rd);
}

void launch_rhs_boundary(const Dims& D, const double* Anbr, const Boundary& bc,
                         double* rd, hipStream_t s) {
  const long long work = (long long)D.real_nodes * D.T;
  hipLaunchKernelGGL(k_rhs_boundary, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                     s, D, Anbr, bc, rd);
}

void launch_ingest_setup_tv(const Dims& D, const ProblemIn& P, const TvSlices& S,
                            const int* nsz, const int* msz, const ProblemIn& in,
                            int* nsz_out, const Coef& C, Scalars* sc, hipStream_t s) {
  const unsigned nb = (unsigned)S.nsl;
  hipLaunchKernelGGL(k_ingest_tv, dim3((D.real_nodes + 127) / 128, nb), dim3(128), 0, s, D, P,
                     S, nsz, msz, in, nsz_out, sc);
  hipLaunchKernelGGL(k_node_prep_tv, dim3((D.nodes + 127) / 128, nb), dim3(128), 0, s, D, in,
                     S, C, sc);
  const long long work = (long long)D.nodes * 18;
  const dim3 g((unsigned)((work + 127) / 128), nb);
  switch (D.n) {
    case 1: hipLaunchKernelGGL(k_stencil_tv<1>, g, dim3(128), 0, s, D, in, S, C); break;
    case 2: hipLaunchKernelGGL(k_stencil_tv<2>, g, dim3(128), 0, s, D, in, S, C); break;
    case 3: hipLaunchKernelGGL(k_stencil_tv<3>, g, dim3(128), 0, s, D, in, S, C); break;
    case 4: hipLaunchKernelGGL(k_stencil_tv<4>, g, dim3(128), 0, s, D, in, S, C); break;
    default: break;
  }
}

void launch_ingest(const Dims& D, const ProblemIn& P, const int* nsz, const int* msz,
                   const ProblemIn& out, int* nsz_out, Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_ingest_mask, dim3((D.real_nodes + 127) / 128), dim3(128), 0, s, D,
                     P, nsz, msz, out, nsz_out, sc);
}

}  // namespace lqg
