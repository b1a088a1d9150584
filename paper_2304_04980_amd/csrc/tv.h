// Launchers of the time-varying-data kernels (tv.hip).
#pragma once
#include "launch.h"

namespace lqg {

// The time-fastest coefficient arrays of the time-varying operator (layouts
// in tv.hip) in element type T, and the block solve's parking vector.
template <typename T>
struct TvCoef {
  const T *G13, *Qi, *Cdn, *Cup, *Fw, *Bw;
  const T *AT5, *RiBT;  // FP64 only (recovery)
  T* w;                 // forward-sweep result of the block solve
  const T *A5 = nullptr, *BRB = nullptr;  // factored Delta apply (TA5, TBRB)
  T* dw = nullptr;      // the factored Delta apply's intermediate w
};

// y = Delta d (and one FP64 partial of d'y per workgroup into partial);
// returns the number of partials.  The factored two-pass form: needs C.A5,
// C.BRB and the intermediate vector C.dw.
template <typename T>
int tv_delta_apply(const Dims& D, const TvCoef<T>& C, const T* d, T* y, double* partial,
                   const Scalars* sc, int check, hipStream_t s);
template <typename T>
void tv_xi_rhs(const Dims& D, const TvCoef<T>& C, const T* r, const T* dl, T* rho,
               const Scalars* sc, int check, hipStream_t s);
template <typename T>
void tv_omega_rhs(const Dims& D, const TvCoef<T>& C, const T* rho, const T* th, T* tau,
                  const Scalars* sc, int check, hipStream_t s);
template <typename T>
void tv_phi_solve(const Dims& D, const TvCoef<T>& C, const T* tau, T* out,
                  const Scalars* sc, int check, hipStream_t s);
void tv_recover(const Dims& D, const TvCoef<double>& C, const double* dl, double* x,
                double* u, hipStream_t s);
// Time slices assembled per batch before their scatter into the time-fastest
// arrays (the assembly scratch holds this many slices).
constexpr int kTvBatch = 16;
// Blocks of the nsl time slices s0 .. s0 + nsl - 1 assembled in the
// time-invariant layouts of S (each array of S holding kTvBatch slices back to
// back) into the time-varying arrays of C; slice T contributes Q_T^-1 only.
void tv_scatter_batch(const Dims& D, const Coef& S, const TvCoef<double>& C, int s0, int nsl,
                      hipStream_t s);
// One-chain factorisation of every Phi_bar_{v,t}, t = 0..T (C.tv_ld = ldt).
void tv_factor(const Dims& D, const Coef& C, Scalars* sc, hipStream_t s);

}  // namespace lqg
