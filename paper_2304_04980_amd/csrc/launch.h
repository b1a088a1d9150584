// Launchers of the lqgrid kernels (host-callable), one per kernel family.
#pragma once
#include "lqg_internal.h"

namespace lqg {

// The caller's problem arrays (device pointers, [N][K][...] layouts).
struct ProblemIn {
  int K, N, n, m;
  const double *A, *A_nbr, *B, *Q, *R, *QT;
};

// setup.hip
void launch_setup(const Dims& D, const ProblemIn& P, const Coef& C,
                  Scalars* sc, hipStream_t s);
void launch_factor(const Dims& D, const Coef& C, Scalars* sc, hipStream_t s);
void launch_rhs_init(const Dims& D, const double* x0, double* rd,
                     hipStream_t s);

// ops.hip (T = double or float).  delta_apply returns the number of partial
// sums it wrote.  check_done != 0 makes the kernels return at once when the
// device flag sc->done is set (converged iterations become no-ops).
template <typename T>
int delta_apply(const Dims& D, const OpCoef<T>& C, const T* d, T* y,
                double* partial, const Scalars* sc, int check_done,
                hipStream_t s);
template <typename T>
void omega_rhs(const Dims& D, const OpCoef<T>& C, const T* rho, const T* th,
               T* tau, const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
void xi_rhs(const Dims& D, const OpCoef<T>& C, const T* r, const T* dl, T* rho,
            const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
void phi_solve(const Dims& D, const OpCoef<T>& C, const T* tau, T* out,
               const Scalars* sc, int check_done, int qt_distinct,
               hipStream_t s);
void recover(const Dims& D, const Coef& C, const double* dl, double* x,
             double* u, hipStream_t s);

// vec.hip: flat vector kernels over D.vlen entries
constexpr int kFlatBlocks = 1024;
template <typename T>
void vec_dir(const Dims& D, const T* q, T* d, const Scalars* sc, hipStream_t s);
template <typename T>
int vec_update(const Dims& D, const T* d, const T* y, T* x, T* r,
               double* partial, const Scalars* sc, hipStream_t s);
template <typename T>
int vec_dot(const Dims& D, const T* a, const T* b, double* partial,
            const Scalars* sc, int check_done, hipStream_t s);
template <typename T>
int vec_norms(const Dims& D, const T* a, double* psum, double* pmax,
              hipStream_t s);
template <typename T>
void vec_zero(T* a, long long len, hipStream_t s);
template <typename T>
void vec_scale_to(const Dims& D, const double* a, double scale, T* out,
                  hipStream_t s);
template <typename T>
void vec_axpy_from(const Dims& D, double scale, const T* e, double* x,
                   hipStream_t s);
int vec_sub_norm(const Dims& D, const double* rd, const double* y, double* r,
                 double* psum, double* pmax, hipStream_t s);
void copy_to_float(const double* a, float* b, long long n, hipStream_t s);

enum ScalarMode {
  kModeRd2 = 0,   // rd2 = sum, rdinf = max; tol2 = tol^2 rd2; done = 0
  kModeYd = 1,    // yd = sum; theta = mu / yd (breakdown if yd <= 0)
  kModeRr = 2,    // rr = sum; iter++; convergence / max_iter test
  kModeMu = 3,    // mu' = sum; beta = mu'/mu; mu = mu'
  kModeMuInit = 4,// mu = sum; beta = 0; done = 0
  kModeTrue = 5   // rr = sum, rinf = max (true residual), no state change
};
void scalar_step(int mode, const double* psum, const double* pmax, int np,
                 Scalars* sc, double tol, hipStream_t s);

// layout conversion between the [T+1][N][K][n] interface order and the
// internal time-fastest order
void to_internal(const Dims& D, const double* abi, double* internal,
                 hipStream_t s);
void to_abi(const Dims& D, const double* internal, double* abi, hipStream_t s);

}  // namespace lqg
