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

// ops.hip -- every launcher returns the number of partial sums it wrote (0
// if none).  check_done != 0 makes the kernels return at once when the
// device flag sc->done is set (converged iterations become no-ops).
int delta_apply(const Dims& D, const Coef& C, const double* d, double* y,
                double* partial, const Scalars* sc, int check_done,
                hipStream_t s);
void omega_rhs(const Dims& D, const Coef& C, const double* rho,
               const double* th, double* tau, const Scalars* sc,
               int check_done, hipStream_t s);
void xi_rhs(const Dims& D, const Coef& C, const double* r, const double* dl,
            double* rho, const Scalars* sc, int check_done, hipStream_t s);
void phi_solve(const Dims& D, const Coef& C, const double* tau, double* out,
               const Scalars* sc, int check_done, int qt_distinct,
               hipStream_t s);

// flat vector kernels over D.vlen entries
constexpr int kFlatBlocks = 1024;
void vec_dir(const Dims& D, const double* q, double* d, const Scalars* sc,
             hipStream_t s);
int vec_update(const Dims& D, const double* d, const double* y, double* dl,
               double* r, double* partial, const Scalars* sc, hipStream_t s);
int vec_dot(const Dims& D, const double* a, const double* b, double* partial,
            const Scalars* sc, int check_done, hipStream_t s);
int vec_sub_norm(const Dims& D, const double* rd, const double* y, double* r,
                 double* psum, double* pmax, hipStream_t s);
int vec_norms(const Dims& D, const double* a, double* psum, double* pmax,
              hipStream_t s);
void vec_copy(const Dims& D, const double* a, double* b, hipStream_t s);
void vec_zero(double* a, long long len, hipStream_t s);

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
void recover(const Dims& D, const Coef& C, const double* dl, double* x,
             double* u, hipStream_t s);

}  // namespace lqg
