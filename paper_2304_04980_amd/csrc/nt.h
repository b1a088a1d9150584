// Launchers of the node-temporal block Jacobi preconditioner (nt.hip).
#pragma once
#include "launch.h"
#include "tv.h"

namespace lqg {

// Doubles of the factor table [t][3][n*n][nodes] (Linv_t, M_t, N_t).
size_t nt_table_doubles(const Dims& D);
// Block Cholesky in t of every node's block of D_node (tv != 0: from the
// time-varying arrays V, else from the time-invariant blocks of C).
void nt_factor(const Dims& D, const Coef& C, const TvCoef<double>& V, int tv, double* tab,
               Scalars* sc, hipStream_t s);
// out = D_node^-1 tau.
template <typename T>
void nt_solve(const Dims& D, const T* tab, const T* tau, T* out, const Scalars* sc, int check,
              hipStream_t s);

}  // namespace lqg
