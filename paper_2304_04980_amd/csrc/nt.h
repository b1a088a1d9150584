// Launchers of the node-temporal block Jacobi preconditioner (nt.hip).
#pragma once
#include "launch.h"
#include "tv.h"

namespace lqg {

// Doubles of the factor table [t][node group of 16][4][16][n][n] (Linv_t, M_t,
// N_t, Linv_t').
size_t nt_table_doubles(const Dims& D);
// Block Cholesky in t of every node's block of D_node (tv != 0: from the
// time-varying arrays V, else from the time-invariant blocks of C).
void nt_factor(const Dims& D, const Coef& C, const TvCoef<double>& V, int tv, double* tab,
               Scalars* sc, hipStream_t s);
// out = D_node^-1 tau; zbuf (a vector, distinct from tau and out) holds the
// forward sweep's result.
template <typename T>
void nt_solve(const Dims& D, const T* tab, const T* tau, T* zbuf, T* out, const Scalars* sc,
              int check, hipStream_t s);

}  // namespace lqg
