// Setup bodies: ingest of the problem arrays, assembly of the time-invariant
// blocks of Delta and of its splittings, and the banded block Cholesky
// factorisation of every distinct Phi_bar_{v,t}.
//
//   Psi_hat_t = Q_t^-1 + A_hat Q^-1 A_hat' + B_hat R^-1 B_hat'   (t >= 1)
//   Psi_hat_0 = Q_0^-1,  Xi_hat_t = -A_hat Q^-1                (eq. "structure_of_Delta")
//   Phi_bar_{v,t} = diagonal super-block of Psi_hat_t over the column pair of v
//                                          (eq. "constructing_Phi_Omega_matrices")
//   each Phi_bar_{v,t} is factored by block Cholesky once per solve (Sec. IV-B)
#pragma once
#include "launch.h"

namespace lqg {
namespace dev {

// Pointer to the n x n block A_hat[p, s] (p's dynamics coupling to s) in the
// caller's [N][K][...] arrays, or nullptr when s is not p or one of its four
// in-grid neighbours.
__device__ inline const double* ahat_block(const ProblemIn& P, int ip, int jp, int is,
                                    int js) {
  const int K = P.K, N = P.N, n = P.n;
  if (is < 0 || is >= K || js < 0 || js >= N) return nullptr;
  const size_t node = (size_t)jp * K + ip;
  const size_t nn = (size_t)n * n;
  if (is == ip && js == jp) return P.A + node * nn;
  int slot = -1;
  if (is == ip && js == jp - 1) slot = 0;       // E
  else if (is == ip && js == jp + 1) slot = 1;  // F
  else if (is == ip - 1 && js == jp) slot = 2;  // G
  else if (is == ip + 1 && js == jp) slot = 3;  // H
  if (slot < 0) return nullptr;
  return P.A_nbr + (node * 4 + slot) * nn;
}

// In-place inverse of a small SPD matrix by Gauss-Jordan with partial
// pivoting (setup only; sizes <= 8).  Returns false on a zero pivot.
__device__ inline bool small_inverse(double* M, int n) {
  double W[kMaxM * 2 * kMaxM];
  const int w2 = 2 * n;
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < w2; ++c)
      W[r * w2 + c] = c < n ? M[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(W[r * w2 + c]) > fabs(W[piv * w2 + c])) piv = r;
    if (!(fabs(W[piv * w2 + c]) > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < w2; ++k) {
        double tmp = W[c * w2 + k];
        W[c * w2 + k] = W[piv * w2 + k];
        W[piv * w2 + k] = tmp;
      }
    const double inv = 1.0 / W[c * w2 + c];
    for (int k = 0; k < w2; ++k) W[c * w2 + k] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = W[r * w2 + c];
      if (f != 0.0)
        for (int k = 0; k < w2; ++k) W[r * w2 + k] -= f * W[c * w2 + k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) M[r * n + c] = W[r * w2 + n + c];
  return true;
}

// True when the small symmetric matrix M (n x n) has a Cholesky
// factorisation with positive pivots (the problem statement requires
// Q, Q_T, R positive definite).
__device__ inline bool small_spd(const double* M, int n) {
  double L[kMaxM * kMaxM];
  for (int c = 0; c < n; ++c) {
    double s = M[c * n + c];
    for (int k = 0; k < c; ++k) s -= L[c * n + k] * L[c * n + k];
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double dg = sqrt(s);
    L[c * n + c] = dg;
    for (int r = c + 1; r < n; ++r) {
      double t = M[r * n + c];
      for (int k = 0; k < c; ++k) t -= L[r * n + k] * L[c * n + k];
      L[r * n + c] = t / dg;
    }
  }
  return true;
}

// Node p: Q^-1, Q_T^-1, Q_T^-1 - Q^-1, Q, R^-1 B'.
__device__ inline void node_prep(const Dims& D, const ProblemIn& P, const Coef& C,
                                 Scalars* sc, int p) {
  if (p >= D.nodes) return;
  const int n = D.n, m = D.m;
  const size_t nn = (size_t)n * n;
  double* Qi = C.Qi + p * nn;
  double* QTi = C.QTi + p * nn;
  double* QTd = C.QTd + p * nn;
  double* Qm = C.Qm + p * nn;
  double* RiBT = C.RiBT + (size_t)p * m * n;
  if (p >= D.real_nodes) {  // dummy column: all zero
    for (size_t k = 0; k < nn; ++k) Qi[k] = QTi[k] = QTd[k] = Qm[k] = 0.0;
    for (int k = 0; k < m * n; ++k) RiBT[k] = 0.0;
    if (C.BRB)
      for (size_t k = 0; k < nn; ++k) C.BRB[p * nn + k] = 0.0;
    return;
  }
  double q[kMaxM * kMaxM], qt[kMaxM * kMaxM], r[kMaxM * kMaxM];
  const double* Qs = P.Q + p * nn;
  const double* QTs = (P.QT ? P.QT : P.Q) + p * nn;
  bool differs = false;
  for (size_t k = 0; k < nn; ++k) {
    q[k] = Qs[k];
    qt[k] = QTs[k];
    Qm[k] = Qs[k];
    differs |= (q[k] != qt[k]);
  }
  for (int k = 0; k < m * m; ++k) r[k] = P.R[(size_t)p * m * m + k];
  bool ok = small_spd(q, n) && small_spd(qt, n) && small_spd(r, m);
  ok = small_inverse(q, n) && small_inverse(qt, n) && small_inverse(r, m) && ok;
  for (size_t k = 0; k < nn; ++k) {
    Qi[k] = q[k];
    QTi[k] = qt[k];
    QTd[k] = qt[k] - q[k];
  }
  const double* Bp = P.B + (size_t)p * n * m;  // [n][m]
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < n; ++b) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += r[a * m + k] * Bp[b * m + k];
      RiBT[a * n + b] = s;
    }
  if (C.BRB) {  // B R^-1 B' = B (R^-1 B')
    double* BRB = C.BRB + p * nn;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Bp[a * m + k] * RiBT[k * n + b];
        BRB[a * n + b] = s;
      }
  }
  if (differs) atomicOr(&sc->qt_differs, 1);
  if (!ok) atomicOr(&sc->flag_notspd, 1);
}

// Work unit gid = 18 p + k of node p: k < 13 -> G13[p][k]; 13 <= k < 18 ->
// the 5-point blocks Cdn, AT5, Cup for k5 = k - 13.  NS = D.n at compile
// time, so the n x n work blocks stay in registers.
template <int NS>
__device__ inline void stencil(const Dims& D, const ProblemIn& P, const Coef& C,
                               long long gid) {
  if (gid >= (long long)D.nodes * 18) return;
  const int p = (int)(gid / 18), k = (int)(gid % 18);
  constexpr int n = NS;
  constexpr size_t nn = (size_t)n * n;
  const int K = D.K, N = D.N;
  const int j = p / K, i = p - j * K;
  double out[nn];
  double out2[nn];
  double out3[nn];
  for (size_t e = 0; e < nn; ++e) out[e] = out2[e] = out3[e] = 0.0;
  const bool real = p < D.real_nodes;
  if (k < 13) {
    const int iq = i + kOff13[k][0], jq = j + kOff13[k][1];
    if (real && iq >= 0 && iq < K && jq >= 0 && jq < N) {
      // sum over s in N1[p] ∩ N1[q] of A_hat[p,s] Q_s^-1 A_hat[q,s]'
      for (int k5 = 0; k5 < 5; ++k5) {
        const int is = i + kOff5[k5][0], js = j + kOff5[k5][1];
        const double* Aps = ahat_block(P, i, j, is, js);
        const double* Aqs = ahat_block(P, iq, jq, is, js);
        if (!Aps || !Aqs) continue;
        const double* Qis = C.Qi + ((size_t)js * K + is) * nn;
        double tmp[nn];
        for (int a = 0; a < n; ++a)  // tmp = A_ps Q_s^-1
          for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += Aps[a * n + c] * Qis[c * n + b];
            tmp[a * n + b] = s;
          }
        for (int a = 0; a < n; ++a)  // out += tmp A_qs'
          for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += tmp[a * n + c] * Aqs[b * n + c];
            out[a * n + b] += s;
          }
      }
      if (k == 0) {  // + B R^-1 B' = B (R^-1 B')
        const double* Bp = P.B + (size_t)p * n * D.m;
        const double* RiBT = C.RiBT + (size_t)p * D.m * n;
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int c = 0; c < D.m; ++c) s += Bp[a * D.m + c] * RiBT[c * n + b];
            out[a * n + b] += s;
          }
      }
    }
    double* G = C.G13 + ((size_t)p * 13 + k) * nn;
    for (size_t e = 0; e < nn; ++e) G[e] = out[e];
    return;
  }
  const int k5 = k - 13;
  const int iq = i + kOff5[k5][0], jq = j + kOff5[k5][1];
  if (real && iq >= 0 && iq < K && jq >= 0 && jq < N) {
    const double* Apq = ahat_block(P, i, j, iq, jq);  // p's coupling to q
    const double* Aqp = ahat_block(P, iq, jq, i, j);  // q's coupling to p
    const double* Qiq = C.Qi + ((size_t)jq * K + iq) * nn;
    const double* Qip = C.Qi + (size_t)p * nn;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Apq[a * n + c] * Qiq[c * n + b];
        out[a * n + b] = s;                 // Cdn = A_hat[p,q] Q_q^-1
        out2[a * n + b] = Aqp[b * n + a];   // AT5 = A_hat[q,p]'
      }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Qip[a * n + c] * out2[c * n + b];
        out3[a * n + b] = s;                // Cup = Q_p^-1 A_hat[q,p]'
      }
  }
  double* Cd = C.Cdn + ((size_t)p * 5 + k5) * nn;
  double* At = C.AT5 + ((size_t)p * 5 + k5) * nn;
  double* Cu = C.Cup + ((size_t)p * 5 + k5) * nn;
  for (size_t e = 0; e < nn; ++e) {
    Cd[e] = out[e];
    At[e] = out2[e];
    Cu[e] = out3[e];
  }
  if (C.A5) {  // A_hat[p, q] itself (the factored Delta apply)
    double* A5 = C.A5 + ((size_t)p * 5 + k5) * nn;
    const double* Apq = (real && iq >= 0 && iq < K && jq >= 0 && jq < N)
                            ? ahat_block(P, i, j, iq, jq) : nullptr;
    for (size_t e = 0; e < nn; ++e) A5[e] = Apq ? Apq[e] : 0.0;
  }
}

// Entry (r, c) of the block Phi_bar[i, i+di] (di = 0, -1, -2) of super-column
// v in (i, column-in-pair, component) order, class cls (0: Q^-1 on the
// diagonal, 1: Q_T^-1).  Dummy nodes get an identity diagonal and no coupling.
__device__ inline double phi_entry(const Dims& D, const Coef& C, int cls, int v,
                            int i, int di, int r, int c) {
  const int n = D.n, K = D.K;
  const int h = r / n, a = r - h * n;
  const int h2 = c / n, b = c - h2 * n;
  const int j = 2 * v + h, j2 = 2 * v + h2;
  const bool dummy1 = j >= D.N, dummy2 = j2 >= D.N;
  if (dummy1 || dummy2)
    return (di == 0 && h == h2 && a == b && dummy1) ? 1.0 : 0.0;
  const int k = off13_index(di, h2 - h);
  if (k < 0) return 0.0;
  const size_t p = (size_t)j * K + i;
  const size_t nn = (size_t)n * n;
  if (C.tv_ld) {  // time-varying data: class cls is the time t, t fastest
    const size_t ld = (size_t)C.tv_ld;
    double val = C.G13[((p * 13 + k) * nn + a * n + b) * ld + cls];
    if (di == 0 && h == h2) val += C.Qi[(p * nn + a * n + b) * ld + cls];
    return val;
  }
  double val = C.G13[(p * 13 + k) * nn + a * n + b];
  if (di == 0 && h == h2)
    val += (cls == 0 ? C.Qi : C.QTi)[p * nn + a * n + b];
  return val;
}

// Addresses of entry (row r, column k) of block row `row` of the forward
// (kFwRow columns) and backward (kBwRow columns) factor tables of class cls,
// super-column v: [cls][v][row][r][k] for time-invariant data, and for
// time-varying data [v][row][k][t][r8] (t = cls, 8 rows per time step)
// so that the eight row threads of eight time steps read one coalesced
// segment per column.
__device__ inline double* fw_at(const Dims& D, const Coef& C, int cls, int v, int row,
                                int r, int k) {
  if (C.tv_ld)
    return C.Fw + ((((size_t)v * fw_rows(D.K) + row) * kFwRow + k) * C.tv_ld + cls) * 8 + r;
  const size_t frows = ((size_t)cls * D.V + v) * fw_rows(D.K);
  return C.Fw + ((frows + row) * (2 * D.n) + r) * kFwRow + k;
}
__device__ inline double* bw_at(const Dims& D, const Coef& C, int cls, int v, int row,
                                int r, int k) {
  if (C.tv_ld)
    return C.Bw + ((((size_t)v * D.K + row) * kBwRow + k) * C.tv_ld + cls) * 8 + r;
  const size_t rows = ((size_t)cls * D.V + v) * D.K;
  return C.Bw + ((rows + row) * (2 * D.n) + r) * kBwRow + k;
}

// Cholesky factor L of the SPD NB x NB block Dm (shared memory, row-major)
// and Li = L^-1, written to Li (shared), by one thread with the block in
// registers.  A non-positive or non-finite pivot sets *bad and is replaced
// by 1 so that the factorisation runs to the end.
template <int NB>
__device__ inline void chol_inv_reg(const double* Dm, double* Li, int* bad) {
  double a[NB][NB], li[NB][NB];
#pragma unroll
  for (int r = 0; r < NB; ++r)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      a[r][c] = Dm[r * NB + c];
      li[r][c] = 0.0;
    }
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    double s = a[cc][cc];
#pragma unroll
    for (int k = 0; k < cc; ++k) s -= a[cc][k] * a[cc][k];
    if (!(s > 0.0) || !isfinite(s)) {
      *bad = 1;
      s = 1.0;
    }
    const double dg = sqrt(s);
    a[cc][cc] = dg;
#pragma unroll
    for (int rr = cc + 1; rr < NB; ++rr) {
      double t = a[rr][cc];
#pragma unroll
      for (int k = 0; k < cc; ++k) t -= a[rr][k] * a[cc][k];
      a[rr][cc] = t / dg;
    }
  }
#pragma unroll
  for (int cc = 0; cc < NB; ++cc) {
    li[cc][cc] = 1.0 / a[cc][cc];
#pragma unroll
    for (int rr = cc + 1; rr < NB; ++rr) {
      double t = 0.0;
#pragma unroll
      for (int k = cc; k < rr; ++k) t += a[rr][k] * li[k][cc];
      li[rr][cc] = -t / a[rr][rr];
    }
  }
#pragma unroll
  for (int r = 0; r < NB; ++r)
#pragma unroll
    for (int c = 0; c < NB; ++c) Li[r * NB + c] = li[r][c];
}
__device__ inline void chol_inv(const double* Dm, double* Li, int NB, int* bad) {
  switch (NB) {
    case 2: chol_inv_reg<2>(Dm, Li, bad); break;
    case 4: chol_inv_reg<4>(Dm, Li, bad); break;
    case 6: chol_inv_reg<6>(Dm, Li, bad); break;
    default: chol_inv_reg<8>(Dm, Li, bad); break;
  }
}

// Banded block Cholesky of Phi_bar_{v,cls} by one 64-thread workgroup.  Block rows of size NB = 2n; block bandwidth 2 (Psi_hat couples
// nodes at Manhattan distance <= 2, so rows i and i-2 meet only in the same
// column).  For each block row i:
//   L_{i,i-2} = Phi[i,i-2] L_{i-2,i-2}^-T
//   L_{i,i-1} = (Phi[i,i-1] - L_{i,i-2} L_{i-1,i-2}') L_{i-1,i-1}^-T
//   L_ii L_ii' = Phi[i,i] - L_{i,i-1} L_{i,i-1}' - L_{i,i-2} L_{i,i-2}'
__device__ inline void factor(const Dims& D, const Coef& C, Scalars* sc, int v,
                              int cls) {
  const int NB = 2 * D.n, NB2 = NB * NB, K = D.K;
  const int tid = threadIdx.x;
  const int r = tid / NB, c = tid - (tid / NB) * NB;
  const bool act = tid < NB2;
  __shared__ double S1[64], S2[64], Dm[64], L1[64], L2[64], T1[64];
  __shared__ double Lp1[64], Lp2[64], L1p[64], Li[64];
  __shared__ int bad;
  if (tid == 0) bad = 0;
  if (act) Lp1[tid] = Lp2[tid] = L1p[tid] = 0.0;
  __syncthreads();
  for (int i = 0; i < K; ++i) {
    if (act) {
      Dm[tid] = phi_entry(D, C, cls, v, i, 0, r, c);
      S1[tid] = i >= 1 ? phi_entry(D, C, cls, v, i, -1, r, c) : 0.0;
      S2[tid] = i >= 2 ? phi_entry(D, C, cls, v, i, -2, r, c) : 0.0;
    }
    __syncthreads();
    if (act) {  // L2 = S2 Linv_{i-2}'
      double s = 0.0;
      for (int k = 0; k < NB; ++k) s += S2[r * NB + k] * Lp2[c * NB + k];
      L2[tid] = s;
    }
    __syncthreads();
    if (act) {  // T1 = S1 - L2 L1p'
      double s = S1[tid];
      for (int k = 0; k < NB; ++k) s -= L2[r * NB + k] * L1p[c * NB + k];
      T1[tid] = s;
    }
    __syncthreads();
    if (act) {  // L1 = T1 Linv_{i-1}'
      double s = 0.0;
      for (int k = 0; k < NB; ++k) s += T1[r * NB + k] * Lp1[c * NB + k];
      L1[tid] = s;
    }
    __syncthreads();
    if (act) {  // Dm -= L1 L1' + L2 L2'
      double s = Dm[tid];
      for (int k = 0; k < NB; ++k)
        s -= L1[r * NB + k] * L1[c * NB + k] + L2[r * NB + k] * L2[c * NB + k];
      Dm[tid] = s;
    }
    __syncthreads();
    if (tid == 0) chol_inv(Dm, Li, NB, &bad);  // Cholesky of Dm, inverse
    __syncthreads();
    if (act) {
      double m1 = 0.0, m2 = 0.0, n1 = 0.0, n2 = 0.0;
      for (int k = 0; k < NB; ++k) {
        m1 += Li[r * NB + k] * L1[k * NB + c];    // Linv_i L_{i,i-1}
        m2 += Li[r * NB + k] * L2[k * NB + c];    // Linv_i L_{i,i-2}
        n1 += Lp1[k * NB + r] * L1[c * NB + k];   // Linv_{i-1}' L_{i,i-1}'
        n2 += Lp2[k * NB + r] * L2[c * NB + k];   // Linv_{i-2}' L_{i,i-2}'
      }
      *fw_at(D, C, cls, v, i, r, c) = m1;
      *fw_at(D, C, cls, v, i, r, 8 + c) = m2;
      *fw_at(D, C, cls, v, i, r, 16 + c) = Li[r * NB + c];
      // Linv_i' is used one block row later (w_i needs all of z_i)
      *fw_at(D, C, cls, v, i + 1, r, 24 + c) = Li[c * NB + r];
      if (i >= 1) *bw_at(D, C, cls, v, i - 1, r, c) = n1;
      if (i >= 2) *bw_at(D, C, cls, v, i - 2, r, 8 + c) = n2;
    }
    __syncthreads();
    if (act) {
      Lp2[tid] = Lp1[tid];
      Lp1[tid] = Li[tid];
      L1p[tid] = L1[tid];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) atomicOr(&sc->flag_notspd, 1);
  __syncthreads();  // the shared arrays may be reused by the next unit
}

// ---------------------------------------------------------------------------
// Twisted factorisation of Phi_bar_{v,cls} (K >= kTwistMin block rows): the
// same banded block Cholesky in the row order [0 .. m-1 (top chain),
// K-1 down to m+2 (bottom chain), m, m+1 (middle)], m = (K-2)/2.  In this
// order the two chains do not couple, so their substitutions run
// concurrently, each over about K/2 block rows.  Rows m and m+1 couple to
// the last two rows of each chain:
//   L_{m,m-2}, L_{m,m-1}  (top chain, as its continuation),   L_{m,m+2};
//   L_{m+1,m+3}, L_{m+1,m+2} (bottom chain, as its continuation),
//   L_{m+1,m-1}, L_{m+1,m}
// (every other block of the two middle rows is zero: Phi couples rows at
// most two apart, and a coupling to the last row of a chain does not fill
// back into it).
//
// Stored (per class and super-column), in the substitution-product form of
// factor():
//   Fw rows 0 .. m+1      top chain positions k = 0 .. m (row i = k), row
//                         m+1 holding only Linv_m'
//   Fw rows m+2 .. K+1    bottom chain positions k = 0 .. |B| (row
//                         i = K-1-k, position |B| = row m+1), the last row
//                         holding only Linv_{m+1}'
//   Bw rows 0 .. m        top positions: N1 = Linv_i' L_{i+1,i}',
//                         N2 = Linv_i' L_{i+2,i}' (row m: N1 = Linv_m'
//                         L_{m+1,m}', N2 = 0)
//   Bw rows m+1 .. K-1    bottom positions: N1 = Linv_i' L_{i-1,i}',
//                         N2 = Linv_i' L_{i-2,i}' (row m+1: zero)
//   Xw                    Linv_m L_{m,m+2} | Linv_{m+1} L_{m+1,m-1} |
//                         Linv_{m+1} L_{m+1,m}
__device__ __forceinline__ int twist_m(int K) { return (K - 2) / 2; }

// (A B')[r][c], (A B)[r][c], (A' B')[r][c] of NB x NB row-major blocks.
__device__ inline double mm_t(const double* A, const double* B, int NB, int r, int c) {
  double s = 0.0;
  for (int k = 0; k < NB; ++k) s += A[r * NB + k] * B[c * NB + k];
  return s;
}
__device__ inline double mm_n(const double* A, const double* B, int NB, int r, int c) {
  double s = 0.0;
  for (int k = 0; k < NB; ++k) s += A[r * NB + k] * B[k * NB + c];
  return s;
}
__device__ inline double mm_tt(const double* A, const double* B, int NB, int r, int c) {
  double s = 0.0;
  for (int k = 0; k < NB; ++k) s += A[k * NB + r] * B[c * NB + k];
  return s;
}

// One 128-thread workgroup per (v, cls): threads 0-63 factor the top chain,
// threads 64-127 the bottom chain (independent in this order, so side by
// side, with the same barriers; the shorter top chain idles), then threads
// 0-63 the two middle rows.
__device__ inline void factor_twisted(const Dims& D, const Coef& C, Scalars* sc,
                                      int v, int cls) {
  const int NB = 2 * D.n, NB2 = NB * NB, K = D.K;
  const int m = twist_m(K), nb = K - 2 - m;  // top and bottom chain lengths
  const int h = threadIdx.x >> 6, tid = threadIdx.x & 63;  // half, thread in half
  const int r = tid / NB, c = tid - (tid / NB) * NB;
  const bool act = tid < NB2;
  const bool top = h == 0;
  __shared__ double S1[2][64], S2[2][64], Dm[2][64], L1[2][64], L2[2][64], T1[2][64];
  __shared__ double Lp1[2][64], Lp2[2][64], L1p[2][64], Li[2][64];
  __shared__ double Lm1[64], Lmx[64], Lmi[64], LA[64], LM[64], SX[64];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  const size_t cv = (size_t)cls * D.V + v;
  const size_t fw0 = cv * fw_rows(K), bw0 = cv * K;
  const size_t fwb = fw0 + m + 2, bwb = bw0 + m + 1;  // bottom chain tables
  auto fwrow = [&](size_t row) { return C.Fw + (row * NB + r) * kFwRow; };
  auto bwrow = [&](size_t row) { return C.Bw + (row * NB + r) * kBwRow; };
  double* xw = C.Xw + (cv * NB + r) * kFwRow;
  if (act && top) xw[24 + c] = 0.0;

  // The two chains: position k, block row i = top ? k : K-1-k, previous rows
  // in the chain i - dir and i - 2 dir.  Afterwards Lp1 / Lp2 hold Linv of
  // the last / second-last position of each chain, L1p the coupling between
  // them.
  {
    const int dir = top ? 1 : -1, len = top ? m : nb;
    const size_t ft = top ? fw0 : fwb, bt = top ? bw0 : bwb;
    double *S1h = S1[h], *S2h = S2[h], *Dmh = Dm[h], *L1h = L1[h], *L2h = L2[h];
    double *T1h = T1[h], *Lp1h = Lp1[h], *Lp2h = Lp2[h], *L1ph = L1p[h], *Lih = Li[h];
    if (act) Lp1h[tid] = Lp2h[tid] = L1ph[tid] = 0.0;
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
      const bool work = act && k < len;
      const int i = top ? k : K - 1 - k;
      if (work) {
        Dmh[tid] = phi_entry(D, C, cls, v, i, 0, r, c);
        S1h[tid] = k >= 1 ? phi_entry(D, C, cls, v, i, -dir, r, c) : 0.0;
        S2h[tid] = k >= 2 ? phi_entry(D, C, cls, v, i, -2 * dir, r, c) : 0.0;
      }
      __syncthreads();
      if (work) L2h[tid] = mm_t(S2h, Lp2h, NB, r, c);
      __syncthreads();
      if (work) T1h[tid] = S1h[tid] - mm_t(L2h, L1ph, NB, r, c);
      __syncthreads();
      if (work) L1h[tid] = mm_t(T1h, Lp1h, NB, r, c);
      __syncthreads();
      if (work) Dmh[tid] -= mm_t(L1h, L1h, NB, r, c) + mm_t(L2h, L2h, NB, r, c);
      __syncthreads();
      if (tid == 0 && k < len) chol_inv(Dmh, Lih, NB, &bad);
      __syncthreads();
      if (work) {
        double* fw = fwrow(ft + k);
        fw[c] = mm_n(Lih, L1h, NB, r, c);
        fw[8 + c] = mm_n(Lih, L2h, NB, r, c);
        fw[16 + c] = Lih[r * NB + c];
        fwrow(ft + k + 1)[24 + c] = Lih[c * NB + r];
        if (k >= 1) bwrow(bt + k - 1)[c] = mm_tt(Lp1h, L1h, NB, r, c);
        if (k >= 2) bwrow(bt + k - 2)[8 + c] = mm_tt(Lp2h, L2h, NB, r, c);
      }
      __syncthreads();
      if (work) {
        Lp2h[tid] = Lp1h[tid];
        Lp1h[tid] = Lih[tid];
        L1ph[tid] = L1h[tid];
      }
      __syncthreads();
    }
  }
  // top chain's end: A1 = Linv_{m-1}, A2 = Linv_{m-2}, A12 = L_{m-1,m-2};
  // bottom chain's end: B1 = Linv_{m+2}, B2 = Linv_{m+3}, B12 = L_{m+2,m+3}
  const double *A1 = Lp1[0], *A2 = Lp2[0], *A12 = L1p[0];
  const double *B1 = Lp1[1], *B2 = Lp2[1], *B12 = L1p[1];
  double *S1m = S1[0], *S2m = S2[0], *Dmm = Dm[0], *L1m = L1[0], *L2m = L2[0];
  double *T1m = T1[0], *Lim = Li[0];
  const bool mact = act && top;  // the middle rows run on threads 0-63

  // ---- row m: top continuation plus L_{m,m+2}
  if (mact) {
    Dmm[tid] = phi_entry(D, C, cls, v, m, 0, r, c);
    S1m[tid] = phi_entry(D, C, cls, v, m, -1, r, c);
    S2m[tid] = phi_entry(D, C, cls, v, m, -2, r, c);
    SX[tid] = phi_entry(D, C, cls, v, m, 2, r, c);
  }
  __syncthreads();
  if (mact) {
    L2m[tid] = mm_t(S2m, A2, NB, r, c);  // L_{m,m-2}
    Lmx[tid] = mm_t(SX, B1, NB, r, c);   // L_{m,m+2}
  }
  __syncthreads();
  if (mact) T1m[tid] = S1m[tid] - mm_t(L2m, A12, NB, r, c);
  __syncthreads();
  if (mact) Lm1[tid] = mm_t(T1m, A1, NB, r, c);  // L_{m,m-1}
  __syncthreads();
  if (mact)
    Dmm[tid] -= mm_t(Lm1, Lm1, NB, r, c) + mm_t(L2m, L2m, NB, r, c) + mm_t(Lmx, Lmx, NB, r, c);
  __syncthreads();
  if (threadIdx.x == 0) chol_inv(Dmm, Lmi, NB, &bad);  // Lmi = Linv_m
  __syncthreads();
  if (mact) {
    double* fw = fwrow(fw0 + m);
    fw[c] = mm_n(Lmi, Lm1, NB, r, c);
    fw[8 + c] = mm_n(Lmi, L2m, NB, r, c);
    fw[16 + c] = Lmi[r * NB + c];
    double* fe = fwrow(fw0 + m + 1);
    fe[c] = fe[8 + c] = fe[16 + c] = 0.0;
    fe[24 + c] = Lmi[c * NB + r];                             // Linv_m'
    xw[c] = mm_n(Lmi, Lmx, NB, r, c);                         // Linv_m L_{m,m+2}
    bwrow(bw0 + m - 1)[c] = mm_tt(A1, Lm1, NB, r, c);         // N1_{m-1}
    bwrow(bw0 + m - 2)[8 + c] = mm_tt(A2, L2m, NB, r, c);     // N2_{m-2}
    bwrow(bwb + nb - 1)[8 + c] = mm_tt(B1, Lmx, NB, r, c);    // N2 of row m+2
  }
  __syncthreads();

  // ---- row m+1: bottom continuation plus L_{m+1,m-1}, L_{m+1,m}
  if (mact) {
    Dmm[tid] = phi_entry(D, C, cls, v, m + 1, 0, r, c);
    S1m[tid] = phi_entry(D, C, cls, v, m + 1, 1, r, c);    // Phi[m+1, m+2]
    S2m[tid] = phi_entry(D, C, cls, v, m + 1, 2, r, c);    // Phi[m+1, m+3]
    SX[tid] = phi_entry(D, C, cls, v, m + 1, -2, r, c);    // Phi[m+1, m-1]
    T1m[tid] = phi_entry(D, C, cls, v, m + 1, -1, r, c);   // Phi[m+1, m]
  }
  __syncthreads();
  if (mact) {
    L2m[tid] = mm_t(S2m, B2, NB, r, c);  // L_{m+1,m+3}
    LA[tid] = mm_t(SX, A1, NB, r, c);    // L_{m+1,m-1}
  }
  __syncthreads();
  if (mact) S1m[tid] -= mm_t(L2m, B12, NB, r, c);
  __syncthreads();
  if (mact) L1m[tid] = mm_t(S1m, B1, NB, r, c);  // L_{m+1,m+2}
  __syncthreads();
  if (mact) T1m[tid] -= mm_t(LA, Lm1, NB, r, c) + mm_t(L1m, Lmx, NB, r, c);
  __syncthreads();
  if (mact) LM[tid] = mm_t(T1m, Lmi, NB, r, c);  // L_{m+1,m}
  __syncthreads();
  if (mact)
    Dmm[tid] -= mm_t(L1m, L1m, NB, r, c) + mm_t(L2m, L2m, NB, r, c) + mm_t(LA, LA, NB, r, c) +
                mm_t(LM, LM, NB, r, c);
  __syncthreads();
  if (threadIdx.x == 0) chol_inv(Dmm, Lim, NB, &bad);  // Lim = Linv_{m+1}
  __syncthreads();
  if (mact) {
    double* fw = fwrow(fwb + nb);
    fw[c] = mm_n(Lim, L1m, NB, r, c);
    fw[8 + c] = mm_n(Lim, L2m, NB, r, c);
    fw[16 + c] = Lim[r * NB + c];
    double* fe = fwrow(fwb + nb + 1);
    fe[c] = fe[8 + c] = fe[16 + c] = 0.0;
    fe[24 + c] = Lim[c * NB + r];                             // Linv_{m+1}'
    xw[8 + c] = mm_n(Lim, LA, NB, r, c);                      // Linv_{m+1} L_{m+1,m-1}
    xw[16 + c] = mm_n(Lim, LM, NB, r, c);                     // Linv_{m+1} L_{m+1,m}
    bwrow(bwb + nb - 1)[c] = mm_tt(B1, L1m, NB, r, c);        // N1 of row m+2
    bwrow(bwb + nb - 2)[8 + c] = mm_tt(B2, L2m, NB, r, c);    // N2 of row m+3
    bwrow(bw0 + m - 1)[8 + c] = mm_tt(A1, LA, NB, r, c);      // N2_{m-1}
    double* bm = bwrow(bw0 + m);
    bm[c] = mm_tt(Lmi, LM, NB, r, c);                         // N1_m
    bm[8 + c] = 0.0;
    double* bl = bwrow(bwb + nb);                             // row m+1: zero
    bl[c] = bl[8 + c] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(&sc->flag_notspd, 1);
  __syncthreads();
}

// r_delta = col(-gamma_hat, 0, ..., 0) in the internal layout, entry g =
// p n + c (the vector is zeroed beforehand).
// r_delta at t = 0: -gamma (Sec. II-A, reading of omega~); components past
// a node's state size (nsz, nullable) are padding and read as zero.
__device__ inline void rhs_init(const Dims& D, const double* __restrict__ x0,
                                const int* __restrict__ nsz, double* __restrict__ rd,
                                int g) {
  if (g >= D.real_nodes * D.n) return;
  const int p = g / D.n, c = g % D.n;
  const bool real = !nsz || c < nsz[p];
  rd[(size_t)g * D.ldt] = real ? -x0[g] : 0.0;  // g = p*n + c in both layouts
}

// Known spatial boundary states (Sec. II, eqs. "boundary_condition_i/j")
// enter the dynamics of the nodes next to the grid's edges as the affine term
// omega_hat_t = M_hat alpha_hat_t + N_hat beta_hat_t, so r_delta at t + 1
// holds -(G x_{0,j,t} + H x_{K+1,j,t} + E x_{i,0,t} + F x_{i,N+1,t}) for the
// couplings of node (i, j) that point outside the grid.  Work unit g = p T + t
// (real node p, t = 0..T-1) writes r_delta(p, ., t + 1); nodes away from the
// edges (and null state arrays) give zero, so the call also clears the
// entries of an earlier solve.  Anbr holds the node's four coupling blocks
// (rows past its state size already zero).
__device__ inline void rhs_boundary(const Dims& D, const double* __restrict__ Anbr,
                                    const double* __restrict__ alo,
                                    const double* __restrict__ ahi,
                                    const double* __restrict__ blo,
                                    const double* __restrict__ bhi,
                                    double* __restrict__ rd, long long g) {
  if (g >= (long long)D.real_nodes * D.T) return;
  const int p = (int)(g / D.T), t = (int)(g % D.T);
  const int n = D.n, K = D.K, N = D.N;
  const int i = p % K, j = p / K;
  double w[kMaxN];
  for (int c = 0; c < n; ++c) w[c] = 0.0;
  // slot 0: E (x_{i,j-1}), 1: F (x_{i,j+1}), 2: G (x_{i-1,j}), 3: H (x_{i+1,j})
  const double* st[4] = {j == 0 && blo ? blo + ((size_t)t * K + i) * n : nullptr,
                         j == N - 1 && bhi ? bhi + ((size_t)t * K + i) * n : nullptr,
                         i == 0 && alo ? alo + ((size_t)t * N + j) * n : nullptr,
                         i == K - 1 && ahi ? ahi + ((size_t)t * N + j) * n : nullptr};
  for (int k = 0; k < 4; ++k) {
    if (!st[k]) continue;
    const double* M = Anbr + ((size_t)p * 4 + k) * n * n;
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) w[a] += M[a * n + c] * st[k][c];
  }
  for (int c = 0; c < n; ++c) rd[((size_t)p * n + c) * D.ldt + t + 1] = -w[c];
}

// Ingest with per-node sizes (Sec. II: x_{i,j} in R^{n_{i,j}}, u_{i,j} in
// R^{m_{i,j}}): every node is padded to n, m with decoupled components --
// rows and columns past its sizes of A, of its coupling blocks (columns past
// the neighbour's size) and of B are zero, Q, Q_T and R are the identity
// there.  A padded state then starts at zero, is driven by nothing and
// drives nothing, and costs nothing; a padded input acts on nothing and is
// zero at the optimum; the multipliers of padded rows are zero.  The copies
// (user layouts) replace the caller's arrays for the rest of the setup.
// nsz / msz may be null (uniform sizes: a plain copy).  One thread per real
// node; a size outside 1..n (1..m) raises flag_badsize.
__device__ inline void ingest_mask(const Dims& D, const ProblemIn P, const int* nsz_in,
                                   const int* msz_in, ProblemIn out, int* nsz_out,
                                   Scalars* sc, int p) {
  if (p >= D.real_nodes) return;
  const int n = D.n, m = D.m, K = D.K, N = D.N;
  const int i = p % K, j = p / K;
  int np_ = nsz_in ? nsz_in[p] : n, mp = msz_in ? msz_in[p] : m;
  if (np_ < 1 || np_ > n || mp < 1 || mp > m) {
    atomicOr(&sc->flag_badsize, 1);
    np_ = n;
    mp = m;
  }
  nsz_out[p] = np_;
  const size_t nn = (size_t)n * n;
  double* A = const_cast<double*>(out.A) + p * nn;
  const double* As = P.A + p * nn;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) A[a * n + b] = (a < np_ && b < np_) ? As[a * n + b] : 0.0;
  const int ni[4] = {i, i, i - 1, i + 1}, nj[4] = {j - 1, j + 1, j, j};
  for (int k = 0; k < 4; ++k) {
    const bool in_grid = ni[k] >= 0 && ni[k] < K && nj[k] >= 0 && nj[k] < N;
    int nq = n;
    if (in_grid && nsz_in) {
      nq = nsz_in[nj[k] * K + ni[k]];
      nq = (nq < 1 || nq > n) ? n : nq;
    }
    double* E = const_cast<double*>(out.A_nbr) + ((size_t)p * 4 + k) * nn;
    const double* Es = P.A_nbr + ((size_t)p * 4 + k) * nn;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) E[a * n + b] = (a < np_ && b < nq) ? Es[a * n + b] : 0.0;
  }
  double* B = const_cast<double*>(out.B) + (size_t)p * n * m;
  const double* Bs = P.B + (size_t)p * n * m;
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < m; ++c) B[a * m + c] = (a < np_ && c < mp) ? Bs[a * m + c] : 0.0;
  const double* QTs = P.QT ? P.QT : P.Q;
  double* Q = const_cast<double*>(out.Q) + p * nn;
  double* QT = const_cast<double*>(out.QT) + p * nn;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const bool in = a < np_ && b < np_;
      Q[a * n + b] = in ? P.Q[p * nn + a * n + b] : (a == b ? 1.0 : 0.0);
      QT[a * n + b] = in ? QTs[p * nn + a * n + b] : (a == b ? 1.0 : 0.0);
    }
  double* R = const_cast<double*>(out.R) + (size_t)p * m * m;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      R[a * m + b] = (a < mp && b < mp) ? P.R[(size_t)p * m * m + a * m + b]
                                        : (a == b ? 1.0 : 0.0);
}

}  // namespace dev
}  // namespace lqg
