// Internal definitions shared by the lqgrid HIP kernels and the host driver.
//
// Device layout (all FP64 unless noted):
//   node id      p = j*K + i over an even number of columns Npad = 2V
//                (V = ceil(N/2) super-columns of the paper, Sec. II-B); when N
//                is odd the extra column j = N holds zero "dummy" nodes so that
//                every super-column is a pair.
//   vectors      v[((p*n + c)*ldt) + t]: time fastest, ldt = T+1 rounded up
//                to 16 (128-byte rows).  A wavefront's 64 lanes cover 64
//                consecutive t of one (node, component): every vector access
//                is a contiguous 512-byte load/store.  Entries with t > T and
//                dummy nodes are kept at zero.
//   coefficients time invariant, per node, n x n row-major blocks:
//     G13[p][k]  13-point blocks of G = A_hat Q^-1 A_hat' + B R^-1 B'
//                (Psi_hat_t = Q_t^-1 + G for t >= 1, eq. "structure_of_Delta")
//     Cdn[p][k]  A_hat[p,q] Q_q^-1  (q = p + off5[k]); Delta_{t,t-1} = -Cdn
//     Cup[p][k]  Q_p^-1 A_hat[q,p]'; Delta_{t,t+1} = -Cup
//     AT5[p][k]  A_hat[q,p]' (recovery x = Q^-1 A~' delta)
//     Qi, QTi, QTd (= QT^-1 - Q^-1), Qm (= Q, the t = 0 block solve), RiBT
//   factors      banded block Cholesky Phi_bar_{v,t} = L L' in (i,
//                column-in-pair, component) order, stored as the products the
//                substitutions use (Linv_i = L_ii^-1):
//                  forward  z_i   = Linv_i tau_i - M1_i z_{i-1} - M2_i z_{i-2}
//                           w_i   = Linv_i' z_i
//                  backward theta_i = w_i - N1_i theta_{i+1} - N2_i theta_{i+2}
//                with M1_i = Linv_i L_{i,i-1}, M2_i = Linv_i L_{i,i-2},
//                N1_i = Linv_i' L_{i+1,i}', N2_i = Linv_i' L_{i+2,i}'.
//                Fw[cls][v][i][r][32] (i = 0..K) = rows r of (M1_i, M2_i,
//                Linv_i, Linv_{i-1}'), each padded to 8 doubles (block row K
//                holds only Linv_{K-1}'); Bw[cls][v][i][r][16] = rows r of
//                (N1_i, N2_i).  One row of a block row is 256 (128) contiguous
//                bytes: one coalesced load per wavefront and block row.
//                cls 0: 1 <= t <= T-1 (and t = T when QT = Q), cls 1: t = T.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lqg {

constexpr int kWave = 64;
constexpr int kMaxN = 4;   // compiled state sizes: 1..kMaxN
constexpr int kMaxM = 8;
constexpr int kFwRow = 32;  // doubles per row of a forward factor block row
constexpr int kBwRow = 16;  // doubles per row of a backward factor block row

// (di, dj) offsets of the 13-point stencil (Manhattan distance <= 2).
constexpr int kOff13[13][2] = {{0, 0},  {-1, 0}, {1, 0},  {0, -1}, {0, 1},
                               {-2, 0}, {2, 0},  {0, -2}, {0, 2},  {-1, -1},
                               {-1, 1}, {1, -1}, {1, 1}};
// (di, dj) offsets of the 5-point stencil: self, north (i-1), south (i+1),
// west (j-1), east (j+1).
constexpr int kOff5[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};

__host__ __device__ constexpr int off13_index(int di, int dj) {
  for (int k = 0; k < 13; ++k)
    if (kOff13[k][0] == di && kOff13[k][1] == dj) return k;
  return -1;
}

struct Dims {
  int K, N, T, n, m;
  int Npad, V, Tt, ldt;
  int nodes;       // Npad*K (including dummy column)
  int real_nodes;  // N*K
  long long vlen;  // nodes*n*ldt
};

struct Coef {
  double *G13, *Cdn, *Cup, *AT5;
  double *Qi, *QTi, *QTd, *Qm, *RiBT;
  double *Fw, *Bw;  // factors in the substitution layout
  double* Xw;       // middle-row couplings of the twisted factorisation
  // A5[p][k] = A_hat[p, p + o5_k] and BRB[p] = B_p R_p^-1 B_p' for the
  // factored Delta apply (null: not assembled)
  double* A5 = nullptr;
  double* BRB = nullptr;
  // Time-varying data (0: the layouts above).  Otherwise the class of a
  // factorisation is the time t = 0..T and the one-chain factorisation reads
  // G13 / Qi and writes Fw / Bw in the time-fastest layouts of the
  // time-varying operator (see tv.hip), with this leading dimension (ldt).
  long long tv_ld = 0;
};

// The operator blocks the hot kernels read, in the element type of the
// vectors they act on (FP64 arrays above, or their FP32 copies).
template <typename T>
struct OpCoef {
  const T *G13, *Cdn, *Cup, *Qi, *QTd, *Qm, *Fw, *Bw, *Xw;
  // the factored form of the Delta apply: A5[p][k] = A_hat[p, p + o5_k],
  // BRB[p] = B_p R_p^-1 B_p', and its intermediate vector W (single-problem
  // path; null in the batched form)
  const T *A5 = nullptr, *BRB = nullptr;
  T* W = nullptr;
};

// Rows of the forward factor table per (class, super-column): the one-chain
// factorisation uses K + 1 of them, the twisted one K + 2.
__host__ __device__ inline int fw_rows(int K) { return K + 2; }

// Phi_bar is factored and solved in the twisted order from this many block
// rows on, in the single-problem and in the batched form alike.
constexpr int kTwistMin = 8;
__host__ __device__ inline bool twisted(const Dims& D) { return D.K >= kTwistMin; }

// Device-resident PCG scalars.
struct Scalars {
  double rd2;      // ||r_delta||^2
  double mu;       // q'r of the current direction
  double yd;       // d' Delta d
  double theta;    // step length
  double beta;     // direction coefficient
  double rr;       // ||r||^2 after the last update
  double tol2;     // tol^2 * rd2
  double rinf;     // ||r||_inf of the last true residual
  double rdinf;    // ||r_delta||_inf
  int done;        // 0 running, 1 converged (recurrence), 2 breakdown, 3 max_iter
  int iter;
  int max_iter;
  int flag_notspd; // factor pivot failure
  int qt_differs;  // QT != Q somewhere
  int active;      // batched form: the problem takes part in the current phase
  int flag_badsize;// a per-node state or input size outside 1..n / 1..m
  int pad;
  double* hist;    // non-null: record theta_k at [2k] and beta_k at [2k+1]
  int hist_cap;    // iterations the history holds
  int pad2;
};

enum Done { kRunning = 0, kConverged = 1, kBreakdown = 2, kMaxIter = 3 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over a block of BS threads (BS multiple of 64); result valid in thread 0.
template <int BS>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[BS / kWave];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < BS / kWave; ++k) s += red[k];
  }
  __syncthreads();
  return s;
}
template <int BS>
__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[BS / kWave];
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < BS / kWave; ++k) s = fmax(s, red[k]);
  }
  __syncthreads();
  return s;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wavefront, which would drain
// the register prefetch rings of the block-row sweeps at every block row.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The 8 XCDs of the MI355X each own an L2 cache and receive workgroups
// round-robin (hardware block b runs on XCD b % 8).  Grids are launched with
// a multiple of 8 blocks and remapped so that each XCD processes one
// contiguous range of logical blocks: neighbouring tiles, whose halos
// overlap, then share an L2.  Returns the logical block (>= the real count
// for the padding blocks, which exit).
constexpr int kXcds = 8;
__host__ __device__ inline int padded_grid(int nblocks) {
  return (nblocks + kXcds - 1) / kXcds * kXcds;
}
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, per = gridDim.x / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

__device__ __forceinline__ int uniform(int x) {
  return __builtin_amdgcn_readfirstlane(x);
}

}  // namespace lqg
