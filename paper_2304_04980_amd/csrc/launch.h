// Launchers of the lqgrid kernels (host-callable), one per kernel family.
#pragma once
#include "lqg_internal.h"

namespace lqg {

// The caller's problem arrays (device pointers, [N][K][...] layouts).
struct ProblemIn {
  int K, N, n, m;
  const double *A, *A_nbr, *B, *Q, *R, *QT;
};

// A batch of time slices s0 .. s0 + nsl - 1 of time-varying data, handled by
// one launch per setup kernel (blockIdx.y = slice b of the batch).  Slice s
// reads the problem arrays of slice min(s, T - 1) at the given strides (the
// terminal slice T: Q = Q_T, or Q_{T-1} without one); slice b's ingested
// copies and assembly scratch sit at b times their strides from the slice-0
// pointers.
struct TvSlices {
  int s0, nsl, T;
  long long sA, sN, sB, sR;      // problem arrays: A and Q, A_nbr, B, R per slice
  const double* QT;              // terminal weight (may be null)
  long long iA, iN, iB, iR;      // ingested copies: A and Q, A_nbr, B, R per slice
  long long cG13, cQi, c5, cRiBT, cBRB;  // scratch: G13; Qi; Cdn, Cup, AT5, A5; RiBT; BRB
};

// setup.hip
void launch_setup(const Dims& D, const ProblemIn& P, const Coef& C,
                  Scalars* sc, hipStream_t s);
// Ingest and assembly of a batch of time slices (P: slice-0 problem arrays,
// in / C: slice-0 ingested copies and assembly scratch; the shared blocks of C
// that time-varying data does not use, Q_T^-1 and the like, are written by
// every slice of the batch).
void launch_ingest_setup_tv(const Dims& D, const ProblemIn& P, const TvSlices& S,
                            const int* nsz, const int* msz, const ProblemIn& in,
                            int* nsz_out, const Coef& C, Scalars* sc, hipStream_t s);
void launch_factor(const Dims& D, const Coef& C, Scalars* sc, hipStream_t s);
void launch_rhs_init(const Dims& D, const double* x0, double* rd,
                     hipStream_t s, const int* nsz = nullptr);
// Known spatial boundary states ([T+1][N][n] for the rows above / below the
// grid, [T+1][K][n] for the columns left / right of it; null: zero).
struct Boundary {
  const double *alo, *ahi, *blo, *bhi;
};
void launch_rhs_boundary(const Dims& D, const double* Anbr, const Boundary& bc,
                         double* rd, hipStream_t s);
// Per-node sizes: padded copies of the problem arrays (see ingest_mask).
void launch_ingest(const Dims& D, const ProblemIn& P, const int* nsz, const int* msz,
                   const ProblemIn& out, int* nsz_out, Scalars* sc, hipStream_t s);

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
  kModeTrue = 5,  // rr = sum, rinf = max (true residual), no state change
  kModeRd2Rel = 6,// as kModeRd2 with the relative target of a refinement
                  // pass, tol_rel = min(tol ||r_delta|| / ||r||, 1/2), taken
                  // from the outer scalars
  kModeDotA = 7,  // mu = sum (a dot product for the host, no state change)
  kModeDotB = 8   // yd = sum (likewise)
};

// The scalar update of Algorithm 1 selected by mode, given the reduced sum s
// and maximum m.  `outer` (kModeRd2Rel only) holds the true residual of the
// outer loop.
__device__ inline void scalar_apply(int mode, double s, double m, Scalars* sc,
                                    const Scalars* outer, double tol) {
  switch (mode) {
    case kModeRd2:
    case kModeRd2Rel: {
      double tr = tol;
      if (mode == kModeRd2Rel)
        tr = fmin(tol * sqrt(outer->rd2 / outer->rr), 0.5);
      sc->rd2 = s;
      sc->rdinf = m;
      sc->rr = s;     // residual of the zero start
      sc->rinf = m;
      sc->tol2 = tr * tr * s;
      sc->done = kRunning;
      break;
    }
    case kModeYd:
      sc->yd = s;
      if (!(s > 0.0) || !isfinite(s) || !isfinite(sc->mu)) {
        sc->done = kBreakdown;
      } else {
        sc->theta = sc->mu / s;
        if (sc->hist && sc->iter < sc->hist_cap) sc->hist[2 * sc->iter] = sc->theta;
      }
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
        // iteration iter - 1 was counted by kModeRr
        if (sc->hist && sc->iter >= 1 && sc->iter - 1 < sc->hist_cap)
          sc->hist[2 * (sc->iter - 1) + 1] = sc->beta;
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
    case kModeDotA:
      sc->mu = s;
      break;
    case kModeDotB:
      sc->yd = s;
      break;
  }
}
__host__ __device__ inline bool scalar_mode_gated(int mode) {
  return mode == kModeYd || mode == kModeRr || mode == kModeMu;
}
void scalar_step(int mode, const double* psum, const double* pmax, int np,
                 Scalars* sc, double tol, hipStream_t s);

// layout conversion between the [T+1][N][K][n] interface order and the
// internal time-fastest order
void to_internal(const Dims& D, const double* abi, double* internal,
                 hipStream_t s);
void to_abi(const Dims& D, const double* internal, double* abi, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched form: many independent problems (uniform n; K, N, T, m free) in one
// set of launches.  Every problem keeps its own coefficient blocks, factors,
// vectors and PCG scalars; kernels walk flattened (problem, tile) work lists.
enum BatchVec { kBX, kBR, kBD, kBY, kBA, kBB, kBC, kBE, kBRd, kBDl, kBRt, kBYt,
                kNumBatchVec };
struct BatchProb {
  Dims D;
  Coef C;
  ProblemIn in;
  const double* x0;
  double* delta_out;
  double* v[kNumBatchVec];
  Scalars* sc;   // the PCG instance
  Scalars* sco;  // the outer (true residual) loop
  int first[3];  // first original work item of each kind
  int count[3];
};
// One work item: problem, two coordinates (node items: node group, time
// chunk; solve items: super-column, time chunk; flat items: element range
// [a, b)), and the slot of its partial sums (its index in the original list).
struct Item {
  int prob, a, b, slot;
};
enum ItemKind { kItemNode = 0, kItemSolve = 1, kItemFlat = 2, kNumItemKinds = 3 };
// Unit items of the setup kernels: problem and unit range [a, b).
enum UnitKind { kUnitPrep = 0, kUnitStencil = 1, kUnitRhs = 2, kUnitFactor = 3,
                kUnitAbi = 4, kNumUnitKinds = 5 };

struct BatchDev {
  BatchProb* probs;
  Scalars* sc;     // [P] PCG instances (probs[p].sc == sc + p)
  Scalars* sco;    // [P] outer loops
  int P;
  Item* orig[kNumItemKinds];
  int norig[kNumItemKinds];
  Item* live[kNumItemKinds];
  int* nlive;      // [kNumItemKinds + 1]: live items per kind, running problems
  int* live_flag;  // [P]
  int* live_off;   // [kNumItemKinds][P]
  int* host_in;    // [2 P] staging: active flags, iteration limits
  Item* units[kNumUnitKinds];
  int nunits[kNumUnitKinds];
  double *psum_node, *psum_flat, *pmax_flat;
  // node list with time chunks fastest: the first chunk item of a node group
  // runs all its chunks in the Delta apply and the Xi~ right-hand side
  int node_rows = 0;
};

enum FlatOp {
  kFlatDir = 0,     // b = a + beta b
  kFlatUpdate = 1,  // x(c) += theta a, r(d) -= theta b, partial |r|^2
  kFlatDot = 2,     // partial a'b
  kFlatNorms = 3,   // partial |a|^2, max |a|
  kFlatSubNorm = 4, // c = a - b, partial |c|^2, max |c|
  kFlatScale = 5,   // b = a / ||r|| (outer scalars)
  kFlatAxpy = 6,    // b += ||r|| a (outer scalars)
  kFlatZero = 7     // a = 0
};

// batch.hip launchers.  `check` selects the gate: 0 = every live item, 1 =
// only problems whose PCG instance is still running.  grid = persistent
// workgroup count.
void batch_delta(const BatchDev& B, int n, int in, int out, int partial,
                 int check, int grid, hipStream_t s);
void batch_omega(const BatchDev& B, int n, int rho, int th, int tau, int check,
                 int grid, hipStream_t s);
void batch_xi(const BatchDev& B, int n, int r, int dl, int rho, int check,
              int grid, hipStream_t s);
void batch_solve(const BatchDev& B, int n, int tau, int out, int check,
                 int grid, hipStream_t s);
void batch_flat(const BatchDev& B, int op, int a, int b, int c, int d,
                int check, int grid, hipStream_t s);
void batch_scalar(const BatchDev& B, int mode, int kind, int outer, double tol,
                  hipStream_t s);
void batch_compact(const BatchDev& B, int running_only, hipStream_t s);
void batch_set_active(const BatchDev& B, hipStream_t s);
void batch_setup(const BatchDev& B, int n, hipStream_t s);
void batch_factor(const BatchDev& B, hipStream_t s);
void batch_rhs_init(const BatchDev& B, hipStream_t s);
void batch_to_abi(const BatchDev& B, hipStream_t s);

}  // namespace lqg
