// Host side of the lqgrid C ABI: argument checks, workspace layout, and the
// driver of Algorithm 1 (PCGM) with the Algorithm 2 preconditioner.
//
// Solve structure.  An outer FP64 loop keeps the iterate delta~ and checks
// the true residual r = r_delta - Delta delta~ (FP64 Delta apply).  Each pass
// solves Delta e = r / ||r|| with Algorithm 1 from e = 0 in the working
// precision (FP64, or FP32 vectors and sweeps for the precision form, with
// FP64 scalars and FP64 accumulation of every dot product) and adds e to
// delta~.  In FP64 the first pass is plain PCG to the requested tolerance and
// the loop only repeats when rounding leaves the true residual above it; in
// FP32 the loop is iterative refinement.  All device work is enqueued on the
// caller's stream; PCG scalars stay on the device and the host reads the
// convergence flag every `check_every` iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "api_common.h"
#include "tv.h"
#include "nt.h"

using namespace lqg;

namespace {

constexpr int kOpF32 = 16;         // lqgrid_apply_operator: FP32 kernels

// FP64 vectors of the outer loop, then the 8 vectors of one PCG instance.
enum OuterVec { kRd, kDl, kRt, kYt, kNumOuter };
enum PcgVec { kX, kR, kD, kY, kBufA, kBufB, kBufC, kBufD, kNumPcg };

struct Plan {
  size_t G13, Cdn, Cup, AT5, Qi, QTi, QTd, Qm, RiBT, Fw, Bw, Xw;
  size_t G13f, Cdnf, Cupf, Qif, QTdf, Qmf, Fwf, Bwf, Xwf;
  size_t A5, BRB, A5f, BRBf, W64, W32;  // the factored Delta apply
  size_t outer[kNumOuter], p64[kNumPcg], p32[kNumPcg];
  size_t psum, pmax, scal, scal_outer, hist;
  size_t inA, inAnbr, inB, inQ, inQT, inR, nsz;  // ingested (size-masked) arrays
  // time-varying data (tv.hip layouts), FP64 and FP32 copies
  size_t tG13, tQi, tCdn, tCup, tAT5, tRiBT, tA5, tBRB, tFw, tBw, tW;
  size_t tG13f, tQif, tCdnf, tCupf, tA5f, tBRBf, tFwf, tBwf, tWf;
  size_t tsG13, tsQi, tsCdn, tsCup, tsAT5, tsRiBT, tsA5, tsBRB;  // kTvBatch assembly slices
  size_t tsInA, tsInN, tsInB, tsInQ, tsInR;  // kTvBatch ingested slices
  bool tv;
  size_t nt64, nt32, total_nt;  // node-temporal tables, past `total` (opt-in)
  int npartial;
  size_t total;
};

// PCG iterations whose coefficients lqgrid_condition_estimate can record.
constexpr int kHistCap = 8192;

Plan make_plan(const Dims& D, bool tv) {
  Plan P{};
  P.tv = tv;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t nn = (size_t)D.n * D.n, nodes = D.nodes, NB = 2 * D.n;
  const size_t fw = (size_t)2 * D.V * fw_rows(D.K) * NB * kFwRow;
  const size_t bw = (size_t)2 * D.V * D.K * NB * kBwRow;
  const size_t xw = (size_t)2 * D.V * NB * kFwRow;
  P.scal = take(sizeof(Scalars));
  P.scal_outer = take(sizeof(Scalars));
  P.hist = take((size_t)kHistCap * 2 * sizeof(double));
  const size_t rn = (size_t)D.real_nodes;
  P.inA = take(rn * nn * 8);
  P.inAnbr = take(rn * 4 * nn * 8);
  P.inB = take(rn * D.n * D.m * 8);
  P.inQ = take(rn * nn * 8);
  P.inQT = take(rn * nn * 8);
  P.inR = take(rn * D.m * D.m * 8);
  P.nsz = take(rn * sizeof(int));
  P.G13 = take(nodes * 13 * nn * 8);
  P.Cdn = take(nodes * 5 * nn * 8);
  P.Cup = take(nodes * 5 * nn * 8);
  P.AT5 = take(nodes * 5 * nn * 8);
  P.Qi = take(nodes * nn * 8);
  P.QTi = take(nodes * nn * 8);
  P.QTd = take(nodes * nn * 8);
  P.Qm = take(nodes * nn * 8);
  P.RiBT = take(nodes * (size_t)D.m * D.n * 8);
  P.Fw = take(fw * 8);
  P.Bw = take(bw * 8);
  P.Xw = take(xw * 8);
  P.G13f = take(nodes * 13 * nn * 4);
  P.Cdnf = take(nodes * 5 * nn * 4);
  P.Cupf = take(nodes * 5 * nn * 4);
  P.Qif = take(nodes * nn * 4);
  P.QTdf = take(nodes * nn * 4);
  P.Qmf = take(nodes * nn * 4);
  P.Fwf = take(fw * 4);
  P.Bwf = take(bw * 4);
  P.Xwf = take(xw * 4);
  P.A5 = take(nodes * 5 * nn * 8);
  P.BRB = take(nodes * nn * 8);
  P.A5f = take(nodes * 5 * nn * 4);
  P.BRBf = take(nodes * nn * 4);
  P.W64 = take((size_t)D.vlen * 8);
  P.W32 = take((size_t)D.vlen * 4);
  const int apply_blocks = padded_grid(((D.real_nodes + 3) / 4) * ((D.Tt + 63) / 64));
  P.npartial = std::max(apply_blocks, kFlatBlocks);
  if (tv) {
    const size_t L = (size_t)D.nodes * D.ldt;
    const size_t fwt = (size_t)D.V * fw_rows(D.K) * kFwRow * D.ldt * 8;
    const size_t bwt = (size_t)D.V * D.K * kBwRow * D.ldt * 8;
    P.tG13 = take(L * 13 * nn * 8);
    P.tQi = take(L * nn * 8);
    P.tCdn = take(L * 5 * nn * 8);
    P.tCup = take(L * 5 * nn * 8);
    P.tAT5 = take(L * 5 * nn * 8);
    P.tRiBT = take(L * D.m * D.n * 8);
    P.tA5 = take(L * 5 * nn * 8);
    P.tBRB = take(L * nn * 8);
    P.tFw = take(fwt * 8);
    P.tBw = take(bwt * 8);
    P.tW = take((size_t)D.vlen * 8);
    P.tG13f = take(L * 13 * nn * 4);
    P.tQif = take(L * nn * 4);
    P.tCdnf = take(L * 5 * nn * 4);
    P.tCupf = take(L * 5 * nn * 4);
    P.tA5f = take(L * 5 * nn * 4);
    P.tBRBf = take(L * nn * 4);
    P.tFwf = take(fwt * 4);
    P.tBwf = take(bwt * 4);
    P.tWf = take((size_t)D.vlen * 4);
    const size_t B = kTvBatch, nd = D.nodes;
    P.tsG13 = take(B * nd * 13 * nn * 8);
    P.tsQi = take(B * nd * nn * 8);
    P.tsCdn = take(B * nd * 5 * nn * 8);
    P.tsCup = take(B * nd * 5 * nn * 8);
    P.tsAT5 = take(B * nd * 5 * nn * 8);
    P.tsRiBT = take(B * nd * D.m * D.n * 8);
    P.tsA5 = take(B * nd * 5 * nn * 8);
    P.tsBRB = take(B * nd * nn * 8);
    P.tsInA = take(B * rn * nn * 8);
    P.tsInN = take(B * rn * 4 * nn * 8);
    P.tsInB = take(B * rn * D.n * D.m * 8);
    P.tsInQ = take(B * rn * nn * 8);
    P.tsInR = take(B * rn * D.m * D.m * 8);
    P.npartial = std::max<int>(P.npartial, (int)(((long long)D.real_nodes * D.ldt + 255) / 256));
  }
  P.psum = take((size_t)P.npartial * 8);
  P.pmax = take((size_t)P.npartial * 8);
  for (int v = 0; v < kNumOuter; ++v) P.outer[v] = take((size_t)D.vlen * 8);
  for (int v = 0; v < kNumPcg; ++v) P.p64[v] = take((size_t)D.vlen * 8);
  for (int v = 0; v < kNumPcg; ++v) P.p32[v] = take((size_t)D.vlen * 4);
  P.total = off;
  P.nt64 = take(nt_table_doubles(D) * 8);
  P.nt32 = take(nt_table_doubles(D) * 4);
  P.total_nt = off;
  return P;
}

template <typename T>
struct PcgBufs {
  T* v[kNumPcg];
};

}  // namespace

struct lqgrid_ctx {
  Dims D;
  Plan P;
  Coef C;
  OpCoef<double> op64;
  OpCoef<float> op32;
  hipStream_t stream;
  char* ws;
  Scalars* sc;        // the PCG instance
  Scalars* sco;       // the outer loop
  double* outer[kNumOuter];
  PcgBufs<double> b64;
  PcgBufs<float> b32;
  double *psum, *pmax;
  bool factored = false;
  bool qt_distinct = false;
  int pmode = LQGRID_PRECOND_NBJM;  // preconditioner of the running solve
  bool nt_ok = false;   // the workspace holds the node-temporal tables
  bool nt_factored = false;
  bool sized = false;     // per-node sizes given: x0 is masked by nsz
  bool rd_dirty = false;  // r_delta holds boundary terms of an earlier solve
  const int* nsz = nullptr;       // per-node state sizes (workspace copy)
  const double* Anbr = nullptr;   // ingested coupling blocks (boundary terms)
  bool tv = false;                // time-varying data
  TvCoef<double> tv64{};
  TvCoef<float> tv32{};
  int host_iter[2];   // staging for resetting the device iteration counters
  // profiling
  bool prof = false;
  int prof_stride = 1;                  // time every prof_stride-th launch
  long long prof_seen[4] = {0, 0, 0, 0};  // launches per kind since enable
  long long prof_launches[4] = {0, 0, 0, 0};
  double prof_ms[4] = {0, 0, 0, 0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  std::vector<int> prof_kind;
  std::vector<int> prof_batch;  // PCG check batch of the sample (-1: none)
  int prof_used = 0;
  int prof_batch_cur = -1;
  int prof_batches = 0;
  ~lqgrid_ctx() {
    for (auto& e : prof_ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
};

namespace {

thread_local char g_last_error[256] = "";

}  // namespace

namespace lqg {

bool make_dims(const lqgrid_problem_desc* d, Dims* D) {
  if (!d || d->K < 1 || d->N < 1 || d->T < 1 || d->n < 1 || d->m < 1) return false;
  D->K = d->K;
  D->N = d->N;
  D->T = d->T;
  D->n = d->n;
  D->m = d->m;
  D->V = (d->N + 1) / 2;
  D->Npad = 2 * D->V;
  D->Tt = d->T + 1;
  D->ldt = (D->Tt + 15) / 16 * 16;
  D->nodes = D->Npad * d->K;
  D->real_nodes = d->N * d->K;
  D->vlen = (long long)D->nodes * d->n * D->ldt;
  return true;
}

int hip_fail(hipError_t e, const char* where) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where,
                hipGetErrorString(e), (int)e);
  return LQGRID_EHIP;
}


// Optional event timing around one launch (profiling mode only).  Events are
// recorded without synchronising and resolved after the next stream sync.
struct ProfScope {
  lqgrid_ctx* c;
  int slot = -1;
  ProfScope(lqgrid_ctx* c_, int k) : c(c_) {
    if (!c->prof) return;
    if (c->prof_seen[k]++ % c->prof_stride != 0) return;
    if (c->prof_used >= (int)c->prof_ev.size()) {
      hipEvent_t a, b;
      // timing only: no system-scope fence (no L2 writeback per sample)
      if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess ||
          hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess)
        return;
      c->prof_ev.push_back({a, b});
      c->prof_kind.push_back(0);
      c->prof_batch.push_back(-1);
    }
    slot = c->prof_used++;
    c->prof_kind[slot] = k;
    c->prof_batch[slot] = c->prof_batch_cur;
    (void)hipEventRecord(c->prof_ev[slot].first, c->stream);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(c->prof_ev[slot].second, c->stream);
  }
};

// Launches of the check batch in which a PCG run stops may exit at once
// (device-side gate); their samples are dropped.
void prof_drop_batch(lqgrid_ctx* c, int batch) {
  for (int e = 0; e < c->prof_used; ++e)
    if (c->prof_batch[e] == batch) c->prof_kind[e] = -1;
}

void prof_resolve(lqgrid_ctx* c) {
  for (int e = 0; e < c->prof_used; ++e) {
    if (c->prof_kind[e] < 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->prof_ev[e].first, c->prof_ev[e].second) ==
        hipSuccess) {
      c->prof_ms[c->prof_kind[e]] += ms;
      c->prof_launches[c->prof_kind[e]] += 1;
    }
  }
  c->prof_used = 0;
}

void opts_fill(const lqgrid_solve_opts* in, lqgrid_solve_opts* o) {
  lqgrid_default_opts(o);
  if (in) *o = *in;
  if (o->max_iter <= 0) o->max_iter = 10000;
  if (o->check_every <= 0) o->check_every = 8;
  if (o->inner_tol <= 0) o->inner_tol = 1e-5;
}

bool opts_valid(const lqgrid_solve_opts& o) {
  return o.outer_S >= 1 && o.inner_L >= 2 && (o.inner_L % 2) == 0 &&
         o.tol > 0 && std::isfinite(o.tol) &&
         (o.precision == LQGRID_FP64 || o.precision == LQGRID_FP32_REFINE) &&
         o.preconditioner >= LQGRID_PRECOND_NBJM && o.preconditioner <= LQGRID_PRECOND_NONE;
}

}  // namespace lqg

namespace {

// Copies the scalars to the host (stream synchronised); pending timing
// samples are resolved unless the caller still has to drop some.
int read_scalars(lqgrid_ctx* c, const Scalars* src, Scalars* h, bool resolve = true) {
  HIPCHECK(hipMemcpyAsync(h, src, sizeof(Scalars), hipMemcpyDeviceToHost,
                          c->stream));
  HIPCHECK(hipStreamSynchronize(c->stream));
  if (resolve && c->prof_used) prof_resolve(c);
  return LQGRID_OK;
}

template <typename T>
const OpCoef<T>& op_coef(const lqgrid_ctx* c);
template <>
const OpCoef<double>& op_coef<double>(const lqgrid_ctx* c) { return c->op64; }
template <>
const OpCoef<float>& op_coef<float>(const lqgrid_ctx* c) { return c->op32; }
template <typename T>
PcgBufs<T>& pcg_bufs(lqgrid_ctx* c);
template <>
PcgBufs<double>& pcg_bufs<double>(lqgrid_ctx* c) { return c->b64; }
template <>
PcgBufs<float>& pcg_bufs<float>(lqgrid_ctx* c) { return c->b32; }

template <typename T>
const TvCoef<T>& tv_coef(const lqgrid_ctx* c);
template <>
const TvCoef<double>& tv_coef<double>(const lqgrid_ctx* c) { return c->tv64; }
template <>
const TvCoef<float>& tv_coef<float>(const lqgrid_ctx* c) { return c->tv32; }

// The operators of the path on the context's data: the time-invariant
// kernels, or the time-varying ones (tv.hip).
template <typename T>
int op_delta(lqgrid_ctx* c, const T* d, T* y, double* partial, const Scalars* sc,
             int check) {
  if (c->tv) return tv_delta_apply<T>(c->D, tv_coef<T>(c), d, y, partial, sc, check, c->stream);
  return delta_apply<T>(c->D, op_coef<T>(c), d, y, partial, sc, check, c->stream);
}
template <typename T>
void op_xi(lqgrid_ctx* c, const T* r, const T* dl, T* rho, int check) {
  if (c->tv) tv_xi_rhs<T>(c->D, tv_coef<T>(c), r, dl, rho, c->sc, check, c->stream);
  else xi_rhs<T>(c->D, op_coef<T>(c), r, dl, rho, c->sc, check, c->stream);
}
template <typename T>
void op_omega(lqgrid_ctx* c, const T* rho, const T* th, T* tau, int check) {
  if (c->tv) tv_omega_rhs<T>(c->D, tv_coef<T>(c), rho, th, tau, c->sc, check, c->stream);
  else omega_rhs<T>(c->D, op_coef<T>(c), rho, th, tau, c->sc, check, c->stream);
}
template <typename T>
void op_phi(lqgrid_ctx* c, const T* tau, T* out, int check) {
  if (c->tv) tv_phi_solve<T>(c->D, tv_coef<T>(c), tau, out, c->sc, check, c->stream);
  else phi_solve<T>(c->D, op_coef<T>(c), tau, out, c->sc, check, c->qt_distinct ? 1 : 0,
                    c->stream);
}
void op_recover(lqgrid_ctx* c, const double* dl, double* x, double* u) {
  if (c->tv) tv_recover(c->D, c->tv64, dl, x, u, c->stream);
  else recover(c->D, c->C, dl, x, u, c->stream);
}

// q = P_S^-1 r by S outer x L inner NBJM sweeps (Alg. 2 with a fixed number
// of sweeps, Theorem 2).  Returns the buffer holding the result (one of the
// two theta buffers of the PCG instance).
template <typename T>
const T* nt_tab(const lqgrid_ctx* c);
template <>
const double* nt_tab<double>(const lqgrid_ctx* c) {
  return reinterpret_cast<const double*>(c->ws + c->P.nt64);
}
template <>
const float* nt_tab<float>(const lqgrid_ctx* c) {
  return reinterpret_cast<const float*>(c->ws + c->P.nt32);
}

template <typename T>
T* precondition(lqgrid_ctx* c, const T* r, int S, int L, int check) {
  const Dims& D = c->D;
  if (c->pmode == LQGRID_PRECOND_NODE_TEMPORAL) {  // one node-temporal Jacobi sweep
    T* q = pcg_bufs<T>(c).v[kBufC];
    ProfScope ps(c, 1);
    nt_solve<T>(D, nt_tab<T>(c), r, pcg_bufs<T>(c).v[kBufD], q, c->sc, check, c->stream);
    return q;
  }
  const OpCoef<T>& C = op_coef<T>(c);
  PcgBufs<T>& b = pcg_bufs<T>(c);
  T* rho = b.v[kBufA];
  T* tau = b.v[kBufB];
  T* thx = b.v[kBufC];
  T* thy = b.v[kBufD];
  T* dprev = nullptr;  // delta^(s) of Alg. 2 (zero for s = 0)
  for (int s = 0; s < S; ++s) {
    const T* rs = r;
    if (s > 0) {  // r_theta^(s) = r + Xi~ delta^(s)
      ProfScope ps(c, 2);
      op_xi<T>(c, r, dprev, rho, check);
      rs = rho;
    }
    T* th = (dprev == thx) ? thy : thx;
    for (int l = 0; l < L; ++l) {
      const T* rhs = rs;
      if (l > 0) {  // tau = r_theta + Omega~ theta^(l)
        ProfScope ps(c, 2);
        op_omega<T>(c, rs, th, tau, check);
        rhs = tau;
      }
      ProfScope ps(c, 1);
      op_phi<T>(c, rhs, th, check);
    }
    dprev = th;
  }
  return dprev;
}

// Algorithm 1 on Delta x = b from x = 0 in element type T.  On entry the PCG
// instance's r vector holds b and x is zero.  Stops when the recursively
// updated residual satisfies ||r|| <= tol_rel ||b||, on breakdown, or after
// max_iter iterations.  Returns a HIP status; *iters and *done report the
// iterations taken and the device stop reason.
template <typename T>
int pcg_core(lqgrid_ctx* c, double tol_rel, int max_iter, int check_every,
             int S, int L, int* iters, int* done) {
  const Dims& D = c->D;
  const OpCoef<T>& C = op_coef<T>(c);
  PcgBufs<T>& b = pcg_bufs<T>(c);
  hipStream_t s = c->stream;
  Scalars* sc = c->sc;
  T* r = b.v[kR];
  T* d = b.v[kD];
  T* y = b.v[kY];
  T* x = b.v[kX];
  int np = vec_norms<T>(D, r, c->psum, c->pmax, s);
  scalar_step(kModeRd2, c->psum, c->pmax, np, sc, tol_rel, s);
  c->host_iter[0] = 0;
  c->host_iter[1] = max_iter;
  HIPCHECK(hipMemcpyAsync(&sc->iter, c->host_iter, 2 * sizeof(int),
                          hipMemcpyHostToDevice, s));
  // P = I (plain CG): q aliases r, every read of q sees the current residual
  const bool ident = c->pmode == LQGRID_PRECOND_NONE;
  T* q = ident ? r : precondition<T>(c, r, S, L, 0);
  np = vec_dot<T>(D, q, r, c->psum, sc, 0, s);
  scalar_step(kModeMuInit, c->psum, nullptr, np, sc, 0.0, s);
  vec_zero<T>(d, D.vlen, s);
  Scalars h{};
  for (;;) {
    c->prof_batch_cur = ++c->prof_batches;
    for (int k = 0; k < check_every; ++k) {
      vec_dir<T>(D, q, d, sc, s);  // d = q + beta d (beta = 0 after init)
      {
        ProfScope ps(c, 0);
        np = op_delta<T>(c, d, y, c->psum, sc, 1);
      }
      scalar_step(kModeYd, c->psum, nullptr, np, sc, 0.0, s);
      {
        ProfScope ps(c, 3);
        np = vec_update<T>(D, d, y, x, r, c->psum, sc, s);
      }
      scalar_step(kModeRr, c->psum, nullptr, np, sc, 0.0, s);
      if (!ident) q = precondition<T>(c, r, S, L, 1);
      np = vec_dot<T>(D, q, r, c->psum, sc, 1, s);
      scalar_step(kModeMu, c->psum, nullptr, np, sc, 0.0, s);
    }
    c->prof_batch_cur = -1;
    HIPCHECK(hipGetLastError());
    const int st = read_scalars(c, sc, &h, false);
    if (st != LQGRID_OK) return st;
    if (h.done != kRunning) prof_drop_batch(c, c->prof_batches);
    if (c->prof_used) prof_resolve(c);
    if (h.done != kRunning) break;
  }
  *iters = h.iter;
  *done = h.done;
  return LQGRID_OK;
}

// r_delta of a solve: -gamma at t = 0 (padding masked with per-node sizes)
// and the boundary terms at t >= 1 (cleared when an earlier solve left some).
void rhs_of(lqgrid_ctx* c, const double* x0, const lqgrid_boundary* bc) {
  launch_rhs_init(c->D, x0, c->outer[kRd], c->stream, c->sized ? c->nsz : nullptr);
  const bool any = bc && (bc->alpha_lo || bc->alpha_hi || bc->beta_lo || bc->beta_hi);
  if (any || c->rd_dirty) {
    Boundary b{any ? bc->alpha_lo : nullptr, any ? bc->alpha_hi : nullptr,
               any ? bc->beta_lo : nullptr, any ? bc->beta_hi : nullptr};
    launch_rhs_boundary(c->D, c->Anbr, b, c->outer[kRd], c->stream);
  }
  c->rd_dirty = any;
}

// r = r_delta - Delta dl (FP64), true residual norms into the outer scalars.
void true_residual(lqgrid_ctx* c, const double* dl = nullptr) {
  const Dims& D = c->D;
  op_delta<double>(c, dl ? dl : c->outer[kDl], c->outer[kYt], nullptr, c->sco, 0);
  const int np = vec_sub_norm(D, c->outer[kRd], c->outer[kYt], c->outer[kRt],
                              c->psum, c->pmax, c->stream);
  scalar_step(kModeTrue, c->psum, c->pmax, np, c->sco, 0.0, c->stream);
}

// One pass in element type T: e = PCG(Delta, r / ||r||), dl += ||r|| e.
template <typename T>
int refine_pass(lqgrid_ctx* c, double rnorm, double tol_rel, int max_iter,
                const lqgrid_solve_opts& o, int* iters, int* done) {
  PcgBufs<T>& b = pcg_bufs<T>(c);
  vec_scale_to<T>(c->D, c->outer[kRt], 1.0 / rnorm, b.v[kR], c->stream);
  vec_zero<T>(b.v[kX], c->D.vlen, c->stream);
  const int st = pcg_core<T>(c, tol_rel, max_iter, o.check_every, o.outer_S,
                             o.inner_L, iters, done);
  if (st != LQGRID_OK) return st;
  vec_axpy_from<T>(c->D, rnorm, b.v[kX], c->outer[kDl], c->stream);
  return LQGRID_OK;
}

// FP32 copies of the operator blocks (after assembly) and of the factors
// (after factorisation) for the precision form.
void make_f32_blocks(lqgrid_ctx* c, bool factors) {
  const Dims& D = c->D;
  const long long nn = (long long)D.n * D.n, nodes = D.nodes, NB = 2 * D.n;
  char* w = c->ws;
  const Plan& P = c->P;
  auto fp = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
  if (!factors) {
    copy_to_float(c->C.G13, fp(P.G13f), nodes * 13 * nn, c->stream);
    copy_to_float(c->C.Cdn, fp(P.Cdnf), nodes * 5 * nn, c->stream);
    copy_to_float(c->C.Cup, fp(P.Cupf), nodes * 5 * nn, c->stream);
    copy_to_float(c->C.Qi, fp(P.Qif), nodes * nn, c->stream);
    copy_to_float(c->C.QTd, fp(P.QTdf), nodes * nn, c->stream);
    copy_to_float(c->C.Qm, fp(P.Qmf), nodes * nn, c->stream);
    copy_to_float(c->C.A5, fp(P.A5f), nodes * 5 * nn, c->stream);
    copy_to_float(c->C.BRB, fp(P.BRBf), nodes * nn, c->stream);
  } else {
    copy_to_float(c->C.Fw, fp(P.Fwf), 2LL * D.V * fw_rows(D.K) * NB * kFwRow, c->stream);
    copy_to_float(c->C.Bw, fp(P.Bwf), 2LL * D.V * D.K * NB * kBwRow, c->stream);
    copy_to_float(c->C.Xw, fp(P.Xwf), 2LL * D.V * NB * kFwRow, c->stream);
  }
}


// Scratch of the allocation-free entry point: the whole workspace of one
// solve, in a file-scope device array that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.
constexpr size_t kNoAllocBytes = (size_t)80 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LQGRID_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) % kAlign) != 0)
      return hip_fail(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LQGRID_OK;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a and off-diagonal b (Sturm sequence of the LDL' pivots).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t k = 0; k < a.size(); ++k) {
    const double off = k ? b[k - 1] * b[k - 1] : 0.0;
    q = a[k] - x - (k ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;  // a zero pivot counts as negative
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// The k-th smallest eigenvalue (k = 0 .. size-1) by bisection inside the
// Gershgorin interval, to a relative width of 1e-14.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) > k) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Argument checks shared by lqgrid_setup and lqgrid_solve_noalloc.
int check_problem(const lqgrid_problem_desc* desc, Dims* D) {
  if (!make_dims(desc, D)) return LQGRID_EINVAL;
  if (!desc->A || !desc->A_nbr || !desc->B || !desc->Q || !desc->R)
    return LQGRID_EINVAL;
  if (D->n > kMaxN || D->m > kMaxM) return LQGRID_EUNSUPPORTED;
  // the block solves address each vector with 32-bit byte offsets
  if (D->vlen * 8 >= (1LL << 31)) return LQGRID_EUNSUPPORTED;
  return LQGRID_OK;
}

// Lays the workspace out for the problem, clears what must start at zero and
// enqueues ingest and assembly into c (a fresh context).
int setup_into(lqgrid_ctx* c, const lqgrid_problem_desc* desc, const Dims& D,
               void* workspace, size_t workspace_bytes, void* hip_stream) {
  const bool tv = desc->time_varying != 0;
  const Plan P = make_plan(D, tv);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 ||
      workspace_bytes < P.total)
    return LQGRID_EWORKSPACE;
  c->D = D;
  c->tv = tv;
  c->nt_ok = workspace_bytes >= P.total_nt;
  c->P = P;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  char* w = c->ws;
  auto dp = [&](size_t off) { return reinterpret_cast<double*>(w + off); };
  auto fp = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
  c->sc = reinterpret_cast<Scalars*>(w + P.scal);
  c->sco = reinterpret_cast<Scalars*>(w + P.scal_outer);
  c->C = Coef{dp(P.G13), dp(P.Cdn), dp(P.Cup), dp(P.AT5), dp(P.Qi), dp(P.QTi),
              dp(P.QTd), dp(P.Qm), dp(P.RiBT), dp(P.Fw), dp(P.Bw), dp(P.Xw)};
  c->C.A5 = dp(P.A5);
  c->C.BRB = dp(P.BRB);
  c->op64 = OpCoef<double>{c->C.G13, c->C.Cdn, c->C.Cup, c->C.Qi, c->C.QTd,
                           c->C.Qm, c->C.Fw, c->C.Bw, c->C.Xw,
                           c->C.A5, c->C.BRB, dp(P.W64)};
  c->op32 = OpCoef<float>{fp(P.G13f), fp(P.Cdnf), fp(P.Cupf), fp(P.Qif),
                          fp(P.QTdf), fp(P.Qmf), fp(P.Fwf), fp(P.Bwf), fp(P.Xwf),
                          fp(P.A5f), fp(P.BRBf), fp(P.W32)};
  for (int v = 0; v < kNumOuter; ++v) c->outer[v] = dp(P.outer[v]);
  for (int v = 0; v < kNumPcg; ++v) {
    c->b64.v[v] = dp(P.p64[v]);
    c->b32.v[v] = fp(P.p32[v]);
  }
  c->psum = dp(P.psum);
  c->pmax = dp(P.pmax);
  clear_stale_error();
  // zero the scalars and every vector (padding entries must stay zero)
  vec_zero<double>(dp(P.scal), (long long)(P.G13 - P.scal) / 8, c->stream);
  for (int v = 0; v < kNumOuter; ++v) vec_zero<double>(c->outer[v], D.vlen, c->stream);
  for (int v = 0; v < kNumPcg; ++v) {
    vec_zero<double>(c->b64.v[v], D.vlen, c->stream);
    vec_zero<float>(c->b32.v[v], D.vlen, c->stream);
  }
  vec_zero<double>(dp(P.W64), D.vlen, c->stream);
  vec_zero<float>(fp(P.W32), D.vlen, c->stream);
  // ingest: copies of the problem arrays, padded where a node is smaller than
  // n, m (a plain copy for uniform sizes); the setup reads only the copies,
  // and the coupling blocks stay for the boundary terms of later solves
  ProblemIn user{D.K, D.N, D.n, D.m, desc->A, desc->A_nbr, desc->B,
                 desc->Q, desc->R, desc->QT};
  ProblemIn in{D.K, D.N, D.n, D.m, dp(P.inA), dp(P.inAnbr), dp(P.inB),
               dp(P.inQ), dp(P.inR), dp(P.inQT)};
  int* nsz = reinterpret_cast<int*>(w + P.nsz);
  c->sized = desc->n_node != nullptr;
  c->nsz = nsz;
  c->Anbr = in.A_nbr;
  if (!tv) {
    launch_ingest(D, user, desc->n_node, desc->m_node, in, nsz, c->sc, c->stream);
    launch_setup(D, in, c->C, c->sc, c->stream);
    make_f32_blocks(c, false);
  } else {
    // time-varying data: each time slice s is ingested and assembled by the
    // time-invariant kernels into the (scratch) blocks of c->C, then
    // scattered into the time-fastest arrays: blocks of slice s at t = s
    // (Cdn, Cup, AT5, R^-1 B', Q^-1) and t = s + 1 (the 13-point G); the
    // terminal weight Q_T gives Q^-1 at t = T
    c->tv64 = TvCoef<double>{dp(P.tG13), dp(P.tQi), dp(P.tCdn), dp(P.tCup), dp(P.tFw),
                             dp(P.tBw), dp(P.tAT5), dp(P.tRiBT), dp(P.tW),
                             dp(P.tA5), dp(P.tBRB), dp(P.W64)};
    c->tv32 = TvCoef<float>{fp(P.tG13f), fp(P.tQif), fp(P.tCdnf), fp(P.tCupf), fp(P.tFwf),
                            fp(P.tBwf), nullptr, nullptr, fp(P.tWf),
                            fp(P.tA5f), fp(P.tBRBf), fp(P.W32)};
    vec_zero<double>(dp(P.tG13), (long long)(P.tFw - P.tG13) / 8, c->stream);
    vec_zero<double>(dp(P.tW), D.vlen, c->stream);
    vec_zero<float>(fp(P.tWf), D.vlen, c->stream);
    const size_t rn = (size_t)D.real_nodes, nn = (size_t)D.n * D.n;
    const size_t sA = rn * nn, sN = rn * 4 * nn, sB = rn * D.n * D.m, sR = rn * D.m * D.m;
    const size_t nd = D.nodes;
    // every slice of a batch in one launch per setup kernel (slice b reads
    // its problem data, writes its ingested copy and assembly scratch)
    const ProblemIn user0{D.K, D.N, D.n, D.m, desc->A, desc->A_nbr, desc->B, desc->Q,
                          desc->R, desc->Q};
    const ProblemIn in0{D.K, D.N, D.n, D.m, dp(P.tsInA), dp(P.tsInN), dp(P.tsInB),
                        dp(P.tsInQ), dp(P.tsInR), dp(P.tsInQ)};
    Coef S0 = c->C;
    S0.G13 = dp(P.tsG13);
    S0.Qi = dp(P.tsQi);
    S0.Cdn = dp(P.tsCdn);
    S0.Cup = dp(P.tsCup);
    S0.AT5 = dp(P.tsAT5);
    S0.RiBT = dp(P.tsRiBT);
    S0.A5 = dp(P.tsA5);
    S0.BRB = dp(P.tsBRB);
    for (int s0 = 0; s0 <= D.T; s0 += kTvBatch) {
      const int nsl = std::min(kTvBatch, D.T + 1 - s0);
      TvSlices S{};
      S.s0 = s0;
      S.nsl = nsl;
      S.T = D.T;
      S.sA = (long long)sA;
      S.sN = (long long)sN;
      S.sB = (long long)sB;
      S.sR = (long long)sR;
      S.QT = desc->QT;
      S.iA = (long long)(rn * nn);
      S.iN = (long long)(rn * 4 * nn);
      S.iB = (long long)(rn * D.n * D.m);
      S.iR = (long long)(rn * D.m * D.m);
      S.cG13 = (long long)(nd * 13 * nn);
      S.cQi = (long long)(nd * nn);
      S.c5 = (long long)(nd * 5 * nn);
      S.cRiBT = (long long)(nd * D.m * D.n);
      S.cBRB = (long long)(nd * nn);
      launch_ingest_setup_tv(D, user0, S, desc->n_node, desc->m_node, in0, nsz, S0, c->sc,
                             c->stream);
      tv_scatter_batch(D, S0, c->tv64, s0, nsl, c->stream);
    }
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "lqgrid_setup launch");
  return LQGRID_OK;
}

}  // namespace

extern "C" {

void lqgrid_default_opts(lqgrid_solve_opts* o) {
  if (!o) return;
  o->outer_S = 2;
  o->inner_L = 2;
  o->tol = 1e-10;
  o->max_iter = 10000;
  o->precision = LQGRID_FP64;
  o->inner_tol = 1e-5;
  o->check_every = 8;
  o->warm_fallback = 1;
  o->preconditioner = LQGRID_PRECOND_NBJM;
}

int lqgrid_abi_version(void) { return LQGRID_ABI_VERSION; }

const char* lqgrid_status_string(int s) {
  switch (s) {
    case LQGRID_OK: return "ok";
    case LQGRID_EINVAL: return "invalid argument";
    case LQGRID_ENOTSPD: return "Phi_bar block not positive definite";
    case LQGRID_EBREAKDOWN: return "PCG breakdown";
    case LQGRID_ENOCONV: return "no convergence within max_iter";
    case LQGRID_EWORKSPACE: return "workspace null, misaligned or too small";
    case LQGRID_EHIP: return "HIP runtime error";
    case LQGRID_EUNSUPPORTED: return "size outside the compiled range";
  }
  return "unknown status";
}

size_t lqgrid_workspace_bytes(const lqgrid_problem_desc* desc,
                              const lqgrid_solve_opts* opts) {
  Dims D;
  if (!make_dims(desc, &D)) return 0;
  const Plan P = make_plan(D, desc->time_varying != 0);
  return (opts && opts->preconditioner == LQGRID_PRECOND_NODE_TEMPORAL) ? P.total_nt : P.total;
}

int lqgrid_setup(const lqgrid_problem_desc* desc, void* workspace,
                 size_t workspace_bytes, void* hip_stream, lqgrid_ctx** out) {
  if (!out) return LQGRID_EINVAL;
  *out = nullptr;
  Dims D;
  const int chk = check_problem(desc, &D);
  if (chk != LQGRID_OK) return chk;
  lqgrid_ctx* c = new (std::nothrow) lqgrid_ctx();
  if (!c) return LQGRID_EHIP;
  const int st = setup_into(c, desc, D, workspace, workspace_bytes, hip_stream);
  if (st != LQGRID_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LQGRID_OK;
}

int lqgrid_factor(lqgrid_ctx* c) {
  if (!c) return LQGRID_EINVAL;
  clear_stale_error();
  // entries never written by the factorisation (padding, N1/N2 of the last
  // block rows) must read as zero
  const long long NB = 2 * c->D.n;
  if (c->tv) {
    // one-chain factorisation of every Phi_bar_{v,t}, t = 0..T, written in
    // the time-fastest table layout; FP32 copies for the precision form
    const Dims& D = c->D;
    const Plan& P = c->P;
    char* w = c->ws;
    auto dp = [&](size_t off) { return reinterpret_cast<double*>(w + off); };
    auto fp = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
    const long long L = (long long)D.nodes * D.ldt, nn = (long long)D.n * D.n;
    const long long fwt = (long long)D.V * fw_rows(D.K) * kFwRow * D.ldt * 8;
    const long long bwt = (long long)D.V * D.K * kBwRow * D.ldt * 8;
    vec_zero<double>(dp(P.tFw), fwt, c->stream);
    vec_zero<double>(dp(P.tBw), bwt, c->stream);
    Coef F{};
    F.G13 = dp(P.tG13);
    F.Qi = dp(P.tQi);
    F.Fw = dp(P.tFw);
    F.Bw = dp(P.tBw);
    F.tv_ld = D.ldt;
    tv_factor(D, F, c->sc, c->stream);
    copy_to_float(dp(P.tG13), fp(P.tG13f), L * 13 * nn, c->stream);
    copy_to_float(dp(P.tQi), fp(P.tQif), L * nn, c->stream);
    copy_to_float(dp(P.tCdn), fp(P.tCdnf), L * 5 * nn, c->stream);
    copy_to_float(dp(P.tCup), fp(P.tCupf), L * 5 * nn, c->stream);
    copy_to_float(dp(P.tA5), fp(P.tA5f), L * 5 * nn, c->stream);
    copy_to_float(dp(P.tBRB), fp(P.tBRBf), L * nn, c->stream);
    copy_to_float(dp(P.tFw), fp(P.tFwf), fwt, c->stream);
    copy_to_float(dp(P.tBw), fp(P.tBwf), bwt, c->stream);
  } else {
    vec_zero<double>(c->C.Fw, 2LL * c->D.V * fw_rows(c->D.K) * NB * kFwRow, c->stream);
    vec_zero<double>(c->C.Bw, 2LL * c->D.V * c->D.K * NB * kBwRow, c->stream);
    vec_zero<double>(c->C.Xw, 2LL * c->D.V * NB * kFwRow, c->stream);
    launch_factor(c->D, c->C, c->sc, c->stream);
    make_f32_blocks(c, true);
  }
  if (c->nt_ok) {  // node-temporal tables (workspace sized for them)
    double* t64 = reinterpret_cast<double*>(c->ws + c->P.nt64);
    nt_factor(c->D, c->C, c->tv64, c->tv ? 1 : 0, t64, c->sc, c->stream);
    copy_to_float(t64, reinterpret_cast<float*>(c->ws + c->P.nt32),
                  (long long)nt_table_doubles(c->D), c->stream);
    c->nt_factored = true;
  }
  HIPCHECK(hipGetLastError());
  Scalars h;
  int st = read_scalars(c, c->sc, &h);
  if (st != LQGRID_OK) return st;
  c->qt_distinct = h.qt_differs != 0;
  if (h.flag_badsize) return LQGRID_EINVAL;
  if (h.flag_notspd) return LQGRID_ENOTSPD;
  c->factored = true;
  return LQGRID_OK;
}

namespace {

// The body of lqgrid_pcg_solve.  With timed_events the device time comes from
// two HIP events around the solve; without (the allocation-free entry point)
// from the host clock around the synchronised solve.
int pcg_solve_impl(lqgrid_ctx* c, const double* x0, const lqgrid_boundary* bc,
                   const lqgrid_solve_opts* opts_in, const double* delta_init,
                   double* delta, double* x, double* u, lqgrid_info* info,
                   bool timed_events) {
  if (info) std::memset(info, 0, sizeof(*info));
  if (!c || !x0 || !delta) return LQGRID_EINVAL;
  lqgrid_solve_opts o;
  opts_fill(opts_in, &o);
  if (!opts_valid(o) || !c->factored) return LQGRID_EINVAL;
  if (o.preconditioner == LQGRID_PRECOND_NODE_TEMPORAL && !c->nt_factored)
    return LQGRID_EWORKSPACE;
  c->pmode = o.preconditioner;
  const Dims& D = c->D;
  hipStream_t s = c->stream;
  clear_stale_error();
  // the solve's timing events, destroyed on every return path
  struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  const auto h0 = std::chrono::steady_clock::now();
  if (timed_events) {
    HIPCHECK(hipEventCreate(&ev.a));
    HIPCHECK(hipEventCreate(&ev.b));
    HIPCHECK(hipEventRecord(ev.a, s));
  }

  // r_delta, ||r_delta||, tol^2 ||r_delta||^2 (outer scalars)
  if (c->tv && bc && (bc->alpha_lo || bc->alpha_hi || bc->beta_lo || bc->beta_hi))
    return LQGRID_EUNSUPPORTED;  // boundary couplings are kept for one time slice only
  rhs_of(c, x0, bc);
  int np = vec_norms<double>(D, c->outer[kRd], c->psum, c->pmax, s);
  scalar_step(kModeRd2, c->psum, c->pmax, np, c->sco, o.tol, s);
  if (delta_init) to_internal(D, delta_init, c->outer[kDl], s);
  else vec_zero<double>(c->outer[kDl], D.vlen, s);

  int status = LQGRID_OK, total_it = 0, passes = 0;
  bool warm = delta_init != nullptr;
  Scalars h{};
  if (warm && o.warm_fallback == 2) {
    // energy line search along the warm start: delta^(0) = alpha delta_init
    // with alpha = delta_init' r_delta / (delta_init' Delta delta_init), the
    // minimiser of the Delta-norm of the error on that line (Sec. III: the
    // norm PCG reduces), never larger than the zero start's
    op_delta<double>(c, c->outer[kDl], c->outer[kYt], c->psum, c->sco, 0);
    int nb = vec_dot<double>(D, c->outer[kDl], c->outer[kYt], c->psum, c->sco, 0, s);
    scalar_step(kModeDotB, c->psum, nullptr, nb, c->sco, 0.0, s);
    nb = vec_dot<double>(D, c->outer[kDl], c->outer[kRd], c->psum, c->sco, 0, s);
    scalar_step(kModeDotA, c->psum, nullptr, nb, c->sco, 0.0, s);
    const int st = read_scalars(c, c->sco, &h);
    if (st != LQGRID_OK) return st;
    const double alpha = h.mu / h.yd;
    if (h.yd > 0.0 && std::isfinite(alpha) && alpha > 0.0) {
      vec_scale_to<double>(D, c->outer[kDl], alpha, c->outer[kRt], s);
      vec_scale_to<double>(D, c->outer[kRt], 1.0, c->outer[kDl], s);
    } else {
      vec_zero<double>(c->outer[kDl], D.vlen, s);
      warm = false;
    }
  }
  for (;;) {
    true_residual(c);
    int st = read_scalars(c, c->sco, &h);
    if (st != LQGRID_OK) return st;
    if (warm && passes == 0 && o.warm_fallback == 1 && !(h.rr < h.rd2)) {
      // the warm start does not lower the residual: start from zero
      vec_zero<double>(c->outer[kDl], D.vlen, s);
      warm = false;
      continue;
    }
    if (h.rr <= h.tol2) break;  // also the exact-start case (0 iterations)
    if (!std::isfinite(h.rr)) {
      status = LQGRID_EBREAKDOWN;
      break;
    }
    if (total_it >= o.max_iter || passes >= kMaxPasses) {
      status = LQGRID_ENOCONV;
      break;
    }
    const double rnorm = std::sqrt(h.rr);
    // relative target of this pass: the absolute tol ||r_delta|| ...
    double tol_rel = o.tol * std::sqrt(h.rd2) / rnorm;
    int it = 0, done = kRunning;
    if (o.precision == LQGRID_FP32_REFINE) {
      // ... but no tighter than FP32 vectors can resolve
      tol_rel = std::max(tol_rel, o.inner_tol);
      st = refine_pass<float>(c, rnorm, tol_rel, o.max_iter - total_it, o, &it, &done);
    } else {
      st = refine_pass<double>(c, rnorm, std::min(tol_rel, 0.5),
                               o.max_iter - total_it, o, &it, &done);
    }
    if (st != LQGRID_OK) return st;
    total_it += it;
    ++passes;
    if (done == kBreakdown && it <= 1) {
      status = LQGRID_EBREAKDOWN;
      break;
    }
  }
  to_abi(D, c->outer[kDl], delta, s);
  if (x || u) op_recover(c, c->outer[kDl], x, u);
  float ms = 0.f;
  if (timed_events) {
    HIPCHECK(hipEventRecord(ev.b, s));
    HIPCHECK(hipEventSynchronize(ev.b));
    (void)hipEventElapsedTime(&ms, ev.a, ev.b);
  } else {
    HIPCHECK(hipStreamSynchronize(s));
    ms = (float)std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now() - h0).count();
  }
  if (c->prof_used) prof_resolve(c);
  HIPCHECK(hipGetLastError());
  if (info) {
    info->status = status;
    info->iterations = total_it;
    info->refinements = passes;
    info->restarts = std::max(0, passes - 1);
    info->rel_kkt_residual = h.rd2 > 0 ? std::sqrt(h.rr / h.rd2) : 0.0;
    info->rel_res_inf = h.rdinf > 0 ? h.rinf / h.rdinf : 0.0;
    info->seconds = ms * 1e-3;
    info->warm_start_used = warm ? 1 : 0;
  }
  return status;
}

}  // namespace

int lqgrid_pcg_solve(lqgrid_ctx* c, const double* x0,
                     const lqgrid_solve_opts* opts_in, const double* delta_init,
                     double* delta, double* x, double* u, lqgrid_info* info) {
  return pcg_solve_impl(c, x0, nullptr, opts_in, delta_init, delta, x, u, info, true);
}

int lqgrid_pcg_solve_bc(lqgrid_ctx* c, const double* x0, const lqgrid_boundary* bc,
                        const lqgrid_solve_opts* opts_in, const double* delta_init,
                        double* delta, double* x, double* u, lqgrid_info* info) {
  return pcg_solve_impl(c, x0, bc, opts_in, delta_init, delta, x, u, info, true);
}

int lqgrid_apply_operator(lqgrid_ctx* c, int op, int S, int L,
                          const double* in, double* out) {
  if (!c || !in || !out) return LQGRID_EINVAL;
  const Dims& D = c->D;
  hipStream_t s = c->stream;
  clear_stale_error();
  const bool f32 = (op & kOpF32) != 0;
  op &= ~kOpF32;
  if (op < LQGRID_OP_DELTA || op > LQGRID_OP_NODE_PRECOND) return LQGRID_EINVAL;
  if (op >= LQGRID_OP_PHI_SOLVE && !c->factored) return LQGRID_EINVAL;
  if (op == LQGRID_OP_NODE_PRECOND && !c->nt_factored) return LQGRID_EWORKSPACE;
  if (op == LQGRID_OP_PRECOND && (S < 1 || L < 1)) return LQGRID_EINVAL;
  double* vin = c->outer[kRt];
  double* vout = c->outer[kYt];
  to_internal(D, in, vin, s);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const OpCoef<T>& C = op_coef<T>(c);
    PcgBufs<T>& b = pcg_bufs<T>(c);
    T* x = b.v[kD];
    T* y = b.v[kY];
    vec_scale_to<T>(D, vin, 1.0, x, s);
    switch (op) {
      case LQGRID_OP_DELTA: op_delta<T>(c, x, y, nullptr, c->sc, 0); break;
      case LQGRID_OP_XI: op_xi<T>(c, (const T*)nullptr, x, y, 0); break;
      case LQGRID_OP_OMEGA: op_omega<T>(c, (const T*)nullptr, x, y, 0); break;
      case LQGRID_OP_PHI_SOLVE:
        op_phi<T>(c, x, y, 0);
        break;
      case LQGRID_OP_NODE_PRECOND:
        nt_solve<T>(D, nt_tab<T>(c), x, b.v[kBufD], y, c->sc, 0, s);
        break;
      default:
        c->pmode = LQGRID_PRECOND_NBJM;
        y = precondition<T>(c, x, S, L, 0);
        break;
    }
    vec_zero<double>(vout, D.vlen, s);
    vec_axpy_from<T>(D, 1.0, y, vout, s);
  };
  if (f32) run(float{});
  else run(double{});
  to_abi(D, vout, out, s);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

int lqgrid_profile_enable(lqgrid_ctx* c, int enable) {
  if (!c) return LQGRID_EINVAL;
  if (c->prof_used) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LQGRID_EHIP;
    prof_resolve(c);
  }
  c->prof = enable > 0;
  c->prof_stride = enable > 0 ? enable : 1;
  for (int k = 0; k < 4; ++k) {
    c->prof_seen[k] = 0;
    c->prof_launches[k] = 0;
    c->prof_ms[k] = 0.0;
  }
  return LQGRID_OK;
}

int lqgrid_profile_read(lqgrid_ctx* c, int kernel, long long* launches,
                        double* total_ms) {
  if (!c || kernel < 0 || kernel > 3) return LQGRID_EINVAL;
  if (c->prof_used) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LQGRID_EHIP;
    prof_resolve(c);
  }
  if (launches) *launches = c->prof_launches[kernel];
  if (total_ms) *total_ms = c->prof_ms[kernel];
  return LQGRID_OK;
}

int lqgrid_nbjm_solve(lqgrid_ctx* c, const double* x0, const lqgrid_solve_opts* opts_in,
                      double* delta, double* x, double* u, lqgrid_info* info) {
  if (info) std::memset(info, 0, sizeof(*info));
  if (!c || !x0 || !delta) return LQGRID_EINVAL;
  lqgrid_solve_opts o;
  opts_fill(opts_in, &o);
  if (!opts_valid(o) || !c->factored) return LQGRID_EINVAL;
  if (o.precision != LQGRID_FP64) return LQGRID_EUNSUPPORTED;
  const Dims& D = c->D;
  hipStream_t s = c->stream;
  clear_stale_error();
  const auto h0 = std::chrono::steady_clock::now();
  double* rd = c->outer[kRd];
  rhs_of(c, x0, nullptr);
  int np = vec_norms<double>(D, rd, c->psum, c->pmax, s);
  scalar_step(kModeRd2, c->psum, c->pmax, np, c->sco, o.tol, s);
  double* dcur = c->b64.v[kX];
  double* dnext = c->b64.v[kD];
  double* rho = c->b64.v[kBufA];
  double* tau = c->b64.v[kBufB];
  vec_zero<double>(dcur, D.vlen, s);
  int sweeps = 0, status = LQGRID_OK;
  Scalars h{};
  for (;;) {
    // delta^(s+1): rho = r_delta + Xi~ delta^(s); the inner iteration starts
    // from theta^(0) = delta^(s), theta^(l+1) = Phi~^-1 (rho + Omega~ theta^(l))
    {
      ProfScope ps(c, 2);
      op_xi<double>(c, rd, dcur, rho, 0);
    }
    const double* th = dcur;
    for (int l = 0; l < o.inner_L; ++l) {
      {
        ProfScope ps(c, 2);
        op_omega<double>(c, rho, th, tau, 0);
      }
      ProfScope ps(c, 1);
      op_phi<double>(c, tau, dnext, 0);
      th = dnext;
    }
    std::swap(dcur, dnext);
    ++sweeps;
    if (sweeps % o.check_every == 0 || sweeps >= o.max_iter) {
      true_residual(c, dcur);
      HIPCHECK(hipGetLastError());
      const int st = read_scalars(c, c->sco, &h);
      if (st != LQGRID_OK) return st;
      if (!std::isfinite(h.rr)) {
        status = LQGRID_EBREAKDOWN;
        break;
      }
      if (h.rr <= h.tol2) break;
      if (sweeps >= o.max_iter) {
        status = LQGRID_ENOCONV;
        break;
      }
    }
  }
  to_abi(D, dcur, delta, s);
  if (x || u) op_recover(c, dcur, x, u);
  HIPCHECK(hipStreamSynchronize(s));
  HIPCHECK(hipGetLastError());
  if (info) {
    info->status = status;
    info->iterations = sweeps;
    info->rel_kkt_residual = h.rd2 > 0 ? std::sqrt(h.rr / h.rd2) : 0.0;
    info->rel_res_inf = h.rdinf > 0 ? h.rinf / h.rdinf : 0.0;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
  }
  return status;
}

int lqgrid_condition_estimate(lqgrid_ctx* c, const double* x0, int preconditioned,
                              int outer_S, int inner_L, double tol, int max_iter,
                              double* kappa, double* lambda_min, double* lambda_max,
                              int* iterations) {
  if (!c || !x0 || !c->factored) return LQGRID_EINVAL;
  lqgrid_solve_opts o;
  opts_fill(nullptr, &o);
  o.outer_S = outer_S;
  o.inner_L = inner_L;
  o.tol = tol;
  o.max_iter = max_iter > 0 ? max_iter : kHistCap;
  if (!opts_valid(o) || o.max_iter > kHistCap || preconditioned < 0 || preconditioned > 2)
    return LQGRID_EINVAL;
  if (preconditioned == 2 && !c->nt_factored) return LQGRID_EWORKSPACE;
  const Dims& D = c->D;
  hipStream_t s = c->stream;
  clear_stale_error();
  rhs_of(c, x0, nullptr);
  int np = vec_norms<double>(D, c->outer[kRd], c->psum, c->pmax, s);
  scalar_step(kModeRd2, c->psum, c->pmax, np, c->sco, o.tol, s);
  vec_zero<double>(c->outer[kDl], D.vlen, s);
  true_residual(c);
  Scalars h{};
  int st = read_scalars(c, c->sco, &h);
  if (st != LQGRID_OK) return st;
  if (!(h.rr > 0.0) || !std::isfinite(h.rr)) return LQGRID_EBREAKDOWN;
  // record the coefficients of this one FP64 run of Algorithm 1 from zero
  struct { double* p; int cap; } stage{reinterpret_cast<double*>(c->ws + c->P.hist), kHistCap};
  HIPCHECK(hipMemcpyAsync(&c->sc->hist, &stage, sizeof(double*) + sizeof(int),
                          hipMemcpyHostToDevice, s));
  c->pmode = preconditioned == 0 ? LQGRID_PRECOND_NONE
            : preconditioned == 2 ? LQGRID_PRECOND_NODE_TEMPORAL : LQGRID_PRECOND_NBJM;
  int it = 0, done = kRunning;
  st = refine_pass<double>(c, std::sqrt(h.rr), o.tol, o.max_iter, o, &it, &done);
  c->pmode = LQGRID_PRECOND_NBJM;
  const decltype(stage) none{nullptr, 0};
  HIPCHECK(hipMemcpyAsync(&c->sc->hist, &none, sizeof(double*) + sizeof(int),
                          hipMemcpyHostToDevice, s));
  if (st != LQGRID_OK) return st;
  if (it < 1) return LQGRID_EBREAKDOWN;
  std::vector<double> coef(2 * (size_t)it);
  HIPCHECK(hipMemcpyAsync(coef.data(), c->ws + c->P.hist, coef.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  // Lanczos matrix of P^-1 Delta from the CG coefficients (Sec. III): diag
  // 1/theta_k + beta_{k-1}/theta_{k-1}, off-diagonal sqrt(beta_k)/theta_k
  std::vector<double> a(it), b(it > 1 ? it - 1 : 0);
  for (int k = 0; k < it; ++k) {
    const double th = coef[2 * k];
    a[k] = 1.0 / th + (k ? coef[2 * (k - 1) + 1] / coef[2 * (k - 1)] : 0.0);
    if (k + 1 < it) b[k] = std::sqrt(coef[2 * k + 1]) / th;
  }
  const double lo = tridiag_eig(a, b, 0), hi = tridiag_eig(a, b, it - 1);
  if (lambda_min) *lambda_min = lo;
  if (lambda_max) *lambda_max = hi;
  if (kappa) *kappa = hi / lo;
  if (iterations) *iterations = it;
  return done == kBreakdown ? LQGRID_EBREAKDOWN : LQGRID_OK;
}

size_t lqgrid_noalloc_capacity(void) { return kNoAllocBytes; }

int lqgrid_solve_noalloc(const lqgrid_problem_desc* desc, const double* x0,
                         const lqgrid_solve_opts* opts, double* delta, double* x,
                         double* u, void* hip_stream, lqgrid_info* info) {
  if (info) std::memset(info, 0, sizeof(*info));
  if (!x0 || !delta) return LQGRID_EINVAL;
  Dims D;
  const int chk = check_problem(desc, &D);
  if (chk != LQGRID_OK) return chk;
  const size_t need = lqgrid_workspace_bytes(desc, opts);
  if (need > kNoAllocBytes) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "lqgrid_solve_noalloc: the problem needs %zu bytes of scratch, "
                  "the library's static scratch holds %zu", need, kNoAllocBytes);
    return LQGRID_EWORKSPACE;
  }
  void* ws = nullptr;
  const int st = scratch_of_current_device(&ws);
  if (st != LQGRID_OK) return st;
  lqgrid_ctx c;  // on the stack: nothing is allocated on the host either
  int r = setup_into(&c, desc, D, ws, kNoAllocBytes, hip_stream);
  if (r != LQGRID_OK) return r;
  r = lqgrid_factor(&c);
  if (r != LQGRID_OK) return r;
  return pcg_solve_impl(&c, x0, nullptr, opts, nullptr, delta, x, u, info, false);
}

void lqgrid_destroy(lqgrid_ctx* c) { delete c; }

const char* lqgrid_last_error(void) { return g_last_error; }

}  // extern "C"
