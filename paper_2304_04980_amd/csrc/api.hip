// Host side of the lqgrid C ABI: argument checks, workspace layout, and the
// driver of Algorithm 1 (PCGM) with the Algorithm 2 preconditioner.  All
// device work is enqueued on the caller's stream; PCG scalars stay on the
// device and the host reads the convergence flag every `check_every`
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "../../include/lqgrid.h"
#include "launch.h"

using namespace lqg;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum Vec { kRd, kDl, kR, kD, kY, kBufA, kBufB, kBufC, kBufD, kNumVec };

struct Plan {
  size_t G13, Cdn, Cup, AT5, Qi, QTi, QTd, Qm, RiBT, Fw, Bw;
  size_t vec[kNumVec];
  size_t psum, pmax, scal;
  int npartial;
  size_t total;
};

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

Plan make_plan(const Dims& D) {
  Plan P{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t nn = (size_t)D.n * D.n, nodes = D.nodes, NB = 2 * D.n;
  P.scal = take(sizeof(Scalars));
  P.G13 = take(nodes * 13 * nn * 8);
  P.Cdn = take(nodes * 5 * nn * 8);
  P.Cup = take(nodes * 5 * nn * 8);
  P.AT5 = take(nodes * 5 * nn * 8);
  P.Qi = take(nodes * nn * 8);
  P.QTi = take(nodes * nn * 8);
  P.QTd = take(nodes * nn * 8);
  P.Qm = take(nodes * nn * 8);
  P.RiBT = take(nodes * (size_t)D.m * D.n * 8);
  P.Fw = take((size_t)2 * D.V * (D.K + 1) * NB * kFwRow * 8);
  P.Bw = take((size_t)2 * D.V * D.K * NB * kBwRow * 8);
  const int apply_blocks = ((D.real_nodes + 3) / 4) * ((D.Tt + 63) / 64);
  P.npartial = std::max(apply_blocks, kFlatBlocks);
  P.psum = take((size_t)P.npartial * 8);
  P.pmax = take((size_t)P.npartial * 8);
  for (int v = 0; v < kNumVec; ++v) P.vec[v] = take((size_t)D.vlen * 8);
  P.total = off;
  return P;
}

}  // namespace

struct lqgrid_ctx {
  Dims D;
  Plan P;
  Coef C;
  hipStream_t stream;
  char* ws;
  Scalars* sc;
  double* vec[kNumVec];
  double *psum, *pmax;
  bool factored = false;
  bool qt_distinct = false;
  // profiling
  bool prof = false;
  long long prof_launches[4] = {0, 0, 0, 0};
  double prof_ms[4] = {0, 0, 0, 0};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  std::vector<int> prof_kind;
  int prof_used = 0;
  ~lqgrid_ctx() {
    for (auto& e : prof_ev) {
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
  }
};

namespace {

thread_local char g_last_error[256] = "";

int hip_fail(hipError_t e, const char* where) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where,
                hipGetErrorString(e), (int)e);
  return LQGRID_EHIP;
}

// Drop an error left behind by earlier, unrelated runtime calls of the
// process (e.g. a not-ready status of a query) so that the checks below see
// only this library's launches.
inline void clear_stale_error() { (void)hipGetLastError(); }

#define HIPCHECK(x)                                          \
  do {                                                       \
    hipError_t e_ = (x);                                     \
    if (e_ != hipSuccess) return hip_fail(e_, #x);           \
  } while (0)

// Optional event timing around one launch (profiling mode only).  Events are
// recorded without synchronising; lqgrid_profile_read resolves them.
struct ProfScope {
  lqgrid_ctx* c;
  int k;
  int slot = -1;
  ProfScope(lqgrid_ctx* c_, int k_) : c(c_), k(k_) {
    if (!c->prof) return;
    if (c->prof_used >= (int)c->prof_ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return;
      c->prof_ev.push_back({a, b});
      c->prof_kind.push_back(0);
    }
    slot = c->prof_used++;
    c->prof_kind[slot] = k;
    hipEventRecord(c->prof_ev[slot].first, c->stream);
  }
  ~ProfScope() {
    if (slot >= 0) hipEventRecord(c->prof_ev[slot].second, c->stream);
  }
};

// Fold recorded event pairs into the per-kernel totals (after a sync).
void prof_resolve(lqgrid_ctx* c) {
  for (int e = 0; e < c->prof_used; ++e) {
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
         (o.precision == LQGRID_FP64 || o.precision == LQGRID_FP32_REFINE);
}

// q = P_S^-1 r by S outer x L inner NBJM sweeps (Alg. 2 with a fixed number
// of sweeps, Theorem 2).  Returns the buffer holding the result (one of the
// two theta buffers).
double* precondition(lqgrid_ctx* c, const double* r, int S, int L, int check) {
  const Dims& D = c->D;
  double* rho = c->vec[kBufA];
  double* tau = c->vec[kBufB];
  double* thx = c->vec[kBufC];
  double* thy = c->vec[kBufD];
  double* dprev = nullptr;  // delta^(s) of Alg. 2 (zero for s = 0)
  for (int s = 0; s < S; ++s) {
    const double* rs = r;
    if (s > 0) {  // r_theta^(s) = r + Xi~ delta^(s)
      ProfScope ps(c, 2);
      xi_rhs(D, c->C, r, dprev, rho, c->sc, check, c->stream);
      rs = rho;
    }
    double* th = (dprev == thx) ? thy : thx;
    for (int l = 0; l < L; ++l) {
      const double* rhs = rs;
      if (l > 0) {  // tau = r_theta + Omega~ theta^(l)
        ProfScope ps(c, 2);
        omega_rhs(D, c->C, rs, th, tau, c->sc, check, c->stream);
        rhs = tau;
      }
      ProfScope ps(c, 1);
      phi_solve(D, c->C, rhs, th, c->sc, check, c->qt_distinct ? 1 : 0,
                c->stream);
    }
    dprev = th;
  }
  return dprev;
}

// r = r_delta - Delta dl (into r), true residual norms into sc.
void true_residual(lqgrid_ctx* c, const double* dl, double* r) {
  const Dims& D = c->D;
  double* y = c->vec[kY];
  delta_apply(D, c->C, dl, y, nullptr, c->sc, 0, c->stream);
  const int np = vec_sub_norm(D, c->vec[kRd], y, r, c->psum, c->pmax, c->stream);
  scalar_step(kModeTrue, c->psum, c->pmax, np, c->sc, 0.0, c->stream);
}

int read_scalars(lqgrid_ctx* c, Scalars* h) {
  HIPCHECK(hipMemcpyAsync(h, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost,
                          c->stream));
  HIPCHECK(hipStreamSynchronize(c->stream));
  if (c->prof_used) prof_resolve(c);
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
  (void)opts;
  Dims D;
  if (!make_dims(desc, &D)) return 0;
  return make_plan(D).total;
}

int lqgrid_setup(const lqgrid_problem_desc* desc, void* workspace,
                 size_t workspace_bytes, void* hip_stream, lqgrid_ctx** out) {
  if (!out) return LQGRID_EINVAL;
  *out = nullptr;
  Dims D;
  if (!make_dims(desc, &D)) return LQGRID_EINVAL;
  if (!desc->A || !desc->A_nbr || !desc->B || !desc->Q || !desc->R)
    return LQGRID_EINVAL;
  if (D.n > kMaxN || D.m > kMaxM) return LQGRID_EUNSUPPORTED;
  // the block solves address each vector with 32-bit byte offsets
  if (D.vlen * 8 >= (1LL << 31)) return LQGRID_EUNSUPPORTED;
  const Plan P = make_plan(D);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 ||
      workspace_bytes < P.total)
    return LQGRID_EWORKSPACE;
  lqgrid_ctx* c = new (std::nothrow) lqgrid_ctx();
  if (!c) return LQGRID_EHIP;
  c->D = D;
  c->P = P;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  char* w = c->ws;
  c->sc = reinterpret_cast<Scalars*>(w + P.scal);
  c->C.G13 = reinterpret_cast<double*>(w + P.G13);
  c->C.Cdn = reinterpret_cast<double*>(w + P.Cdn);
  c->C.Cup = reinterpret_cast<double*>(w + P.Cup);
  c->C.AT5 = reinterpret_cast<double*>(w + P.AT5);
  c->C.Qi = reinterpret_cast<double*>(w + P.Qi);
  c->C.QTi = reinterpret_cast<double*>(w + P.QTi);
  c->C.QTd = reinterpret_cast<double*>(w + P.QTd);
  c->C.Qm = reinterpret_cast<double*>(w + P.Qm);
  c->C.RiBT = reinterpret_cast<double*>(w + P.RiBT);
  c->C.Fw = reinterpret_cast<double*>(w + P.Fw);
  c->C.Bw = reinterpret_cast<double*>(w + P.Bw);
  for (int v = 0; v < kNumVec; ++v)
    c->vec[v] = reinterpret_cast<double*>(w + P.vec[v]);
  c->psum = reinterpret_cast<double*>(w + P.psum);
  c->pmax = reinterpret_cast<double*>(w + P.pmax);
  clear_stale_error();
  // zero scalars and every vector (padding entries must stay zero)
  vec_zero(reinterpret_cast<double*>(w + P.scal), sizeof(Scalars) / 8, c->stream);
  for (int v = 0; v < kNumVec; ++v) vec_zero(c->vec[v], D.vlen, c->stream);
  ProblemIn in{D.K, D.N, D.n, D.m, desc->A, desc->A_nbr, desc->B,
               desc->Q, desc->R, desc->QT};
  launch_setup(D, in, c->C, c->sc, c->stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "lqgrid_setup launch");
  }
  *out = c;
  return LQGRID_OK;
}

int lqgrid_factor(lqgrid_ctx* c) {
  if (!c) return LQGRID_EINVAL;
  clear_stale_error();
  // entries never written by the factorisation (padding, N1/N2 of the last
  // block rows) must read as zero
  vec_zero(c->C.Fw, (long long)2 * c->D.V * (c->D.K + 1) * 2 * c->D.n * kFwRow, c->stream);
  vec_zero(c->C.Bw, (long long)2 * c->D.V * c->D.K * 2 * c->D.n * kBwRow, c->stream);
  launch_factor(c->D, c->C, c->sc, c->stream);
  HIPCHECK(hipGetLastError());
  Scalars h;
  int st = read_scalars(c, &h);
  if (st != LQGRID_OK) return st;
  c->qt_distinct = h.qt_differs != 0;
  if (h.flag_notspd) return LQGRID_ENOTSPD;
  c->factored = true;
  return LQGRID_OK;
}

int lqgrid_pcg_solve(lqgrid_ctx* c, const double* x0,
                     const lqgrid_solve_opts* opts_in, const double* delta_init,
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
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  HIPCHECK(hipEventRecord(e0, s));

  double* rd = c->vec[kRd];
  double* dl = c->vec[kDl];
  double* r = c->vec[kR];
  double* d = c->vec[kD];
  double* y = c->vec[kY];
  Scalars* sc = c->sc;

  // r_delta, ||r_delta||^2, tol^2 ||r_delta||^2
  launch_rhs_init(D, x0, rd, s);
  int np = vec_norms(D, rd, c->psum, c->pmax, s);
  scalar_step(kModeRd2, c->psum, c->pmax, np, sc, o.tol, s);
  // delta^(0) and r^(0) = r_delta - Delta delta^(0)
  if (delta_init) {
    to_internal(D, delta_init, dl, s);
    true_residual(c, dl, r);
  } else {
    vec_zero(dl, D.vlen, s);
    vec_copy(D, rd, r, s);
  }
  Scalars h{};
  {
    // set iteration state
    Scalars init{};
    int st = read_scalars(c, &h);
    if (st != LQGRID_OK) return st;
    init = h;
    init.iter = 0;
    init.max_iter = o.max_iter;
    init.done = kRunning;
    HIPCHECK(hipMemcpyAsync(sc, &init, sizeof(Scalars), hipMemcpyHostToDevice, s));
    h = init;
  }
  int status = LQGRID_OK;
  int restarts = 0;
  bool need_init = true;
  double* q = nullptr;
  // a start that already meets the tolerance needs no iteration
  const bool start_converged = h.rr <= h.tol2;
  for (; !start_converged;) {
    if (need_init) {
      // d^(0) = P^-1 r^(0), mu^(0) = d'r
      q = precondition(c, r, o.outer_S, o.inner_L, 0);
      np = vec_dot(D, q, r, c->psum, sc, 0, s);
      scalar_step(kModeMuInit, c->psum, nullptr, np, sc, 0.0, s);
      vec_zero(d, D.vlen, s);
      need_init = false;
    }
    for (int k = 0; k < o.check_every; ++k) {
      vec_dir(D, q, d, sc, s);  // d = q + beta d (beta = 0 after init)
      {
        ProfScope ps(c, 0);
        np = delta_apply(D, c->C, d, y, c->psum, sc, 1, s);
      }
      scalar_step(kModeYd, c->psum, nullptr, np, sc, 0.0, s);
      {
        ProfScope ps(c, 3);
        np = vec_update(D, d, y, dl, r, c->psum, sc, s);
      }
      scalar_step(kModeRr, c->psum, nullptr, np, sc, 0.0, s);
      q = precondition(c, r, o.outer_S, o.inner_L, 1);
      np = vec_dot(D, q, r, c->psum, sc, 1, s);
      scalar_step(kModeMu, c->psum, nullptr, np, sc, 0.0, s);
    }
    HIPCHECK(hipGetLastError());
    int st = read_scalars(c, &h);
    if (st != LQGRID_OK) return st;
    if (h.done == kRunning) continue;
    if (h.done == kBreakdown) {
      status = LQGRID_EBREAKDOWN;
      break;
    }
    // converged by the recurrence, or out of iterations: check the true residual
    true_residual(c, dl, r);
    st = read_scalars(c, &h);
    if (st != LQGRID_OK) return st;
    if (h.rr <= h.tol2) break;
    if (h.iter >= o.max_iter) {
      status = LQGRID_ENOCONV;
      break;
    }
    // restart from the true residual
    ++restarts;
    Scalars fix = h;
    fix.done = kRunning;
    HIPCHECK(hipMemcpyAsync(sc, &fix, sizeof(Scalars), hipMemcpyHostToDevice, s));
    need_init = true;
  }
  // final true residual (already in h when converged; recompute otherwise)
  if (status != LQGRID_OK) {
    true_residual(c, dl, r);
    read_scalars(c, &h);
  }
  to_abi(D, dl, delta, s);
  if (x || u) recover(D, c->C, dl, x, u, s);
  HIPCHECK(hipEventRecord(e1, s));
  HIPCHECK(hipEventSynchronize(e1));
  if (c->prof_used) prof_resolve(c);
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIPCHECK(hipGetLastError());
  if (info) {
    info->status = status;
    info->iterations = h.iter;
    info->refinements = 0;
    info->restarts = restarts;
    info->rel_kkt_residual = h.rd2 > 0 ? std::sqrt(h.rr / h.rd2) : 0.0;
    info->seconds = ms * 1e-3;
    // ||r_delta||_inf = max |x0| (r_delta = col(-gamma, 0, ...))
    info->rel_res_inf = h.rdinf > 0 ? h.rinf / h.rdinf : 0.0;
  }
  return status;
}

size_t lqgrid_batch_workspace_bytes(int P, const lqgrid_problem_desc* descs,
                                    const lqgrid_solve_opts* opts) {
  if (P < 1 || !descs) return 0;
  size_t tot = 0;
  for (int p = 0; p < P; ++p) {
    const size_t b = lqgrid_workspace_bytes(&descs[p], opts);
    if (!b) return 0;
    tot += align_up(b);
  }
  return tot;
}

int lqgrid_batch_solve(int P, const lqgrid_problem_desc* descs,
                       const double* const* x0s, const lqgrid_solve_opts* opts,
                       double* const* deltas, void* workspace,
                       size_t workspace_bytes, void* hip_stream,
                       lqgrid_info* infos) {
  if (P < 1 || !descs || !x0s || !deltas) return LQGRID_EINVAL;
  if (workspace_bytes < lqgrid_batch_workspace_bytes(P, descs, opts))
    return LQGRID_EWORKSPACE;
  char* w = static_cast<char*>(workspace);
  int worst = LQGRID_OK;
  for (int p = 0; p < P; ++p) {
    const size_t b = align_up(lqgrid_workspace_bytes(&descs[p], opts));
    lqgrid_ctx* c = nullptr;
    int st = lqgrid_setup(&descs[p], w, b, hip_stream, &c);
    if (st == LQGRID_OK) st = lqgrid_factor(c);
    lqgrid_info inf{};
    if (st == LQGRID_OK)
      st = lqgrid_pcg_solve(c, x0s[p], opts, nullptr, deltas[p], nullptr,
                            nullptr, &inf);
    inf.status = st;
    if (infos) infos[p] = inf;
    if (st != LQGRID_OK) worst = st;
    lqgrid_destroy(c);
    w += b;
  }
  return worst;
}

int lqgrid_apply_operator(lqgrid_ctx* c, int op, int S, int L,
                          const double* in, double* out) {
  if (!c || !in || !out) return LQGRID_EINVAL;
  const Dims& D = c->D;
  hipStream_t s = c->stream;
  clear_stale_error();
  double* vin = c->vec[kD];
  double* vout = c->vec[kY];
  to_internal(D, in, vin, s);
  switch (op) {
    case LQGRID_OP_DELTA:
      delta_apply(D, c->C, vin, vout, nullptr, c->sc, 0, s);
      break;
    case LQGRID_OP_XI:
      xi_rhs(D, c->C, nullptr, vin, vout, c->sc, 0, s);
      break;
    case LQGRID_OP_OMEGA:
      omega_rhs(D, c->C, nullptr, vin, vout, c->sc, 0, s);
      break;
    case LQGRID_OP_PHI_SOLVE:
      if (!c->factored) return LQGRID_EINVAL;
      phi_solve(D, c->C, vin, vout, c->sc, 0, c->qt_distinct ? 1 : 0, s);
      break;
    case LQGRID_OP_PRECOND: {
      if (!c->factored || S < 1 || L < 1) return LQGRID_EINVAL;
      vout = precondition(c, vin, S, L, 0);
      break;
    }
    default:
      return LQGRID_EINVAL;
  }
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
  c->prof = enable != 0;
  for (int k = 0; k < 4; ++k) {
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

void lqgrid_destroy(lqgrid_ctx* c) { delete c; }

const char* lqgrid_last_error(void) { return g_last_error; }

}  // extern "C"
