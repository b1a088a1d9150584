// Host driver of the batched form (lqgrid_batch_solve): many independent
// problems with uneven K, N, T (uniform n) solved together by Algorithm 1
// with the Algorithm 2 preconditioner, in FP64, each to its own relative
// tolerance confirmed on its true residual.
//
// Structure.  The workspace holds, per problem, the FP64 operator blocks and
// factors of the single-problem path, and, per vector role, one region
// with every problem's vector back to back.  Work lists of (problem, tile)
// items cover the node tiles, the block-solve tiles and element ranges of
// the vectors; a persistent grid walks each list.  One PCG iteration of all
// problems is the same launch sequence as for one problem, with per-problem
// scalars and convergence flags.  A block of `check_every` iterations plus
// the compaction of the live item lists is captured once in a HIP graph and
// replayed until no problem is running.  The outer loop (true FP64 residual,
// restart of the problems that miss the tolerance) runs around it.
//
// Autotuning.  The persistent grid of each kernel family and the order of
// the node tiles (node-major, or time-major = consecutive time chunks of the
// same nodes in one workgroup) are chosen by timing the candidate settings on
// the batch itself, after factorisation, on pure operator applications whose
// outputs are scratch.  The choice is cached per set of problem sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "api_common.h"

using namespace lqg;

namespace {

constexpr int kFlatSeg = 8192;  // vector elements per flat work item
constexpr int kUnitPrepSize = 128, kUnitStencilSize = 128, kUnitRhsSize = 256;
constexpr int kUnitAbiSize = 65536;

struct Tuned {
  int node_order = 0;  // 0: node groups fastest, 1: time chunks fastest
  int g_node = 2048, g_solve = 1024, g_flat = 2048;
};

std::mutex g_tune_mu;
std::map<uint64_t, Tuned> g_tune_cache;

// Workspace layout of a batch.
struct Layout {
  size_t probs, sc, sco, nlive, live_flag, live_off, host_in;
  size_t orig[kNumItemKinds], live[kNumItemKinds], units[kNumUnitKinds];
  size_t psum_node, psum_flat, pmax_flat;
  std::vector<size_t> coef;             // per problem: start of its blocks
  std::vector<size_t> vec[kNumBatchVec];  // per role, per problem
  int nitems[kNumItemKinds];
  int nunits[kNumUnitKinds];
  size_t total;
};

size_t coef_bytes(const Dims& D) {
  const size_t nn = (size_t)D.n * D.n, nodes = D.nodes, NB = 2 * D.n;
  size_t b = 0;
  b += align_up(nodes * 13 * nn * 8);           // G13
  b += 3 * align_up(nodes * 5 * nn * 8);        // Cdn, Cup, AT5
  b += 4 * align_up(nodes * nn * 8);            // Qi, QTi, QTd, Qm
  b += align_up(nodes * (size_t)D.m * D.n * 8); // RiBT
  b += align_up((size_t)2 * D.V * fw_rows(D.K) * NB * kFwRow * 8);
  b += align_up((size_t)2 * D.V * D.K * NB * kBwRow * 8);
  b += align_up((size_t)2 * D.V * NB * kFwRow * 8);  // Xw
  return b;
}

Coef coef_at(char* base, const Dims& D) {
  const size_t nn = (size_t)D.n * D.n, nodes = D.nodes, NB = 2 * D.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    double* p = reinterpret_cast<double*>(base + off);
    off += align_up(bytes);
    return p;
  };
  Coef C{};
  C.G13 = take(nodes * 13 * nn * 8);
  C.Cdn = take(nodes * 5 * nn * 8);
  C.Cup = take(nodes * 5 * nn * 8);
  C.AT5 = take(nodes * 5 * nn * 8);
  C.Qi = take(nodes * nn * 8);
  C.QTi = take(nodes * nn * 8);
  C.QTd = take(nodes * nn * 8);
  C.Qm = take(nodes * nn * 8);
  C.RiBT = take(nodes * (size_t)D.m * D.n * 8);
  C.Fw = take((size_t)2 * D.V * fw_rows(D.K) * NB * kFwRow * 8);
  C.Bw = take((size_t)2 * D.V * D.K * NB * kBwRow * 8);
  C.Xw = take((size_t)2 * D.V * NB * kFwRow * 8);
  return C;
}

int node_items(const Dims& D) {
  return ((D.real_nodes + 3) / 4) * ((D.Tt + kWave - 1) / kWave);
}
int solve_items(const Dims& D) { return D.V * ((D.Tt + kWave - 1) / kWave); }
int flat_items(const Dims& D) { return (int)((D.vlen + kFlatSeg - 1) / kFlatSeg); }

Layout make_layout(const std::vector<Dims>& Ds) {
  Layout L{};
  const int P = (int)Ds.size();
  for (int k = 0; k < kNumItemKinds; ++k) L.nitems[k] = 0;
  for (int k = 0; k < kNumUnitKinds; ++k) L.nunits[k] = 0;
  for (const Dims& D : Ds) {
    L.nitems[kItemNode] += node_items(D);
    L.nitems[kItemSolve] += solve_items(D);
    L.nitems[kItemFlat] += flat_items(D);
    L.nunits[kUnitPrep] += (D.nodes + kUnitPrepSize - 1) / kUnitPrepSize;
    L.nunits[kUnitStencil] += (D.nodes * 18 + kUnitStencilSize - 1) / kUnitStencilSize;
    L.nunits[kUnitRhs] += (D.real_nodes * D.n + kUnitRhsSize - 1) / kUnitRhsSize;
    L.nunits[kUnitFactor] += 2 * D.V;
    L.nunits[kUnitAbi] +=
        (int)(((long long)D.real_nodes * D.n * D.Tt + kUnitAbiSize - 1) / kUnitAbiSize);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.probs = take(P * sizeof(BatchProb));
  L.sc = take(P * sizeof(Scalars));
  L.sco = take(P * sizeof(Scalars));
  L.nlive = take((kNumItemKinds + 1) * sizeof(int));
  L.live_flag = take(P * sizeof(int));
  L.live_off = take((size_t)kNumItemKinds * P * sizeof(int));
  L.host_in = take(2 * (size_t)P * sizeof(int));
  for (int k = 0; k < kNumItemKinds; ++k) L.orig[k] = take(L.nitems[k] * sizeof(Item));
  for (int k = 0; k < kNumItemKinds; ++k) L.live[k] = take(L.nitems[k] * sizeof(Item));
  for (int k = 0; k < kNumUnitKinds; ++k) L.units[k] = take(L.nunits[k] * sizeof(Item));
  L.psum_node = take(L.nitems[kItemNode] * sizeof(double));
  L.psum_flat = take(L.nitems[kItemFlat] * sizeof(double));
  L.pmax_flat = take(L.nitems[kItemFlat] * sizeof(double));
  L.coef.resize(P);
  for (int p = 0; p < P; ++p) L.coef[p] = take(coef_bytes(Ds[p]));
  for (int r = 0; r < kNumBatchVec; ++r) {
    L.vec[r].resize(P);
    for (int p = 0; p < P; ++p) L.vec[r][p] = take((size_t)Ds[p].vlen * 8);
  }
  L.total = off;
  return L;
}

// Host copies of the work lists.
struct Lists {
  std::vector<Item> items[kNumItemKinds];
  std::vector<Item> units[kNumUnitKinds];
  std::vector<int> first[kNumItemKinds], count[kNumItemKinds];
};

void build_node_items(const std::vector<Dims>& Ds, int order, Lists* Ls) {
  auto& v = Ls->items[kItemNode];
  v.clear();
  for (int p = 0; p < (int)Ds.size(); ++p) {
    const Dims& D = Ds[p];
    const int ng = (D.real_nodes + 3) / 4, nc = (D.Tt + kWave - 1) / kWave;
    Ls->first[kItemNode][p] = (int)v.size();
    Ls->count[kItemNode][p] = ng * nc;
    if (order == 0) {
      for (int c = 0; c < nc; ++c)
        for (int g = 0; g < ng; ++g) v.push_back({p, g, c, (int)v.size()});
    } else {
      for (int g = 0; g < ng; ++g)
        for (int c = 0; c < nc; ++c) v.push_back({p, g, c, (int)v.size()});
    }
  }
}

Lists build_lists(const std::vector<Dims>& Ds, int order) {
  Lists Ls;
  const int P = (int)Ds.size();
  for (int k = 0; k < kNumItemKinds; ++k) {
    Ls.first[k].assign(P, 0);
    Ls.count[k].assign(P, 0);
  }
  build_node_items(Ds, order, &Ls);
  for (int p = 0; p < P; ++p) {
    const Dims& D = Ds[p];
    const int nc = (D.Tt + kWave - 1) / kWave;
    auto& s = Ls.items[kItemSolve];
    Ls.first[kItemSolve][p] = (int)s.size();
    Ls.count[kItemSolve][p] = D.V * nc;
    for (int v = 0; v < D.V; ++v)
      for (int c = 0; c < nc; ++c) s.push_back({p, v, c, (int)s.size()});
    auto& f = Ls.items[kItemFlat];
    Ls.first[kItemFlat][p] = (int)f.size();
    Ls.count[kItemFlat][p] = flat_items(D);
    for (long long e = 0; e < D.vlen; e += kFlatSeg)
      f.push_back({p, (int)e, (int)std::min<long long>(e + kFlatSeg, D.vlen),
                   (int)f.size()});
    auto ranges = [&](int kind, long long n, int size) {
      for (long long e = 0; e < n; e += size)
        Ls.units[kind].push_back({p, (int)e, (int)std::min<long long>(e + size, n), 0});
    };
    ranges(kUnitPrep, D.nodes, kUnitPrepSize);
    ranges(kUnitStencil, (long long)D.nodes * 18, kUnitStencilSize);
    ranges(kUnitRhs, (long long)D.real_nodes * D.n, kUnitRhsSize);
    for (int v = 0; v < D.V; ++v)
      for (int cls = 0; cls < 2; ++cls) Ls.units[kUnitFactor].push_back({p, v, cls, 0});
    ranges(kUnitAbi, (long long)D.real_nodes * D.n * D.Tt, kUnitAbiSize);
  }
  return Ls;
}

uint64_t dims_key(const std::vector<Dims>& Ds) {
  uint64_t h = 1469598103934665603ULL;  // FNV-1a over the sizes
  auto mix = [&](int x) {
    h ^= (uint64_t)(uint32_t)x;
    h *= 1099511628211ULL;
  };
  mix((int)Ds.size());
  for (const Dims& D : Ds) {
    mix(D.K);
    mix(D.N);
    mix(D.T);
    mix(D.n);
    mix(D.m);
  }
  return h;
}

struct Batch {
  BatchDev B;
  int n = 0;
  int S = 2, L = 2;
  Tuned tp;
  hipStream_t s = nullptr;
};

// q = P_S^-1 r for every live problem (Alg. 2, S x L sweeps); returns the
// role holding q.  Roles: rho = A, tau = B, theta = C / E alternately.
int b_precondition(Batch& b, int r, int check) {
  const BatchDev& B = b.B;
  int dprev = -1;
  for (int s = 0; s < b.S; ++s) {
    int rs = r;
    if (s > 0) {  // r_theta^(s) = r + Xi~ delta^(s)
      batch_xi(B, b.n, r, dprev, kBA, check, b.tp.g_node, b.s);
      rs = kBA;
    }
    const int th = (dprev == kBC) ? kBE : kBC;
    for (int l = 0; l < b.L; ++l) {
      int rhs = rs;
      if (l > 0) {  // tau = r_theta + Omega~ theta^(l)
        batch_omega(B, b.n, rs, th, kBB, check, b.tp.g_node, b.s);
        rhs = kBB;
      }
      batch_solve(B, b.n, rhs, th, check, b.tp.g_solve, b.s);
    }
    dprev = th;
  }
  return dprev;
}

// One PCG iteration of every running problem (Algorithm 1).
void b_iteration(Batch& b, int q) {
  const BatchDev& B = b.B;
  batch_flat(B, kFlatDir, q, kBD, -1, -1, 1, b.tp.g_flat, b.s);  // d = q + beta d
  batch_delta(B, b.n, kBD, kBY, 1, 1, b.tp.g_node, b.s);          // y = Delta d
  batch_scalar(B, kModeYd, kItemNode, 0, 0.0, b.s);
  batch_flat(B, kFlatUpdate, kBD, kBY, kBX, kBR, 1, b.tp.g_flat, b.s);
  batch_scalar(B, kModeRr, kItemFlat, 0, 0.0, b.s);
  const int q2 = b_precondition(b, kBR, 1);
  batch_flat(B, kFlatDot, q2, kBR, -1, -1, 1, b.tp.g_flat, b.s);
  batch_scalar(B, kModeMu, kItemFlat, 0, 0.0, b.s);
}

int upload_active(Batch& b, const std::vector<int>& act, const std::vector<int>& maxit,
                  std::vector<int>* staging) {
  const int P = b.B.P;
  staging->assign(2 * P, 0);
  for (int p = 0; p < P; ++p) {
    (*staging)[p] = act[p];
    (*staging)[P + p] = maxit[p];
  }
  HIPCHECK(hipMemcpyAsync(b.B.host_in, staging->data(), 2 * P * sizeof(int),
                          hipMemcpyHostToDevice, b.s));
  HIPCHECK(hipStreamSynchronize(b.s));  // staging is reused by the caller
  batch_set_active(b.B, b.s);
  return LQGRID_OK;
}

int read_all(Batch& b, Scalars* dev, std::vector<Scalars>* h) {
  h->resize(b.B.P);
  HIPCHECK(hipMemcpyAsync(h->data(), dev, b.B.P * sizeof(Scalars),
                          hipMemcpyDeviceToHost, b.s));
  HIPCHECK(hipStreamSynchronize(b.s));
  return LQGRID_OK;
}

int upload_items(Batch& b, const Layout& Lay, char* w, const Lists& Ls, int kind) {
  const auto& v = Ls.items[kind];
  if (!v.empty())
    HIPCHECK(hipMemcpyAsync(w + Lay.orig[kind], v.data(), v.size() * sizeof(Item),
                            hipMemcpyHostToDevice, b.s));
  return LQGRID_OK;
}

// Average milliseconds of `reps` back-to-back runs of f on the stream.
template <typename F>
float time_ms(hipStream_t s, int reps, F f) {
  hipEvent_t a, z;
  if (hipEventCreate(&a) != hipSuccess) return 1e30f;
  if (hipEventCreate(&z) != hipSuccess) {
    (void)hipEventDestroy(a);
    return 1e30f;
  }
  f();  // warm
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r) f();
  (void)hipEventRecord(z, s);
  float ms = 1e30f;
  if (hipEventSynchronize(z) == hipSuccess) (void)hipEventElapsedTime(&ms, a, z);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  return ms / reps;
}

// LQGRID_BATCH_NODE_ORDER = 0 or 1 fixes the node-tile order (tests run both
// the per-chunk and the all-chunks stencil paths); -1 when unset.
int forced_node_order() {
  const char* e = std::getenv("LQGRID_BATCH_NODE_ORDER");
  if (!e) return -1;
  if (e[0] == '0' && e[1] == 0) return 0;
  if (e[0] == '1' && e[1] == 0) return 1;
  return -1;
}

// Autotune the persistent grids and the node-tile order on pure operator
// applications (inputs: r_delta; outputs: scratch roles).  Leaves the node
// list in the chosen order and every item live.
int autotune(Batch& b, const Layout& Lay, char* w, const std::vector<Dims>& Ds,
             Lists* Ls) {
  const BatchDev& B = b.B;
  const int reps = 3;
  Tuned best = b.tp;
  float best_node = 1e30f;
  const int forced = forced_node_order();
  for (int order = 0; order < 2; ++order) {
    if (forced >= 0 && order != forced) continue;
    build_node_items(Ds, order, Ls);
    int st = upload_items(b, Lay, w, *Ls, kItemNode);
    if (st != LQGRID_OK) return st;
    batch_compact(B, 0, b.s);
    b.B.node_rows = order == 1;
    for (int g : {1024, 2048, 4096, 8192}) {
      const float ms = time_ms(b.s, reps, [&] {
        batch_delta(B, b.n, kBRd, kBYt, 1, 0, g, b.s);
        batch_xi(B, b.n, -1, kBRd, kBA, 0, g, b.s);
      });
      if (ms < best_node) {
        best_node = ms;
        best.node_order = order;
        best.g_node = g;
      }
    }
  }
  float best_solve = 1e30f;
  for (int g : {512, 1024, 2048, 4096}) {
    const float ms = time_ms(b.s, reps, [&] { batch_solve(B, b.n, kBRd, kBA, 0, g, b.s); });
    if (ms < best_solve) {
      best_solve = ms;
      best.g_solve = g;
    }
  }
  float best_flat = 1e30f;
  for (int g : {1024, 2048, 4096, 8192}) {
    const float ms = time_ms(b.s, reps, [&] {
      batch_flat(B, kFlatDot, kBRd, kBYt, -1, -1, 0, g, b.s);
    });
    if (ms < best_flat) {
      best_flat = ms;
      best.g_flat = g;
    }
  }
  b.tp = best;
  b.B.node_rows = best.node_order == 1;
  build_node_items(Ds, best.node_order, Ls);
  const int st = upload_items(b, Lay, w, *Ls, kItemNode);
  if (st != LQGRID_OK) return st;
  batch_compact(B, 0, b.s);
  HIPCHECK(hipGetLastError());
  return LQGRID_OK;
}

bool batch_dims(int P, const lqgrid_problem_desc* descs, std::vector<Dims>* Ds) {
  if (P < 1 || !descs) return false;
  Ds->resize(P);
  for (int p = 0; p < P; ++p)
    if (!make_dims(&descs[p], &(*Ds)[p])) return false;
  return true;
}

struct StreamGuard {  // the batch's own stream, ordered after the caller's
  hipStream_t caller, own = nullptr;
  hipEvent_t ev = nullptr;
  ~StreamGuard() {
    if (own) {
      if (ev && hipEventRecord(ev, own) == hipSuccess)
        (void)hipStreamWaitEvent(caller, ev, 0);
      (void)hipStreamSynchronize(own);
      (void)hipStreamDestroy(own);
    }
    if (ev) (void)hipEventDestroy(ev);
  }
};

struct GraphGuard {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  ~GraphGuard() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
  }
};

}  // namespace

extern "C" {

size_t lqgrid_batch_workspace_bytes(int P, const lqgrid_problem_desc* descs,
                                    const lqgrid_solve_opts* opts) {
  (void)opts;
  std::vector<Dims> Ds;
  if (!batch_dims(P, descs, &Ds)) return 0;
  return make_layout(Ds).total;
}

int lqgrid_batch_solve(int P, const lqgrid_problem_desc* descs,
                       const double* const* x0s, const lqgrid_solve_opts* opts_in,
                       double* const* deltas, void* workspace,
                       size_t workspace_bytes, void* hip_stream,
                       lqgrid_info* infos) {
  if (infos && P > 0) std::memset(infos, 0, sizeof(lqgrid_info) * P);
  std::vector<Dims> Ds;
  if (!batch_dims(P, descs, &Ds) || !x0s || !deltas) return LQGRID_EINVAL;
  lqgrid_solve_opts o;
  opts_fill(opts_in, &o);
  if (!opts_valid(o)) return LQGRID_EINVAL;
  if (o.precision != LQGRID_FP64) return LQGRID_EUNSUPPORTED;
  if (o.preconditioner != LQGRID_PRECOND_NBJM) return LQGRID_EUNSUPPORTED;
  for (int p = 0; p < P; ++p) {
    const lqgrid_problem_desc& d = descs[p];
    if (!d.A || !d.A_nbr || !d.B || !d.Q || !d.R || !x0s[p] || !deltas[p])
      return LQGRID_EINVAL;
    if (d.n_node || d.m_node || d.time_varying)  // uniform, time-invariant only
      return LQGRID_EUNSUPPORTED;
    if (Ds[p].n != Ds[0].n) return LQGRID_EUNSUPPORTED;
    if (Ds[p].n > kMaxN || Ds[p].m > kMaxM) return LQGRID_EUNSUPPORTED;
    if (Ds[p].vlen * 8 >= (1LL << 31)) return LQGRID_EUNSUPPORTED;
  }
  const Layout Lay = make_layout(Ds);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0 ||
      workspace_bytes < Lay.total)
    return LQGRID_EWORKSPACE;
  clear_stale_error();
  char* w = static_cast<char*>(workspace);

  StreamGuard sg;
  sg.caller = reinterpret_cast<hipStream_t>(hip_stream);
  HIPCHECK(hipStreamCreateWithFlags(&sg.own, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(sg.ev, sg.caller));
  HIPCHECK(hipStreamWaitEvent(sg.own, sg.ev, 0));
  hipEvent_t t0, t1;
  HIPCHECK(hipEventCreate(&t0));
  HIPCHECK(hipEventCreate(&t1));
  HIPCHECK(hipEventRecord(t0, sg.own));

  Batch b;
  b.n = Ds[0].n;
  b.S = o.outer_S;
  b.L = o.inner_L;
  b.s = sg.own;
  const uint64_t key = dims_key(Ds) ^ ((uint64_t)(forced_node_order() + 2) << 60);
  bool tuned = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      b.tp = it->second;
      tuned = true;
    }
  }
  Lists Ls = build_lists(Ds, b.tp.node_order);

  BatchDev& B = b.B;
  B.P = P;
  B.probs = reinterpret_cast<BatchProb*>(w + Lay.probs);
  B.nlive = reinterpret_cast<int*>(w + Lay.nlive);
  B.live_flag = reinterpret_cast<int*>(w + Lay.live_flag);
  B.live_off = reinterpret_cast<int*>(w + Lay.live_off);
  B.host_in = reinterpret_cast<int*>(w + Lay.host_in);
  for (int k = 0; k < kNumItemKinds; ++k) {
    B.orig[k] = reinterpret_cast<Item*>(w + Lay.orig[k]);
    B.live[k] = reinterpret_cast<Item*>(w + Lay.live[k]);
    B.norig[k] = Lay.nitems[k];
  }
  for (int k = 0; k < kNumUnitKinds; ++k) {
    B.units[k] = reinterpret_cast<Item*>(w + Lay.units[k]);
    B.nunits[k] = Lay.nunits[k];
  }
  B.psum_node = reinterpret_cast<double*>(w + Lay.psum_node);
  B.node_rows = b.tp.node_order == 1;
  B.psum_flat = reinterpret_cast<double*>(w + Lay.psum_flat);
  B.pmax_flat = reinterpret_cast<double*>(w + Lay.pmax_flat);
  Scalars* sc = reinterpret_cast<Scalars*>(w + Lay.sc);
  Scalars* sco = reinterpret_cast<Scalars*>(w + Lay.sco);
  B.sc = sc;
  B.sco = sco;

  std::vector<BatchProb> hp(P);
  for (int p = 0; p < P; ++p) {
    BatchProb& q = hp[p];
    q.D = Ds[p];
    q.C = coef_at(w + Lay.coef[p], Ds[p]);
    const lqgrid_problem_desc& d = descs[p];
    q.in = ProblemIn{d.K, d.N, d.n, d.m, d.A, d.A_nbr, d.B, d.Q, d.R, d.QT};
    q.x0 = x0s[p];
    q.delta_out = deltas[p];
    for (int r = 0; r < kNumBatchVec; ++r)
      q.v[r] = reinterpret_cast<double*>(w + Lay.vec[r][p]);
    q.sc = sc + p;
    q.sco = sco + p;
    for (int k = 0; k < kNumItemKinds; ++k) {
      q.first[k] = Ls.first[k][p];
      q.count[k] = Ls.count[k][p];
    }
  }
  // zero everything the kernels read before writing (scalars, coefficient
  // padding, vector padding), then upload descriptors and work lists
  vec_zero<double>(reinterpret_cast<double*>(w + Lay.sc), (long long)(Lay.nlive - Lay.sc) / 8,
                   b.s);
  vec_zero<double>(reinterpret_cast<double*>(w + Lay.coef[0]),
                   (long long)(Lay.total - Lay.coef[0]) / 8, b.s);
  HIPCHECK(hipMemcpyAsync(B.probs, hp.data(), P * sizeof(BatchProb),
                          hipMemcpyHostToDevice, b.s));
  for (int k = 0; k < kNumItemKinds; ++k) {
    const int st = upload_items(b, Lay, w, Ls, k);
    if (st != LQGRID_OK) return st;
  }
  for (int k = 0; k < kNumUnitKinds; ++k)
    if (!Ls.units[k].empty())
      HIPCHECK(hipMemcpyAsync(B.units[k], Ls.units[k].data(),
                              Ls.units[k].size() * sizeof(Item),
                              hipMemcpyHostToDevice, b.s));

  // a1-a3: ingest, assembly, factorisation of every problem
  batch_setup(B, b.n, b.s);
  batch_factor(B, b.s);
  HIPCHECK(hipGetLastError());
  std::vector<Scalars> hs;
  int st = read_all(b, sc, &hs);  // also completes the uploads above
  if (st != LQGRID_OK) return st;

  std::vector<int> status(P, LQGRID_OK), total_it(P, 0), passes(P, 0);
  std::vector<int> open(P, 1), maxit(P, o.max_iter), staging;
  for (int p = 0; p < P; ++p)
    if (hs[p].flag_notspd) {
      status[p] = LQGRID_ENOTSPD;
      open[p] = 0;
    }

  // a4: r_delta and its norms (outer scalars)
  batch_rhs_init(B, b.s);
  st = upload_active(b, open, maxit, &staging);
  if (st != LQGRID_OK) return st;
  batch_compact(B, 0, b.s);
  batch_flat(B, kFlatNorms, kBRd, -1, -1, -1, 0, b.tp.g_flat, b.s);
  batch_scalar(B, kModeRd2, kItemFlat, 1, o.tol, b.s);

  if (!tuned) {
    st = autotune(b, Lay, w, Ds, &Ls);
    if (st != LQGRID_OK) return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = b.tp;
  }

  // The captured iteration block (q lives in the role the preconditioner
  // returns, the same for every iteration).
  GraphGuard gg;
  const int block = std::max(1, o.check_every);
  int q_role = -1;
  std::vector<Scalars> ho;
  // problems whose true residual is evaluated this round: every open one at
  // first, then those that just had a pass (including ones it closed)
  std::vector<int> eval = open;
  for (;;) {
    // true residual r = r_delta - Delta delta~
    st = upload_active(b, eval, maxit, &staging);
    if (st != LQGRID_OK) return st;
    batch_compact(B, 0, b.s);
    batch_delta(B, b.n, kBDl, kBYt, 0, 0, b.tp.g_node, b.s);
    batch_flat(B, kFlatSubNorm, kBRd, kBYt, kBRt, -1, 0, b.tp.g_flat, b.s);
    batch_scalar(B, kModeTrue, kItemFlat, 1, 0.0, b.s);
    HIPCHECK(hipGetLastError());
    st = read_all(b, sco, &ho);
    if (st != LQGRID_OK) return st;
    std::vector<int> need(P, 0);
    int nneed = 0;
    for (int p = 0; p < P; ++p) {
      if (!open[p]) continue;
      const Scalars& h = ho[p];
      if (h.rr <= h.tol2) {
        open[p] = 0;  // converged (also the zero right-hand side)
      } else if (!std::isfinite(h.rr)) {
        status[p] = LQGRID_EBREAKDOWN;
        open[p] = 0;
      } else if (total_it[p] >= o.max_iter || passes[p] >= kMaxPasses) {
        status[p] = LQGRID_ENOCONV;
        open[p] = 0;
      } else {
        need[p] = 1;
        maxit[p] = o.max_iter - total_it[p];
        ++nneed;
      }
    }
    if (nneed == 0) break;

    // one PCG pass on Delta e = r / ||r|| for the problems that need it
    st = upload_active(b, need, maxit, &staging);
    if (st != LQGRID_OK) return st;
    batch_compact(B, 0, b.s);
    batch_flat(B, kFlatScale, kBRt, kBR, -1, -1, 0, b.tp.g_flat, b.s);
    batch_flat(B, kFlatZero, kBX, -1, -1, -1, 0, b.tp.g_flat, b.s);
    batch_flat(B, kFlatNorms, kBR, -1, -1, -1, 0, b.tp.g_flat, b.s);
    batch_scalar(B, kModeRd2Rel, kItemFlat, 0, o.tol, b.s);
    const int q = b_precondition(b, kBR, 0);
    batch_flat(B, kFlatDot, q, kBR, -1, -1, 0, b.tp.g_flat, b.s);
    batch_scalar(B, kModeMuInit, kItemFlat, 0, 0.0, b.s);
    batch_flat(B, kFlatZero, kBD, -1, -1, -1, 0, b.tp.g_flat, b.s);
    batch_compact(B, 1, b.s);
    HIPCHECK(hipGetLastError());
    if (!gg.x) {
      q_role = q;
      HIPCHECK(hipStreamBeginCapture(b.s, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < block; ++k) b_iteration(b, q_role);
      batch_compact(B, 1, b.s);
      HIPCHECK(hipStreamEndCapture(b.s, &gg.g));
      HIPCHECK(hipGraphInstantiate(&gg.x, gg.g, nullptr, nullptr, 0));
    }
    const int max_replays = o.max_iter / block + 2;
    for (int rep = 0; rep < max_replays; ++rep) {
      int running = 0;
      HIPCHECK(hipGraphLaunch(gg.x, b.s));
      HIPCHECK(hipMemcpyAsync(&running, B.nlive + kNumItemKinds, sizeof(int),
                              hipMemcpyDeviceToHost, b.s));
      HIPCHECK(hipStreamSynchronize(b.s));
      if (running == 0) break;
    }
    st = read_all(b, sc, &hs);
    if (st != LQGRID_OK) return st;
    for (int p = 0; p < P; ++p) {
      if (!need[p]) continue;
      total_it[p] += hs[p].iter;
      passes[p] += 1;
      if (hs[p].done == kBreakdown && hs[p].iter <= 1) {
        status[p] = LQGRID_EBREAKDOWN;
        open[p] = 0;
      } else if (hs[p].done == kRunning) {
        status[p] = LQGRID_ENOCONV;  // replay cap reached
        open[p] = 0;
      }
    }
    // delta~ += ||r|| e for every problem of this pass
    st = upload_active(b, need, maxit, &staging);
    if (st != LQGRID_OK) return st;
    batch_compact(B, 0, b.s);
    batch_flat(B, kFlatAxpy, kBX, kBDl, -1, -1, 0, b.tp.g_flat, b.s);
    for (int p = 0; p < P; ++p) open[p] = open[p] && need[p];
    eval = need;
  }
  batch_to_abi(B, b.s);
  HIPCHECK(hipEventRecord(t1, b.s));
  HIPCHECK(hipEventSynchronize(t1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  HIPCHECK(hipGetLastError());
  int worst = LQGRID_OK;
  for (int p = 0; p < P; ++p) {
    if (infos) {
      lqgrid_info& inf = infos[p];
      const Scalars& h = ho[p];
      inf.status = status[p];
      inf.iterations = total_it[p];
      inf.refinements = passes[p];
      inf.restarts = std::max(0, passes[p] - 1);
      inf.rel_kkt_residual = h.rd2 > 0 ? std::sqrt(h.rr / h.rd2) : 0.0;
      inf.rel_res_inf = h.rdinf > 0 ? h.rinf / h.rdinf : 0.0;
      inf.seconds = ms * 1e-3;
    }
    if (status[p] != LQGRID_OK && worst == LQGRID_OK) worst = status[p];
  }
  return worst;
}

}  // extern "C"
