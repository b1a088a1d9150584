// Batched form: the kernels of the single-problem path for many independent
// problems at once.  Each kernel is persistent: a fixed grid walks a
// flattened list of (problem, tile) work items, each workgroup a contiguous
// (node and flat items) or strided (block-solve items, whose cost grows with
// the problem's K) share of it, and calls the same tile bodies as the
// single-problem kernels with that problem's dimensions, coefficients and
// vectors.  The item lists are compacted on the device between iteration
// blocks so that converged problems cost nothing; inside a block the
// per-problem convergence flag masks the items of problems that finish early.
// Item counts are read from device memory, so the launches can be captured
// once in a graph and replayed while the lists shrink.
#include "bodies_ops.h"
#include "bodies_setup.h"

namespace lqg {
namespace {
using namespace dev;

__device__ __forceinline__ OpCoef<double> op64(const Coef& C) {
  return OpCoef<double>{C.G13, C.Cdn, C.Cup, C.Qi, C.QTd, C.Qm, C.Fw, C.Bw, C.Xw};
}

// Contiguous share [*lo, *hi) of n items for this workgroup (XCD-remapped, so
// that an XCD's workgroups hold neighbouring items).
__device__ __forceinline__ void share(int n, int* lo, int* hi) {
  const int G = gridDim.x, lb = xcd_block();
  const int per = (n + G - 1) / G;
  *lo = min(n, lb * per);
  *hi = min(n, *lo + per);
}

// Per-problem records, work lists and counts are passed as separate
// read-only, non-aliasing kernel arguments: nothing a kernel stores can
// alias them, so their uniform fields are read through the scalar cache
// instead of vector loads that would wait behind the previous item's stores.
// The convergence flags are not written while these kernels run.
#define LQG_BATCH_ARGS                                                   \
  const BatchProb* __restrict__ probs, const Scalars* __restrict__ scs,   \
      const Item* __restrict__ live, const int* __restrict__ nlive
__device__ __forceinline__ bool gated_out(const Scalars& sc, int check) {
  return check && sc.done != kRunning;
}

template <int NS, bool ROWS>
__global__ __launch_bounds__(256) void kb_delta(LQG_BATCH_ARGS,
                                                double* __restrict__ psum,
                                                int in, int out, int partial,
                                                int check) {
  int lo, hi;
  share(*nlive, &lo, &hi);
  for (int it = lo; it < hi; ++it) {
    const Item w = live[it];
    const BatchProb& P = probs[w.prob];
    if (gated_out(scs[w.prob], check)) continue;
    if constexpr (ROWS) {  // the group's first chunk item covers every chunk
      if (w.b != 0) {
        if (partial && threadIdx.x == 0) psum[w.slot] = 0.0;
        continue;
      }
      delta_rows<double, NS>(P.D, op64(P.C), P.v[in], P.v[out],
                             partial ? psum + w.slot : nullptr, w.a);
    } else {
      delta_tile<double, NS>(P.D, op64(P.C), P.v[in], P.v[out],
                             partial ? psum + w.slot : nullptr, w.a, w.b);
    }
  }
}

template <int NS>
__global__ __launch_bounds__(256) void kb_omega(LQG_BATCH_ARGS, int rho, int th,
                                                int tau, int check) {
  int lo, hi;
  share(*nlive, &lo, &hi);
  for (int it = lo; it < hi; ++it) {
    const Item w = live[it];
    const BatchProb& P = probs[w.prob];
    if (gated_out(scs[w.prob], check)) continue;
    omega_tile<double, NS>(P.D, op64(P.C), rho >= 0 ? P.v[rho] : nullptr,
                           P.v[th], P.v[tau], w.a, w.b, w.b + 1);
  }
}

template <int NS, bool ROWS>
__global__ __launch_bounds__(256) void kb_xi(LQG_BATCH_ARGS, int r, int dl,
                                             int rho, int check) {
  int lo, hi;
  share(*nlive, &lo, &hi);
  for (int it = lo; it < hi; ++it) {
    const Item w = live[it];
    const BatchProb& P = probs[w.prob];
    if (gated_out(scs[w.prob], check)) continue;
    if constexpr (ROWS) {  // as in kb_delta
      if (w.b != 0) continue;
      xi_rows<double, NS>(P.D, op64(P.C), r >= 0 ? P.v[r] : nullptr, P.v[dl], P.v[rho],
                          w.a);
    } else {
      xi_tile<double, NS>(P.D, op64(P.C), r >= 0 ? P.v[r] : nullptr, P.v[dl],
                          P.v[rho], w.a, w.b, w.b + 1);
    }
  }
}

// Block-solve items are dealt out round-robin (item = lb + k G) so that the
// long sweeps of large-K problems spread over all workgroups.  A problem with
// K >= kTwistMin is solved in the twisted order (the same 2n wavefronts: two
// rows each, half per chain), smaller ones in the one-chain order; both use
// the one LDS buffer.
template <int NS>
__global__ __launch_bounds__(2 * NS * kWave) void kb_solve(LQG_BATCH_ARGS,
                                                           int tau, int out,
                                                           int check) {
  static_assert(2 * kWavesPerHalf<NS> == 2 * NS, "twisted and one-chain solves share the grid");
  constexpr int NB = 2 * NS, WK = kWKeepAlloc<double, NS>;
  __shared__ double zb2[2][2][NB][kWave];
  __shared__ double wb[2][WK][NB][kWave];
  auto* zb1 = zb2[0];  // the one-chain exchange buffer
  const int n = *nlive;
  for (int it = xcd_block(); it < n; it += gridDim.x) {
    const Item w = live[it];
    const BatchProb& P = probs[w.prob];
    if (gated_out(scs[w.prob], check)) continue;
    const int qt = scs[w.prob].qt_differs != 0;
    if (twisted(P.D))
      phi_tile_twisted<double, NS>(P.D, op64(P.C), P.v[tau], P.v[out], qt, w.a, w.b, zb2, wb);
    else
      phi_tile<double, NS>(P.D, op64(P.C), P.v[tau], P.v[out], qt, w.a, w.b, zb1);
  }
}

// Flat vector operations on element ranges of one problem's vectors; the
// step lengths come from that problem's scalars.
__global__ __launch_bounds__(256) void kb_flat(LQG_BATCH_ARGS,
                                               const Scalars* __restrict__ scos,
                                               double* __restrict__ psum,
                                               double* __restrict__ pmax,
                                               int op, int ra, int rb, int rc,
                                               int rd, int check) {
  int lo, hi;
  share(*nlive, &lo, &hi);
  for (int it = lo; it < hi; ++it) {
    const Item w = live[it];
    const BatchProb& P = probs[w.prob];
    if (gated_out(scs[w.prob], check)) continue;
    const Scalars& sc = scs[w.prob];
    double* a = P.v[ra];
    double* b = rb >= 0 ? P.v[rb] : nullptr;
    double* c = rc >= 0 ? P.v[rc] : nullptr;
    double* d = rd >= 0 ? P.v[rd] : nullptr;
    double acc = 0.0, mx = 0.0;
    const int e0 = w.a, e1 = w.b;
    switch (op) {
      case kFlatDir: {
        const double beta = sc.beta;
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x)
          b[g] = fma(beta, b[g], a[g]);
        break;
      }
      case kFlatUpdate: {
        const double th = sc.theta;
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x) {
          c[g] = fma(th, a[g], c[g]);
          const double rn = fma(-th, b[g], d[g]);
          d[g] = rn;
          acc = fma(rn, rn, acc);
        }
        break;
      }
      case kFlatDot:
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x)
          acc = fma(a[g], b[g], acc);
        break;
      case kFlatNorms:
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x) {
          acc = fma(a[g], a[g], acc);
          mx = fmax(mx, fabs(a[g]));
        }
        break;
      case kFlatSubNorm:
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x) {
          const double v = a[g] - b[g];
          c[g] = v;
          acc = fma(v, v, acc);
          mx = fmax(mx, fabs(v));
        }
        break;
      case kFlatScale: {
        const double s = 1.0 / sqrt(scos[w.prob].rr);
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x) b[g] = s * a[g];
        break;
      }
      case kFlatAxpy: {
        const double s = sqrt(scos[w.prob].rr);
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x)
          b[g] = fma(s, a[g], b[g]);
        break;
      }
      case kFlatZero:
        for (int g = e0 + threadIdx.x; g < e1; g += blockDim.x) a[g] = 0.0;
        break;
    }
    if (op == kFlatUpdate || op == kFlatDot || op == kFlatNorms ||
        op == kFlatSubNorm) {
      acc = block_sum<256>(acc);
      if (op == kFlatNorms || op == kFlatSubNorm) {
        mx = block_max<256>(mx);
        if (threadIdx.x == 0) pmax[w.slot] = mx;
      }
      if (threadIdx.x == 0) psum[w.slot] = acc;
    }
  }
}

// One workgroup per problem: fixed-order reduction of the problem's partial
// sums (its original item slots of `kind`), then the scalar update.
__global__ __launch_bounds__(256) void kb_scalar(BatchDev B, int mode, int kind,
                                                 int outer, double tol) {
  const BatchProb& P = B.probs[blockIdx.x];
  Scalars* sc = outer ? P.sco : P.sc;
  if (!sc->active) return;
  if (scalar_mode_gated(mode) && sc->done != kRunning) return;
  const double* psum = kind == kItemNode ? B.psum_node : B.psum_flat;
  const bool want_max = kind == kItemFlat;
  const int f = P.first[kind], n = P.count[kind];
  double s = 0.0, m = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    s += psum[f + k];
    if (want_max) m = fmax(m, B.pmax_flat[f + k]);
  }
  s = block_sum<256>(s);
  if (want_max) m = block_max<256>(m);
  if (threadIdx.x != 0) return;
  scalar_apply(mode, s, want_max ? m : 0.0, sc, P.sco, tol);
}

// Live problems (active, and when running_only also still iterating) and
// the offsets of their items in the compacted lists: one workgroup, chunks
// of 256 problems with a workgroup-wide exclusive scan per item kind.
__global__ __launch_bounds__(256) void kb_compact_scan(BatchDev B,
                                                       int running_only) {
  __shared__ int wsum[kNumItemKinds + 1][4];
  int carry[kNumItemKinds + 1] = {0, 0, 0, 0};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int base = 0; base < B.P; base += 256) {
    const int p = base + threadIdx.x;
    int live = 0;
    int cnt[kNumItemKinds] = {0, 0, 0};
    if (p < B.P) {
      const Scalars* sc = B.probs[p].sc;
      live = sc->active && (!running_only || sc->done == kRunning);
      B.live_flag[p] = live;
      if (live)
        for (int k = 0; k < kNumItemKinds; ++k) cnt[k] = B.probs[p].count[k];
    }
#pragma unroll
    for (int k = 0; k <= kNumItemKinds; ++k) {
      const int v = k < kNumItemKinds ? cnt[k] : live;
      // inclusive scan within the wavefront
      int x = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane == 63) wsum[k][wv] = x;
      __syncthreads();
      int before = carry[k];
      for (int q = 0; q < wv; ++q) before += wsum[k][q];
      if (p < B.P && k < kNumItemKinds) B.live_off[k * B.P + p] = before + x - v;
      int total = 0;
      for (int q = 0; q < 4; ++q) total += wsum[k][q];
      carry[k] += total;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0)
    for (int k = 0; k <= kNumItemKinds; ++k) B.nlive[k] = carry[k];
}

__global__ __launch_bounds__(256) void kb_compact_scatter(BatchDev B) {
  for (int k = 0; k < kNumItemKinds; ++k) {
    const Item* src = B.orig[k];
    Item* dst = B.live[k];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B.norig[k];
         i += gridDim.x * blockDim.x) {
      const Item w = src[i];
      if (!B.live_flag[w.prob]) continue;
      dst[B.live_off[k * B.P + w.prob] + (i - B.probs[w.prob].first[k])] = w;
    }
  }
}

// Active flags and iteration limits from the host staging area.
__global__ void kb_set_active(BatchDev B) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.P) return;
  const int act = B.host_in[p];
  Scalars* sc = B.probs[p].sc;
  sc->active = act;
  B.probs[p].sco->active = act;
  if (act) {
    sc->done = kRunning;
    sc->iter = 0;
    sc->max_iter = B.host_in[B.P + p];
  }
}

// Setup unit kernels (one unit per thread, or per workgroup for the factor).
__global__ void kb_node_prep(BatchDev B) {
  const Item* u = B.units[kUnitPrep];
  for (int it = blockIdx.x; it < B.nunits[kUnitPrep]; it += gridDim.x) {
    const Item w = u[it];
    BatchProb& P = B.probs[w.prob];
    const int q = w.a + threadIdx.x;
    if (q < w.b) node_prep(P.D, P.in, P.C, P.sc, q);
  }
}
template <int NS>
__global__ void kb_stencil(BatchDev B) {
  const Item* u = B.units[kUnitStencil];
  for (int it = blockIdx.x; it < B.nunits[kUnitStencil]; it += gridDim.x) {
    const Item w = u[it];
    const BatchProb& P = B.probs[w.prob];
    const int q = w.a + threadIdx.x;
    if (q < w.b) stencil<NS>(P.D, P.in, P.C, q);
  }
}
// Factor units of the problems factored in the twisted order (128 threads,
// one chain per half) or in the one-chain order (64 threads); each kernel
// skips the other kind.
__global__ __launch_bounds__(128) void kb_factor_twisted(BatchDev B) {
  const Item* u = B.units[kUnitFactor];
  for (int it = blockIdx.x; it < B.nunits[kUnitFactor]; it += gridDim.x) {
    const Item w = u[it];
    const BatchProb& P = B.probs[w.prob];
    if (twisted(P.D)) factor_twisted(P.D, P.C, P.sc, w.a, w.b);
  }
}
__global__ __launch_bounds__(64) void kb_factor(BatchDev B) {
  const Item* u = B.units[kUnitFactor];
  for (int it = blockIdx.x; it < B.nunits[kUnitFactor]; it += gridDim.x) {
    const Item w = u[it];
    const BatchProb& P = B.probs[w.prob];
    if (!twisted(P.D)) factor(P.D, P.C, P.sc, w.a, w.b);
  }
}
__global__ void kb_rhs_init(BatchDev B) {
  const Item* u = B.units[kUnitRhs];
  for (int it = blockIdx.x; it < B.nunits[kUnitRhs]; it += gridDim.x) {
    const Item w = u[it];
    const BatchProb& P = B.probs[w.prob];
    const int q = w.a + threadIdx.x;
    if (q < w.b) rhs_init(P.D, P.x0, nullptr, P.v[kBRd], q);
  }
}
// delta~ of each problem from the internal to the interface layout
// [T+1][N][K][n]; unit q is an entry of the output.
__global__ void kb_to_abi(BatchDev B) {
  const Item* u = B.units[kUnitAbi];
  for (int it = blockIdx.x; it < B.nunits[kUnitAbi]; it += gridDim.x) {
    const Item w = u[it];
    const BatchProb& P = B.probs[w.prob];
    const Dims& D = P.D;
    const long long per_t = (long long)D.real_nodes * D.n;
    const double* in = P.v[kBDl];
    for (int q = w.a + threadIdx.x; q < w.b; q += blockDim.x) {
      const int t = (int)(q / per_t);
      const long long pc = q - (long long)t * per_t;
      P.delta_out[q] = in[pc * D.ldt + t];
    }
  }
}

}  // namespace

#define LQG_DISPATCH_N(n, CALL) \
  switch (n) {                  \
    case 1: CALL(1); break;     \
    case 2: CALL(2); break;     \
    case 3: CALL(3); break;     \
    case 4: CALL(4); break;     \
    default: break;             \
  }

void batch_delta(const BatchDev& B, int n, int in, int out, int partial,
                 int check, int grid, hipStream_t s) {
#define CALL(NS)                                                                     \
  if (B.node_rows)                                                                    \
    hipLaunchKernelGGL((kb_delta<NS, true>), dim3(grid), dim3(256), 0, s, B.probs, B.sc, \
                       B.live[kItemNode], B.nlive + kItemNode, B.psum_node, in, out,  \
                       partial, check);                                               \
  else                                                                                \
    hipLaunchKernelGGL((kb_delta<NS, false>), dim3(grid), dim3(256), 0, s, B.probs,   \
                       B.sc, B.live[kItemNode], B.nlive + kItemNode, B.psum_node, in, \
                       out, partial, check)
  LQG_DISPATCH_N(n, CALL)
#undef CALL
}
void batch_omega(const BatchDev& B, int n, int rho, int th, int tau, int check,
                 int grid, hipStream_t s) {
#define CALL(NS)                                                         \
  hipLaunchKernelGGL(kb_omega<NS>, dim3(grid), dim3(256), 0, s, B.probs, B.sc, \
                     B.live[kItemNode], B.nlive + kItemNode, rho, th, tau, check)
  LQG_DISPATCH_N(n, CALL)
#undef CALL
}
void batch_xi(const BatchDev& B, int n, int r, int dl, int rho, int check,
              int grid, hipStream_t s) {
#define CALL(NS)                                                                      \
  if (B.node_rows)                                                                     \
    hipLaunchKernelGGL((kb_xi<NS, true>), dim3(grid), dim3(256), 0, s, B.probs, B.sc,  \
                       B.live[kItemNode], B.nlive + kItemNode, r, dl, rho, check);     \
  else                                                                                 \
    hipLaunchKernelGGL((kb_xi<NS, false>), dim3(grid), dim3(256), 0, s, B.probs, B.sc, \
                       B.live[kItemNode], B.nlive + kItemNode, r, dl, rho, check)
  LQG_DISPATCH_N(n, CALL)
#undef CALL
}
void batch_solve(const BatchDev& B, int n, int tau, int out, int check,
                 int grid, hipStream_t s) {
#define CALL(NS)                                                            \
  hipLaunchKernelGGL(kb_solve<NS>, dim3(grid), dim3(2 * NS * kWave), 0, s, \
                     B.probs, B.sc, B.live[kItemSolve], B.nlive + kItemSolve, \
                     tau, \
                     out, check)
  LQG_DISPATCH_N(n, CALL)
#undef CALL
}
void batch_flat(const BatchDev& B, int op, int a, int b, int c, int d,
                int check, int grid, hipStream_t s) {
  hipLaunchKernelGGL(kb_flat, dim3(grid), dim3(256), 0, s, B.probs, B.sc,
                     B.live[kItemFlat], B.nlive + kItemFlat, B.sco, B.psum_flat,
                     B.pmax_flat, op, a, b, c, d, check);
}
void batch_scalar(const BatchDev& B, int mode, int kind, int outer, double tol,
                  hipStream_t s) {
  hipLaunchKernelGGL(kb_scalar, dim3(B.P), dim3(256), 0, s, B, mode, kind,
                     outer, tol);
}
void batch_compact(const BatchDev& B, int running_only, hipStream_t s) {
  hipLaunchKernelGGL(kb_compact_scan, dim3(1), dim3(256), 0, s, B, running_only);
  hipLaunchKernelGGL(kb_compact_scatter, dim3(512), dim3(256), 0, s, B);
}
void batch_set_active(const BatchDev& B, hipStream_t s) {
  hipLaunchKernelGGL(kb_set_active, dim3((B.P + 255) / 256), dim3(256), 0, s, B);
}
void batch_setup(const BatchDev& B, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_node_prep, dim3(1024), dim3(128), 0, s, B);
#define CALL(NS) hipLaunchKernelGGL(kb_stencil<NS>, dim3(2048), dim3(128), 0, s, B)
  LQG_DISPATCH_N(n, CALL)
#undef CALL
}
void batch_factor(const BatchDev& B, hipStream_t s) {
  const dim3 g(std::max(1, std::min(B.nunits[kUnitFactor], 16384)));
  hipLaunchKernelGGL(kb_factor, g, dim3(64), 0, s, B);
  hipLaunchKernelGGL(kb_factor_twisted, g, dim3(128), 0, s, B);
}
void batch_rhs_init(const BatchDev& B, hipStream_t s) {
  hipLaunchKernelGGL(kb_rhs_init, dim3(1024), dim3(256), 0, s, B);
}
void batch_to_abi(const BatchDev& B, hipStream_t s) {
  hipLaunchKernelGGL(kb_to_abi, dim3(2048), dim3(256), 0, s, B);
}

}  // namespace lqg
