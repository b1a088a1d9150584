/*
 * lqgrid -- MI355X (gfx950) solver for finite-horizon LQ optimal control over
 * a K x N grid of coupled sub-systems, by the preconditioned conjugate
 * gradient method of Zafar & Manchester, "Structured linear quadratic control
 * computations over 2D grids" (arXiv 2304.04980).
 *
 * The library solves the Schur-complement system  Delta delta~ = r_delta
 * (Sec. II-B, eq. "block_tridiagonal_system") with Algorithm 1 (PCGM,
 * Sec. III), preconditioned by a fixed number of sweeps of Algorithm 2
 * (nested block Jacobi, Sec. IV, Theorem 2), and recovers
 * x~ = Q~^-1 A~' delta~, u~ = R~^-1 B~' delta~.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every pointer argument named as an array is DEVICE memory owned
 *           by the caller.  The library never allocates device memory: all
 *           scratch lives in the caller's workspace (size from
 *           lqgrid_workspace_bytes).  It allocates only the small host-side
 *           context, freed by lqgrid_destroy, and HIP events for timing.
 * Streams.  Device work is enqueued on the caller's HIP stream (hipStream_t
 *           passed as void*; NULL = the null stream); lqgrid_batch_solve
 *           alone also uses an internal stream of its own (see there).
 * Layout.   Row-major C arrays, node (i, j) with i = 0..K-1 the vertical and
 *           j = 0..N-1 the horizontal grid index, column j outermost exactly as
 *           in the paper's stacking x_hat_t = col_j col_i x_{i,j,t}
 *           (Sec. II-A).  Vectors over the horizon are [T+1][N][K][n]
 *           (t outermost), i.e. the order of delta~ = col(delta_hat_0, ...,
 *           delta_hat_T).
 * Sign.     delta~ follows the Schur-complement convention of Sec. II-B:
 *           Q~ x~ = A~' delta~, R~ u~ = B~' delta~, Delta delta~ = r_delta.
 * Data.     Time-invariant A, B, Q, R, or time-varying ones (desc
 *           time_varying).  Spatial boundary states: zero, or given
 *           per solve to lqgrid_pcg_solve_bc.  Per-node sizes: optional
 *           (lqgrid_problem_desc n_node / m_node).
 * Errors.   Every call returns an lqgrid_status; none aborts.
 * Threads.  A context is not thread safe; distinct contexts are independent.
 */
#ifndef LQGRID_H
#define LQGRID_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LQGRID_ABI_VERSION 3

#if defined(__GNUC__) || defined(__clang__)
#define LQGRID_API __attribute__((visibility("default")))
#else
#define LQGRID_API
#endif

typedef struct lqgrid_ctx lqgrid_ctx; /* opaque, host side */

typedef enum {
  LQGRID_OK = 0,
  LQGRID_EINVAL = 1,      /* bad dimension, option, or null required pointer */
  LQGRID_ENOTSPD = 2,     /* a Phi_bar block Cholesky pivot was <= 0 or not finite */
  LQGRID_EBREAKDOWN = 3,  /* PCG breakdown: d'Delta d <= 0, mu <= 0, or non-finite */
  LQGRID_ENOCONV = 4,     /* max_iter reached; outputs and info are still written */
  LQGRID_EWORKSPACE = 5,  /* workspace null, misaligned (256 B) or too small */
  LQGRID_EHIP = 6,        /* a HIP runtime call failed */
  LQGRID_EUNSUPPORTED = 7 /* a size outside the compiled range (n > 4, m > 8) */
} lqgrid_status;

typedef enum {
  LQGRID_FP64 = 0,        /* every vector and sweep in FP64 */
  LQGRID_FP32_REFINE = 1  /* FP32 operator/sweeps inside FP64 iterative refinement */
} lqgrid_precision;

/* Preconditioner of Algorithm 1. */
typedef enum {
  /* The paper's: S outer x L inner nested block Jacobi sweeps of Algorithm 2
   * (time split first, then column pairs; per (v, t) solves along the rows). */
  LQGRID_PRECOND_NBJM = 0,
  /* The alternative nesting: one block Jacobi sweep over the grid nodes with
   * each node's whole temporal block of Delta (block tridiagonal in t, its
   * blocks Psi_hat_t[p,p] and Delta_{t+1,t}[p,p] = -A_hat_t[p,p] Q_{t,p}^-1),
   * solved exactly by a block Cholesky in t.  That part of Delta is positive
   * definite, so P is too.  Needs the workspace sized with this choice in
   * opts (lqgrid_workspace_bytes), else the solve returns LQGRID_EWORKSPACE. */
  LQGRID_PRECOND_NODE_TEMPORAL = 1,
  /* P = I: plain conjugate gradients. */
  LQGRID_PRECOND_NONE = 2
} lqgrid_preconditioner;

/* One problem (Sec. II, eq. "2d_graph_dynamics" and the LQ problem):
 *   x_{i,j,t+1} = A x_{i,j,t} + B u_{i,j,t} + E x_{i,j-1,t} + F x_{i,j+1,t}
 *                 + G x_{i-1,j,t} + H x_{i+1,j,t}
 * cost 1/2 sum (x'Qx + u'Ru) over t < T plus 1/2 x_T' QT x_T. */
typedef struct {
  int K, N, T, n, m;       /* grid rows, grid columns, horizon, state, input dims */
  const double *A;         /* [N][K][n][n]    A_{i,j}                             */
  const double *A_nbr;     /* [N][K][4][n][n] neighbour blocks of node (i,j):
                              0: E (couples x_{i,j-1}), 1: F (x_{i,j+1}),
                              2: G (x_{i-1,j}),         3: H (x_{i+1,j});
                              slots that point outside the grid are ignored     */
  const double *B;         /* [N][K][n][m]                                        */
  const double *Q;         /* [N][K][n][n] SPD stage weight, t = 0..T-1          */
  const double *R;         /* [N][K][m][m] SPD input weight                       */
  const double *QT;        /* [N][K][n][n] SPD terminal weight; NULL means QT = Q */
  /* Heterogeneous sub-systems (Sec. II: x_{i,j} in R^{n_{i,j}}, u_{i,j} in
   * R^{m_{i,j}}); NULL means n (m) at every node.  [N][K] int arrays with
   * 1 <= n_node <= n, 1 <= m_node <= m.  The arrays above keep their padded
   * shapes; only the leading n_{i,j} x n_{i,j} part of A_{i,j}, Q, QT, the
   * leading n_{i,j} x n_q part of the block coupling neighbour q, the leading
   * n_{i,j} x m_{i,j} part of B and m_{i,j} x m_{i,j} of R are read, and the
   * other entries may hold anything.  Outputs keep the padded layouts with
   * zeros past each node's sizes; x0 entries there are ignored.  A size
   * outside its range makes lqgrid_factor return LQGRID_EINVAL.  (ABI 2.)  */
  const int *n_node;
  const int *m_node;
  /* Time-varying data (Sec. II: A_{i,j,t}, B_{i,j,t}, E..H_{i,j,t},
   * Q_{i,j,t}, R_{i,j,t}).  0: the arrays above are time invariant.  1: A,
   * A_nbr, B, Q and R carry a leading time index t = 0..T-1 ([T][N][K][n][n]
   * etc.), A_t coupling x_t to x_{t+1}, Q_t and R_t weighting stage t; QT
   * keeps its shape (NULL: Q_{T-1}).  Every Phi_bar_{v,t} is then factored
   * (V (T+1) systems) and the operators read per-time blocks; the workspace
   * grows accordingly (about 30 n^2 doubles per node and time step).  Not
   * supported with boundary states, by the batched form or by the warm
   * start (EUNSUPPORTED).  (ABI 3.) */
  int time_varying;
} lqgrid_problem_desc;

typedef struct {
  int outer_S;        /* S >= 1: outer block-Jacobi sweeps (Alg. 2); paper: 2   */
  int inner_L;        /* L >= 2 and even (Theorem 2 needs even L); paper: 2     */
  double tol;         /* stop when ||r||_2 <= tol * ||r_delta||_2, confirmed on
                         the true FP64 residual r_delta - Delta delta~          */
  int max_iter;       /* PCG iteration cap (<= 0: 10000)                         */
  int precision;      /* lqgrid_precision                                        */
  double inner_tol;   /* FP32_REFINE: relative tolerance of each inner solve
                         (<= 0: 1e-5)                                            */
  int check_every;    /* iterations between host convergence reads (<= 0: 8)    */
  int warm_fallback;  /* with delta_init: 0 use it as given; 1 start from zero
                         instead if ||r_delta - Delta delta_init|| >= ||r_delta||
                         (the warm start is then no better than none); 2
                         energy line search: start from alpha delta_init,
                         alpha = delta_init' r_delta / (delta_init' Delta
                         delta_init), which minimises the Delta-norm of the
                         error along delta_init (so it is never larger than
                         the zero start's), or from zero if alpha <= 0       */
  int preconditioner; /* lqgrid_preconditioner (default NBJM); S and L apply to
                         NBJM only (ABI 3)                                     */
} lqgrid_solve_opts;

typedef struct {
  int status;              /* lqgrid_status of the solve                        */
  int iterations;          /* PCG iterations (all refinement passes summed)     */
  int refinements;         /* outer FP64 refinement passes (FP32_REFINE)        */
  int restarts;            /* restarts after a failed true-residual check       */
  double rel_kkt_residual; /* ||r_delta - Delta delta~||_2 / ||r_delta||_2 (FP64) */
  double rel_res_inf;      /* ||r_delta - Delta delta~||_inf / ||r_delta||_inf    */
  double seconds;          /* device time of the solve (HIP events)             */
  int warm_start_used;     /* 1 if delta_init was given and kept                */
} lqgrid_info;

/* Fills opts with the paper's settings: S = L = 2, tol 1e-10, FP64. */
LQGRID_API void lqgrid_default_opts(lqgrid_solve_opts *opts);

/* Bytes of device workspace that lqgrid_setup needs for this problem (0 if
 * the description is invalid); it covers both precisions.  Workspace must be
 * 256-byte aligned.  opts may be NULL; with opts->preconditioner ==
 * LQGRID_PRECOND_NODE_TEMPORAL the size includes that preconditioner's
 * factor tables (a setup given at least that much workspace factors them in
 * lqgrid_factor and can use either preconditioner). */
LQGRID_API size_t lqgrid_workspace_bytes(const lqgrid_problem_desc *desc,
                              const lqgrid_solve_opts *opts);

/* Ingest and Schur-block assembly (Sec. II-B eq. "structure_of_Delta";
 * Sec. II-B eq. "constructing_Phi_Omega_matrices").  Reads the problem
 * arrays once (they may be freed after the call's work completes on the
 * stream), writes the time-invariant operator blocks into the workspace and
 * returns a context.  Enqueue only; no synchronisation.
 * Errors: EINVAL (dims < 1, null A/A_nbr/B/Q/R), EUNSUPPORTED, EWORKSPACE. */
LQGRID_API int lqgrid_setup(const lqgrid_problem_desc *desc, void *workspace,
                 size_t workspace_bytes, void *hip_stream, lqgrid_ctx **out);

/* Banded block Cholesky factorisation of every distinct Phi_bar_{v,t}
 * (Sec. IV-B: factored once, before the PCG loop).  Synchronises
 * the stream to read the pivot check.  Errors: ENOTSPD, EHIP. */
LQGRID_API int lqgrid_factor(lqgrid_ctx *ctx);

/* Algorithm 1 with the Algorithm 2 preconditioner (S outer x L inner sweeps).
 *   x0         [N][K][n]       initial state gamma (DEVICE)
 *   delta_init [T+1][N][K][n]  optional warm start (NULL: zero start); any
 *                              value is allowed -- it only sets delta^(0)
 *   delta      [T+1][N][K][n]  output multipliers delta~
 *   x          [T+1][N][K][n]  optional primal state trajectory (NULL: skip)
 *   u          [T][N][K][m]    optional inputs (NULL: skip)
 *   info       host struct, always written when non-NULL
 * Synchronises the stream before returning.  Errors: EINVAL (bad opts or
 * factor not run), EBREAKDOWN, ENOCONV, EHIP. */
LQGRID_API int lqgrid_pcg_solve(lqgrid_ctx *ctx, const double *x0,
                     const lqgrid_solve_opts *opts, const double *delta_init,
                     double *delta, double *x, double *u, lqgrid_info *info);

/* Known spatial boundary states (Sec. II, eqs. "boundary_condition_i" and
 * "boundary_condition_j"), DEVICE arrays over t = 0..T (entries at t = T do
 * not enter the dynamics), each nullable (zero):
 *   alpha_lo [T+1][N][n]  x_{0,j,t}    the row above the grid (coupled by G
 *                                       of the nodes with i = 1)
 *   alpha_hi [T+1][N][n]  x_{K+1,j,t}  the row below (H of i = K)
 *   beta_lo  [T+1][K][n]  x_{i,0,t}    the column left of it (E of j = 1)
 *   beta_hi  [T+1][K][n]  x_{i,N+1,t}  the column right of it (F of j = N)
 * They enter only the right-hand side: r_delta at t+1 gets -(G alpha_lo +
 * H alpha_hi + E beta_lo + F beta_hi) of time t for the nodes on the edges
 * (the affine term omega_hat_t of Sec. II-A).  With per-node sizes the
 * boundary states are padded to n and the coupling blocks' columns are used
 * as given (zero-pad both past the boundary node's size). */
typedef struct {
  const double *alpha_lo, *alpha_hi, *beta_lo, *beta_hi;
} lqgrid_boundary;

/* lqgrid_pcg_solve with known boundary states (bc NULL: zero, which is
 * lqgrid_pcg_solve). */
LQGRID_API int lqgrid_pcg_solve_bc(lqgrid_ctx *ctx, const double *x0,
                                   const lqgrid_boundary *bc,
                                   const lqgrid_solve_opts *opts, const double *delta_init,
                                   double *delta, double *x, double *u, lqgrid_info *info);

/* Several independent problems solved together.  descs[p], x0s[p], deltas[p]
 * describe problem p (device pointers, layouts as above); all share n and
 * opts, while K, N, T and m may differ from problem to problem.  Uniform
 * sizes per problem (n_node / m_node non-null: EUNSUPPORTED) and zero
 * boundary states.  workspace
 * sized by lqgrid_batch_workspace_bytes.  infos[p] receives problem p's
 * result.  Synchronises the stream before returning.  Device memory: none
 * is allocated (everything lives in the workspace), but each call creates one
 * internal HIP stream and a few events (the iteration block is captured on
 * that stream into a HIP graph, instantiated and replayed, ordered after the
 * caller's stream by an event) and destroys them before returning.
 * Returns LQGRID_OK only if every problem converged.  The first call for a
 * set of problem sizes times the persistent grids and the order of the node
 * work items and caches the choice; the environment variable
 * LQGRID_BATCH_NODE_ORDER = 0 or 1 fixes that order (0: node groups
 * fastest, per-chunk stencil tiles; 1: time chunks fastest, the Delta apply
 * and Xi~ right-hand side run each node group over all its chunks). */
LQGRID_API size_t lqgrid_batch_workspace_bytes(int P, const lqgrid_problem_desc *descs,
                                    const lqgrid_solve_opts *opts);
LQGRID_API int lqgrid_batch_solve(int P, const lqgrid_problem_desc *descs,
                       const double *const *x0s, const lqgrid_solve_opts *opts,
                       double *const *deltas, void *workspace,
                       size_t workspace_bytes, void *hip_stream,
                       lqgrid_info *infos);

/* Single operator applications on vectors in the [T+1][N][K][n] layout, for
 * parity testing of each step of the path against a reference:
 *   LQGRID_OP_DELTA     out = Delta in                       (Sec. II-B)
 *   LQGRID_OP_XI        out = Xi~ in,  Xi~ = Psi~ - Delta    (eq. "splitting_Delta")
 *   LQGRID_OP_OMEGA     out = Omega~ in, Omega~ = Phi~ - Psi~ (eq. "splitting_Psi")
 *   LQGRID_OP_PHI_SOLVE out = Phi~^-1 in                     (eq. "decomposed_problem")
 *   LQGRID_OP_PRECOND   out = P_S^-1 in  (Alg. 2, S x L sweeps; Theorem 2)
 * Or-ing LQGRID_OP_F32 into op runs the FP32 kernels of the precision form
 * (input rounded to FP32, output widened back).  Requires lqgrid_factor for
 * PHI_SOLVE / PRECOND.  Enqueue only. */
typedef enum {
  LQGRID_OP_DELTA = 0,
  LQGRID_OP_XI = 1,
  LQGRID_OP_OMEGA = 2,
  LQGRID_OP_PHI_SOLVE = 3,
  LQGRID_OP_PRECOND = 4,
  LQGRID_OP_NODE_PRECOND = 5, /* out = D_node^-1 in (LQGRID_PRECOND_NODE_TEMPORAL) */
  LQGRID_OP_F32 = 16
} lqgrid_op;
LQGRID_API int lqgrid_apply_operator(lqgrid_ctx *ctx, int op, int outer_S, int inner_L,
                          const double *in, double *out);

/* Per-kernel device timing over the calls that follow: HIP events on the
 * context's stream around every enable-th launch of each hot kernel
 * (enable = 1: every launch; enable <= 0 stops recording).  An event pair
 * between two launches serialises their dispatch, so a stride above 1 keeps
 * the timed calls close to untimed ones.  Samples from the last convergence
 * check batch (opts.check_every iterations) of each PCG run are dropped:
 * launches enqueued after the run converged exit at once.  Used by the
 * benchmark to time the dominant kernel.  Returns LQGRID_EINVAL for a null
 * ctx, LQGRID_EHIP if resolving pending events fails. */
LQGRID_API int lqgrid_profile_enable(lqgrid_ctx *ctx, int enable);
/* kernel: 0 = Delta apply, 1 = Phi solve, 2 = Omega/Xi right-hand side,
 * 3 = vector update.  Returns the timed launches and their summed
 * milliseconds since enable. */
LQGRID_API int lqgrid_profile_read(lqgrid_ctx *ctx, int kernel, long long *launches,
                        double *total_ms);

/* ------------------------------------------------------------------------
 * Learned warm start.  A convolutional network over the K x N grid maps each
 * node's x0, A_ii and B_ii to 16 Chebyshev-in-time coefficients per state
 * component of delta~; their expansion over t = 0..T (tau = 2t/T - 1) is a
 * delta_init for lqgrid_pcg_solve.  Algorithm 1 allows any initial iterate,
 * so the preconditioner and the convergence test are unchanged, and
 * opts.warm_fallback restarts from zero when the prediction does not lower
 * the residual.  `layers` 3 x 3 convolutions, 64 channels, ReLU between
 * them, zero padding; BF16 weights and activations, FP32 accumulation on the
 * matrix cores; FP32 master weights trained with Adam on solves.
 * Supported: n = 4, n + n^2 + n m <= 32, K a multiple of 8, K N a multiple
 * of 256, 2 <= layers <= 8 (0 / LQGRID_EINVAL otherwise).
 *
 * Parameters: one FP32 array; for each layer l, W_l[64][3][3][cin_l] (cin_0
 * = 32, cin_l = 64; tap (a, b) couples pixel (i, j) to (i + a - 1, j + b - 1))
 * followed by b_l[64].  Features of one problem: lqgrid_wsnet_sample_bytes(,
 * 0) bytes (BF16, pixel-major then channel-major copy).  Targets of one
 * solved problem: lqgrid_wsnet_sample_bytes(, 1) bytes (FP32 projections of
 * delta* on the basis and |delta*|^2).  Batched calls read sample index[b]
 * (device int array; NULL: b) of arrays of such samples.  Workspaces:
 * lqgrid_wsnet_workspace_bytes(desc, batch), 256-byte aligned.  Enqueue only,
 * except lqgrid_wsnet_gradient when loss is non-NULL (synchronises). */
typedef struct {
  int K, N, n, m, T; /* the problem sizes the network is built for */
  int layers;        /* convolution layers (6) */
} lqgrid_wsnet_desc;
LQGRID_API size_t lqgrid_wsnet_param_count(const lqgrid_wsnet_desc *desc);
LQGRID_API size_t lqgrid_wsnet_sample_bytes(const lqgrid_wsnet_desc *desc, int which);
LQGRID_API size_t lqgrid_wsnet_workspace_bytes(const lqgrid_wsnet_desc *desc, int batch);
/* Input features of one problem (x0: [N][K][n]) into feat. */
LQGRID_API int lqgrid_wsnet_features(const lqgrid_wsnet_desc *desc,
                                     const lqgrid_problem_desc *prob, const double *x0,
                                     void *feat, void *hip_stream);
/* Training target of one solved problem (delta: [T+1][N][K][n]). */
LQGRID_API int lqgrid_wsnet_targets(const lqgrid_wsnet_desc *desc, const double *delta,
                                    float *target, void *workspace, size_t workspace_bytes,
                                    void *hip_stream);
/* Network output (FP32 [batch][K N][64], pixel p = j K + i). */
LQGRID_API int lqgrid_wsnet_forward(const lqgrid_wsnet_desc *desc, int batch,
                                    const void *feats, const int *index,
                                    const float *params, float *out, void *workspace,
                                    size_t workspace_bytes, void *hip_stream);
/* Mean over the batch of the relative squared error of the expansion,
 * sum_t |delta0_t - delta*_t|^2 / sum_t |delta*_t|^2, and its gradient with
 * respect to params (FP32, same layout). */
LQGRID_API int lqgrid_wsnet_gradient(const lqgrid_wsnet_desc *desc, int batch,
                                     const void *feats, const float *targets,
                                     const int *index, const float *params, float *grad,
                                     double *loss, void *workspace,
                                     size_t workspace_bytes, void *hip_stream);
/* Gradient with respect to params of a loss whose gradient with respect to
 * the network output is dout (FP32 [batch][K N][64], rounded to BF16 like
 * the back-propagated gradients): the backward pass of lqgrid_wsnet_gradient
 * from a given output gradient, for losses formed outside the network (e.g.
 * from operator products) and for exact tests. */
LQGRID_API int lqgrid_wsnet_backward(const lqgrid_wsnet_desc *desc, int batch,
                                     const void *feats, const int *index,
                                     const float *params, const float *dout, float *grad,
                                     void *workspace, size_t workspace_bytes,
                                     void *hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8); moments: 2 x param_count
 * FP32, zero before step 1. */
LQGRID_API int lqgrid_wsnet_adam(const lqgrid_wsnet_desc *desc, float *params,
                                 const float *grad, float *moments, int step, float lr,
                                 void *hip_stream);
/* delta_init [T+1][N][K][n] (FP64) predicted for one problem's features. */
LQGRID_API int lqgrid_wsnet_predict(const lqgrid_wsnet_desc *desc, const void *feat,
                                    const float *params, double *delta_init,
                                    void *workspace, size_t workspace_bytes,
                                    void *hip_stream);

/* Standalone NBJM solver (the paper's comparison method, Sec. IV eq.
 * "outer_jacobi_iterations" with opts->inner_L inner sweeps of eq.
 * "inner_iteration_NBJM", Algorithm 2 run to convergence): from delta = 0,
 *   rho = r_delta + Xi~ delta^(s),  theta^(0) = delta^(s),
 *   theta^(l+1) = Phi~^-1 (rho + Omega~ theta^(l)),  delta^(s+1) = theta^(L).
 * Each inner iteration starts from the outer iterate (with theta^(0) = 0, as
 * in the preconditioner, the iteration would converge to another point for
 * finite L).  Stops when the FP64 relative residual ||r_delta - Delta
 * delta||_2 / ||r_delta||_2 <= opts->tol, tested every opts->check_every
 * sweeps (1: every sweep); opts->max_iter caps the sweeps (ENOCONV).
 * info->iterations = outer sweeps.  FP64 only (FP32_REFINE: EUNSUPPORTED).
 * Outputs as lqgrid_pcg_solve (x, u optional).  Requires lqgrid_factor.
 * Synchronises the stream. */
LQGRID_API int lqgrid_nbjm_solve(lqgrid_ctx *ctx, const double *x0,
                                 const lqgrid_solve_opts *opts, double *delta,
                                 double *x, double *u, lqgrid_info *info);

/* Spectrum of the (preconditioned) Schur complement from the coefficients of
 * Algorithm 1 (Sec. III: the CG rate is set by the condition number; Sec. V
 * compares kappa(Delta) with kappa(P_S^-1/2 Delta P_S^-1/2)).  Runs one FP64
 * Algorithm 1 from zero on Delta delta = r_delta(x0) to the relative
 * tolerance tol (at most max_iter <= 8192 iterations; <= 0: 8192) with the
 * S x L NBJM preconditioner (preconditioned = 1), the node-temporal one
 * (preconditioned = 2) or P = I (preconditioned = 0, plain CG), and
 * returns the extreme eigenvalues of the Lanczos matrix built from its step
 * lengths theta_k and direction coefficients beta_k (diagonal 1/theta_k +
 * beta_{k-1}/theta_{k-1}, off-diagonal sqrt(beta_k)/theta_k), which converge
 * to those of P^-1 Delta from inside its spectrum; kappa = lambda_max /
 * lambda_min.  Output pointers are host memory and may be NULL.  Requires
 * lqgrid_factor; synchronises the stream.  Errors: EINVAL, EBREAKDOWN, EHIP. */
LQGRID_API int lqgrid_condition_estimate(lqgrid_ctx *ctx, const double *x0,
                                         int preconditioned, int outer_S, int inner_L,
                                         double tol, int max_iter, double *kappa,
                                         double *lambda_min, double *lambda_max,
                                         int *iterations);

/* ------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same computation as lqgrid_setup + lqgrid_factor +
 * lqgrid_pcg_solve (zero start, same kernels and results), with the
 * workspace in a static device array of the library instead of the caller's
 * buffer: lqgrid_noalloc_capacity() bytes (80 MiB, enough for the
 * 32 x 32 x 100, n = 4, m = 2 workload), held by every GPU the library runs
 * on until the process ends.  The caller passes inputs and outputs as for
 * the three calls it replaces; the call runs on the stream's device, which
 * must be the current device.  It calls no hipMalloc, hipFree or other
 * allocating routine, creates no event and keeps its context on the stack
 * (info->seconds is host time around the synchronised solve).
 * Errors: as lqgrid_setup / lqgrid_factor / lqgrid_pcg_solve, and
 * LQGRID_EWORKSPACE when lqgrid_workspace_bytes(desc) exceeds the capacity
 * (lqgrid_last_error() names both sizes).  Every call on one GPU uses that
 * GPU's one array: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller. */
LQGRID_API size_t lqgrid_noalloc_capacity(void);
LQGRID_API int lqgrid_solve_noalloc(const lqgrid_problem_desc *desc, const double *x0,
                                    const lqgrid_solve_opts *opts, double *delta,
                                    double *x, double *u, void *hip_stream,
                                    lqgrid_info *info);

LQGRID_API void lqgrid_destroy(lqgrid_ctx *ctx);
LQGRID_API const char *lqgrid_status_string(int status);
LQGRID_API int lqgrid_abi_version(void);
/* Text of the last HIP runtime failure seen by this thread (for EHIP), or of
 * the scratch-size error of lqgrid_solve_noalloc. */
LQGRID_API const char *lqgrid_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LQGRID_H */
