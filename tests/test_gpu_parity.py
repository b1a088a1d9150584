"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Operators: element-wise comparison on the same seeded inputs at sizes that
span several 64-wide time tiles with a ragged tail, odd and even N (the odd
case exercises the single-column last super-column), K = 1, N = 1, T = 1 and
n = 1..4; K < 8 runs the one-chain Phi_bar factorisation, K >= 8 (even and
odd, up to the headline K = 128) the twisted one.

Tolerances (FP64, derived from the arithmetic): each operator output is a sum
of at most 23 n-by-n block products, evaluated in a different order than the
oracle; the element-wise bound used is 1e-12 * max|ref|.  Phi~^-1 multiplies
by the explicit inverse of each Cholesky diagonal block instead of a banded
triangular solve: bound 1e-11 * max|ref| (kappa of the 2n x 2n blocks is
O(10^2) on these inputs).  Whole solves: the relative residual must meet the
requested tolerance, and the error to the exact solution obeys
||e|| / ||delta*|| <= kappa(Delta) * relative residual.
"""
import sys

import numpy as np
import pytest

from lqgrid_synth import make_problem, config_problem
from oracle import kkt, slab, nbjm, pcg, residual

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_abi(p, v):
    """(T+1, KNn) oracle array -> [T+1][N][K][n]."""
    return v.reshape(p.T + 1, p.N, p.K, p.n)


def rand_vec(p, seed):
    return np.random.default_rng(seed).standard_normal((p.T + 1, p.N, p.K, p.n))


CASES = [
    # K, N, T, n, m, qt_scale
    (4, 4, 20, 2, 1, 1.0),
    (5, 7, 150, 3, 2, 1.0),     # odd N, three time tiles, ragged tail
    (6, 6, 63, 4, 2, 2.5),      # T+1 = 64 exactly, distinct terminal weight
    (3, 5, 64, 4, 2, 0.7),      # T+1 = 65: one-lane second tile, QT != Q
    (1, 5, 9, 2, 1, 1.0),       # K = 1
    (6, 1, 9, 2, 2, 1.0),       # N = 1 (single dummy-padded super-column)
    (4, 3, 1, 1, 1, 1.0),       # T = 1, n = 1
    (7, 8, 40, 4, 3, 1.0),      # K = 7: the last one-chain Phi_bar factor
    # K >= 8: the twisted factorisation and two-chain sweep
    (8, 4, 70, 4, 2, 1.0),      # K = 8: chains of 3 + 3 rows, two time tiles
    (9, 6, 40, 3, 2, 2.5),      # odd K: bottom chain one row longer, QT != Q
    (12, 3, 9, 2, 2, 1.3),      # odd N, QT != Q
    (16, 5, 130, 2, 1, 0.7),    # three time tiles with a ragged tail, QT != Q
    (33, 2, 20, 4, 3, 1.0),     # odd K
    (64, 2, 64, 1, 1, 1.0),     # T+1 = 65, n = 1
    (128, 2, 20, 4, 2, 1.0),    # K of the headline workload
    # T+1 a multiple of 64: the t-1 / t+1 terms cross every chunk boundary
    # at full lanes (lane 63 from the previous chunk, lane 0 from the next)
    (4, 3, 127, 2, 1, 1.0),     # two full time tiles, odd N
    (9, 4, 191, 3, 2, 1.5),     # three full time tiles, twisted, QT != Q
]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


# per-node random SPD Q, Q_T and R (a weight of the wrong node, or Q in place
# of Q_T, changes every operator): one-chain and twisted factorisations,
# odd N, ragged time tiles
SPD_CASES = [
    (4, 4, 20, 2, 1, 1.0, "spd"),
    (5, 7, 150, 3, 2, 1.3, "spd"),
    (7, 6, 64, 4, 2, 0.8, "spd"),
    (9, 5, 40, 4, 3, 1.0, "spd"),
    (16, 4, 70, 4, 2, 2.0, "spd"),
    (33, 3, 20, 2, 2, 1.0, "spd"),
]


@pytest.mark.parametrize("case", CASES + SPD_CASES, ids=[str(c) for c in CASES + SPD_CASES])
def test_operators_match_oracle(lib, torch, case):
    from paper_2304_04980_amd import lqgrid
    K, N, T, n, m, qt = case[:6]
    w = case[6] if len(case) > 6 else "identity"
    say("operators case", case)
    p = make_problem(K, N, T, n, m, seed=K * 100 + N * 10 + T, qt_scale=qt, weights=w)
    ctx = lqgrid.Context(p)
    ops = slab.SlabOperators(p)
    v = rand_vec(p, 7)
    vf = v.reshape(T + 1, -1)
    checks = [
        (lqgrid.OP_DELTA, ops.delta(vf), 1e-12),
        (lqgrid.OP_XI, ops.xi(vf), 1e-12),
        (lqgrid.OP_OMEGA, ops.omega(vf), 1e-12),
        (lqgrid.OP_PHI_SOLVE, ops.phi_solve(vf), 1e-11),
    ]
    for op, ref, tol in checks:
        got = ctx.apply(op, v).cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        say(f"  op {op}: max err {err:.3e} (scale {np.abs(ref).max():.3e})")
        assert err <= tol * np.abs(ref).max(), (op, err)
    for S, L in [(2, 2), (1, 2), (3, 4)]:
        ref = nbjm.slab_preconditioner(ops, S, L)(vf)
        got = ctx.apply(lqgrid.OP_PRECOND, v, S=S, L=L).cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        say(f"  precond S={S} L={L}: max err {err:.3e}")
        assert err <= 1e-10 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("seed,w", [(0, "identity"), (1, "identity"), (2, "identity"),
                                    (3, "spd"), (4, "spd")])
def test_tiny_solve_matches_dense_kkt(lib, torch, seed, w):
    """Tiny configuration: GPU PCG vs brute-force dense KKT LDL' (also with
    per-node SPD weights and Q_T != Q)."""
    from paper_2304_04980_amd import lqgrid
    if w == "identity":
        p, tol = config_problem("tiny", seed)
    else:
        tol = 1e-10
        p = make_problem(4, 4, 20, 2, 1, rho=0.9, seed=seed, qt_scale=1.6, weights=w)
    say("tiny solve seed", seed, w)
    ctx = lqgrid.Context(p)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0), lqgrid.default_opts(tol=tol),
                                  want_primal=True)
    ref = kkt.solve_kkt(p)
    d = delta.cpu().numpy().ravel()
    err = np.linalg.norm(d - ref["delta"]) / np.linalg.norm(ref["delta"])
    ops = slab.SlabOperators(p)
    gate = residual.kkt_residual(ops, d.reshape(p.T + 1, -1))
    from oracle import stack
    D = stack.delta_matrix(p).toarray()
    ev = np.linalg.eigvalsh(D)
    kappa = ev[-1] / ev[0]
    say(f"  iters {info['iterations']} gpu-res {info['rel_kkt_residual']:.2e} "
        f"oracle-res {gate['rel2']:.2e} err {err:.2e} kappa {kappa:.1f}")
    assert info["status"] == lqgrid.OK
    assert gate["rel2"] <= tol * 1.01
    assert abs(info["rel_kkt_residual"] - gate["schur_rel2"]) <= 1e-3 * tol + 1e-15
    assert err <= kappa * gate["rel2"] * 1.01 + 1e-14
    xr = ref["x"].reshape(p.T + 1, p.N, p.K, p.n)
    ur = ref["u"].reshape(p.T, p.N, p.K, p.m)
    assert np.abs(x.cpu().numpy() - xr).max() <= kappa * tol * 10 * np.abs(xr).max()
    assert np.abs(u.cpu().numpy() - ur).max() <= kappa * tol * 10 * np.abs(ur).max()
    # same iteration count as the oracle's Algorithm 1 (rounding may move the
    # exit by an iteration)
    pre = nbjm.slab_preconditioner(ops, 2, 2)
    _, it, _ = pcg.pcg(ops.delta, pre, ops.r_delta(), tol=tol)
    assert abs(info["iterations"] - it) <= 2
    ctx.close()


@pytest.mark.parametrize("w", ["identity", "spd"])
def test_riccati_single_node(lib, torch, w):
    """K = N = 1: the GPU solution equals the textbook Riccati LQR (scaled
    identity weights, and full SPD Q, R, Q_T)."""
    from paper_2304_04980_amd import lqgrid
    from oracle import riccati
    p = make_problem(1, 1, 60, 4, 2, rho=1.05, seed=3, qt_scale=2.0, weights=w)
    R = riccati.lqr_of_problem(p)
    ctx = lqgrid.Context(p)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0),
                                  lqgrid.default_opts(tol=1e-12), want_primal=True)
    assert info["status"] == lqgrid.OK
    assert np.abs(x.cpu().numpy()[:, 0, 0] - R["x"]).max() <= 1e-8 * np.abs(R["x"]).max()
    assert np.abs(u.cpu().numpy()[:, 0, 0] - R["u"]).max() <= 1e-8 * np.abs(R["u"]).max()
    assert np.abs(delta.cpu().numpy()[:, 0, 0] - R["delta"]).max() <= 1e-8 * np.abs(R["delta"]).max()


def test_plain_config_solve(lib, torch):
    """K = N = 32, T = 100, n = 4, m = 2 (the plain FP64 GPU configuration):
    oracle-evaluated residual below tol, iteration count equal to the oracle's
    Algorithm 1 within 2, and agreement with the oracle's PCG solution."""
    from paper_2304_04980_amd import lqgrid
    p, tol = config_problem("plain", 0)
    say("plain config solve")
    ctx = lqgrid.Context(p)
    delta, _, _, info = ctx.solve(torch.as_tensor(p.x0), lqgrid.default_opts(tol=tol))
    ops = slab.SlabOperators(p)
    d = delta.cpu().numpy().reshape(p.T + 1, -1)
    gate = residual.kkt_residual(ops, d)
    pre = nbjm.slab_preconditioner(ops, 2, 2)
    xo, it, _ = pcg.pcg(ops.delta, pre, ops.r_delta(), tol=tol)
    rel = np.linalg.norm(d - xo) / np.linalg.norm(xo)
    say(f"  gpu iters {info['iterations']} oracle iters {it} res {gate['rel2']:.2e} "
        f"diff {rel:.2e} t {info['seconds']*1e3:.1f} ms")
    assert info["status"] == lqgrid.OK
    assert gate["rel2"] <= tol * 1.01
    assert abs(info["iterations"] - it) <= 2
    assert rel <= 1e-6


def test_warm_start_and_exact_start(lib, torch):
    """Any warm start reaches the same tolerance; starting at the solution
    takes zero iterations."""
    from paper_2304_04980_amd import lqgrid
    p, tol = config_problem("tiny", 4)
    ctx = lqgrid.Context(p)
    x0 = torch.as_tensor(p.x0)
    opts = lqgrid.default_opts(tol=tol)
    d0, _, _, i0 = ctx.solve(x0, opts)
    garbage = np.random.default_rng(1).standard_normal((p.T + 1, p.N, p.K, p.n)) * 10
    d1, _, _, i1 = ctx.solve(x0, opts, delta_init=torch.as_tensor(garbage))
    assert i1["status"] == lqgrid.OK and i1["rel_kkt_residual"] <= tol
    ref = kkt.solve_kkt(p)["delta"].reshape(d0.shape)
    d2, _, _, i2 = ctx.solve(x0, opts, delta_init=torch.as_tensor(ref))
    assert i2["iterations"] == 0 and i2["rel_kkt_residual"] <= tol


def test_error_paths(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p, tol = config_problem("tiny", 0)
    ctx = lqgrid.Context(p)
    x0 = torch.as_tensor(p.x0)
    # odd L is rejected (Theorem 2 needs even L)
    with pytest.raises(lqgrid.LqgridError) as e:
        ctx.solve(x0, lqgrid.default_opts(inner_L=3))
    assert e.value.status == lqgrid.EINVAL
    # iteration cap
    _, _, _, info = ctx.solve(x0, lqgrid.default_opts(tol=1e-14, max_iter=3,
                                                      check_every=1),
                              raise_on_error=False)
    assert info["status"] == lqgrid.ENOCONV and info["iterations"] == 3
    # indefinite weight -> not SPD factor
    q = make_problem(3, 3, 4, 2, 1, seed=0)
    q.Q[1, 1] = -np.eye(2)
    with pytest.raises(lqgrid.LqgridError) as e:
        lqgrid.Context(q)
    assert e.value.status == lqgrid.ENOTSPD
    # non-finite initial state -> breakdown
    bad = x0.clone()
    bad[0, 0, 0] = float("nan")
    _, _, _, info = ctx.solve(bad, lqgrid.default_opts(), raise_on_error=False)
    assert info["status"] == lqgrid.EBREAKDOWN


# ------------------------------------------------------------ precision form
F32_CASES = [(4, 4, 20, 2, 1, 1.0), (5, 7, 150, 3, 2, 1.0), (3, 5, 64, 4, 2, 0.7),
             (6, 1, 9, 2, 2, 1.0), (8, 4, 70, 4, 2, 1.0), (9, 6, 40, 3, 2, 2.5),
             (33, 2, 20, 4, 3, 1.0), (128, 2, 20, 4, 2, 1.3),
             # a short last 64-step tile, node count not a multiple of 4,
             # n = 3 and n = 2
             (7, 3, 129, 3, 2, 1.0), (5, 3, 66, 2, 1, 1.0),
             # T+1 a multiple of 64 (full-lane chunk boundaries)
             (4, 3, 127, 2, 1, 1.0), (9, 4, 191, 3, 2, 1.5),
             # n = 1: one coefficient register per 16 blocks' worth
             (4, 3, 70, 1, 1, 1.0), (16, 2, 129, 1, 1, 0.7)]


@pytest.mark.parametrize("case", F32_CASES + SPD_CASES, ids=[str(c) for c in F32_CASES + SPD_CASES])
def test_fp32_operators_match_oracle(lib, torch, case):
    """FP32 kernels of the precision form against the FP64 oracle.  Inputs and
    coefficients are rounded to FP32 (unit roundoff u = 2^-24 ~ 6e-8); each
    output is a sum of at most 23 n x n block products (<= 92 terms), so the
    element-wise bound used is 1e-5 * max|ref| (~170 u, covering the
    cancellation of terms of either sign).  Phi~^-1 adds the conditioning of
    the 2n x 2n Cholesky blocks: 1e-4 * max|ref|."""
    from paper_2304_04980_amd import lqgrid
    K, N, T, n, m, qt = case[:6]
    w = case[6] if len(case) > 6 else "identity"
    say("fp32 operators case", case)
    p = make_problem(K, N, T, n, m, seed=K * 100 + N * 10 + T, qt_scale=qt, weights=w)
    ctx = lqgrid.Context(p)
    ops = slab.SlabOperators(p)
    v = rand_vec(p, 7)
    vf = v.reshape(T + 1, -1)
    checks = [
        (lqgrid.OP_DELTA, ops.delta(vf), 1e-5),
        (lqgrid.OP_XI, ops.xi(vf), 1e-5),
        (lqgrid.OP_OMEGA, ops.omega(vf), 1e-5),
        (lqgrid.OP_PHI_SOLVE, ops.phi_solve(vf), 1e-4),
    ]
    for op, ref, tol in checks:
        got = ctx.apply(op | lqgrid.OP_F32, v).cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max()
        say(f"  op {op} f32: max err {err:.3e} (scale {np.abs(ref).max():.3e})")
        assert err <= tol * np.abs(ref).max(), (op, err)
    ref = nbjm.slab_preconditioner(ops, 2, 2)(vf)
    got = ctx.apply(lqgrid.OP_PRECOND | lqgrid.OP_F32, v).cpu().numpy().reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_fp32_refinement_reaches_fp64_accuracy(lib, torch, tol):
    """FP32 sweeps inside FP64 iterative refinement reach the same relative
    KKT residual as plain FP64 PCG (checked by the oracle's FP64 residual)."""
    from paper_2304_04980_amd import lqgrid
    p, _ = config_problem("plain", 1)
    ctx = lqgrid.Context(p)
    x0 = torch.as_tensor(p.x0)
    d64, _, _, i64 = ctx.solve(x0, lqgrid.default_opts(tol=tol))
    d32, _, _, i32 = ctx.solve(x0, lqgrid.default_opts(tol=tol, precision=lqgrid.FP32_REFINE,
                                                       inner_tol=1e-4))
    ops = slab.SlabOperators(p)
    g64 = residual.kkt_residual(ops, d64.cpu().numpy().reshape(p.T + 1, -1))
    g32 = residual.kkt_residual(ops, d32.cpu().numpy().reshape(p.T + 1, -1))
    say(f"  tol {tol}: fp64 {i64['iterations']} it res {g64['rel2']:.2e}; fp32+refine "
        f"{i32['iterations']} it in {i32['refinements']} passes res {g32['rel2']:.2e}")
    assert i32["status"] == lqgrid.OK and i32["refinements"] >= 2
    assert g32["rel2"] <= tol * 1.01 and g64["rel2"] <= tol * 1.01
    rel = np.linalg.norm((d32 - d64).cpu().numpy()) / np.linalg.norm(d64.cpu().numpy())
    assert rel <= 1e-3   # both within kappa * tol of delta*


# ------------------------------------------------------------ headline size
@pytest.fixture(scope="module")
def headline():
    """The 128 x 128 x 200 workload and the oracle's slab operators of it."""
    p, tol = config_problem("headline", 0)
    return p, tol, slab.SlabOperators(p)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_headline_solve_checked_by_oracle(lib, torch, headline, precision):
    """K = N = 128, T = 200, n = 4, m = 2 (the benchmarked workload) at
    tol 1e-8 in both forms: the oracle's FP64 KKT residual of the returned
    delta~, x~ and u~ (all three blocks of the KKT system) meets the
    tolerance, and the library's own reported residual agrees with the
    oracle's Schur-complement residual to 1e-3 tol."""
    from paper_2304_04980_amd import lqgrid
    p, tol, ops = headline
    say("headline solve", precision)
    ctx = lqgrid.Context(p)
    prec = lqgrid.FP64 if precision == "fp64" else lqgrid.FP32_REFINE
    opts = lqgrid.default_opts(tol=tol, precision=prec, inner_tol=1e-4)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0), opts, want_primal=True)
    d = delta.cpu().numpy().reshape(p.T + 1, -1)
    xs = x.cpu().numpy().reshape(p.T + 1, -1)
    us = u.cpu().numpy().reshape(p.T, -1)
    gate = residual.kkt_residual(ops, d, xs, us)
    own = residual.kkt_residual(ops, d)
    say(f"  {info['iterations']} it, {info['refinements']} passes; reported "
        f"{info['rel_kkt_residual']:.3e}, oracle {gate['rel2']:.3e} "
        f"(with recovered primal {own['rel2']:.3e})")
    assert info["status"] == lqgrid.OK
    assert gate["rel2"] <= 1.01 * tol
    assert own["rel2"] <= 1.01 * tol
    assert abs(info["rel_kkt_residual"] - own["schur_rel2"]) <= 1e-3 * tol
    ctx.close()


# ------------------------------------------------------------ kernel timing
def test_profile_samples_leave_out_the_stopping_batch(lib, torch):
    """The per-kernel timing (lqgrid_profile_*) counts the block-solve
    launches of the initial preconditioner and of every check batch before
    the one in which the run stops: with one iteration per batch, a run that
    stops in iteration k keeps 4 + 4 (k - 1) samples (S = L = 2: four solves
    per preconditioner); with every iteration in one batch, only the initial
    four."""
    from paper_2304_04980_amd import lqgrid
    p = make_problem(4, 4, 20, 2, 1, seed=21)
    ctx = lqgrid.Context(p)
    x0 = torch.as_tensor(p.x0)
    ctx.profile_enable(True, stride=1)
    _, _, _, info = ctx.solve(x0, lqgrid.default_opts(tol=1e-8, check_every=1))
    n1, ms1 = ctx.profile_read(1)
    say(f"  check_every 1: {info['iterations']} it, {info['refinements']} passes, "
        f"{n1} timed solves, {ms1:.3f} ms")
    assert info["status"] == lqgrid.OK and info["refinements"] == 1
    assert n1 == 4 * info["iterations"] and ms1 > 0.0
    ctx.profile_enable(True, stride=1)
    _, _, _, info = ctx.solve(x0, lqgrid.default_opts(tol=1e-8, check_every=64))
    n2, _ = ctx.profile_read(1)
    say(f"  check_every 64: {info['iterations']} it, {n2} timed solves")
    assert info["status"] == lqgrid.OK and info["refinements"] == 1
    assert info["iterations"] < 64 and n2 == 4
    ctx.profile_enable(False)
    ctx.close()
