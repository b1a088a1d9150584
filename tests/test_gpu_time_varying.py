"""Time-varying data (A_t, B_t, E..H_t, Q_t, R_t) on the GPU through the C
ABI against the FP64 oracle (oracle/slab.py with per-time slice matrices,
oracle/kkt.py dense LDL', oracle/riccati.py time-varying recursion).

Element-wise operator bounds as for time-invariant data (test_gpu_parity.py:
FP64 1e-12 of the largest entry, the block solve 1e-11; FP32 1e-5 and 1e-4),
since every output is the same number of block products; only the blocks
differ from step to step.  The weights are per-node, per-time random SPD
matrices and Q_T differs from Q_{T-1}, so a block taken at the wrong time (or
node) fails.  Whole solves: the oracle's KKT residual of the returned delta~,
x~, u~ meets the tolerance and the error to the dense solution is within
kappa * residual (1e-6 relative at tol 1e-10).
"""
import sys

import numpy as np
import pytest

from lqgrid_synth import make_problem
from oracle import kkt, slab, nbjm, residual, riccati

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


CASES = [
    # K, N, T, n, m, qt_scale
    (4, 4, 20, 2, 1, 1.3),
    (5, 7, 70, 3, 2, 1.0),      # odd N, two time tiles of 32 steps and a tail
    (9, 6, 40, 4, 2, 2.0),      # K >= 8
    (3, 5, 64, 4, 2, 0.7),      # T + 1 = 65
    (1, 5, 9, 2, 1, 1.0),       # K = 1
    (6, 1, 9, 2, 2, 1.0),       # N = 1
    (4, 3, 1, 1, 1, 1.0),       # T = 1, n = 1
    (16, 4, 33, 4, 3, 1.5),
    # the setup assembles and scatters 16 time slices per batch: T + 1 = 16
    # and 32 fill the batches exactly (T + 1 = 65 above leaves the terminal
    # slice alone in the last batch)
    (4, 4, 15, 2, 1, 1.0),
    (3, 3, 31, 4, 2, 1.2),
]


def tv_problem(case, seed_off=0):
    K, N, T, n, m, qt = case
    return make_problem(K, N, T, n, m, seed=K * 100 + N * 10 + T + seed_off, qt_scale=qt,
                        weights="spd", time_varying=True)


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_time_varying_operators_match_oracle(lib, torch, case):
    from paper_2304_04980_amd import lqgrid
    p = tv_problem(case)
    say("time-varying operators", case)
    ctx = lqgrid.Context(p)
    ops = slab.SlabOperators(p)
    v = np.random.default_rng(7).standard_normal((p.T + 1, p.N, p.K, p.n))
    vf = v.reshape(p.T + 1, -1)
    refs = [(lqgrid.OP_DELTA, ops.delta(vf), 1e-12, 1e-5),
            (lqgrid.OP_XI, ops.xi(vf), 1e-12, 1e-5),
            (lqgrid.OP_OMEGA, ops.omega(vf), 1e-12, 1e-5),
            (lqgrid.OP_PHI_SOLVE, ops.phi_solve(vf), 1e-11, 1e-4)]
    for op, ref, tol64, tol32 in refs:
        scale = max(np.abs(ref).max(), 1e-300)
        e64 = np.abs(ctx.apply(op, v).cpu().numpy().reshape(ref.shape) - ref).max()
        e32 = np.abs(ctx.apply(op | lqgrid.OP_F32, v).cpu().numpy().reshape(ref.shape)
                     - ref).max()
        say(f"  op {op}: fp64 {e64 / scale:.2e}, fp32 {e32 / scale:.2e} (scale {scale:.2e})")
        assert e64 <= tol64 * scale and e32 <= tol32 * scale, op
    for S, L in [(2, 2), (1, 2), (3, 4)]:
        ref = nbjm.slab_preconditioner(ops, S, L)(vf)
        got = ctx.apply(lqgrid.OP_PRECOND, v, S=S, L=L).cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"  precond S={S} L={L}: {err:.2e}")
        assert err <= 1e-10
    ctx.close()


@pytest.mark.parametrize("seed,precision", [(0, "fp64"), (1, "fp64"), (2, "fp32_refine")])
def test_time_varying_solve_matches_dense_kkt(lib, torch, seed, precision):
    from paper_2304_04980_amd import lqgrid
    p = make_problem(4, 4, 20, 2, 1, rho=0.9, seed=seed, weights="spd", qt_scale=1.6,
                     time_varying=True)
    tol = 1e-10
    prec = lqgrid.FP64 if precision == "fp64" else lqgrid.FP32_REFINE
    ctx = lqgrid.Context(p)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0),
                                  lqgrid.default_opts(tol=tol, precision=prec, inner_tol=1e-4),
                                  want_primal=True)
    ref = kkt.solve_kkt(p)
    ops = slab.SlabOperators(p)
    g = residual.kkt_residual(ops, delta.cpu().numpy().reshape(p.T + 1, -1),
                              x.cpu().numpy().reshape(p.T + 1, -1),
                              u.cpu().numpy().reshape(p.T, -1))
    errs = [np.abs(a.cpu().numpy().ravel() - ref[k]).max() / np.abs(ref[k]).max()
            for a, k in ((delta, "delta"), (x, "x"), (u, "u"))]
    say(f"  seed {seed} {precision}: {info['iterations']} it, oracle res {g['rel2']:.2e}, "
        f"errors {errs}")
    assert info["status"] == lqgrid.OK
    assert g["rel2"] <= 1.01 * tol
    assert max(errs) <= 1e-6
    # iteration count of the oracle's Algorithm 1 within 2 (plain FP64)
    if precision == "fp64":
        from oracle import pcg
        _, it, _ = pcg.pcg(ops.delta, nbjm.slab_preconditioner(ops, 2, 2), ops.r_delta(),
                           tol=tol)
        assert abs(info["iterations"] - it) <= 2
    ctx.close()


def test_time_varying_riccati_single_node(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p = make_problem(1, 1, 50, 4, 2, rho=1.05, seed=6, weights="spd", qt_scale=2.0,
                     time_varying=True)
    R = riccati.lqr_of_tv_problem(p)
    ctx = lqgrid.Context(p)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0), lqgrid.default_opts(tol=1e-12),
                                  want_primal=True)
    assert info["status"] == lqgrid.OK
    for got, key in ((x, "x"), (u, "u"), (delta, "delta")):
        err = np.abs(got.cpu().numpy()[:, 0, 0] - R[key]).max() / np.abs(R[key]).max()
        say(f"  {key}: {err:.2e}")
        assert err <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_time_varying_larger_grid(lib, torch, precision):
    from paper_2304_04980_amd import lqgrid
    p = make_problem(16, 9, 70, 4, 2, seed=8, weights="spd", qt_scale=1.2, time_varying=True)
    tol = 1e-9
    prec = lqgrid.FP64 if precision == "fp64" else lqgrid.FP32_REFINE
    ctx = lqgrid.Context(p)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0),
                                  lqgrid.default_opts(tol=tol, precision=prec, inner_tol=1e-4),
                                  want_primal=True)
    ops = slab.SlabOperators(p)
    d = delta.cpu().numpy().reshape(p.T + 1, -1)
    g = residual.kkt_residual(ops, d, x.cpu().numpy().reshape(p.T + 1, -1),
                              u.cpu().numpy().reshape(p.T, -1))
    say(f"  {precision}: {info['iterations']} it in {info['refinements']} passes, reported "
        f"{info['rel_kkt_residual']:.2e}, oracle {g['rel2']:.2e}")
    assert info["status"] == lqgrid.OK and g["rel2"] <= 1.01 * tol
    assert abs(info["rel_kkt_residual"] - residual.kkt_residual(ops, d)["schur_rel2"]) <= 1e-3 * tol
    ctx.close()


def test_time_varying_refusals(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p = make_problem(3, 3, 5, 2, 1, seed=1, time_varying=True, boundary=True)
    ctx = lqgrid.Context(p)
    with pytest.raises(lqgrid.LqgridError) as e:
        ctx.solve(torch.as_tensor(p.x0), lqgrid.default_opts(),
                  boundary=dict(alpha_lo=p.alpha_lo))
    assert e.value.status == lqgrid.EUNSUPPORTED
    ctx.close()
    b = lqgrid.Batch([make_problem(3, 3, 5, 2, 1, seed=2)])
    b.descs[0].time_varying = 1
    _, _, st = b.solve()
    assert st == lqgrid.EUNSUPPORTED
