"""The node-temporal block Jacobi preconditioner (the alternative nesting:
time kept whole, space split into nodes) on the GPU through the C ABI
against the FP64 oracle (oracle/nodetemporal.py).

Operator parity: out = D_node^-1 in element by element, FP64 to 1e-11 of the
largest entry (a block Cholesky along T+1 steps, explicit inverses of the
n x n pivots, kappa of the node blocks O(10^2..10^3)) and FP32 to 1e-4.
Solves: the oracle's FP64 KKT residual meets the tolerance, iteration counts
within 2 of the oracle's Algorithm 1 with the same preconditioner, and the
Lanczos estimate of kappa(D_node^-1 Delta) within 5 % of the dense
eigenvalue ratio.
"""
import sys

import numpy as np
import pytest

from lqgrid_synth import make_problem, config_problem
from oracle import kkt, slab, residual, pcg, stack, nodetemporal

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


CASES = [
    # K, N, T, n, m, qt, weights, time_varying
    (4, 4, 20, 2, 1, 1.0, "identity", False),
    (5, 7, 150, 3, 2, 1.3, "spd", False),    # odd N (dummy column), ragged tiles
    (9, 6, 40, 4, 2, 2.0, "spd", False),
    (1, 5, 9, 2, 1, 1.0, "identity", False),  # K = 1
    (6, 1, 9, 2, 2, 1.0, "identity", False),  # N = 1
    (4, 3, 1, 1, 1, 1.0, "identity", False),  # T = 1, n = 1
    (5, 3, 30, 4, 2, 1.4, "spd", True),       # time-varying data
    # horizons against the solve's 16-step (FP32) / 8-step (FP64) tiles and
    # its 8- / 4-step coefficient ring: steps past the end of the last tile
    # from none to more than the ring is deep (T + 1 = 101: 11 in FP32, where
    # an index clamped at 0 only once read past the coefficient table)
    (4, 4, 100, 4, 2, 1.0, "identity", False),
    (3, 2, 3, 4, 2, 1.0, "identity", False),    # T + 1 = 4, shorter than the ring
    (4, 4, 16, 4, 2, 1.0, "spd", False),        # T + 1 = 17
    (4, 4, 63, 4, 2, 1.0, "identity", False),   # T + 1 = 64: no step past the end
    (2, 4, 104, 2, 1, 1.0, "identity", False),  # T + 1 = 105: 7 past the end in FP64
    (4, 2, 120, 4, 2, 2.0, "spd", False),       # T + 1 = 121
]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_node_temporal_operator_matches_oracle(lib, torch, case):
    from paper_2304_04980_amd import lqgrid
    K, N, T, n, m, qt, w, tv = case
    p = make_problem(K, N, T, n, m, seed=K * 100 + N * 10 + T, qt_scale=qt, weights=w,
                     time_varying=tv)
    say("node-temporal operator", case)
    ctx = lqgrid.Context(p, node_temporal=True)
    ops = slab.SlabOperators(p)
    P = nodetemporal.NodeTemporal(ops)
    v = np.random.default_rng(7).standard_normal((T + 1, N, K, n))
    ref = P(v.reshape(T + 1, -1))
    scale = np.abs(ref).max()
    e64 = np.abs(ctx.apply(lqgrid.OP_NODE_PRECOND, v).cpu().numpy().reshape(ref.shape) - ref).max()
    e32 = np.abs(ctx.apply(lqgrid.OP_NODE_PRECOND | lqgrid.OP_F32, v).cpu().numpy()
                 .reshape(ref.shape) - ref).max()
    say(f"  fp64 {e64 / scale:.2e}, fp32 {e32 / scale:.2e}")
    assert e64 <= 1e-11 * scale and e32 <= 1e-4 * scale
    ctx.close()


@pytest.mark.parametrize("case", [("tiny", 0, "fp64"), ("tiny", 1, "fp32_refine"),
                                  ("tv", 2, "fp64")])
def test_node_temporal_solve_matches_dense_kkt(lib, torch, case):
    from paper_2304_04980_amd import lqgrid
    kind, seed, precision = case
    if kind == "tiny":
        p, _ = config_problem("tiny", seed)
    else:
        p = make_problem(4, 4, 20, 2, 1, rho=0.9, seed=seed, weights="spd", time_varying=True)
    tol = 1e-10
    prec = lqgrid.FP64 if precision == "fp64" else lqgrid.FP32_REFINE
    ctx = lqgrid.Context(p, node_temporal=True)
    opts = lqgrid.default_opts(tol=tol, precision=prec, inner_tol=1e-4,
                               preconditioner=lqgrid.PRECOND_NODE_TEMPORAL)
    delta, x, u, info = ctx.solve(torch.as_tensor(p.x0), opts, want_primal=True)
    ref = kkt.solve_kkt(p)
    ops = slab.SlabOperators(p)
    g = residual.kkt_residual(ops, delta.cpu().numpy().reshape(p.T + 1, -1),
                              x.cpu().numpy().reshape(p.T + 1, -1),
                              u.cpu().numpy().reshape(p.T, -1))
    err = np.abs(delta.cpu().numpy().ravel() - ref["delta"]).max() / np.abs(ref["delta"]).max()
    _, it, _ = pcg.pcg(ops.delta, nodetemporal.NodeTemporal(ops), ops.r_delta(), tol=tol)
    say(f"  {case}: {info['iterations']} it (oracle {it}), oracle res {g['rel2']:.2e}, "
        f"error {err:.2e}")
    assert info["status"] == lqgrid.OK and g["rel2"] <= 1.01 * tol and err <= 1e-6
    if precision == "fp64":
        assert abs(info["iterations"] - it) <= 2
    ctx.close()


def test_node_temporal_plain_config(lib, torch):
    """The 32 x 32 x 100 workload at tol 1e-8: iterations within 2 of the
    oracle's, residual checked by the oracle, and fewer iterations than the
    paper's S = L = 2 preconditioner on the same problem."""
    from paper_2304_04980_amd import lqgrid
    p, _ = config_problem("plain", 0)
    tol = 1e-8
    ctx = lqgrid.Context(p, node_temporal=True)
    x0 = torch.as_tensor(p.x0)
    d, _, _, info = ctx.solve(x0, lqgrid.default_opts(
        tol=tol, preconditioner=lqgrid.PRECOND_NODE_TEMPORAL))
    _, _, _, inb = ctx.solve(x0, lqgrid.default_opts(tol=tol))
    ops = slab.SlabOperators(p)
    g = residual.kkt_residual(ops, d.cpu().numpy().reshape(p.T + 1, -1))
    _, it, _ = pcg.pcg(ops.delta, nodetemporal.NodeTemporal(ops), ops.r_delta(), tol=tol)
    say(f"  node-temporal {info['iterations']} it (oracle {it}) in "
        f"{info['seconds'] * 1e3:.1f} ms; NBJM {inb['iterations']} it in "
        f"{inb['seconds'] * 1e3:.1f} ms; oracle res {g['rel2']:.2e}")
    assert info["status"] == lqgrid.OK and g["rel2"] <= 1.01 * tol
    assert abs(info["iterations"] - it) <= 2
    ctx.close()


def test_node_temporal_condition_estimate_and_refusals(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p, _ = config_problem("tiny", 0)
    ctx = lqgrid.Context(p, node_temporal=True)
    est = ctx.condition_estimate(torch.as_tensor(p.x0), preconditioned=2, tol=1e-10)
    D = stack.delta_matrix(p).toarray()
    Dn = nodetemporal.node_blocks_dense(p, stack.delta_matrix(p)).toarray()
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(Dn, D)).real)
    say(f"  kappa(D_node^-1 Delta) gpu {est['kappa']:.4e} dense {ev[-1] / ev[0]:.4e}")
    assert abs(est["kappa"] / (ev[-1] / ev[0]) - 1) <= 0.05
    ctx.close()
    small = lqgrid.Context(p)   # workspace without the node-temporal tables
    with pytest.raises(lqgrid.LqgridError) as e:
        small.solve(torch.as_tensor(p.x0),
                    lqgrid.default_opts(preconditioner=lqgrid.PRECOND_NODE_TEMPORAL))
    assert e.value.status == lqgrid.EWORKSPACE
    small.close()
    _, _, st = lqgrid.batch_solve([p], opts=lqgrid.default_opts(
        preconditioner=lqgrid.PRECOND_NODE_TEMPORAL))
    assert st == lqgrid.EUNSUPPORTED
