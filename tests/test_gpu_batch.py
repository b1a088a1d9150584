"""Batched form (lqgrid_batch_solve) against the FP64 oracle.

Every problem of a batch must meet its own relative KKT residual (evaluated
by the oracle in FP64 on the returned delta~), take the oracle's Algorithm 1
iteration count within 2, and agree with the oracle's PCG solution within
kappa * tol (the bound used is 1e-6 relative, as for the single-problem
path).  The batches mix odd and even N, K = 1 and N = 1, one to four 64-wide
time tiles with ragged tails, a distinct terminal weight, and K below and
above 8 (one-chain and twisted Phi_bar factorisations in one batch).
"""
import sys

import numpy as np
import pytest

from lqgrid_synth import make_problem, batched_problems, BATCHED_TOL
from oracle import slab, nbjm, pcg, residual

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


UNEVEN = [
    # K, N, T, n, m, qt_scale
    (4, 4, 20, 4, 2, 1.0),
    (5, 7, 150, 4, 2, 1.0),     # odd N, three time tiles, ragged tail
    (6, 6, 63, 4, 1, 2.5),      # T+1 = 64, distinct terminal weight
    (3, 5, 64, 4, 2, 0.7),      # T+1 = 65
    (1, 5, 9, 4, 2, 1.0),       # K = 1
    (6, 1, 9, 4, 3, 1.0),       # N = 1
    (9, 8, 200, 4, 2, 1.0),     # four time tiles; K >= 8: twisted Phi_bar order
    (2, 3, 1, 4, 2, 1.0),       # T = 1
    (12, 5, 70, 4, 2, 2.0),     # twisted, odd N, QT != Q
    (17, 4, 30, 4, 3, 1.0),     # twisted, odd K
]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def uneven_problems(weights="identity"):
    return [make_problem(K, N, T, n, m, seed=11 * k + 5, qt_scale=qt, weights=weights)
            for k, (K, N, T, n, m, qt) in enumerate(UNEVEN)]


def check_against_oracle(p, delta, info, tol):
    ops = slab.SlabOperators(p)
    d = delta.cpu().numpy().reshape(p.T + 1, -1)
    gate = residual.kkt_residual(ops, d)
    xo, it, _ = pcg.pcg(ops.delta, nbjm.slab_preconditioner(ops, 2, 2),
                        ops.r_delta(), tol=tol)
    rel = np.linalg.norm(d - xo) / max(np.linalg.norm(xo), 1e-300)
    say(f"  K={p.K} N={p.N} T={p.T}: {info['iterations']} it (oracle {it}), "
        f"res {gate['rel2']:.2e} (reported {info['rel_kkt_residual']:.2e}), diff {rel:.2e}")
    assert info["status"] == 0
    assert gate["rel2"] <= tol * 1.01
    assert abs(info["rel_kkt_residual"] - gate["schur_rel2"]) <= 1e-3 * tol + 1e-15
    assert abs(info["iterations"] - it) <= 2
    assert rel <= 1e-6


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_uneven_batch_matches_oracle(lib, torch, tol):
    from paper_2304_04980_amd import lqgrid
    probs = uneven_problems()
    say("uneven batch, tol", tol)
    outs, infos, st = lqgrid.batch_solve(probs, opts=lqgrid.default_opts(tol=tol))
    assert st == lqgrid.OK, [i["status"] for i in infos]
    for p, d, info in zip(probs, outs, infos):
        check_against_oracle(p, d, info, tol)


def test_uneven_batch_with_spd_weights(lib, torch):
    """The uneven batch with per-node random SPD Q, Q_T and R."""
    from paper_2304_04980_amd import lqgrid
    probs = uneven_problems("spd")
    say("uneven batch, spd weights")
    outs, infos, st = lqgrid.batch_solve(probs, opts=lqgrid.default_opts(tol=1e-9))
    assert st == lqgrid.OK, [i["status"] for i in infos]
    for p, d, info in zip(probs, outs, infos):
        check_against_oracle(p, d, info, 1e-9)


@pytest.mark.parametrize("order", ["0", "1"])
def test_uneven_batch_in_each_node_order(lib, torch, order, monkeypatch):
    """Both node-item orders (per-chunk stencil tiles; all-chunks Delta and
    Xi~ with the other chunk items idle) against the oracle."""
    from paper_2304_04980_amd import lqgrid
    monkeypatch.setenv("LQGRID_BATCH_NODE_ORDER", order)
    probs = uneven_problems()
    say("uneven batch, node order", order)
    outs, infos, st = lqgrid.batch_solve(probs, opts=lqgrid.default_opts(tol=1e-9))
    assert st == lqgrid.OK, [i["status"] for i in infos]
    for p, d, info in zip(probs, outs, infos):
        check_against_oracle(p, d, info, 1e-9)


def test_batch_equals_single_problem_path(lib, torch):
    """Each problem of a batch takes the same iterations as the
    single-problem solve and lands within kappa * tol of it."""
    from paper_2304_04980_amd import lqgrid
    allp = uneven_problems()
    probs = [allp[k] for k in (0, 1, 6, 8)]  # one-chain and twisted Phi_bar orders
    opts = lqgrid.default_opts(tol=1e-10)
    outs, infos, st = lqgrid.batch_solve(probs, opts=opts)
    assert st == lqgrid.OK
    for p, d, info in zip(probs, outs, infos):
        ctx = lqgrid.Context(p)
        d1, _, _, i1 = ctx.solve(torch.as_tensor(p.x0), opts)
        ctx.close()
        rel = (torch.linalg.norm(d - d1) / torch.linalg.norm(d1)).item()
        say(f"  K={p.K} N={p.N} T={p.T}: batch {info['iterations']} it, single "
            f"{i1['iterations']} it, diff {rel:.2e}")
        assert abs(info["iterations"] - i1["iterations"]) <= 1
        assert rel <= 1e-7


def test_repeated_batch_solves_are_identical(lib, torch):
    """The second call (autotuned settings cached) gives bitwise the same
    result as the first: every reduction has a fixed order."""
    from paper_2304_04980_amd import lqgrid
    b = lqgrid.Batch(uneven_problems(), opts=lqgrid.default_opts(tol=1e-9))
    outs1, infos1, st1 = b.solve()
    first = [o.clone() for o in outs1]
    outs2, infos2, st2 = b.solve()
    assert st1 == st2 == lqgrid.OK
    for a, c in zip(first, outs2):
        assert torch.equal(a, c)
    assert [i["iterations"] for i in infos1] == [i["iterations"] for i in infos2]


def test_full_batched_workload(lib, torch):
    """The 256-problem batched workload (K, N ~ U{8..64}, T ~ U{50..200}) at
    tol 1e-8: every problem converges; the oracle confirms the residual of a
    sample of problems."""
    from paper_2304_04980_amd import lqgrid
    probs, tol = batched_problems(), BATCHED_TOL
    say(f"batched workload: {len(probs)} problems, "
        f"{sum(p.unknowns for p in probs) / 1e6:.1f} M unknowns")
    b = lqgrid.Batch(probs, opts=lqgrid.default_opts(tol=tol))
    outs, infos, st = b.solve()
    its = [i["iterations"] for i in infos]
    say(f"  status {st}; iterations {min(its)}..{max(its)}; "
        f"max residual {max(i['rel_kkt_residual'] for i in infos):.2e}; "
        f"{infos[0]['seconds']:.3f} s")
    assert st == lqgrid.OK
    assert all(i["status"] == lqgrid.OK and i["rel_kkt_residual"] <= tol for i in infos)
    order = sorted(range(len(probs)), key=lambda k: probs[k].unknowns)
    for k in order[:2] + order[-1:]:
        p = probs[k]
        ops = slab.SlabOperators(p)
        gate = residual.kkt_residual(ops, outs[k].cpu().numpy().reshape(p.T + 1, -1))
        say(f"  problem {k} (K={p.K} N={p.N} T={p.T}): oracle residual {gate['rel2']:.2e}")
        assert gate["rel2"] <= tol * 1.01


def test_batch_error_paths(lib, torch):
    from paper_2304_04980_amd import lqgrid
    probs = uneven_problems()[:3]
    # one indefinite weight: that problem reports ENOTSPD, the others solve
    bad = make_problem(3, 3, 10, 4, 2, seed=0)
    bad.Q[1, 1] = -np.eye(4)
    outs, infos, st = lqgrid.batch_solve(probs + [bad], opts=lqgrid.default_opts(tol=1e-8))
    assert st == lqgrid.ENOTSPD
    assert [i["status"] for i in infos] == [0, 0, 0, lqgrid.ENOTSPD]
    for p, d, info in zip(probs, outs, infos):
        check_against_oracle(p, d, info, 1e-8)
    # iteration cap
    outs, infos, st = lqgrid.batch_solve(
        probs, opts=lqgrid.default_opts(tol=1e-14, max_iter=3, check_every=1))
    assert st == lqgrid.ENOCONV
    assert all(i["status"] == lqgrid.ENOCONV and i["iterations"] == 3 for i in infos)
    # mixed state sizes and the FP32 form are not batched
    mixed = probs + [make_problem(3, 3, 10, 2, 1, seed=1)]
    _, _, st = lqgrid.batch_solve(mixed)
    assert st == lqgrid.EUNSUPPORTED
    _, _, st = lqgrid.batch_solve(probs, opts=lqgrid.default_opts(precision=lqgrid.FP32_REFINE))
    assert st == lqgrid.EUNSUPPORTED
