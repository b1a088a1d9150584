"""Bitwise reproducibility of the single-problem path: every reduction on the
device has a fixed order (wavefront shuffles, one partial per workgroup, a
fixed-order sum of the partials), no atomics accumulate floating point, and
the iteration count is decided on the device, so two solves of the same
problem, each from its own setup, must agree bit for bit in delta~, x~, u~
and in the number of iterations.  Covered: FP64 and FP32 sweeps inside FP64
refinement with the paper's preconditioner, the node-temporal preconditioner,
and time-varying data."""
import sys

import numpy as np
import pytest

from lqgrid_synth import config_problem, make_problem

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def solve_twice(torch, p, opts, node_temporal=False):
    from paper_2304_04980_amd import lqgrid
    runs = []
    for _ in range(2):
        ctx = lqgrid.Context(p, node_temporal=node_temporal)
        d, x, u, info = ctx.solve(p.x0, opts, want_primal=True)
        torch.cuda.synchronize()
        runs.append((d.cpu().numpy(), x.cpu().numpy(), u.cpu().numpy(), info))
        ctx.close()
    return runs


def check_identical(runs, tol, label):
    (d1, x1, u1, i1), (d2, x2, u2, i2) = runs
    say(f"{label}: {i1['iterations']} / {i2['iterations']} it, "
        f"res {i1['rel_kkt_residual']:.2e}")
    assert i1["status"] == 0 and i1["rel_kkt_residual"] <= tol
    assert i1["iterations"] == i2["iterations"]
    assert i1["refinements"] == i2["refinements"]
    for a, b in ((d1, d2), (x1, x2), (u1, u2)):
        assert np.array_equal(a, b)  # bitwise: the same floats in the same places


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_repeated_solves_are_identical(lib, torch, precision):
    from paper_2304_04980_amd import lqgrid
    p, tol = config_problem("plain", 0)
    kw = {} if precision == "fp64" else dict(precision=lqgrid.FP32_REFINE)
    opts = lqgrid.default_opts(tol=tol, **kw)
    check_identical(solve_twice(torch, p, opts), tol, f"32x32x100 {precision}")


def test_repeated_node_temporal_solves_are_identical(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p, _ = config_problem("plain", 0)
    opts = lqgrid.default_opts(tol=1e-8, preconditioner=lqgrid.PRECOND_NODE_TEMPORAL,
                               precision=lqgrid.FP32_REFINE)
    check_identical(solve_twice(torch, p, opts, node_temporal=True), 1e-8,
                    "32x32x100 node-temporal fp32r")


def test_repeated_time_varying_solves_are_identical(lib, torch):
    from paper_2304_04980_amd import lqgrid
    p = make_problem(12, 9, 70, 4, 2, seed=5, weights="spd", time_varying=True)
    opts = lqgrid.default_opts(tol=1e-9)
    check_identical(solve_twice(torch, p, opts), 1e-9, "12x9x70 time-varying fp64")
