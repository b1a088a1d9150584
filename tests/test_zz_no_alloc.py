"""The allocation-free entry point lqgrid_solve_noalloc (static device
scratch) against the entry points it replaces (lqgrid_setup + lqgrid_factor +
lqgrid_pcg_solve on a caller workspace), called through the C ABI.

Both run the same kernels with the same launch shapes on the same inputs and
every reduction has a fixed order, so the outputs are expected to be
identical; the bound asserted is the FP64 operator bound of the parity tests
(1e-12 of the largest entry), with equal iteration counts.  Two calls in a
row, the second on a smaller problem (the scratch keeps the first call's
contents, which the second must not see), then an oversized problem, which
is rejected with LQGRID_EWORKSPACE before any device work.
"""
import sys

import numpy as np
import pytest

from lqgrid_synth import make_problem
from oracle import slab, residual

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def noalloc_solve(torch, L, p, opts):
    from paper_2304_04980_amd import lqgrid
    f64 = dict(dtype=torch.float64, device="cuda")
    a = {k: torch.as_tensor(getattr(p, k)).to(**f64).contiguous()
         for k in ("A", "A_nbr", "B", "Q", "R", "QT")}
    x0 = torch.as_tensor(p.x0).to(**f64).contiguous()
    desc = lqgrid.problem_desc(p.K, p.N, p.T, p.n, p.m, a["A"], a["A_nbr"], a["B"],
                               a["Q"], a["R"], a["QT"])
    d = torch.full((p.T + 1, p.N, p.K, p.n), float("nan"), **f64)
    x = torch.full((p.T + 1, p.N, p.K, p.n), float("nan"), **f64)
    u = torch.full((p.T, p.N, p.K, p.m), float("nan"), **f64)
    st, info = lqgrid.solve_noalloc(desc, x0, opts, d, x, u)
    torch.cuda.synchronize()
    return st, d, x, u, info


def reference_solve(torch, p, opts):
    from paper_2304_04980_amd import lqgrid
    ctx = lqgrid.Context(p)
    d, x, u, info = ctx.solve(torch.as_tensor(p.x0), opts, want_primal=True)
    torch.cuda.synchronize()
    ctx.close()
    return d, x, u, info


def test_noalloc_matches_workspace_entry_points(lib, torch):
    from paper_2304_04980_amd import lqgrid
    L = lib
    cap = L.lqgrid_noalloc_capacity()
    say(f"noalloc capacity {cap / 2**20:.1f} MiB")
    cases = [((24, 20, 100, 4, 2), 1e-10, lqgrid.FP64),   # twisted order, 3 time tiles
             ((6, 5, 40, 3, 2), 1e-8, lqgrid.FP32_REFINE)]  # smaller, odd N, one-chain
    for (K, N, T, n, m), tol, prec in cases:
        p = make_problem(K, N, T, n, m, seed=K + N + T, qt_scale=1.5, weights="spd")
        need = lqgrid.workspace_bytes(K, N, T, n, m)
        assert need <= cap
        opts = lqgrid.default_opts(tol=tol, precision=prec, inner_tol=1e-4)
        say(f"case K={K} N={N} T={T} n={n} m={m} precision {prec}: scratch {need} bytes")
        st, d, x, u, info = noalloc_solve(torch, L, p, opts)
        assert st == lqgrid.OK, lqgrid.LqgridError(st, "lqgrid_solve_noalloc")
        dr, xr, ur, ir = reference_solve(torch, p, opts)
        same = torch.equal(d, dr) and torch.equal(x, xr) and torch.equal(u, ur)
        errs = [float((a - b).abs().max() / b.abs().max()) for a, b in
                ((d, dr), (x, xr), (u, ur))]
        say(f"  noalloc {info['iterations']} it res {info['rel_kkt_residual']:.3e}; "
            f"workspace path {ir['iterations']} it; bitwise equal {same}; rel errs {errs}")
        assert info["iterations"] == ir["iterations"]
        assert max(errs) <= 1e-12
        ops = slab.SlabOperators(p)
        g = residual.kkt_residual(ops, d.cpu().numpy().reshape(T + 1, -1),
                                  x.cpu().numpy().reshape(T + 1, -1),
                                  u.cpu().numpy().reshape(T, -1))
        say(f"  oracle residual {g['rel2']:.3e}")
        assert g["rel2"] <= 1.01 * tol


def test_noalloc_rejects_oversized_problem(lib, torch):
    from paper_2304_04980_amd import lqgrid
    L = lib
    cap = L.lqgrid_noalloc_capacity()
    p = make_problem(64, 64, 100, 4, 2, seed=0)
    assert lqgrid.workspace_bytes(64, 64, 100, 4, 2) > cap
    st, d, _, _, _ = noalloc_solve(torch, L, p, lqgrid.default_opts(tol=1e-8))
    assert st == lqgrid.EWORKSPACE
    msg = L.lqgrid_last_error().decode()
    say("  rejected:", msg)
    assert "scratch" in msg
    assert bool(torch.isnan(d).all())   # nothing was written
