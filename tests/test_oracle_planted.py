"""Planted mistakes: each test breaks the oracle on the CPU in one plausible
way and checks that an independent pin notices.  This is evidence that the
pins in test_oracle_pins.py constrain the oracle, not a test of the oracle's
correct behaviour (that is test_oracle_pins.py)."""
import numpy as np
import pytest

from lqgrid_synth import make_problem, config_problem
from oracle import stack, kkt, splitting, slab, nbjm, pcg
from test_oracle_pins import simulate, shapes


def test_swapped_east_west_coupling_is_caught(monkeypatch):
    p = make_problem(3, 4, 6, 2, 1, seed=1)
    good = kkt.solve_kkt(p)
    x, u = shapes(p, good)
    assert np.abs(simulate(p, u) - x).max() < 1e-10
    q = make_problem(3, 4, 6, 2, 1, seed=1)
    q.A_nbr = q.A_nbr[:, :, [1, 0, 2, 3]].copy()      # E <-> F in the oracle's input
    real_A_hat = stack.A_hat
    monkeypatch.setattr(stack, "A_hat", lambda _p: real_A_hat(q))
    bad = kkt.solve_kkt(p)
    xb, ub = shapes(p, bad)
    assert np.abs(simulate(p, ub) - xb).max() > 1e-3


def test_flipped_omega_sign_is_caught():
    p = make_problem(3, 4, 3, 2, 1, rho=0.5, seed=9)
    s = splitting.splittings(p)
    s_bad = dict(s, Omega=-s["Omega"])
    Dinv = np.linalg.inv(s["Delta"].toarray())
    good = splitting.preconditioner_inverse(s, 600, 30)
    bad = splitting.preconditioner_inverse(s_bad, 600, 30)
    assert np.abs(good - Dinv).max() <= 1e-9 * np.abs(Dinv).max()
    assert np.abs(bad - Dinv).max() > 1e-3 * np.abs(Dinv).max()


def test_flipped_xi_sign_is_caught():
    p = make_problem(3, 4, 3, 2, 1, rho=0.5, seed=9)
    s = splitting.splittings(p)
    s_bad = dict(s, Xi=-s["Xi"])
    Dinv = np.linalg.inv(s["Delta"].toarray())
    bad = splitting.preconditioner_inverse(s_bad, 600, 30)
    assert np.abs(bad - Dinv).max() > 1e-3 * np.abs(Dinv).max()


def test_printed_direction_update_is_caught():
    """The literal direction update d = r + beta d (instead of q + beta d)
    fails to reach the dense solution within the iteration budget."""
    p, tol = config_problem("tiny", 0)
    ops = slab.SlabOperators(p)
    pre = nbjm.slab_preconditioner(ops, 2, 2)
    rd = ops.r_delta()
    ds = kkt.solve_schur_dense(p).reshape(rd.shape)

    def literal_pcg(max_iter=300):
        x = np.zeros_like(rd)
        r = rd.copy()
        d = pre(r)
        mu = np.vdot(d, r)
        for _ in range(max_iter):
            y = ops.delta(d)
            th = mu / np.vdot(y, d)
            x += th * d
            r -= th * y
            q = pre(r)
            mu2 = np.vdot(q, r)
            d = r + (mu2 / mu) * d
            mu = mu2
        return x

    xg, it, _ = pcg.pcg(ops.delta, pre, rd, tol=tol)
    assert np.linalg.norm(xg - ds) <= 1e-8 * np.linalg.norm(ds)
    xl = literal_pcg()
    assert np.linalg.norm(xl - ds) > 1e-6 * np.linalg.norm(ds)


def test_missing_terminal_weight_is_caught(monkeypatch):
    """Using Q instead of Q_T at t = T breaks the Riccati pin."""
    from oracle import riccati
    p = make_problem(1, 1, 10, 2, 1, rho=1.1, seed=2, qt_scale=5.0)
    R = riccati.lqr_of_problem(p)
    monkeypatch.setattr(stack, "Q_hat", lambda _p, t: stack._blkdiag_nodes(_p, _p.Q))
    bad = kkt.solve_kkt(p)
    assert np.abs(bad["x"].reshape(11, 2) - R["x"]).max() > 1e-4
