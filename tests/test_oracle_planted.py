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


def test_weight_of_the_wrong_node_is_caught(monkeypatch):
    """With per-node SPD weights, a Q^-1 taken from the wrong node (the node
    order of the weight blocks reversed) breaks the node-level feasibility
    pin of the KKT solution."""
    p = make_problem(3, 4, 6, 2, 1, seed=3, weights="spd")
    good = kkt.solve_kkt(p)
    x, u = shapes(p, good)
    assert np.abs(simulate(p, u) - x).max() < 1e-10
    real = stack._blkdiag_nodes

    def reversed_nodes(_p, blocks):
        flip = blocks[::-1, ::-1].copy() if blocks.shape[-1] == _p.n else blocks
        return real(_p, flip)

    monkeypatch.setattr(stack, "_blkdiag_nodes", reversed_nodes)
    bad = kkt.solve_kkt(p)
    xb, ub = shapes(p, bad)
    # the wrong weights give another (feasible) trajectory: its cost is higher
    from test_oracle_pins import cost
    assert cost(p, xb, ub) > cost(p, x, u) * (1 + 1e-6)


def test_boundary_state_on_the_wrong_edge_is_caught(monkeypatch):
    """Boundary states of the north edge fed through the south coupling (G
    and H swapped in the boundary term of omega~) break the node-level
    feasibility pin."""
    p = make_problem(4, 3, 6, 2, 1, seed=5, boundary=True)
    good = kkt.solve_kkt(p)
    x, u = shapes(p, good)
    assert np.abs(simulate(p, u) - x).max() < 1e-10
    q = make_problem(4, 3, 6, 2, 1, seed=5, boundary=True)
    q.alpha_lo, q.alpha_hi = p.alpha_hi, p.alpha_lo
    real = stack.omega_hat
    monkeypatch.setattr(stack, "omega_hat", lambda _p, t: real(q, t))
    bad = kkt.solve_kkt(p)
    xb, ub = shapes(p, bad)
    assert np.abs(simulate(p, ub) - xb).max() > 1e-3


# ------------------------------------------------------------ warm start
def _fd_check_fails(monkeypatch_fn=None):
    """Runs the network finite-difference pin; returns True when it fails."""
    import test_oracle_warmstart as t
    try:
        t.test_network_gradient_matches_finite_differences()
    except AssertionError:
        return True
    return False


def test_flipped_input_gradient_tap_is_caught(monkeypatch):
    from oracle import warmstart as ws
    real = ws.conv3x3_backward

    def bad(x, W, dy):
        dW, db, dx = real(x, W[:, ::-1, ::-1, :].copy(), dy)   # taps not flipped back
        return real(x, W, dy)[0], db, dx
    monkeypatch.setattr(ws, "conv3x3_backward", bad)
    assert _fd_check_fails()


def test_missing_relu_mask_is_caught(monkeypatch):
    from oracle import warmstart as ws
    real_forward = ws.forward

    def no_mask_backward(params, x, acts, dout, round_bf16=False):
        grads = [None] * len(params)
        dy = dout
        for li in range(len(params) - 1, -1, -1):
            xin = x if li == 0 else acts[li - 1]
            dW, db, dx = ws.conv3x3_backward(xin, params[li][0], dy)
            grads[li] = (dW, db)
            dy = dx                                  # ReLU mask dropped
        return grads
    monkeypatch.setattr(ws, "backward", no_mask_backward)
    assert real_forward is ws.forward
    assert _fd_check_fails()


def test_wrong_chebyshev_recurrence_is_caught(monkeypatch):
    from oracle import warmstart as ws
    import test_oracle_warmstart as t

    def bad_basis(T, k):
        tau = 2.0 * np.arange(T + 1) / T - 1.0
        B = np.empty((T + 1, k))
        B[:, 0] = 1.0
        B[:, 1] = tau
        for c in range(2, k):
            B[:, c] = tau * B[:, c - 1] - B[:, c - 2]      # factor 2 dropped
        return B
    monkeypatch.setattr(ws, "cheb_basis", bad_basis)
    with pytest.raises(AssertionError):
        t.test_chebyshev_basis_matches_numpy_chebval()


def test_truncating_bf16_is_caught(monkeypatch):
    from oracle import warmstart as ws
    import test_oracle_warmstart as t

    def trunc(x):
        f = np.asarray(x, dtype=np.float32)
        u = (f.view(np.uint32) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    monkeypatch.setattr(ws, "bf16", trunc)
    with pytest.raises(AssertionError):
        t.test_bf16_rounding()
