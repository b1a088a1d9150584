"""Primal recovery and the relative KKT residual (Sec. II-B).

    x~ = Q~^-1 A~' delta~,   u~ = R~^-1 B~' delta~
    rho = ( Q~ x~ - A~' delta~,  R~ u~ - B~' delta~,  A~ x~ + B~ u~ - r_delta )
    relative KKT residual = ||rho||_2 / ||r_delta||_2

(Schur-complement sign convention, see ``kkt``.)  The first two blocks vanish
up to rounding by construction, so the gate equals ||Delta delta~ - r_delta||_2
/ ||r_delta||_2 up to rounding.  The infinity norm (the paper's stopping norm)
is reported as well.

Vectors are arrays of shape (T+1, K*N*n) for delta~/x~ and (T, K*N*m) for u~,
in the paper's stacking order, so the [T+1][N][K][n] arrays of the library's
interface reshape onto them directly.
"""
from __future__ import annotations

import numpy as np

from .slab import SlabOperators


def recover(ops: SlabOperators, delta: np.ndarray):
    T = ops.T
    if ops.tv:
        X = np.empty_like(delta)
        for t in range(T + 1):
            a = -delta[t] + (ops.AT_t(t) @ delta[t + 1] if t < T else 0.0)
            X[t] = ops.Qinv_t(t) @ a
        U = np.stack([ops.Rinv_t(t) @ (ops.BT_t(t) @ delta[t + 1]) for t in range(T)])
        return X, U
    D = delta.T
    AtD = -D.copy()
    AtD[:, :T] += ops.AhT @ D[:, 1:]
    X = np.empty_like(AtD)
    X[:, :T] = ops.Qinv @ AtD[:, :T]
    X[:, T] = ops.QTinv @ AtD[:, T]
    U = ops.Rinv @ (ops.BhT @ D[:, 1:])
    return np.ascontiguousarray(X.T), np.ascontiguousarray(U.T)


def kkt_residual(ops: SlabOperators, delta: np.ndarray, x=None, u=None):
    """Relative KKT residual of a candidate delta~ (and optionally a given
    primal pair; by default the primal pair is recovered from delta~)."""
    T = ops.T
    if x is None or u is None:
        x, u = recover(ops, delta)
    if ops.tv:
        return _kkt_residual_tv(ops, delta, x, u)
    D, X, Uu = delta.T, x.T, u.T
    # block 1: Q~ x~ - A~' delta~
    Qx = np.empty_like(X)
    Qhat = ops_q(ops)
    Qx[:, :T] = Qhat[0] @ X[:, :T]
    Qx[:, T] = Qhat[1] @ X[:, T]
    AtD = -D.copy()
    AtD[:, :T] += ops.AhT @ D[:, 1:]
    r1 = Qx - AtD
    # block 2: R~ u~ - B~' delta~
    r2 = Qhat[2] @ Uu - ops.BhT @ D[:, 1:]
    # block 3: A~ x~ + B~ u~ - r_delta
    AX = -X.copy()
    AX[:, 1:] += ops.Ah @ X[:, :T] + ops.Bh @ Uu
    r3 = AX - ops.r_delta().T
    rd = ops.r_delta()
    nrd = np.linalg.norm(rd)
    tot = np.sqrt(np.sum(r1 ** 2) + np.sum(r2 ** 2) + np.sum(r3 ** 2))
    inf = max(np.max(np.abs(r1)), np.max(np.abs(r2)), np.max(np.abs(r3)))
    return dict(rel2=tot / nrd, inf=inf, rel_inf=inf / np.max(np.abs(rd)),
                schur_rel2=np.linalg.norm(r3) / nrd)


def ops_q(ops: SlabOperators):
    from . import stack
    if not hasattr(ops, "_qhat"):
        ops._qhat = (stack.Q_hat(ops.p, 0), stack.Q_hat(ops.p, ops.T),
                     stack.R_hat(ops.p))
    return ops._qhat


def _kkt_residual_tv(ops, delta, x, u):
    """kkt_residual for time-varying data (every slice matrix at its t)."""
    from . import stack
    p, T = ops.p, ops.T
    rd = ops.r_delta()
    r1 = np.empty_like(x)
    r3 = np.empty_like(x)
    r2 = np.empty_like(u)
    for t in range(T + 1):
        AtD = -delta[t] + (ops.AT_t(t) @ delta[t + 1] if t < T else 0.0)
        r1[t] = stack.Q_hat(p, t) @ x[t] - AtD
        AX = -x[t] + (ops.A_t(t - 1) @ x[t - 1] + ops.B_t(t - 1) @ u[t - 1] if t >= 1 else 0.0)
        r3[t] = AX - rd[t]
    for t in range(T):
        r2[t] = stack.R_hat(p, t) @ u[t] - ops.BT_t(t) @ delta[t + 1]
    nrd = np.linalg.norm(rd)
    tot = np.sqrt(np.sum(r1 ** 2) + np.sum(r2 ** 2) + np.sum(r3 ** 2))
    inf = max(np.max(np.abs(r1)), np.max(np.abs(r2)) if r2.size else 0.0, np.max(np.abs(r3)))
    return dict(rel2=tot / nrd, inf=inf, rel_inf=inf / np.max(np.abs(rd)),
                schur_rel2=np.linalg.norm(r3) / nrd)
