"""Special case K = N = 1: a single linear system, for which the LQ problem
(Sec. II, eq. "LQ_problem" with no neighbours) is solved by the textbook
backward Riccati recursion.  Used as an external pin of the whole solution.

    P_T = Q_T
    K_t = (R + B' P_{t+1} B)^-1 B' P_{t+1} A
    P_t = Q + A' P_{t+1} A - A' P_{t+1} B K_t
    u_t = -K_t x_t,  x_{t+1} = A x_t + B u_t,  x_0 = gamma
    optimal cost = 1/2 gamma' P_0 gamma

The Schur-complement multipliers then satisfy delta_t = -P_t x_t (from
Q_T x_T = -delta_T at the last stage and the costate recursion).
"""
from __future__ import annotations

import numpy as np


def lqr(A, B, Q, R, QT, x0, T):
    n = A.shape[0]
    P = [None] * (T + 1)
    Kg = [None] * T
    P[T] = QT.copy()
    for t in range(T - 1, -1, -1):
        Pn = P[t + 1]
        S = R + B.T @ Pn @ B
        Kg[t] = np.linalg.solve(S, B.T @ Pn @ A)
        P[t] = Q + A.T @ Pn @ A - A.T @ Pn @ B @ Kg[t]
        P[t] = 0.5 * (P[t] + P[t].T)
    x = np.zeros((T + 1, n))
    u = np.zeros((T, B.shape[1]))
    x[0] = x0
    for t in range(T):
        u[t] = -Kg[t] @ x[t]
        x[t + 1] = A @ x[t] + B @ u[t]
    delta = np.stack([-P[t] @ x[t] for t in range(T + 1)])
    cost = 0.5 * x0 @ P[0] @ x0
    return dict(x=x, u=u, delta=delta, P=P, cost=cost)


def lqr_of_problem(p):
    assert p.K == 1 and p.N == 1, "Riccati pin needs a single node"
    return lqr(p.A[0, 0], p.B[0, 0], p.Q[0, 0], p.R[0, 0], p.QT[0, 0],
               p.x0[0, 0], p.T)


def lqr_tv(As, Bs, Qs, Rs, QT, x0):
    """The same recursion with time-varying A_t, B_t, Q_t, R_t (lists over
    t = 0..T-1): P_T = Q_T, K_t = (R_t + B_t' P_{t+1} B_t)^-1 B_t' P_{t+1} A_t,
    P_t = Q_t + A_t' P_{t+1} A_t - A_t' P_{t+1} B_t K_t."""
    T = len(As)
    n = As[0].shape[0]
    P = [None] * (T + 1)
    Kg = [None] * T
    P[T] = QT.copy()
    for t in range(T - 1, -1, -1):
        A, B, Pn = As[t], Bs[t], P[t + 1]
        S = Rs[t] + B.T @ Pn @ B
        Kg[t] = np.linalg.solve(S, B.T @ Pn @ A)
        P[t] = Qs[t] + A.T @ Pn @ A - A.T @ Pn @ B @ Kg[t]
        P[t] = 0.5 * (P[t] + P[t].T)
    x = np.zeros((T + 1, n))
    u = np.zeros((T, Bs[0].shape[1]))
    x[0] = x0
    for t in range(T):
        u[t] = -Kg[t] @ x[t]
        x[t + 1] = As[t] @ x[t] + Bs[t] @ u[t]
    delta = np.stack([-P[t] @ x[t] for t in range(T + 1)])
    return dict(x=x, u=u, delta=delta, P=P, cost=0.5 * x0 @ P[0] @ x0)


def lqr_of_tv_problem(p):
    assert p.K == 1 and p.N == 1 and p.time_varying
    T = p.T
    return lqr_tv([p.A[t, 0, 0] for t in range(T)], [p.B[t, 0, 0] for t in range(T)],
                  [p.Q[t, 0, 0] for t in range(T)], [p.R[t, 0, 0] for t in range(T)],
                  p.QT[0, 0], p.x0[0, 0])
