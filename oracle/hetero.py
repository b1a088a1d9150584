"""Heterogeneous sub-system sizes (Sec. II: x_{i,j,t} in R^{n_{i,j}},
u_{i,j,t} in R^{m_{i,j}}): the KKT system of eq. "LQ_problem" assembled
with per-node block sizes and solved by the dense LDL' of ``kkt`` (tiny
problems only).

The problem arrays use the padded layouts of the library's interface
(A [N][K][n][n], A_nbr [N][K][4][n][n], B [N][K][n][m], Q, QT [N][K][n][n],
R [N][K][m][m], x0 [N][K][n] with n = max n_{i,j}, m = max m_{i,j}); only
the leading n_p x n_q (n_p x m_p, ...) part of each block belongs to the
problem and nothing else is read here.  The stacking is the paper's (node
(i, j) at position j K + i inside each time slice) with variable block
sizes, so this module shares no layout with the padded formulation: the
tests compare its solution with a padded solve entry by entry.
Zero spatial boundary states.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import kkt


def _offsets(sizes):
    off = np.zeros(len(sizes) + 1, dtype=int)
    off[1:] = np.cumsum(sizes)
    return off


def solve(p, n_node, m_node) -> dict:
    """Returns delta~, x~, u~ in padded arrays ([T+1][N][K][n], same,
    [T][N][K][m]; entries past a node's size are zero) and in the compressed
    stacking."""
    K, N, T = p.K, p.N, p.T
    ns = [int(n_node[j, i]) for j in range(N) for i in range(K)]
    ms = [int(m_node[j, i]) for j in range(N) for i in range(K)]
    on, om = _offsets(ns), _offsets(ms)
    X, Uu = on[-1], om[-1]              # states / inputs per time slice
    nx, nu = (T + 1) * X, T * Uu

    def node(i, j):
        return j * K + i

    # A_hat (X x X), B_hat (X x Uu) with per-node blocks
    Ah = np.zeros((X, X))
    Bh = np.zeros((X, Uu))
    Qd = np.zeros((X, X))
    QTd = np.zeros((X, X))
    Rd = np.zeros((Uu, Uu))
    for j in range(N):
        for i in range(K):
            a = node(i, j)
            na, ma = ns[a], ms[a]
            ra = slice(on[a], on[a] + na)
            Ah[ra, ra] = p.A[j, i][:na, :na]
            for slot, (ii, jj) in enumerate([(i, j - 1), (i, j + 1), (i - 1, j), (i + 1, j)]):
                if 0 <= ii < K and 0 <= jj < N:
                    b = node(ii, jj)
                    Ah[ra, on[b]:on[b] + ns[b]] = p.A_nbr[j, i, slot][:na, :ns[b]]
            Bh[ra, om[a]:om[a] + ma] = p.B[j, i][:na, :ma]
            Qd[ra, ra] = p.Q[j, i][:na, :na]
            QTd[ra, ra] = p.QT[j, i][:na, :na]
            Rd[om[a]:om[a] + ma, om[a]:om[a] + ma] = p.R[j, i][:ma, :ma]
    I = np.eye(X)
    At = np.zeros((nx, nx))
    Bt = np.zeros((nx, nu))
    for t in range(T + 1):
        At[t * X:(t + 1) * X, t * X:(t + 1) * X] = -I
        if t >= 1:
            At[t * X:(t + 1) * X, (t - 1) * X:t * X] = Ah
            Bt[t * X:(t + 1) * X, (t - 1) * Uu:t * Uu] = Bh
    Qt = sp.block_diag([Qd] * T + [QTd]).toarray()
    Rt = sp.block_diag([Rd] * T).toarray() if T > 0 else np.zeros((0, 0))
    gamma = np.concatenate([p.x0[j, i][:ns[node(i, j)]] for j in range(N) for i in range(K)])
    rd = np.zeros(nx)
    rd[:X] = -gamma
    M = np.block([[Qt, np.zeros((nx, nu)), At.T],
                  [np.zeros((nu, nx)), Rt, Bt.T],
                  [At, Bt, np.zeros((nx, nx))]])
    z = kkt.ldl_solve(M, np.concatenate([np.zeros(nx + nu), rd]))
    x, u, delta = z[:nx], z[nx:nx + nu], -z[nx + nu:]

    def pad(v, sizes, off, width, steps):
        out = np.zeros((steps, N, K, width))
        per = off[-1]
        for t in range(steps):
            for j in range(N):
                for i in range(K):
                    a = node(i, j)
                    out[t, j, i, :sizes[a]] = v[t * per + off[a]:t * per + off[a] + sizes[a]]
        return out

    return dict(delta=pad(delta, ns, on, p.n, T + 1), x=pad(x, ns, on, p.n, T + 1),
                u=pad(u, ms, om, p.m, T), delta_c=delta, x_c=x, u_c=u,
                residual=np.linalg.norm(M @ z - np.concatenate([np.zeros(nx + nu), rd])))
