"""Stacked formulation of the grid LQ problem (Sec. II-A "Structured
Reformulation", Sec. II-B "KKT Conditions").

Ordering follows the paper's stacking exactly:
    x_bar_{j,t} = col_i x_{i,j,t}     (vertical stack, i = 1..K)
    x_hat_t     = col_j x_bar_{j,t}   (horizontal stack, j = 1..N)
    x_tilde     = col_t x_hat_t       (temporal stack, t = 0..T)
so (0-based) entry c of node (i, j) at time t sits at
    t*K*N*n + (j*K + i)*n + c.
The multiplier vector delta_tilde uses the same ordering.

Readings used here (the paper is garbled or silent at these points):
  * omega_tilde = col(gamma_hat, omega_hat_0, ..., omega_hat_{T-1}): the
    printed col(0, omega_hat_0, ...) with gamma_hat inside omega_hat_0
    would contradict x_{i,j,0} = gamma; the first block row of A_tilde is -I,
    so the constraint reads -x_hat_0 + gamma_hat = 0.  omega_hat_t holds the
    known boundary states' contribution to x_hat_{t+1} (M_hat alpha_hat_t +
    N_hat beta_hat_t): for node (i, j) the coupling blocks whose neighbour
    lies just outside the grid (G at i = 0, H at i = K-1, E at j = 0, F at
    j = N-1, 0-based) times that boundary state at time t; zero boundary
    states give omega_hat_t = 0.
  * r_delta = -omega_tilde (Sec. II-B).
  * Q_hat_T = Q_T, Q_hat_t = Q for t < T; R_tilde stops at t = T-1 because
    R_T = 0 removes u_T (Sec. II, after the cost).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def data(p, name: str, t: int):
    """The problem array `name` at time t: the array itself for time-invariant
    data, its slice t when the problem is time varying (A, A_nbr, B, Q, R
    carry a leading time index t = 0..T-1 there; Q_T has none)."""
    arr = getattr(p, name)
    return arr[t] if getattr(p, "time_varying", False) else arr


def node(i: int, j: int, K: int) -> int:
    """Position of node (i, j) inside x_hat_t (column j outermost)."""
    return j * K + i


def A_hat(p, t: int = 0) -> sp.csr_matrix:
    """A_hat_t: block tri-diagonal over columns j with block tri-diagonal
    diagonal blocks A_bar_j (Sec. II-A).  Block row of node (i,j): A at (i,j),
    E at (i,j-1), F at (i,j+1), G at (i-1,j), H at (i+1,j), each only when
    that neighbour lies inside the grid (the boundary states enter omega~)."""
    K, N, n = p.K, p.N, p.n
    Ad, An = data(p, "A", t), data(p, "A_nbr", t)
    rows, cols, vals = [], [], []

    def put(bi, bj, M):
        r0, c0 = bi * n, bj * n
        for a in range(n):
            for b in range(n):
                rows.append(r0 + a)
                cols.append(c0 + b)
                vals.append(M[a, b])

    for j in range(N):
        for i in range(K):
            me = node(i, j, K)
            put(me, me, Ad[j, i])
            if j - 1 >= 0:
                put(me, node(i, j - 1, K), An[j, i, 0])   # E
            if j + 1 < N:
                put(me, node(i, j + 1, K), An[j, i, 1])   # F
            if i - 1 >= 0:
                put(me, node(i - 1, j, K), An[j, i, 2])   # G
            if i + 1 < K:
                put(me, node(i + 1, j, K), An[j, i, 3])   # H
    KNn = K * N * n
    return sp.csr_matrix((vals, (rows, cols)), shape=(KNn, KNn))


def _blkdiag_nodes(p, blocks) -> sp.csr_matrix:
    """blkdiag over nodes in stacking order of blocks[j, i]."""
    mats = [blocks[j, i] for j in range(p.N) for i in range(p.K)]
    return sp.block_diag(mats, format="csr")


def B_hat(p, t: int = 0) -> sp.csr_matrix:
    return _blkdiag_nodes(p, data(p, "B", t))


def Q_hat(p, t: int) -> sp.csr_matrix:
    return _blkdiag_nodes(p, p.QT if t == p.T else data(p, "Q", t))


def Q_hat_inv(p, t: int) -> sp.csr_matrix:
    Qs = p.QT if t == p.T else data(p, "Q", t)
    return _blkdiag_nodes(p, np.linalg.inv(Qs))


def R_hat(p, t: int = 0) -> sp.csr_matrix:
    return _blkdiag_nodes(p, data(p, "R", t))


def R_hat_inv(p, t: int = 0) -> sp.csr_matrix:
    return _blkdiag_nodes(p, np.linalg.inv(data(p, "R", t)))


def gamma_hat(p) -> np.ndarray:
    """col_j col_i gamma_{i,j} -- x0 is stored [N][K][n], i.e. already in
    stacking order."""
    return np.asarray(p.x0, dtype=np.float64).reshape(-1).copy()


def omega_hat(p, t: int) -> np.ndarray:
    """Boundary contribution to x_hat_{t+1} (stacking order), t = 0..T-1,
    written out per node from eq. "2d_graph_dynamics"."""
    K, N, n = p.K, p.N, p.n
    An = data(p, "A_nbr", t)
    w = np.zeros((N, K, n))
    if getattr(p, "alpha_lo", None) is not None:
        for j in range(N):
            w[j, 0] += An[j, 0, 2] @ p.alpha_lo[t, j]        # G x_{0,j}
    if getattr(p, "alpha_hi", None) is not None:
        for j in range(N):
            w[j, K - 1] += An[j, K - 1, 3] @ p.alpha_hi[t, j]  # H x_{K+1,j}
    if getattr(p, "beta_lo", None) is not None:
        for i in range(K):
            w[0, i] += An[0, i, 0] @ p.beta_lo[t, i]         # E x_{i,0}
    if getattr(p, "beta_hi", None) is not None:
        for i in range(K):
            w[N - 1, i] += An[N - 1, i, 1] @ p.beta_hi[t, i]   # F x_{i,N+1}
    return w.reshape(-1)


def omega_tilde(p) -> np.ndarray:
    KNn = p.K * p.N * p.n
    omega = np.zeros((p.T + 1) * KNn)
    omega[:KNn] = gamma_hat(p)
    for t in range(p.T):
        omega[(t + 1) * KNn:(t + 2) * KNn] = omega_hat(p, t)
    return omega


def stacked(p) -> dict:
    """A_tilde, B_tilde, Q_tilde, R_tilde, omega_tilde, r_delta
    (eq. "t_stacked_LQ_problem" and the definitions after it)."""
    T = p.T
    tv = getattr(p, "time_varying", False)
    Ahs = [A_hat(p, t) for t in range(T)] if tv else [A_hat(p)] * T
    Bhs = [B_hat(p, t) for t in range(T)] if tv else [B_hat(p)] * T
    KNn = p.K * p.N * p.n
    KNm = p.K * p.N * p.m
    I = sp.identity(KNn, format="csr")
    # A_tilde: -I on the block diagonal, A_hat_t at block (t+1, t).
    blocks = [[None] * (T + 1) for _ in range(T + 1)]
    for t in range(T + 1):
        blocks[t][t] = -I
        if t >= 1:
            blocks[t][t - 1] = Ahs[t - 1]
    At = sp.bmat(blocks, format="csr")
    # B_tilde: B_hat_t at block (t+1, t), first block row zero.
    bb = [[None] * T for _ in range(T + 1)]
    for t in range(T):
        bb[t + 1][t] = Bhs[t]
    bb[0][0] = sp.csr_matrix((KNn, KNm))
    Bt = sp.bmat(bb, format="csr")
    Qt = sp.block_diag([Q_hat(p, t) for t in range(T + 1)], format="csr")
    Rt = sp.block_diag([R_hat(p, t) for t in range(T)], format="csr")
    omega = omega_tilde(p)
    return dict(At=At, Bt=Bt, Qt=Qt, Rt=Rt, omega=omega, r_delta=-omega)


def Q_tilde_inv(p) -> sp.csr_matrix:
    return sp.block_diag([Q_hat_inv(p, t) for t in range(p.T + 1)], format="csr")


def R_tilde_inv(p) -> sp.csr_matrix:
    return sp.block_diag([R_hat_inv(p, t) for t in range(p.T)], format="csr")


def delta_matrix(p, S: dict | None = None) -> sp.csr_matrix:
    """Delta = A~ Q~^-1 A~' + B~ R~^-1 B~'  (Sec. II-B, after eq.
    "block_tridiagonal_system")."""
    S = stacked(p) if S is None else S
    At, Bt = S["At"], S["Bt"]
    D = At @ Q_tilde_inv(p) @ At.T + Bt @ R_tilde_inv(p) @ Bt.T
    return sp.csr_matrix(D)


def r_delta(p) -> np.ndarray:
    """r_delta = -omega_tilde = col(-gamma_hat, -omega_hat_0, ...,
    -omega_hat_{T-1})."""
    return -omega_tilde(p)
