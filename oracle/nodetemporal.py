"""Alternative nesting: a block Jacobi preconditioner over the grid nodes
whose blocks are each node's whole temporal problem (every t at once).

The paper's preconditioner (Algorithm 2) splits Delta by time first (Psi~
holds the t-diagonal blocks) and by column pairs second; the innermost solves
are per (column pair, time) along the grid rows.  The other nesting keeps the
time axis whole and splits space instead: with D_node the part of Delta that
couples a node only to itself (its diagonal blocks Psi_hat_t[p,p] and its
temporal blocks Delta_{t+1,t}[p,p] = -A_hat_t[p,p] Q_{t,p}^-1 and their
transposes), each node's block of D_node is a block-tridiagonal n(T+1) x
n(T+1) matrix in time -- a single-node LQ problem's Schur complement -- and

    P^-1 r = D_node^-1 r

is one block Jacobi sweep.  D_node is a principal-block-diagonal part of the
positive definite Delta, hence positive definite, so P is a valid PCG
preconditioner (no even-L condition is needed).  The paper does not study
this nesting; it is the alternative its problem structure suggests (a
per-node temporal solve, like a Riccati sweep).

This module applies D_node^-1 with per-node banded Cholesky factorisations
(scipy ``cholesky_banded``, half-bandwidth 2n - 1 in (t, component) order).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def node_blocks_dense(p, Delta) -> sp.csr_matrix:
    """D_node from an explicit Delta (tiny problems): the entries of Delta
    whose row and column belong to the same grid node."""
    K, N, n = p.K, p.N, p.n
    KNn = K * N * n
    C = sp.coo_matrix(Delta)
    node_r = (C.row % KNn) // n
    node_c = (C.col % KNn) // n
    keep = node_r == node_c
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=Delta.shape)


class NodeTemporal:
    """D_node^-1 for ``slab.SlabOperators`` vectors (shape (T+1, KNn))."""

    def __init__(self, ops):
        self.ops = ops
        p = ops.p
        self.n, self.T, self.nodes = p.n, p.T, p.K * p.N
        n, T = self.n, self.T
        size = n * (T + 1)
        u = 2 * n - 1
        # the node's diagonal blocks over t and the blocks coupling t, t+1
        psi = [sp.csr_matrix(ops.psi_hat(t)) for t in range(T + 1)]
        sub = [sp.csr_matrix(-(ops.A_t(t) @ ops.Qinv_t(t))) for t in range(T)]
        self.factors = []
        for q in range(self.nodes):
            sl = slice(q * n, (q + 1) * n)
            M = np.zeros((size, size))
            for t in range(T + 1):
                M[t * n:(t + 1) * n, t * n:(t + 1) * n] = psi[t][sl, sl].toarray()
                if t < T:
                    E = sub[t][sl, sl].toarray()       # Delta_{t+1,t}[q,q]
                    M[(t + 1) * n:(t + 2) * n, t * n:(t + 1) * n] = E
                    M[t * n:(t + 1) * n, (t + 1) * n:(t + 2) * n] = E.T
            ab = np.zeros((u + 1, size))
            for k in range(u + 1):
                ab[u - k, k:] = np.diagonal(M, offset=k)
            self.factors.append(sla.cholesky_banded(ab, lower=False))

    def __call__(self, r: np.ndarray) -> np.ndarray:
        n, T = self.n, self.T
        out = np.empty_like(r)
        R = r.reshape(T + 1, self.nodes, n)
        O = out.reshape(T + 1, self.nodes, n)
        for q, cb in enumerate(self.factors):
            rhs = R[:, q, :].reshape(-1)
            O[:, q, :] = sla.cho_solve_banded((cb, False), rhs).reshape(T + 1, n)
        return out
