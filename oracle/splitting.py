"""Explicit splittings of Delta and the closed forms of Sec. IV.

    Delta = Psi~ - Xi~,   Psi~ = blkdiag_t(Psi_hat_t),  Xi~ = Psi~ - Delta
                                                    (eq. "splitting_Delta")
    Psi~  = Phi~ - Omega~, Phi~ = blkdiag_{t,v}(Phi_bar_{v,t}),
                           Omega~ = Phi~ - Psi~     (eq. "splitting_Psi")
    Upsilon_L = sum_{l<L} (Phi~^-1 Omega~)^l Phi~^-1            (Lemma 1)
    P_S^-1    = sum_{s<S} (Upsilon_L Xi~)^s Upsilon_L           (Theorem 2)

Readings:
  * Phi_bar_{v,t} is the diagonal super-block of Psi_hat_t over the column
    pair (2v-1, 2v) (1-based), the last column alone when N is odd; the
    printed "V even / V odd" cases are read as "N even / N odd", and the
    printed formulas for Z_bar, Y_bar, V_bar are read as "the exact sub-blocks
    of Psi_hat_t" (they omit Q^-1 and B R^-1 B' and mix time indices).
  * Signs come only from the definitions Xi~ = Psi~ - Delta and
    Omega~ = Phi~ - Psi~ (the drawn blocks of eq. "structure_of_Psi_t" and
    eq. "structure_of_Delta" carry the opposite sign).
These matrices are U x U; use them on small problems only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import stack


def index_maps(p):
    """For every unknown: its time t and its super-column v (0-based)."""
    K, N, n, T = p.K, p.N, p.n, p.T
    KNn = K * N * n
    idx = np.arange((T + 1) * KNn)
    t = idx // KNn
    j = (idx % KNn) // (K * n)
    v = j // 2
    return t, v


def _mask(M: sp.spmatrix, keep_fn) -> sp.csr_matrix:
    C = sp.coo_matrix(M)
    keep = keep_fn(C.row, C.col)
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])),
                         shape=M.shape)


def splittings(p, Delta: sp.spmatrix | None = None) -> dict:
    D = stack.delta_matrix(p) if Delta is None else sp.csr_matrix(Delta)
    t, v = index_maps(p)
    Psi = _mask(D, lambda r, c: t[r] == t[c])
    Xi = sp.csr_matrix(Psi - D)
    Phi = _mask(Psi, lambda r, c: v[r] == v[c])
    Omega = sp.csr_matrix(Phi - Psi)
    return dict(Delta=D, Psi=Psi, Xi=Xi, Phi=Phi, Omega=Omega)


def upsilon(Phi, Omega, L: int) -> np.ndarray:
    """Lemma 1: Upsilon_L = sum_{l=0}^{L-1} (Phi^-1 Omega)^l Phi^-1."""
    Phid, Omd = _dense(Phi), _dense(Omega)
    Phi_inv = np.linalg.inv(Phid)
    G = Phi_inv @ Omd
    term = Phi_inv.copy()
    acc = np.zeros_like(Phi_inv)
    for _ in range(L):
        acc += term
        term = G @ term
    return acc


def preconditioner_inverse(spl: dict, S: int, L: int) -> np.ndarray:
    """Theorem 2: P_S^-1 = sum_{s=0}^{S-1} (Upsilon_L Xi)^s Upsilon_L."""
    U = upsilon(spl["Phi"], spl["Omega"], L)
    H = U @ _dense(spl["Xi"])
    term = U.copy()
    acc = np.zeros_like(U)
    for _ in range(S):
        acc += term
        term = H @ term
    return acc


def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)
