"""The operators of Secs. II-B and IV applied one time slice at a time.

The full U x U matrices of ``stack``/``splitting`` do not fit for large grids;
here every operator is built from the slice matrices A_hat, B_hat, Q_hat^-1,
R_hat^-1 (size K*N*n) and applied to a vector held as an array of shape
(T+1, K*N*n) in the paper's stacking order (row t = delta_hat_t).

  Delta d   = A~ (Q~^-1 (A~' d)) + B~ (R~^-1 (B~' d))          (Sec. II-B)
              with (A~' d)_t = -d_t + A_hat' d_{t+1} (t < T), -d_T;
                   (A~ w)_0 = -w_0, (A~ w)_t = A_hat w_{t-1} - w_t;
                   (B~' d)_t = B_hat' d_{t+1} (t < T);
                   (B~ z)_0 = 0,    (B~ z)_t = B_hat z_{t-1}.
  Psi_hat_0 = Q_hat_0^-1,
  Psi_hat_t = Q_hat_t^-1 + A_hat Q_hat_{t-1}^-1 A_hat' + B_hat R_hat^-1 B_hat'
                                             (eq. "structure_of_Delta")
  Xi~ d     = Psi~ d - Delta d                 (eq. "splitting_Delta")
  Phi_hat_t = Psi_hat_t restricted to the column-pair diagonal super-blocks,
  Omega_hat_t = Phi_hat_t - Psi_hat_t          (eq. "splitting_Psi")
  Phi_hat_t^-1 tau: V independent solves with Phi_bar_{v,t}
                                             (eq. "decomposed_problem")

Phi_bar_{v,t} solves use a banded Cholesky factorisation (scipy
``cholesky_banded``) after ordering the unknowns of the super-column as
(i, column-in-pair, component): in that order Phi_bar_{v,t} is banded with
half-bandwidth 3*w*n - 1 (w = columns in the pair), because Psi_hat_t couples
nodes at Manhattan distance <= 2 only.  The paper only says "block Cholesky";
any exact solver gives the same result up to rounding.

For time-invariant data Psi_hat_t takes three values: t = 0, 1 <= t <= T-1
and t = T (the latter differs through Q_T).  For time-varying data (Sec. II:
A_{i,j,t}, B_{i,j,t}, E...H_{i,j,t}, Q_{i,j,t}, R_{i,j,t}) every slice
matrix carries its time index -- A_hat_t, B_hat_t, Q_hat_t, R_hat_t -- and

  (A~' d)_t = -d_t + A_hat_t' d_{t+1},  (A~ w)_t = A_hat_{t-1} w_{t-1} - w_t,
  (B~' d)_t = B_hat_t' d_{t+1},         (B~ z)_t = B_hat_{t-1} z_{t-1},
  Psi_hat_t = Q_hat_t^-1 + A_hat_{t-1} Q_hat_{t-1}^-1 A_hat_{t-1}'
              + B_hat_{t-1} R_hat_{t-1}^-1 B_hat_{t-1}'   (t >= 1),

so every t is a class of its own.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import stack


def time_class(t: int, T: int) -> int:
    return 0 if t == 0 else (2 if t == T else 1)


class SlabOperators:
    def __init__(self, p):
        self.p = p
        self.K, self.N, self.n, self.T = p.K, p.N, p.n, p.T
        self.KNn = p.K * p.N * p.n
        self.tv = bool(getattr(p, "time_varying", False))
        self.QTinv = stack.Q_hat_inv(p, p.T)       # Q_hat_T^-1
        if self.tv:
            T = p.T
            self.Ahs = [stack.A_hat(p, t) for t in range(T)]
            self.AhTs = [sp.csr_matrix(A.T) for A in self.Ahs]
            self.Bhs = [stack.B_hat(p, t) for t in range(T)]
            self.BhTs = [sp.csr_matrix(B.T) for B in self.Bhs]
            self.Qinvs = [stack.Q_hat_inv(p, t) for t in range(T)] + [self.QTinv]
            self.Rinvs = [stack.R_hat_inv(p, t) for t in range(T)]
        else:
            self.Ah = stack.A_hat(p)
            self.AhT = sp.csr_matrix(self.Ah.T)
            self.Bh = stack.B_hat(p)
            self.BhT = sp.csr_matrix(self.Bh.T)
            self.Qinv = stack.Q_hat_inv(p, 0)          # Q_hat_t^-1, t < T
            self.Rinv = stack.R_hat_inv(p)
        self._psi, self._phi, self._omega, self._chol = {}, {}, {}, {}
        # column of every slice unknown, and its super-column
        idx = np.arange(self.KNn)
        self.col = idx // (self.K * self.n)
        self.sup = self.col // 2
        self.V = (self.N + 1) // 2

    # -- slice matrices -------------------------------------------------
    def Qinv_t(self, t):
        if self.tv:
            return self.Qinvs[t]
        return self.QTinv if t == self.T else self.Qinv

    def A_t(self, t):
        return self.Ahs[t] if self.tv else self.Ah

    def AT_t(self, t):
        return self.AhTs[t] if self.tv else self.AhT

    def B_t(self, t):
        return self.Bhs[t] if self.tv else self.Bh

    def BT_t(self, t):
        return self.BhTs[t] if self.tv else self.BhT

    def Rinv_t(self, t):
        return self.Rinvs[t] if self.tv else self.Rinv

    def cls(self, t):
        return t if self.tv else time_class(t, self.T)

    def psi_hat(self, t) -> sp.csr_matrix:
        c = self.cls(t)
        if c not in self._psi:
            if t == 0:
                M = self.Qinv_t(0)
            else:
                M = (self.Qinv_t(t) + self.A_t(t - 1) @ self.Qinv_t(t - 1) @ self.AT_t(t - 1)
                     + self.B_t(t - 1) @ self.Rinv_t(t - 1) @ self.BT_t(t - 1))
            self._psi[c] = sp.csr_matrix(M)
        return self._psi[c]

    def phi_hat(self, t) -> sp.csr_matrix:
        c = self.cls(t)
        if c not in self._phi:
            C = sp.coo_matrix(self.psi_hat(t))
            keep = self.sup[C.row] == self.sup[C.col]
            self._phi[c] = sp.csr_matrix(
                (C.data[keep], (C.row[keep], C.col[keep])), shape=C.shape)
        return self._phi[c]

    def omega_hat(self, t) -> sp.csr_matrix:
        c = self.cls(t)
        if c not in self._omega:
            self._omega[c] = sp.csr_matrix(self.phi_hat(t) - self.psi_hat(t))
        return self._omega[c]

    # -- operators on (T+1, KNn) arrays ---------------------------------
    def delta(self, d: np.ndarray) -> np.ndarray:
        T = self.T
        if self.tv:
            W = np.empty_like(d)
            for t in range(T + 1):
                a = -d[t] + (self.AT_t(t) @ d[t + 1] if t < T else 0.0)
                W[t] = self.Qinv_t(t) @ a
            Y = -W.copy()
            for t in range(1, T + 1):
                z = self.Rinv_t(t - 1) @ (self.BT_t(t - 1) @ d[t])
                Y[t] += self.A_t(t - 1) @ W[t - 1] + self.B_t(t - 1) @ z
            return Y
        D = d.T                                   # (KNn, T+1)
        AtD = -D.copy()
        AtD[:, :T] += self.AhT @ D[:, 1:]         # (A~' d)_t
        W = np.empty_like(AtD)
        W[:, :T] = self.Qinv @ AtD[:, :T]
        W[:, T] = self.QTinv @ AtD[:, T]
        Z = self.Rinv @ (self.BhT @ D[:, 1:])     # R~^-1 B~' d, t = 0..T-1
        Y = -W.copy()
        Y[:, 1:] += self.Ah @ W[:, :T] + self.Bh @ Z
        return np.ascontiguousarray(Y.T)

    def psi(self, d: np.ndarray) -> np.ndarray:
        return self._per_slice(self.psi_hat, d)

    def xi(self, d: np.ndarray) -> np.ndarray:
        return self.psi(d) - self.delta(d)

    def omega(self, th: np.ndarray) -> np.ndarray:
        return self._per_slice(self.omega_hat, th)

    def phi(self, th: np.ndarray) -> np.ndarray:
        return self._per_slice(self.phi_hat, th)

    def _per_slice(self, getter, d):
        out = np.empty_like(d)
        for c, ts in self._classes().items():
            M = getter(ts[0])
            out[ts] = (M @ d[ts].T).T
        return out

    def _classes(self):
        T = self.T
        cls = {}
        for t in range(T + 1):
            cls.setdefault(self.cls(t), []).append(t)
        return {c: np.array(ts) for c, ts in cls.items()}

    # -- Phi_bar_{v,t} solves -------------------------------------------
    def _perm(self, v):
        K, n, N = self.K, self.n, self.N
        j0 = 2 * v
        w = 2 if j0 + 1 < N else 1
        perm = [((j0 + h) * K + i) * n + c
                for i in range(K) for h in range(w) for c in range(n)]
        return np.array(perm), w

    def _factor(self, t):
        c = self.cls(t)
        if c not in self._chol:
            Phi = self.phi_hat(t).tocsr()
            facs = []
            for v in range(self.V):
                perm, w = self._perm(v)
                M = Phi[perm][:, perm].toarray()
                u = 3 * w * self.n - 1
                size = M.shape[0]
                ab = np.zeros((u + 1, size))
                for k in range(u + 1):          # upper form: ab[u+i-j, j]
                    ab[u - k, k:] = np.diagonal(M, offset=k)
                cb = sla.cholesky_banded(ab, lower=False)
                facs.append((perm, cb))
            self._chol[c] = facs
        return self._chol[c]

    def phi_solve(self, tau: np.ndarray) -> np.ndarray:
        out = np.empty_like(tau)
        for c, ts in self._classes().items():
            for perm, cb in self._factor(ts[0]):
                rhs = tau[np.ix_(ts, perm)].T         # (size, #t)
                sol = sla.cho_solve_banded((cb, False), rhs)
                out[np.ix_(ts, perm)] = sol.T
        return out

    # -- problem data ---------------------------------------------------
    def r_delta(self) -> np.ndarray:
        return stack.r_delta(self.p).reshape(self.T + 1, self.KNn)
