"""Pins of the FP64 oracle against facts it does not compute itself:
textbook special cases, brute force, the paper's theorems and invariants.

Every test here is CPU-only.  Node-level helpers in this file re-derive the
problem from the per-node dynamics equation (Sec. II, eq. "2d_graph_dynamics")
with explicit loops, so that a mistake in the oracle's stacking (a transposed
coupling block, a wrong neighbour, a missing 1/2) shows up as a mismatch.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from lqgrid_synth import make_problem, config_problem
from oracle import stack, kkt, riccati, splitting, slab, nbjm, pcg, residual


# ---------------------------------------------------------------- helpers
def simulate(p, u):
    """x_{i,j,t+1} = A x + B u + E x_{i,j-1} + F x_{i,j+1} + G x_{i-1,j}
    + H x_{i+1,j}, x_{.,.,0} = gamma; a neighbour outside the grid is the
    boundary state of eqs. "boundary_condition_i/j" (zero when the problem
    has none).  u: [T][N][K][m] -> x: [T+1][N][K][n]."""
    K, N, T, n = p.K, p.N, p.T, p.n
    x = np.zeros((T + 1, N, K, n))
    x[0] = p.x0
    zero = np.zeros(n)

    def bnd(arr, t, k):
        return zero if arr is None else arr[t, k]

    for t in range(T):
        A, An, B = at(p, "A", t), at(p, "A_nbr", t), at(p, "B", t)
        for j in range(N):
            for i in range(K):
                acc = A[j, i] @ x[t, j, i] + B[j, i] @ u[t, j, i]
                west = x[t, j - 1, i] if j - 1 >= 0 else bnd(p.beta_lo, t, i)
                east = x[t, j + 1, i] if j + 1 < N else bnd(p.beta_hi, t, i)
                north = x[t, j, i - 1] if i - 1 >= 0 else bnd(p.alpha_lo, t, j)
                south = x[t, j, i + 1] if i + 1 < K else bnd(p.alpha_hi, t, j)
                acc += An[j, i, 0] @ west + An[j, i, 1] @ east
                acc += An[j, i, 2] @ north + An[j, i, 3] @ south
                x[t + 1, j, i] = acc
    return x


def at(p, name, t):
    """Problem array `name` at time t (time-varying data carry a leading t)."""
    a = getattr(p, name)
    return a[t] if p.time_varying else a


def cost(p, x, u):
    """1/2 sum_t sum_{i,j} (x'Qx + u'Ru), terminal 1/2 x_T' Q_T x_T."""
    J = 0.0
    for t in range(p.T + 1):
        for j in range(p.N):
            for i in range(p.K):
                Qm = p.QT[j, i] if t == p.T else at(p, "Q", t)[j, i]
                J += x[t, j, i] @ Qm @ x[t, j, i]
                if t < p.T:
                    J += u[t, j, i] @ at(p, "R", t)[j, i] @ u[t, j, i]
    return 0.5 * J


def shapes(p, sol):
    x = sol["x"].reshape(p.T + 1, p.N, p.K, p.n)
    u = sol["u"].reshape(p.T, p.N, p.K, p.m)
    return x, u


# ---------------------------------------------------------------- pins
@pytest.mark.parametrize("seed,n,m,T,qt,w", [(0, 2, 1, 12, 1.0, "identity"),
                                             (1, 3, 2, 25, 1.0, "identity"),
                                             (2, 4, 2, 40, 3.0, "identity"),
                                             (3, 1, 1, 7, 0.5, "identity"),
                                             # full SPD Q, R and Q_T != Q
                                             (4, 4, 2, 30, 1.0, "spd"),
                                             (5, 3, 3, 17, 2.0, "spd")])
def test_riccati_special_case(seed, n, m, T, qt, w):
    """K = N = 1 must equal the textbook Riccati LQR solution."""
    p = make_problem(1, 1, T, n, m, rho=1.1, seed=seed, qt_scale=qt, weights=w)
    R = riccati.lqr_of_problem(p)
    sol = kkt.solve_kkt(p)
    x, u = shapes(p, sol)
    assert np.abs(x[:, 0, 0] - R["x"]).max() <= 1e-12 * max(1, np.abs(R["x"]).max())
    assert np.abs(u[:, 0, 0] - R["u"]).max() <= 1e-12 * max(1, np.abs(R["u"]).max())
    dl = sol["delta"].reshape(T + 1, n)
    assert np.abs(dl - R["delta"]).max() <= 1e-11 * max(1, np.abs(R["delta"]).max())
    assert abs(cost(p, x, u) - R["cost"]) <= 1e-12 * R["cost"]
    # and the matrix-free Schur path agrees with Riccati too
    ops = slab.SlabOperators(p)
    d = ops.phi_solve(ops.r_delta()) if T == 0 else None
    xs, it, _ = pcg.cg(ops.delta, ops.r_delta(), tol=1e-13, max_iter=5000)
    assert np.abs(xs - R["delta"]).max() <= 1e-9 * max(1, np.abs(R["delta"]).max())


@pytest.mark.parametrize("seed,n,m,T", [(0, 2, 1, 10), (1, 4, 2, 25), (2, 3, 3, 6)])
def test_time_varying_riccati_special_case(seed, n, m, T):
    """K = N = 1 with time-varying A_t, B_t, Q_t, R_t: the KKT solution and the
    matrix-free slab CG equal the time-varying Riccati recursion."""
    p = make_problem(1, 1, T, n, m, rho=1.1, seed=seed, weights="spd", qt_scale=2.0,
                     time_varying=True)
    R = riccati.lqr_of_tv_problem(p)
    sol = kkt.solve_kkt(p)
    x, u = shapes(p, sol)
    assert np.abs(x[:, 0, 0] - R["x"]).max() <= 1e-11 * max(1, np.abs(R["x"]).max())
    assert np.abs(u[:, 0, 0] - R["u"]).max() <= 1e-11 * max(1, np.abs(R["u"]).max())
    assert np.abs(sol["delta"].reshape(T + 1, n) - R["delta"]).max() <= \
        1e-10 * max(1, np.abs(R["delta"]).max())
    assert abs(cost(p, x, u) - R["cost"]) <= 1e-11 * R["cost"]
    ops = slab.SlabOperators(p)
    xs, _, _ = pcg.cg(ops.delta, ops.r_delta(), tol=1e-13, max_iter=5000)
    assert np.abs(xs - R["delta"]).max() <= 1e-9 * max(1, np.abs(R["delta"]).max())


@pytest.mark.parametrize("seed,w,bnd,tv", [(s, "identity", False, False) for s in range(5)]
                         + [(5, "spd", False, False), (6, "spd", False, False),
                            (7, "identity", True, False), (8, "spd", True, False),
                            (9, "spd", False, True), (10, "spd", True, True)])
def test_kkt_solution_is_feasible_and_optimal(seed, w, bnd, tv):
    """Brute force on the tiny configuration: the LDL' KKT solution obeys the
    node-level dynamics (with the boundary states as the neighbours outside
    the grid), and no random feasible perturbation lowers the cost (the cost
    written with loops over the per-node weights)."""
    if w == "identity" and not bnd:
        p, _ = config_problem("tiny", seed)
    else:
        p = make_problem(4, 4, 20, 2, 1, rho=0.9, seed=seed, qt_scale=1.7, weights=w,
                         boundary=bnd, time_varying=tv)
    sol = kkt.solve_kkt(p)
    x, u = shapes(p, sol)
    xs = simulate(p, u)
    assert np.abs(xs - x).max() <= 1e-11 * np.abs(x).max()
    J = cost(p, x, u)
    rng = np.random.default_rng(100 + seed)
    for _ in range(4):
        du = 1e-3 * rng.standard_normal(u.shape)
        u2 = u + du
        J2 = cost(p, simulate(p, u2), u2)
        assert J2 > J
    # first-order optimality: the directional derivative of J vanishes, i.e.
    # the central difference J(u + e du) - J(u - e du) = 2 e J'(u) du + O(e^3)
    du = rng.standard_normal(u.shape)
    e = 1e-4
    d1 = cost(p, simulate(p, u + e * du), u + e * du) - cost(p, simulate(p, u - e * du),
                                                             u - e * du)
    assert abs(d1) < 1e-7 * abs(J) + 1e-12


@pytest.mark.parametrize("K,N,T,n,m", [(4, 4, 20, 2, 1), (3, 5, 6, 3, 2),
                                       (5, 2, 4, 4, 2), (1, 6, 5, 2, 1),
                                       (6, 1, 5, 2, 1), (2, 3, 1, 2, 2)])
def test_schur_solve_equals_kkt_ldl(K, N, T, n, m):
    """Dense Cholesky of Delta == Bunch-Kaufman LDL' of the KKT system."""
    p = make_problem(K, N, T, n, m, rho=0.95, seed=K * 7 + N)
    a = kkt.solve_kkt(p)["delta"]
    b = kkt.solve_schur_dense(p)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("K,N,T,n,m,qt,w", [(4, 4, 20, 2, 1, 1.0, "identity"),
                                            (3, 5, 6, 3, 2, 2.0, "identity"),
                                            (5, 3, 3, 4, 2, 1.0, "identity"),
                                            (2, 7, 4, 2, 1, 0.3, "identity"),
                                            (1, 1, 3, 2, 2, 1.0, "identity"),
                                            (4, 5, 6, 3, 2, 1.0, "spd"),
                                            (5, 3, 4, 4, 2, 0.6, "spd"),
                                            (4, 5, 6, 3, 2, 1.2, "tv"),
                                            (3, 3, 2, 2, 2, 1.0, "tv")])
def test_slab_operators_match_full_matrices(K, N, T, n, m, qt, w):
    p = make_problem(K, N, T, n, m, seed=11, qt_scale=qt,
                     weights="spd" if w == "tv" else w, time_varying=w == "tv")
    ops = slab.SlabOperators(p)
    spl = splitting.splittings(p)
    rng = np.random.default_rng(5)
    d = rng.standard_normal((T + 1, K * N * n))
    for name, f in [("Delta", ops.delta), ("Psi", ops.psi), ("Xi", ops.xi),
                    ("Omega", ops.omega), ("Phi", ops.phi)]:
        ref = spl[name] @ d.ravel()
        got = f(d).ravel()
        assert np.linalg.norm(got - ref) <= 1e-13 * max(1.0, np.linalg.norm(ref)), name
    tau = ops.phi_solve(d)
    assert np.linalg.norm(spl["Phi"] @ tau.ravel() - d.ravel()) <= 1e-12 * np.linalg.norm(d)


@pytest.mark.parametrize("w", ["identity", "spd", "tv"])
def test_delta_from_node_level_definition(w):
    """Delta d equals A~(Q~^-1 A~' d) + B~(R~^-1 B~' d) evaluated with
    node-level loops (no stacked matrices); with per-node SPD weights a weight
    taken from the wrong node changes the result, and with time-varying data
    a block taken at the wrong time does."""
    p = make_problem(3, 4, 5, 2, 2, seed=4, weights="spd" if w == "tv" else w,
                     qt_scale=1.0 if w == "identity" else 1.4, time_varying=w == "tv")
    rng = np.random.default_rng(0)
    d = rng.standard_normal((p.T + 1, p.N, p.K, p.n))
    T = p.T
    Qi = [np.linalg.inv(at(p, "Q", t)) for t in range(T)] + [np.linalg.inv(p.QT)]
    Ri = [np.linalg.inv(at(p, "R", t)) for t in range(T)]

    def nbrs(i, j, t):   # (coupling block of node (i,j) at t, neighbour position)
        A, An = at(p, "A", t), at(p, "A_nbr", t)
        out = [(A[j, i], (i, j))]
        if j - 1 >= 0:
            out.append((An[j, i, 0], (i, j - 1)))
        if j + 1 < p.N:
            out.append((An[j, i, 1], (i, j + 1)))
        if i - 1 >= 0:
            out.append((An[j, i, 2], (i - 1, j)))
        if i + 1 < p.K:
            out.append((An[j, i, 3], (i + 1, j)))
        return out

    # a = A~' d : a_t = -d_t + A_hat_t' d_{t+1}
    a = -d.copy()
    for t in range(T):
        for j in range(p.N):
            for i in range(p.K):
                for M, (ii, jj) in nbrs(i, j, t):
                    a[t, jj, ii] += M.T @ d[t + 1, j, i]
    w = np.zeros_like(a)
    for t in range(T + 1):
        for j in range(p.N):
            for i in range(p.K):
                w[t, j, i] = Qi[t][j, i] @ a[t, j, i]
    y = -w.copy()
    for t in range(1, T + 1):
        for j in range(p.N):
            for i in range(p.K):
                for M, (ii, jj) in nbrs(i, j, t - 1):
                    y[t, j, i] += M @ w[t - 1, jj, ii]
                Bm = at(p, "B", t - 1)[j, i]
                y[t, j, i] += Bm @ Ri[t - 1][j, i] @ Bm.T @ d[t, j, i]
    ops = slab.SlabOperators(p)
    got = ops.delta(d.reshape(T + 1, -1)).reshape(y.shape)
    assert np.abs(got - y).max() <= 1e-13 * np.abs(y).max()


def test_splitting_definiteness_and_convergence():
    """Lemma 1 / Remark 1 / the convergence conditions of Sec. IV:
    Delta, Psi~, Phi~, Phi~+Omega~, Psi~+Xi~ are positive definite and
    rho(Phi~^-1 Omega~) < 1, rho(Psi~^-1 Xi~) < 1."""
    for seed in range(3):
        p, _ = config_problem("tiny", seed)
        spl = splitting.splittings(p)
        d = {k: v.toarray() for k, v in spl.items()}
        for name, M in [("Delta", d["Delta"]), ("Psi", d["Psi"]), ("Phi", d["Phi"]),
                        ("Phi+Omega", d["Phi"] + d["Omega"]),
                        ("Psi+Xi", d["Psi"] + d["Xi"])]:
            assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max(), name
            assert np.linalg.eigvalsh(M).min() > 0, name
        r1 = np.abs(np.linalg.eigvals(np.linalg.solve(d["Phi"], d["Omega"]))).max()
        r2 = np.abs(np.linalg.eigvals(np.linalg.solve(d["Psi"], d["Xi"]))).max()
        assert r1 < 1 and r2 < 1


def test_13_point_pattern_and_band():
    """Psi_hat_t couples nodes at Manhattan distance <= 2 only; in the
    interleaved order Phi_bar_{v,t} is banded with half-bandwidth 3*w*n-1."""
    p = make_problem(6, 5, 3, 2, 1, seed=2)
    ops = slab.SlabOperators(p)
    C = ops.psi_hat(1).tocoo()
    n, K = p.n, p.K
    ni, nj = (C.row // n) % K, (C.row // n) // K
    mi, mj = (C.col // n) % K, (C.col // n) // K
    dist = np.abs(ni - mi) + np.abs(nj - mj)
    assert dist.max() == 2
    pairs = set(zip((ni - mi)[np.abs(C.data) > 0], (nj - mj)[np.abs(C.data) > 0]))
    assert len(pairs) == 13
    Phi = ops.phi_hat(1).tocsr()
    for v in range(ops.V):
        perm, w = ops._perm(v)
        M = Phi[perm][:, perm].toarray()
        r, c = np.nonzero(M)
        assert np.abs(r - c).max() <= 3 * w * n - 1


def test_theorem2_closed_form_and_spd():
    """Theorem 2: S outer x L inner sweeps from zero apply P_S^-1 =
    sum_s (Upsilon_L Xi)^s Upsilon_L, which is symmetric positive definite for
    even L."""
    for seed, (S, L) in [(0, (2, 2)), (1, (3, 2)), (2, (1, 4)), (3, (2, 6))]:
        p, _ = config_problem("tiny", seed)
        spl = splitting.splittings(p)
        Pinv = splitting.preconditioner_inverse(spl, S, L)
        apply = nbjm.sparse_preconditioner(spl, S, L)
        rng = np.random.default_rng(seed)
        for _ in range(3):
            r = rng.standard_normal(Pinv.shape[0])
            a, b = Pinv @ r, apply(r)
            assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)
        assert np.abs(Pinv - Pinv.T).max() <= 1e-13 * np.abs(Pinv).max()
        assert np.linalg.eigvalsh(0.5 * (Pinv + Pinv.T)).min() > 0


def test_preconditioner_special_cases():
    # S = L = 1: block Jacobi with Phi~.
    p = make_problem(3, 4, 5, 2, 1, seed=9)
    spl = splitting.splittings(p)
    Phi = spl["Phi"].toarray()
    assert np.allclose(splitting.preconditioner_inverse(spl, 1, 1),
                       np.linalg.inv(Phi), rtol=1e-12, atol=1e-14)
    # S = 1: P^-1 = Upsilon_L.
    assert np.allclose(splitting.preconditioner_inverse(spl, 1, 2),
                       splitting.upsilon(spl["Phi"], spl["Omega"], 2),
                       rtol=1e-12, atol=1e-14)
    # One super-column (N <= 2): Omega~ = 0, Phi~ = Psi~, Upsilon_L = Psi~^-1.
    p2 = make_problem(4, 2, 5, 2, 1, seed=3)
    s2 = splitting.splittings(p2)
    assert s2["Omega"].count_nonzero() == 0
    U = splitting.upsilon(s2["Phi"], s2["Omega"], 4)
    assert np.allclose(U, np.linalg.inv(s2["Psi"].toarray()), rtol=1e-12, atol=1e-14)
    # Many sweeps: the nested iteration converges to Delta^-1 (the splittings
    # are convergent), so P^-1 -> Delta^-1.  A sign error in Xi~ or Omega~
    # converges elsewhere and fails here.
    # (instance with rho(Psi~^-1 Xi~) ~ 0.92 so 600 sweeps reach ~1e-20)
    p3 = make_problem(3, 4, 3, 2, 1, rho=0.5, seed=9)
    s3 = splitting.splittings(p3)
    Dinv = np.linalg.inv(s3["Delta"].toarray())
    far = splitting.preconditioner_inverse(s3, 600, 30)
    assert np.abs(far - Dinv).max() <= 1e-9 * np.abs(Dinv).max()


def test_pcg_matches_dense_and_energy_norm_monotone():
    """PCG converges to the dense solution; the Delta-norm of the error
    decreases monotonically (the CG error bound of Sec. III); with P = Delta
    (exact preconditioner) one step suffices; P = I is textbook CG."""
    p, tol = config_problem("tiny", 0)
    ops = slab.SlabOperators(p)
    spl = splitting.splittings(p)
    rd = ops.r_delta()
    ds = kkt.solve_schur_dense(p).reshape(rd.shape)
    pre = nbjm.slab_preconditioner(ops, 2, 2)
    x, it, h = pcg.pcg(ops.delta, pre, rd, tol=tol, keep_iterates=True)
    assert np.linalg.norm(x - ds) <= 1e-8 * np.linalg.norm(ds)
    D = spl["Delta"]
    en = [float(np.sqrt((xi - ds).ravel() @ (D @ (xi - ds).ravel())))
          for xi in h["iterates"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(en, en[1:]))
    # CG error bound with kappa(Delta) (applied with P = I)
    xc, itc, hc = pcg.cg(ops.delta, rd, tol=tol, keep_iterates=True)
    ev = np.linalg.eigvalsh(D.toarray())
    kap = ev[-1] / ev[0]
    q = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    enc = [float(np.sqrt((xi - ds).ravel() @ (D @ (xi - ds).ravel())))
           for xi in hc["iterates"]]
    for k, e in enumerate(enc):
        assert e <= 2 * q ** k * enc[0] * (1 + 1e-9) + 1e-12
    # exact preconditioner
    Dd = D.toarray()
    c = sla.cho_factor(Dd)
    xe, ite, _ = pcg.pcg(ops.delta, lambda r: sla.cho_solve(c, r.ravel()).reshape(r.shape),
                         rd, tol=1e-12)
    assert ite == 1
    # PCG beats CG in iterations with the NBJM preconditioner
    assert it < itc


def test_kkt_residual_gate():
    p, tol = config_problem("tiny", 1)
    ops = slab.SlabOperators(p)
    ds = kkt.solve_schur_dense(p).reshape(p.T + 1, -1)
    g = residual.kkt_residual(ops, ds)
    assert g["rel2"] < 1e-13
    bad = ds.copy()
    bad[3, 5] += 1e-3
    assert residual.kkt_residual(ops, bad)["rel2"] > 1e-6
    # the primal pair recovered from delta equals the KKT LDL' primal pair
    sol = kkt.solve_kkt(p)
    x, u = residual.recover(ops, ds)
    assert np.abs(x.ravel() - sol["x"]).max() <= 1e-11 * np.abs(sol["x"]).max()
    assert np.abs(u.ravel() - sol["u"]).max() <= 1e-11 * np.abs(sol["u"]).max()


def test_per_iteration_cost_is_linear():
    """Table I: every operator in a PCG step has O(1) nonzeros per unknown, so
    a step costs O(KNT).  Per row: Delta <= (13 + 5 + 5) n (13-point Psi_hat
    plus two 5-point Xi_hat blocks), Xi~ <= 10 n, Phi~ and Omega~ <= 13 n;
    interior rows reach these bounds, so the count saturates, not grows."""
    n = 2
    per = []
    for K, N, T in [(3, 3, 4), (6, 6, 8), (10, 12, 16), (14, 14, 6)]:
        p = make_problem(K, N, T, n, 1, seed=0)
        spl = splitting.splittings(p)
        rows = {k: np.diff(spl[k].tocsr().indptr) for k in spl}
        nz = {k: np.array([np.count_nonzero(r) for r in
                           np.split(spl[k].tocsr().data, spl[k].tocsr().indptr[1:-1])])
              for k in ("Delta", "Xi", "Phi", "Omega")}
        assert nz["Delta"].max() <= 23 * n
        assert nz["Xi"].max() <= 10 * n
        assert nz["Phi"].max() <= 13 * n and nz["Omega"].max() <= 13 * n
        per.append(spl["Delta"].count_nonzero() / p.unknowns)
    assert per[-1] <= 23 * n and per[-1] > 0.5 * 23 * n


# ------------------------------------------------ standalone NBJM, spectra
def test_lanczos_estimate_on_a_known_spectrum():
    """CG on a diagonal matrix with a known spectrum: the Lanczos matrix built
    from the CG coefficients has the exact extreme eigenvalues (textbook
    equivalence of CG and Lanczos)."""
    from oracle import lanczos
    ev = np.concatenate([[1.0], np.linspace(2.0, 50.0, 60), [100.0]])
    rng = np.random.default_rng(0)
    b = rng.standard_normal(ev.size)
    est = lanczos.condition_from_cg(lambda x: ev * x, lambda r: r.copy(), b, tol=1e-13)
    assert abs(est["lambda_min"] - 1.0) <= 1e-8
    assert abs(est["lambda_max"] - 100.0) <= 1e-8 * 100
    # with a diagonal preconditioner P = diag(ev): P^-1 A = I, one step, kappa 1
    est = lanczos.condition_from_cg(lambda x: ev * x, lambda r: r / ev, b, tol=1e-13)
    assert est["iterations"] == 1 and abs(est["kappa"] - 1.0) <= 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_lanczos_estimates_match_dense_spectra(seed):
    """On the tiny configuration, the CG estimate of kappa(Delta) and the
    PCG estimate of kappa(P_S^-1 Delta) (S = L = 2) agree with the dense
    eigenvalues (Sec. V's conditioning comparison) to 1 %."""
    from oracle import lanczos
    p, _ = config_problem("tiny", seed)
    ops = slab.SlabOperators(p)
    spl = splitting.splittings(p)
    D = spl["Delta"].toarray()
    ev = np.linalg.eigvalsh(D)
    Pinv = splitting.preconditioner_inverse(spl, 2, 2)
    evp = np.sort(np.linalg.eigvals(Pinv @ D).real)
    cg = lanczos.condition_from_cg(ops.delta, lambda r: r.copy(), ops.r_delta(), tol=1e-10)
    pc = lanczos.condition_from_cg(ops.delta, nbjm.slab_preconditioner(ops, 2, 2),
                                   ops.r_delta(), tol=1e-10)
    assert abs(cg["kappa"] / (ev[-1] / ev[0]) - 1) <= 1e-2
    assert abs(pc["kappa"] / (evp[-1] / evp[0]) - 1) <= 1e-2
    assert pc["kappa"] < cg["kappa"] / 10        # the preconditioner's gain


def test_standalone_nbjm_converges_at_the_predicted_rate():
    """Standalone NBJM (inner iterations started from the outer iterate):
    converges to the dense solution, at the rate rho(G) of its iteration
    matrix G = Upsilon_L Xi~ + (Phi~^-1 Omega~)^L; started from theta = 0 in
    every outer iteration (as printed, for the preconditioner) it converges to
    (Upsilon_L^-1 - Xi~)^-1 r_delta instead, which is not the solution."""
    p, _ = config_problem("tiny", 0)
    ops = slab.SlabOperators(p)
    spl = splitting.splittings(p)
    Phi, Om, Xi = (spl[k].toarray() for k in ("Phi", "Omega", "Xi"))
    U = splitting.upsilon(spl["Phi"], spl["Omega"], 2)
    G = U @ Xi + np.linalg.matrix_power(np.linalg.solve(Phi, Om), 2)
    rho = np.abs(np.linalg.eigvals(G)).max()
    d, s, h = nbjm.slab_nbjm_solve(ops, 2, tol=1e-10)
    ds = kkt.solve_schur_dense(p)
    assert np.linalg.norm(d.ravel() - ds) <= 1e-8 * np.linalg.norm(ds)
    rate = (h["res"][-1] / h["res"][-201]) ** (1 / 200)
    assert abs(rate - rho) <= 1e-3
    assert 100 < s < 5000
    # the printed zero inner start: fixed point (Upsilon_L^-1 - Xi~)^-1 r
    rd = ops.r_delta().ravel()
    fixed = np.linalg.solve(np.linalg.inv(U) - Xi, rd)
    x = np.zeros_like(rd)
    for _ in range(3000):
        x = U @ (rd + Xi @ x)
    assert np.linalg.norm(x - fixed) <= 1e-8 * np.linalg.norm(fixed)
    assert np.linalg.norm(fixed - ds) >= 1e-2 * np.linalg.norm(ds)


# ------------------------------------------------ heterogeneous sizes
def simulate_hetero(p, u):
    """The dynamics with per-node sizes n_{i,j}, m_{i,j} (only the leading
    n_p x n_q part of each coupling block), written with loops."""
    K, N, T = p.K, p.N, p.T
    ns, ms = p.n_node, p.m_node
    x = [[[np.asarray(p.x0[j, i][:ns[j, i]], dtype=float) for i in range(K)]
          for j in range(N)]]
    for t in range(T):
        nxt = []
        for j in range(N):
            col = []
            for i in range(K):
                a = ns[j, i]
                acc = p.A[j, i][:a, :a] @ x[t][j][i] + p.B[j, i][:a, :ms[j, i]] @ u[t][j][i]
                for slot, (ii, jj) in enumerate([(i, j - 1), (i, j + 1), (i - 1, j), (i + 1, j)]):
                    if 0 <= ii < K and 0 <= jj < N:
                        acc = acc + p.A_nbr[j, i, slot][:a, :ns[jj, ii]] @ x[t][jj][ii]
                col.append(acc)
            nxt.append(col)
        x.append(nxt)
    return x


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_heterogeneous_sizes(seed):
    """Per-node sizes: the variable-block KKT solution obeys the node-level
    dynamics and is optimal against random feasible perturbations; with
    every size at its maximum it is the uniform solution; and padding each
    node to n, m with decoupled rows (zero coupling rows and columns, unit
    weights, zero initial state) reproduces it, with zero multipliers and
    inputs in the padding."""
    from oracle import hetero
    p = make_problem(3, 4, 6, 3, 2, seed=seed, sizes=True, weights="spd")
    h = hetero.solve(p, p.n_node, p.m_node)
    ns, ms = p.n_node, p.m_node
    K, N, T = p.K, p.N, p.T
    uu = [[[h["u"][t, j, i, :ms[j, i]] for i in range(K)] for j in range(N)] for t in range(T)]
    xs = simulate_hetero(p, uu)
    err = max(np.abs(xs[t][j][i] - h["x"][t, j, i, :ns[j, i]]).max()
              for t in range(T + 1) for j in range(N) for i in range(K))
    assert err <= 1e-11 * np.abs(h["x"]).max()

    def J(xs, uu):
        s = 0.0
        for t in range(T + 1):
            for j in range(N):
                for i in range(K):
                    a = ns[j, i]
                    Qm = (p.QT if t == T else p.Q)[j, i][:a, :a]
                    s += xs[t][j][i] @ Qm @ xs[t][j][i]
                    if t < T:
                        b = ms[j, i]
                        s += uu[t][j][i] @ p.R[j, i][:b, :b] @ uu[t][j][i]
        return 0.5 * s

    J0 = J(xs, uu)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        u2 = [[[v + 1e-3 * rng.standard_normal(v.shape) for v in col] for col in sl] for sl in uu]
        assert J(simulate_hetero(p, u2), u2) > J0
    # all sizes at the maximum: the uniform problem
    full = hetero.solve(p, np.full((N, K), p.n), np.full((N, K), p.m))
    ref = kkt.solve_kkt(p)
    assert np.abs(full["delta"].ravel() - ref["delta"]).max() <= 1e-11 * np.abs(ref["delta"]).max()
    # padding with decoupled rows
    q = make_problem(3, 4, 6, 3, 2, seed=seed, sizes=True, weights="spd")
    for j in range(N):
        for i in range(K):
            a, b = ns[j, i], ms[j, i]
            q.A[j, i][a:, :] = 0.0
            q.A[j, i][:, a:] = 0.0
            q.B[j, i][a:, :] = 0.0
            q.B[j, i][:, b:] = 0.0
            q.x0[j, i][a:] = 0.0
            for slot, (ii, jj) in enumerate([(i, j - 1), (i, j + 1), (i - 1, j), (i + 1, j)]):
                q.A_nbr[j, i, slot][a:, :] = 0.0
                if 0 <= ii < K and 0 <= jj < N:
                    q.A_nbr[j, i, slot][:, ns[jj, ii]:] = 0.0
            for W, k in ((q.Q, a), (q.QT, a), (q.R, b)):
                blk = W[j, i].copy()
                W[j, i] = np.eye(W.shape[-1])
                W[j, i][:k, :k] = blk[:k, :k]
    padded = kkt.solve_kkt(q)
    for key in ("delta", "x"):
        got = padded[key].reshape(T + 1, N, K, p.n)
        assert np.abs(got - h[key]).max() <= 1e-11 * np.abs(h[key]).max()
    gotu = padded["u"].reshape(T, N, K, p.m)
    assert np.abs(gotu - h["u"]).max() <= 1e-11 * np.abs(h["u"]).max()


# ------------------------------------------------ node-temporal nesting
@pytest.mark.parametrize("case", [("tiny", False), ("spd", False), ("tv", True)])
def test_node_temporal_preconditioner(case):
    """The node-temporal block Jacobi preconditioner (oracle/nodetemporal.py,
    per-node banded Cholesky in t) equals the inverse of the node-diagonal
    part of the explicit Delta, which is symmetric positive definite; PCG with
    it converges to the dense solution in fewer iterations than plain CG; for
    a single node it is Delta itself, so PCG takes one step."""
    from oracle import nodetemporal
    import scipy.sparse.linalg as spla
    kind, tv = case
    if kind == "tiny":
        p, _ = config_problem("tiny", 1)
    else:
        p = make_problem(3, 5, 8, 3, 2, seed=4, weights="spd", qt_scale=1.5, time_varying=tv)
    ops = slab.SlabOperators(p)
    D = stack.delta_matrix(p)
    Dn = nodetemporal.node_blocks_dense(p, D)
    Dd = Dn.toarray()
    assert np.abs(Dd - Dd.T).max() <= 1e-14 * np.abs(Dd).max()
    assert np.linalg.eigvalsh(Dd).min() > 0
    P = nodetemporal.NodeTemporal(ops)
    r = np.random.default_rng(3).standard_normal((p.T + 1, p.K * p.N * p.n))
    ref = spla.spsolve(Dn.tocsc(), r.ravel())
    assert np.abs(P(r).ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
    rd = ops.r_delta()
    x, it, _ = pcg.pcg(ops.delta, P, rd, tol=1e-10)
    _, itc, _ = pcg.cg(ops.delta, rd, tol=1e-10)
    ds = kkt.solve_schur_dense(p).reshape(rd.shape)
    assert np.linalg.norm(x - ds) <= 1e-7 * np.linalg.norm(ds)
    assert it < itc
    q = make_problem(1, 1, 25, 3, 2, seed=2, weights="spd", time_varying=tv)
    oq = slab.SlabOperators(q)
    _, it1, _ = pcg.pcg(oq.delta, nodetemporal.NodeTemporal(oq), oq.r_delta(), tol=1e-12)
    assert it1 == 1
