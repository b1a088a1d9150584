"""Pins of the warm-start oracle (oracle/warmstart.py) against library
routines, finite differences and exact values.  CPU only."""
import numpy as np
import pytest
import scipy.signal

from lqgrid_synth import make_problem
from oracle import warmstart as ws


def test_chebyshev_basis_matches_numpy_chebval():
    T, k = 37, 16
    B = ws.cheb_basis(T, k)
    tau = 2.0 * np.arange(T + 1) / T - 1.0
    for c in range(k):
        e = np.zeros(k)
        e[c] = 1.0
        assert np.allclose(B[:, c], np.polynomial.chebyshev.chebval(tau, e), atol=1e-13)
    # |T_c| <= 1 on [-1, 1], T_c(1) = 1, T_c(-1) = (-1)^c
    assert np.all(np.abs(B) <= 1 + 1e-12)
    assert np.allclose(B[-1], 1.0) and np.allclose(B[0], (-1.0) ** np.arange(k))


def test_conv3x3_matches_scipy_correlate2d():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 5, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = ws.conv3x3(x, W, b)
    for o in range(4):
        ref = b[o] + sum(scipy.signal.correlate2d(x[:, :, c], W[o, :, :, c], mode="same")
                         for c in range(3))
        assert np.allclose(y[:, :, o], ref, atol=1e-12)


def _fd(f, v, idx, h=1e-6):
    old = v[idx]
    v[idx] = old + h
    fp = f()
    v[idx] = old - h
    fm = f()
    v[idx] = old
    return (fp - fm) / (2 * h)


def test_conv3x3_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 6, 3))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    R = rng.standard_normal((5, 6, 2))
    f = lambda: np.sum(ws.conv3x3(x, W, b) * R)
    dW, db, dx = ws.conv3x3_backward(x, W, R)
    for idx in [(0, 0, 0, 0), (1, 2, 1, 2), (0, 1, 2, 1), (1, 0, 2, 0)]:
        assert abs(_fd(f, W, idx) - dW[idx]) < 1e-6
    for o in range(2):
        assert abs(_fd(f, b, (o,)) - db[o]) < 1e-6
    for idx in [(0, 0, 0), (4, 5, 2), (2, 3, 1), (0, 5, 1), (4, 0, 0)]:
        assert abs(_fd(f, x, idx) - dx[idx]) < 1e-6


def _tiny_net(rng, cin=5, width=6, layers=3, cout=8):
    params = []
    c = cin
    for li in range(layers):
        o = cout if li == layers - 1 else width
        params.append((rng.standard_normal((o, 3, 3, c)) * 0.5, rng.standard_normal(o) * 0.1))
        c = o
    return params


def test_network_gradient_matches_finite_differences():
    """Three layers with ReLU, Chebyshev expansion and relative loss."""
    rng = np.random.default_rng(2)
    n, ncheb, T = 2, 4, 9
    K, N = 4, 3
    params = _tiny_net(rng, cin=5, width=6, layers=3, cout=n * ncheb)
    x = rng.standard_normal((K, N, 5))
    delta = rng.standard_normal((T + 1, N, K, n))

    def f():
        out = ws.forward(params, x)[-1]
        return ws.loss_and_grad(out, delta, n, ncheb, T)[0]

    acts = ws.forward(params, x)
    loss, dout = ws.loss_and_grad(acts[-1], delta, n, ncheb, T)
    grads = ws.backward(params, x, acts, dout)
    for li, (W, b) in enumerate(params):
        dW, db = grads[li]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            assert abs(_fd(f, W, idx) - dW[idx]) <= 1e-6 * max(1.0, abs(dW[idx]))
        o = int(rng.integers(0, b.shape[0]))
        assert abs(_fd(f, b, (o,)) - db[o]) <= 1e-6 * max(1.0, abs(db[o]))


def test_loss_equals_direct_expansion_error():
    rng = np.random.default_rng(3)
    n, ncheb, T, K, N = 3, 5, 11, 3, 4
    out = rng.standard_normal((K, N, n * ncheb))
    delta = rng.standard_normal((T + 1, N, K, n))
    d0 = ws.expand(out, n, ncheb, T)
    loss, g = ws.loss_and_grad(out, delta, n, ncheb, T)
    assert np.isclose(loss, np.sum((d0 - delta) ** 2) / np.sum(delta ** 2))
    # the exact expansion coefficients give zero loss
    lsq, *_ = np.linalg.lstsq(ws.cheb_basis(T, ncheb), delta.reshape(T + 1, -1), rcond=None)
    exact = lsq.reshape(ncheb, N, K, n).transpose(2, 1, 3, 0).reshape(K, N, n * ncheb)
    target = ws.expand(exact, n, ncheb, T)
    l0, g0 = ws.loss_and_grad(exact, target, n, ncheb, T)
    assert l0 < 1e-24 and np.abs(g0).max() < 1e-10


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7
    assert ws.bf16(one) == one
    assert ws.bf16(one + ulp / 2) == one                    # tie -> even (1.0)
    assert ws.bf16(one + 1.5 * ulp) == one + 2 * ulp        # tie -> even
    assert ws.bf16(one + ulp / 2 + 2.0 ** -20) == one + ulp
    assert ws.bf16(-3.0) == -3.0
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(4).standard_normal(20000) * 10.0 ** np.random.default_rng(5).integers(-8, 8, 20000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ws.bf16(x), ref)


def test_features_layout():
    p = make_problem(5, 3, 4, 4, 2, seed=9)
    f = ws.features(p, 32)
    i, j = 3, 2
    assert np.array_equal(f[i, j, :4], p.x0[j, i])
    assert np.array_equal(f[i, j, 4:20], p.A[j, i].ravel())
    assert np.array_equal(f[i, j, 20:28], p.B[j, i].ravel())
    assert np.all(f[:, :, 28:] == 0)
