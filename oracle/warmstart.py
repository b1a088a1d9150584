"""Oracle of the learned warm start: a convolutional network over the K x N
grid that predicts the Chebyshev-in-time coefficients of the multipliers
delta~, whose expansion is the PCG initial iterate delta^(0) (Algorithm 1
allows any initial iterate).  Test infrastructure only.

Everything here is plain FP64 numpy written from the definitions:

* features(p):  per node (i, j) the channels x0 (n), A_ii row-major (n^2) and
  B_ii row-major (n m), zero-padded to cin channels.  Image rows are i
  (0..K-1), columns j (0..N-1).
* cheb_basis(T, k): T_c(tau_t) for tau_t = 2 t / T - 1, t = 0..T, by the
  three-term recurrence T_0 = 1, T_1 = tau, T_{c+1} = 2 tau T_c - T_{c-1}.
* conv3x3(x, W, b): y[i, j, o] = b[o] + sum_{di, dj, c} W[o, di+1, dj+1, c]
  x[i+di, j+dj, c] with zeros outside the grid (cross-correlation, 'same').
* forward / backward: layers conv3x3 -> ReLU, the last one without ReLU;
  gradients of the weights, biases and inputs from the chain rule written out
  (dW[o, a, b, c] = sum_ij dy[i, j, o] x[i+a-1, j+b-1, c], db = sum dy,
  dx[i, j, c] = sum dy[i-a+1, j-b+1, o] W[o, a, b, c], ReLU mask y > 0).
* loss: output channel s*ncheb + c of node (i, j) is coefficient c of state
  component s; delta0_t = sum_c coef_c T_c(tau_t); loss = sum (delta0 -
  delta*)^2 / sum delta*^2 (relative squared error of the expansion).
* bf16(x): round to the nearest bfloat16, ties to even, through float32
  (the rounding the kernels apply when they store an FP32 value as BF16).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) and return as float64.
    The value is first rounded to float32 (as an FP32 accumulator holds it)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def cheb_basis(T: int, k: int) -> np.ndarray:
    """(T+1, k) array of T_c(tau_t), tau_t = 2 t / T - 1."""
    tau = 2.0 * np.arange(T + 1) / T - 1.0
    B = np.empty((T + 1, k))
    B[:, 0] = 1.0
    if k > 1:
        B[:, 1] = tau
    for c in range(2, k):
        B[:, c] = 2.0 * tau * B[:, c - 1] - B[:, c - 2]
    return B


def features(p, cin: int) -> np.ndarray:
    """(K, N, cin) input image of problem p."""
    K, N, n, m = p.K, p.N, p.n, p.m
    f = np.zeros((K, N, cin))
    # arrays are [N][K][...]: transpose to rows i, columns j
    f[:, :, :n] = np.transpose(p.x0, (1, 0, 2))
    f[:, :, n:n + n * n] = np.transpose(p.A.reshape(N, K, n * n), (1, 0, 2))
    f[:, :, n + n * n:n + n * n + n * m] = np.transpose(p.B.reshape(N, K, n * m), (1, 0, 2))
    return f


def conv3x3(x, W, b):
    """x (H, Wd, C), W (O, 3, 3, C), b (O,) -> (H, Wd, O)."""
    H, Wd, _ = x.shape
    xp = np.zeros((H + 2, Wd + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    y = np.broadcast_to(b, (H, Wd, W.shape[0])).copy()
    for a in range(3):
        for c in range(3):
            y += xp[a:a + H, c:c + Wd] @ W[:, a, c, :].T
    return y


def conv3x3_backward(x, W, dy):
    """Gradients of conv3x3 w.r.t. W, b and x for upstream gradient dy."""
    H, Wd, _ = x.shape
    xp = np.zeros((H + 2, Wd + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    dW = np.empty_like(W)
    for a in range(3):
        for c in range(3):
            dW[:, a, c, :] = np.einsum("ijo,ijk->ok", dy, xp[a:a + H, c:c + Wd])
    db = dy.sum(axis=(0, 1))
    dyp = np.zeros((H + 2, Wd + 2, dy.shape[2]))
    dyp[1:-1, 1:-1] = dy
    dx = np.zeros_like(x)
    for a in range(3):
        for c in range(3):
            # x[i, j] meets dy[i - (a-1), j - (c-1)] through W[:, a, c, :]
            dx += dyp[2 - a:2 - a + H, 2 - c:2 - c + Wd] @ W[:, a, c, :]
    return dW, db, dx


def forward(params, x, round_bf16=False):
    """params: list of (W, b).  Returns the list of layer outputs (the last
    one linear).  With round_bf16 the weights and every stored activation
    are rounded to bfloat16 as the kernels store them (the network input is
    expected to be rounded by the caller)."""
    acts = []
    h = x
    for li, (W, b) in enumerate(params):
        Wq = bf16(W) if round_bf16 else W
        y = conv3x3(h, Wq, b)
        if li < len(params) - 1:
            y = np.maximum(y, 0.0)
            if round_bf16:
                y = bf16(y)
        else:
            if round_bf16:
                y = y.astype(np.float32).astype(np.float64)
        acts.append(y)
        h = y
    return acts


def loss_and_grad(out, delta, n, ncheb, T):
    """out (K, N, n*ncheb); delta (T+1, N, K, n) target multipliers.
    Returns (loss, dloss/dout)."""
    Bc = cheb_basis(T, ncheb)                         # (T+1, ncheb)
    K, N = out.shape[:2]
    coef = out.reshape(K, N, n, ncheb)
    d0 = np.einsum("ijsc,tc->tjis", coef, Bc)         # (T+1, N, K, n)
    dd = np.sum(delta ** 2)
    e = d0 - delta
    loss = np.sum(e ** 2) / dd
    g = 2.0 * np.einsum("tjis,tc->ijsc", e, Bc) / dd
    return loss, g.reshape(K, N, n * ncheb)


def expand(out, n, ncheb, T):
    """delta^(0) (T+1, N, K, n) from the network output (K, N, n*ncheb)."""
    K, N = out.shape[:2]
    coef = out.reshape(K, N, n, ncheb)
    return np.einsum("ijsc,tc->tjis", coef, cheb_basis(T, ncheb))


def backward(params, x, acts, dout, round_bf16=False):
    """Gradients (list of (dW, db)) of the loss whose gradient w.r.t. the
    network output is dout.  With round_bf16 the weights and the gradients
    that the kernels store between layers are rounded to bfloat16."""
    grads = [None] * len(params)
    dy = bf16(dout) if round_bf16 else dout
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        Wq = bf16(W) if round_bf16 else W
        xin = x if li == 0 else acts[li - 1]
        dW, db, dx = conv3x3_backward(xin, Wq, dy)
        grads[li] = (dW, db)
        if li > 0:
            dx = dx * (acts[li - 1] > 0)
            dy = bf16(dx) if round_bf16 else dx
    return grads
