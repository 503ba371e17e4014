"""FP64 reference of the learned warm-start network (test infrastructure only).

The warm start extends the method (it is not in the paper): a small 1-D
convolutional network predicts the initial guess of each shifted system
C_q u = b_i (Appendix E, eq. E.1), C_q = (1 + s_q) I + S, over the m
observation rows.  The shift enters only at the end, so the convolutions run
once per member i, not once per system (q, i):
  * trunk, per member: the input channel bh_i = sqrt(m) b_i / ||b_i|| (unit
    root-mean-square entries) through 1 -> H -> H -> H -> D channels, GELU
    after the first three layers, gives Y_i (D x m);
  * head, per system: with c_q = 1 / (1 + s_q),
        y_{q,i} = sum_d c_q^(d+1) Y_i[d],   u0_{q,i} = (||b_i|| / sqrt(m)) y_{q,i}.
    The Neumann series u = sum_d c^(d+1) (-S)^d b (valid for c ||S|| < 1) has
    this form with Y_i[d] = (-S)^d bh_i, so D channels can hold a truncation
    of it, or any other shift profile the training data favour; u0 scales
    with b_i.  Training targets are u* sqrt(m) / ||b_i||.

Its arithmetic is standard and is written out here from the definitions:
  * cross-correlation with zero "same" padding:
        y[o, t] = bias[o] + sum_c sum_k W[o, c, k] x[c, t + k - K//2];
  * GELU(x) = x Phi(x), Phi the standard normal CDF (Hendrycks & Gimpel);
  * relative L2 loss, mean over the systems of ||y - t|| / ||t||;
  * Adam (Kingma & Ba, Algorithm 1) with bias-corrected moments.

Parity: every function is pinned in tests/test_warmstart_pins.py (SciPy's
correlate, the normal CDF, central finite differences through the trunk, the
head and the loss, Adam's first step in closed form, the scaling of the
prediction, the exact start at S = 0 and the truncated Neumann series).
"""
from __future__ import annotations

import numpy as np
import scipy.special as ss


def conv1d_same(x, W, bias):
    """x (B, Cin, m), W (Cout, Cin, K), bias (Cout,) -> (B, Cout, m), zero 'same' padding."""
    B, Cin, m = x.shape
    Cout, Cin2, K = W.shape
    assert Cin == Cin2
    h = K // 2
    xp = np.zeros((B, Cin, m + 2 * h))
    xp[:, :, h:h + m] = x
    y = np.zeros((B, Cout, m))
    for k in range(K):
        # tap k reads x[t + k - h]
        y += np.einsum("oc,bct->bot", W[:, :, k], xp[:, :, k:k + m])
    return y + bias[None, :, None]


def conv1d_same_grads(x, W, gy):
    """Gradients of conv1d_same w.r.t. its input, weights and bias, given dL/dy = gy."""
    B, Cin, m = x.shape
    Cout, _, K = W.shape
    h = K // 2
    xp = np.zeros((B, Cin, m + 2 * h))
    xp[:, :, h:h + m] = x
    gW = np.zeros_like(W)
    gxp = np.zeros_like(xp)
    for k in range(K):
        gW[:, :, k] = np.einsum("bot,bct->oc", gy, xp[:, :, k:k + m])
        gxp[:, :, k:k + m] += np.einsum("oc,bot->bct", W[:, :, k], gy)
    gb = gy.sum(axis=(0, 2))
    return gxp[:, :, h:h + m], gW, gb


def gelu(x):
    """x Phi(x) with Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
    return 0.5 * x * (1.0 + ss.erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    Phi = 0.5 * (1.0 + ss.erf(x / np.sqrt(2.0)))
    phi = np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)
    return Phi + x * phi


def init_params(channels=(1, 64, 64, 64, 4), K=9, seed=0):
    """He-style uniform weights, zero biases (for CPU experiments; the library has its own)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        bound = np.sqrt(6.0 / (cin * K))
        params.append((rng.uniform(-bound, bound, (cout, cin, K)), np.zeros(cout)))
    return params


def forward(params, X):
    """Trunk output (B, D, m) of member inputs X (B, 1, m) and the pre-activations backward needs."""
    cache = []
    a = X
    for li, (W, b) in enumerate(params):
        z = conv1d_same(a, W, b)
        cache.append((a, z))
        a = gelu(z) if li < len(params) - 1 else z
    return a, cache


def backward(params, cache, gout):
    """Gradients (gW, gb) per layer of the loss whose gradient w.r.t. the trunk output is gout."""
    grads = [None] * len(params)
    g = gout
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        a_in, z = cache[li]
        if li < len(params) - 1:
            g = g * gelu_grad(z)
        gx, gW, gb = conv1d_same_grads(a_in, W, g)
        grads[li] = (gW, gb)
        g = gx
    return grads


def member_features(b):
    """Trunk input (B, 1, m) of members with right-hand sides b (B, m): bh = sqrt(m) b / ||b||."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    m = b.shape[1]
    return (np.sqrt(m) * b / np.linalg.norm(b, axis=1)[:, None])[:, None, :]


def shift_basis(s, D):
    """phi (Q, D): phi[q, d] = c_q^(d+1), c_q = 1 / (1 + s_q)."""
    c = 1.0 / (1.0 + np.asarray(s, dtype=np.float64))
    return np.stack([c ** (d + 1) for d in range(D)], axis=1)


def head(Y, phi):
    """Per-system outputs y (B, Q, m) = sum_d phi[q, d] Y[b, d] of trunk outputs Y (B, D, m)."""
    return np.einsum("qd,bdt->bqt", phi, Y)


def head_grad(gy, phi):
    """Gradient w.r.t. the trunk output Y (B, D, m) given dL/dy = gy (B, Q, m)."""
    return np.einsum("qd,bqt->bdt", phi, gy)


def predict(params, b, s):
    """Warm starts u0 (B, Q, m) of members with right-hand sides b (B, m) at the shifts s (Q,)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    Y, _ = forward(params, member_features(b))
    y = head(Y, shift_basis(s, Y.shape[1]))
    return (np.linalg.norm(b, axis=1) / np.sqrt(b.shape[1]))[:, None, None] * y


def targets(u, b):
    """Training targets u* sqrt(m) / ||b|| of exact solutions u (B, Q, m) for members b (B, m)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    return np.sqrt(b.shape[1]) * np.asarray(u) / np.linalg.norm(b, axis=1)[:, None, None]


def loss_rel_l2(Y, T):
    """mean over rows of ||Y_r - T_r|| / ||T_r|| for arrays (..., m) (every leading index a row),
    and its gradient w.r.t. Y."""
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    shape = Y.shape
    Y2 = Y.reshape(-1, shape[-1])
    T2 = T.reshape(-1, shape[-1])
    B = Y2.shape[0]
    diff = Y2 - T2
    dn = np.linalg.norm(diff, axis=1)
    tn = np.linalg.norm(T2, axis=1)
    loss = float(np.mean(dn / tn))
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(dn[:, None] > 0, diff / (dn * tn)[:, None], 0.0) / B
    return loss, g.reshape(shape)


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); state = {'t': int, 'm': [...], 'v': [...]}."""
    if not state:
        state.update(t=0, m=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                     v=[(np.zeros_like(W), np.zeros_like(b)) for W, b in params])
    state["t"] += 1
    t = state["t"]
    new = []
    for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            mj = state["m"][li][j]
            vj = state["v"][li][j]
            mj[...] = beta1 * mj + (1 - beta1) * g
            vj[...] = beta2 * vj + (1 - beta2) * g * g
            mhat = mj / (1 - beta1 ** t)
            vhat = vj / (1 - beta2 ** t)
            out.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        new.append((out[0], out[1]))
    return new
