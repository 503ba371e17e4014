"""Pins of the warm-start oracle against independent definitions (CPU only).

* the correlation against scipy.signal.correlate, channel by channel;
* GELU against x * (standard normal CDF) and its derivative against a
  central difference;
* every gradient of the loss against central finite differences (FP64);
* Adam's first step in closed form: m_hat = g, v_hat = g^2, so the step is
  -lr g / (|g| + eps);
* the prediction scales with the right-hand side (u0(c b) = c u0(b), c > 0);
* the loss and its gradient vanish at the target.
"""
import numpy as np
import pytest
import scipy.signal as sg
import scipy.stats as st

from oracle import warmstart_ref as wr


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    B, Cin, Cout, K, m = 2, 3, 4, 9, 17
    x = rng.standard_normal((B, Cin, m))
    W = rng.standard_normal((Cout, Cin, K))
    b = rng.standard_normal(Cout)
    y = wr.conv1d_same(x, W, b)
    for bi in range(B):
        for o in range(Cout):
            want = b[o] + sum(sg.correlate(x[bi, c], W[o, c], mode="same") for c in range(Cin))
            assert np.allclose(y[bi, o], want, rtol=1e-13, atol=1e-13)


def test_gelu_definition_and_derivative():
    x = np.linspace(-6, 6, 241)
    assert np.allclose(wr.gelu(x), x * st.norm.cdf(x), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (wr.gelu(x + h) - wr.gelu(x - h)) / (2 * h)
    assert np.allclose(wr.gelu_grad(x), fd, rtol=1e-8, atol=1e-9)


def _loss(params, X, phi, T):
    Y, _ = wr.forward(params, X)
    return wr.loss_rel_l2(wr.head(Y, phi), T)[0]


def test_gradients_match_finite_differences():
    """Trunk, shift head and loss together: every parameter's gradient against central
    differences of the loss."""
    rng = np.random.default_rng(2)
    params = wr.init_params(channels=(1, 4, 4, 4, 3), K=9, seed=3)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    B, m, Q = 3, 13, 4
    X = rng.standard_normal((B, 1, m))
    phi = wr.shift_basis(np.array([0.02, 0.3, 2.0, 15.0]), 3)
    T = rng.standard_normal((B, Q, m))
    Y, cache = wr.forward(params, X)
    _, gy = wr.loss_rel_l2(wr.head(Y, phi), T)
    grads = wr.backward(params, cache, wr.head_grad(gy, phi))
    h = 1e-6
    worst = 0.0
    for li, (W, b) in enumerate(params):
        for j, arr in enumerate((W, b)):
            flat = arr.reshape(-1)
            idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
            for k in idx:
                old = flat[k]
                flat[k] = old + h
                lp = _loss(params, X, phi, T)
                flat[k] = old - h
                lm = _loss(params, X, phi, T)
                flat[k] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][j].reshape(-1)[k]
                worst = max(worst, abs(fd - an) / max(1e-6, abs(fd) + abs(an)))
    assert worst < 1e-6, worst


def test_head_gradient_matches_finite_differences():
    """The head's gradient w.r.t. the trunk output, entry by entry."""
    rng = np.random.default_rng(12)
    B, D, Q, m = 2, 3, 5, 7
    Y = rng.standard_normal((B, D, m))
    phi = wr.shift_basis(rng.uniform(0.0, 20.0, Q), D)
    T = rng.standard_normal((B, Q, m))
    _, gy = wr.loss_rel_l2(wr.head(Y, phi), T)
    gY = wr.head_grad(gy, phi)
    h = 1e-6
    for idx in np.ndindex(Y.shape):
        Yp, Ym = Y.copy(), Y.copy()
        Yp[idx] += h
        Ym[idx] -= h
        fd = (wr.loss_rel_l2(wr.head(Yp, phi), T)[0] - wr.loss_rel_l2(wr.head(Ym, phi), T)[0]) / (2 * h)
        assert abs(fd - gY[idx]) <= 1e-7 * max(1.0, abs(fd)), idx


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    params = [(rng.standard_normal((2, 3, 9)), rng.standard_normal(2))]
    grads = [(rng.standard_normal((2, 3, 9)), rng.standard_normal(2))]
    lr, eps = 1e-3, 1e-8
    new = wr.adam_step(params, grads, {}, lr, eps=eps)
    for (W, b), (gW, gb), (W1, b1) in zip(params, grads, new):
        assert np.allclose(W1, W - lr * gW / (np.abs(gW) + eps), rtol=0, atol=1e-15)
        assert np.allclose(b1, b - lr * gb / (np.abs(gb) + eps), rtol=0, atol=1e-15)


def test_prediction_scales_with_rhs():
    rng = np.random.default_rng(5)
    params = wr.init_params(channels=(1, 8, 8, 8, 4), K=9, seed=6)
    b = rng.standard_normal((4, 30))
    s = np.array([0.0, 1.5, 10.0, 100.0])
    u1 = wr.predict(params, b, s)
    u2 = wr.predict(params, 7.5 * b, s)
    assert u1.shape == (4, 4, 30)
    assert np.allclose(u2, 7.5 * u1, rtol=1e-13, atol=0)


def test_shift_head_solves_the_unlocalized_limit():
    """With S = 0, C_q = (1 + s_q) I: a trunk whose first channel is its input and whose other
    channels are zero predicts the exact solution b / (1 + s_q) at every shift (the basis starts
    at c, not 1)."""
    rng = np.random.default_rng(8)
    b = rng.standard_normal((3, 20))
    s = np.array([0.5, 3.0, 40.0, 0.0])
    X = wr.member_features(b)
    Y = np.zeros((3, 4, 20))
    Y[:, 0, :] = X[:, 0, :]
    y = wr.head(Y, wr.shift_basis(s, 4))
    scale = (np.linalg.norm(b, axis=1) / np.sqrt(b.shape[1]))[:, None, None]
    exact = b[:, None, :] / (1 + s)[None, :, None]
    assert np.allclose(scale * y, exact, rtol=1e-14, atol=0)
    assert np.allclose(wr.targets(exact, b), y, rtol=1e-14)


def test_shift_head_is_the_truncated_neumann_series():
    """With Y[d] = (-S)^d bh the head is sum_{d<D} c^(d+1) (-S)^d b, the Neumann series of
    ((1 + s) I + S)^{-1} b truncated after D terms: its error against a dense solve falls like
    (c ||S||)^D for a small S (each added channel divides it by about c ||S||)."""
    rng = np.random.default_rng(9)
    m = 12
    A = rng.standard_normal((m, m))
    S = 0.05 * (A @ A.T) / m
    b = rng.standard_normal(m)
    s = np.array([0.0, 0.7])
    bh = wr.member_features(b[None, :])[0, 0]
    scale = np.linalg.norm(b) / np.sqrt(m)
    errs = []
    for D in (1, 2, 3, 4):
        Y = np.zeros((1, D, m))
        v = bh.copy()
        for d in range(D):
            Y[0, d] = v
            v = -S @ v
        u = scale * wr.head(Y, wr.shift_basis(s, D))[0]
        exact = np.stack([np.linalg.solve((1 + sq) * np.eye(m) + S, b) for sq in s])
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    rho = np.linalg.norm(S, 2)
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 1.1 * rho * e0
    assert errs[-1] < 2 * rho ** 4


def test_loss_zero_at_target():
    rng = np.random.default_rng(7)
    T = rng.standard_normal((3, 10))
    loss, g = wr.loss_rel_l2(T.copy(), T)
    assert loss == 0.0 and np.all(g == 0.0)
    loss2, _ = wr.loss_rel_l2(2 * T, T)
    assert np.isclose(loss2, 1.0)
