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


def _loss(params, X, T):
    Y, _ = wr.forward(params, X)
    return wr.loss_rel_l2(Y[:, 0, :], T)[0]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = wr.init_params(channels=(3, 4, 4, 4, 1), K=9, seed=3)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    B, m = 3, 13
    X = rng.standard_normal((B, 3, m))
    T = rng.standard_normal((B, m))
    Y, cache = wr.forward(params, X)
    _, gY = wr.loss_rel_l2(Y[:, 0, :], T)
    grads = wr.backward(params, cache, gY[:, None, :])
    h = 1e-6
    worst = 0.0
    for li, (W, b) in enumerate(params):
        for j, arr in enumerate((W, b)):
            flat = arr.reshape(-1)
            idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
            for k in idx:
                old = flat[k]
                flat[k] = old + h
                lp = _loss(params, X, T)
                flat[k] = old - h
                lm = _loss(params, X, T)
                flat[k] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][j].reshape(-1)[k]
                worst = max(worst, abs(fd - an) / max(1e-6, abs(fd) + abs(an)))
    assert worst < 1e-6, worst


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
    params = wr.init_params(channels=(3, 8, 8, 8, 1), K=9, seed=6)
    b = rng.standard_normal((4, 30))
    s = np.array([0.0, 1.5, 10.0, 100.0])
    u1 = wr.predict(params, b, s)
    u2 = wr.predict(params, 7.5 * b, s)
    assert np.allclose(u2, 7.5 * u1, rtol=1e-13, atol=0)


def test_neumann_features_solve_the_unlocalized_limit():
    """With S = 0 the first feature times ||b|| is the exact solution b / (1 + s)."""
    rng = np.random.default_rng(8)
    b = rng.standard_normal((3, 20))
    s = np.array([0.5, 3.0, 40.0])
    X = wr.features(b, s)
    scale = (np.linalg.norm(b, axis=1) / np.sqrt(b.shape[1]))[:, None]
    assert np.allclose(scale * X[:, 0, :], b / (1 + s)[:, None], rtol=1e-14)
    assert np.allclose(X[:, 1, :] * (1 + s)[:, None], X[:, 0, :], rtol=1e-14)
    # the exact solution's target is the first feature when S = 0
    assert np.allclose(wr.targets(b / (1 + s)[:, None], b), X[:, 0, :], rtol=1e-14)


def test_loss_zero_at_target():
    rng = np.random.default_rng(7)
    T = rng.standard_normal((3, 10))
    loss, g = wr.loss_rel_l2(T.copy(), T)
    assert loss == 0.0 and np.all(g == 0.0)
    loss2, _ = wr.loss_rel_l2(2 * T, T)
    assert np.isclose(loss2, 1.0)
