"""Pins of the cycled-model oracle (CPU only).

* the advection term conserves energy: sum_i X_i X_{i-1}(X_{i+1} - X_{i-2}) = 0
  for any state (a telescoping identity of Lorenz-96);
* the layer coupling only exchanges between layers: its sum over the column is 0;
* a uniform state X = F is a fixed point (advection and coupling vanish);
* RK4 is fourth order: halving dt divides the error at a fixed time by ~16;
* RTPS: alpha = 0 leaves the analysis unchanged, alpha = 1 restores the
  forecast spread exactly, and the factor is one per row.
"""
import numpy as np

from oracle import cycle_ref as cr


def test_advection_conserves_energy():
    rng = np.random.default_rng(1)
    for nz, nx in ((1, 40), (3, 17), (8, 12)):
        x = rng.standard_normal(nz * nx) * 3
        adv = cr.advection(x, nz, nx)
        for j in range(nz):
            row = slice(j * nx, (j + 1) * nx)
            assert abs(np.dot(x[row], adv[row])) < 1e-11 * np.dot(x[row], x[row]) * np.abs(x).max()


def test_coupling_exchanges_only():
    rng = np.random.default_rng(2)
    nz, nx, g = 5, 9, 0.7
    x = rng.standard_normal(nz * nx)
    # with the other terms removed (F = X = damping cancels) the column sum of the coupling is 0
    full = cr.l96_tendency(x, nz, nx, 0.0, g)
    base = cr.l96_tendency(x, nz, nx, 0.0, 0.0)
    coup = (full - base).reshape(nz, nx)
    assert np.allclose(coup.sum(axis=0), 0.0, atol=1e-13)
    assert np.abs(coup).max() > 0.1


def test_uniform_forcing_state_is_fixed_point():
    nz, nx = 4, 11
    F = np.array([8.0, 7.0, 6.0, 5.0])
    x = np.repeat(F, nx)
    t = cr.l96_tendency(x, nz, nx, F, 0.0)
    assert np.allclose(t, 0.0, atol=1e-14)
    assert np.allclose(cr.l96_tendency(np.full(nz * nx, 8.0), nz, nx, 8.0, 0.3), 0.0, atol=1e-14)


def test_rk4_is_fourth_order():
    rng = np.random.default_rng(3)
    nz, nx, F, g = 2, 20, 8.0, 0.1
    x0 = F + rng.standard_normal(nz * nx)
    T = 0.2
    ref = cr.l96_forecast(x0[:, None], 800, T / 800, nz, nx, F, g)
    errs = []
    for steps in (10, 20, 40):
        e = np.linalg.norm(cr.l96_forecast(x0[:, None], steps, T / steps, nz, nx, F, g) - ref)
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_rtps_limits():
    rng = np.random.default_rng(4)
    n, N = 30, 10
    Xf = rng.standard_normal((n, N)) * 2
    Xf -= Xf.mean(axis=1, keepdims=True)
    Xa = 0.3 * Xf + 0.1 * rng.standard_normal((n, N))
    Xa -= Xa.mean(axis=1, keepdims=True)
    assert np.array_equal(cr.rtps(Xf, Xa, 0.0), Xa)
    out = cr.rtps(Xf, Xa, 1.0)
    assert np.allclose(out.std(axis=1, ddof=1), Xf.std(axis=1, ddof=1), rtol=1e-13)
    half = cr.rtps(Xf, Xa, 0.5)
    ratio = half / Xa
    assert np.allclose(ratio, ratio[:, :1], rtol=1e-13)   # one factor per state variable
