"""FP64 reference of the cycled-assimilation model pieces (test infrastructure only).

* The coupled multi-layer Lorenz-96 tendency (Sec. 5.1, eq. 5.1): for site i
  (periodic) and layer j,
      dX_ij/dt = X_{i-1,j} (X_{i+1,j} - X_{i-2,j}) - X_ij + F_j
                 + [j > 0] g (X_{i,j-1} - X_ij) + [j < nz-1] g (X_{i,j+1} - X_ij),
  state index j * nx + i, written here with explicit loops.
* The classical fourth-order Runge-Kutta step.
* Relaxation to prior spread (Whitaker & Hamill 2012), the posterior inflation
  of the cycled experiment (Sec. 5.3): per state variable k,
      X_a'[k, :] <- X_a'[k, :] (1 + alpha (sigma_f[k] - sigma_a[k]) / sigma_a[k]),
  sigma the ensemble standard deviations of the deviation rows.

Pinned in tests/test_cycle_pins.py: energy conservation of the advection term,
zero net exchange of the layer coupling, the uniform fixed point, the fourth-
order convergence of RK4 and the limits alpha = 0 and alpha = 1 of RTPS.
"""
from __future__ import annotations

import numpy as np


def l96_tendency(x, nz, nx, forcing, gamma):
    """Tendency of states x (nz*nx,) or (nz*nx, k); forcing scalar or (nz,) per layer."""
    x = np.asarray(x, dtype=np.float64)
    squeeze = x.ndim == 1
    X = x.reshape(nz * nx, -1)
    F = np.broadcast_to(np.asarray(forcing, dtype=np.float64), (nz,))
    out = np.empty_like(X)
    for j in range(nz):
        for i in range(nx):
            k = j * nx + i
            xm1 = X[j * nx + (i - 1) % nx]
            xp1 = X[j * nx + (i + 1) % nx]
            xm2 = X[j * nx + (i - 2) % nx]
            v = xm1 * (xp1 - xm2) - X[k] + F[j]
            if j > 0:
                v = v + gamma * (X[(j - 1) * nx + i] - X[k])
            if j < nz - 1:
                v = v + gamma * (X[(j + 1) * nx + i] - X[k])
            out[k] = v
    return out[:, 0] if squeeze else out


def advection(x, nz, nx):
    """The quadratic term X_{i-1}(X_{i+1} - X_{i-2}) alone."""
    X = np.asarray(x, dtype=np.float64).reshape(nz, nx)
    out = np.empty_like(X)
    for j in range(nz):
        for i in range(nx):
            out[j, i] = X[j, (i - 1) % nx] * (X[j, (i + 1) % nx] - X[j, (i - 2) % nx])
    return out.reshape(-1)


def rk4_step(x, dt, f):
    """One classical Runge-Kutta step of dx/dt = f(x)."""
    k1 = f(x)
    k2 = f(x + 0.5 * dt * k1)
    k3 = f(x + 0.5 * dt * k2)
    k4 = f(x + dt * k3)
    return x + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def l96_forecast(X, steps, dt, nz, nx, forcing, gamma):
    """States X (n, k) advanced by `steps` RK4 steps."""
    f = lambda v: l96_tendency(v, nz, nx, forcing, gamma)  # noqa: E731
    out = np.array(X, dtype=np.float64, copy=True)
    for _ in range(steps):
        out = rk4_step(out, dt, f)
    return out


def rtps(Xf_pert, Xa_pert, alpha):
    """Relaxation to prior spread of the analysis deviations (n, N) given the forecast deviations."""
    Xf_pert = np.asarray(Xf_pert, dtype=np.float64)
    Xa_pert = np.asarray(Xa_pert, dtype=np.float64)
    N = Xf_pert.shape[1]
    sf = np.sqrt(np.sum(Xf_pert ** 2, axis=1) / (N - 1))
    sa = np.sqrt(np.sum(Xa_pert ** 2, axis=1) / (N - 1))
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(sa > 0, 1.0 + alpha * (sf - sa) / sa, 1.0)
    return Xa_pert * fac[:, None]
