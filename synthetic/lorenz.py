"""Multi-layer Lorenz-96 workload (stand-in for the cycled test of Sec. 5).

State layout: index = layer * nx + site, layers 0..nz-1, sites periodic.
Tendency (Sec. 5.1, eq. 5.1): advection + damping + forcing within each layer,
plus linear relaxation towards the layers directly above and below (no flux
through the top and bottom layers).
"""
from __future__ import annotations

import numpy as np

from .gaussian import Problem, config_seed, gc_table_2d


def l96_tendency(x, nz, nx, forcing, gamma):
    """x: (nz*nx, k) states; returns dx/dt with the same shape."""
    s = x.reshape(nz, nx, -1)
    adv = np.roll(s, 1, axis=1) * (np.roll(s, -1, axis=1) - np.roll(s, 2, axis=1))
    out = adv - s + forcing
    if nz > 1:
        out[1:] += gamma * (s[:-1] - s[1:])
        out[:-1] += gamma * (s[1:] - s[:-1])
    return out.reshape(nz * nx, -1)


def l96_rk4_step(x, dt, nz, nx, forcing, gamma):
    k1 = l96_tendency(x, nz, nx, forcing, gamma)
    k2 = l96_tendency(x + 0.5 * dt * k1, nz, nx, forcing, gamma)
    k3 = l96_tendency(x + 0.5 * dt * k2, nz, nx, forcing, gamma)
    k4 = l96_tendency(x + dt * k3, nz, nx, forcing, gamma)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def lorenz_problem(trial: int = 0, nz: int = 8, nx: int = 480, N: int = 20,
                   forcing: float = 8.0, gamma: float = 0.1, dt: float = 0.01,
                   steps_per_cycle: int = 5, spinup_time: float = 10.0,
                   member_sigma: float = 1.0, obs_stride: int = 3, r_var: float = 1.0,
                   c_h: float = 7.5, c_v: float = 1.0, Q: int = 12, ell: float = 1000.0):
    """One forecast ensemble of the multi-layer system with its observations.

    Truth: forcing + 0.01 noise, integrated ``spinup_time``.  Members: truth +
    N(0, member_sigma^2) noise; then truth and members are integrated one
    cycle (steps_per_cycle RK4 steps) to give the forecast ensemble.
    """
    seed = config_seed(3, trial)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = nz * nx
    pert = rng.standard_normal((n, N))                      # members first
    x0 = forcing + 0.01 * rng.standard_normal((n, 1))       # then the truth
    t = x0
    for _ in range(int(round(spinup_time / dt))):
        t = l96_rk4_step(t, dt, nz, nx, forcing, gamma)
    ens = t + member_sigma * pert
    state = np.concatenate([ens, t], axis=1)
    for _ in range(steps_per_cycle):
        state = l96_rk4_step(state, dt, nz, nx, forcing, gamma)
    X = np.asfortranarray(state[:, :N])
    truth = state[:, N].copy()
    idx = np.array([z * nx + x for z in range(nz) for x in range(0, nx, obs_stride)],
                   dtype=np.int32)
    m = idx.size
    h_ptr = np.arange(m + 1, dtype=np.int32)
    h_w = np.ones(m)
    y = truth[idx] + rng.standard_normal(m) * np.sqrt(r_var)   # then observation noise
    bz, bx, table = gc_table_2d(c_h, c_v)
    return Problem(n=n, N=N, m=m, X=X, h_ptr=h_ptr, h_idx=idx, h_w=h_w,
                   r_var=np.full(m, float(r_var)), y=y, nz=nz, nx=nx,
                   periodic_z=0, periodic_x=1, bz=bz, bx=bx, table=table, truth=truth,
                   Q=Q, ell=ell, name=f"lorenz-{nz}x{nx}-N{N}-m{m}-Q{Q}",
                   meta=dict(forcing=forcing, gamma=gamma, dt=dt, seed=seed,
                             steps_per_cycle=steps_per_cycle))
