"""The paper's own workloads (Sec. 4 and Sec. 5), as seeded synthetic inputs.

* Section 4: a Gaussian prior on n = 2000 points of a circle, Sigma(i,j) =
  eta delta_ij + exp(-c(i,j)^2 / (2 nu^2)) with chordal distance
  c(i,j) = (n/pi) sin(pi |i-j| / n), nu = 10, eta = 1e-4; d = 100 observed
  weighted sums H(i,j) = exp(-c(j, 20 i)^2 / (2 b^2)), b = 10; R = r^2 I with
  r^2 = 10% of the mean observable variance; Gaussian localization
  exp(-c^2 / (2 L^2)), L = 12; 20 members.  H's rows and L are kept where
  their entries exceed 1e-17 of their peak (below FP64 resolution).
* Section 5: the coupled Lorenz-96 atmosphere with 32 layers of 40 sites,
  coupling 1, forcing decreasing linearly from 8 (bottom) to 4 (top); 8
  evenly spaced observed columns, 5 channels each with weights
  f_r(j) = exp(-(j - 6r)^2 / (2 8^2)) / W_r, sum_j f_r(j)^2 = 1, noise
  variance 0.25; localization G_2(sqrt(c(x,x')^2 + (y-y')^2) / 3) with the
  chordal distance on the circle of 40 sites; 40 members from 41 random
  fields integrated over 0 <= t <= 10 (the last is the truth).
"""
from __future__ import annotations

import numpy as np

from .gaussian import Problem, config_seed, gaspari_cohn
from .lorenz import l96_rk4_step


def chordal(d, n):
    return (n / np.pi) * np.sin(np.pi * np.abs(d) / n)


def experiment1_prior_row(n: int = 2000, nu: float = 10.0, eta: float = 1e-4):
    """First row of the circulant prior covariance of Sec. 4 (eq. of Sec. 4.1)."""
    row = np.exp(-chordal(np.arange(n), n) ** 2 / (2 * nu * nu))
    row[0] += eta
    return row


def experiment2_noise(cycles: int, m: int = 40, noise_var: float = 0.25, trial: int = 0):
    """Observation noise of the cycled experiment, one row per cycle."""
    rng = np.random.Generator(np.random.PCG64(config_seed(13, trial)))
    return rng.standard_normal((cycles, m)) * np.sqrt(noise_var)


def experiment1_problem(trial: int = 0, n: int = 2000, N: int = 20, d_obs: int = 100, nu: float = 10.0,
                        eta: float = 1e-4, b: float = 10.0, L: float = 12.0, Q: int = 8, ell: float = 1000.0):
    seed = config_seed(11, trial)
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.arange(n)
    row = experiment1_prior_row(n, nu, eta)
    # circulant covariance: eigenvalues are the real DFT of its first row
    lam = np.maximum(np.fft.rfft(row).real, 0.0)
    sq = np.sqrt(lam)

    def draw(k):
        w = rng.standard_normal((n, k))
        return np.fft.irfft(np.fft.rfft(w, axis=0) * sq[:, None], n=n, axis=0)

    X = np.asfortranarray(draw(N))                 # members first
    truth = draw(1)[:, 0]                          # then the truth
    h_ptr = [0]
    h_idx, h_w = [], []
    for i in range(1, d_obs + 1):
        w = np.exp(-chordal(idx - 20 * i, n) ** 2 / (2 * b * b))
        keep = np.nonzero(w > 1e-17)[0]
        h_idx.extend(keep.tolist())
        h_w.extend(w[keep].tolist())
        h_ptr.append(len(h_idx))
    h_ptr = np.asarray(h_ptr, dtype=np.int32)
    h_idx = np.asarray(h_idx, dtype=np.int32)
    h_w = np.asarray(h_w)
    # R = 10% of the mean observable variance diag(H Sigma H^T)
    Hd = np.zeros((d_obs, n))
    for k in range(d_obs):
        Hd[k, h_idx[h_ptr[k]:h_ptr[k + 1]]] = h_w[h_ptr[k]:h_ptr[k + 1]]
    HS = np.fft.irfft(np.fft.rfft(Hd, axis=1) * lam[None, :], n=n, axis=1)   # H Sigma (circulant)
    r2 = 0.1 * float(np.mean(np.sum(HS * Hd, axis=1)))
    y = Hd @ truth + rng.standard_normal(d_obs) * np.sqrt(r2)   # then observation noise
    dx = np.arange(-n // 2, n // 2 + 1)
    g = np.exp(-chordal(dx, n) ** 2 / (2 * L * L))
    bx = int(np.max(np.abs(dx[g > 1e-17])))
    dxs = np.arange(-bx, bx + 1)
    table = np.exp(-chordal(dxs, n) ** 2 / (2 * L * L)).reshape(1, -1)
    return Problem(n=n, N=N, m=d_obs, X=X, h_ptr=h_ptr, h_idx=h_idx, h_w=h_w, r_var=np.full(d_obs, r2), y=y,
                   nz=1, nx=n, periodic_z=0, periodic_x=1, bz=0, bx=bx, table=table, truth=truth, Q=Q, ell=ell,
                   name=f"paper-sec4-n{n}-N{N}-d{d_obs}", meta=dict(seed=seed, r2=r2))


def experiment2_forcing(nz: int = 32):
    return np.linspace(8.0, 4.0, nz)


def experiment2_problem(trial: int = 0, nz: int = 32, nx: int = 40, N: int = 40, gamma: float = 1.0,
                        dt: float = 0.01, steps_per_cycle: int = 5, spinup_time: float = 10.0,
                        Lloc: float = 3.0, Q: int = 8, ell: float = 1000.0, noise_var: float = 0.25):
    seed = config_seed(12, trial)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = nz * nx
    F = experiment2_forcing(nz)
    # 41 independent Gaussian random fields (white, unit variance, around the forcing of each
    # layer), integrated to t = 10; the first N are the ensemble, the last the truth
    fields = rng.standard_normal((n, N + 1))
    state = F.repeat(nx)[:, None] + fields
    forcing = F[:, None, None]   # per layer, broadcast over sites and columns
    for _ in range(int(round(spinup_time / dt))):
        state = l96_rk4_step(state, dt, nz, nx, forcing, gamma)
    X = np.asfortranarray(state[:, :N])
    truth = state[:, N].copy()
    cols = np.arange(0, nx, nx // 8)[:8]
    h_ptr, h_idx, h_w = [0], [], []
    j = np.arange(1, nz + 1)
    for c in cols:
        for r in range(1, 6):
            f = np.exp(-(j - 6 * r) ** 2 / (2 * 8.0 ** 2))
            f /= np.sqrt(np.sum(f * f))
            h_idx.extend((np.arange(nz) * nx + c).tolist())
            h_w.extend(f.tolist())
            h_ptr.append(len(h_idx))
    h_ptr = np.asarray(h_ptr, dtype=np.int32)
    h_idx = np.asarray(h_idx, dtype=np.int32)
    h_w = np.asarray(h_w)
    m = len(h_ptr) - 1
    Hd = np.zeros((m, n))
    for k in range(m):
        Hd[k, h_idx[h_ptr[k]:h_ptr[k + 1]]] = h_w[h_ptr[k]:h_ptr[k + 1]]
    y = Hd @ truth + rng.standard_normal(m) * np.sqrt(noise_var)   # then observation noise
    # localization G_2(sqrt(c(dx)^2 + dz^2) / L) with chordal horizontal distance, support 2 L
    bz = int(np.ceil(2 * Lloc)) - 1
    dxs = np.arange(-nx // 2 + 1, nx // 2)
    keep = dxs[chordal(dxs, nx) < 2 * Lloc]
    bx = int(np.max(np.abs(keep)))
    dz = np.arange(-bz, bz + 1)[:, None]
    dx = np.arange(-bx, bx + 1)[None, :]
    table = gaspari_cohn(np.sqrt(chordal(dx, nx) ** 2 + dz ** 2) / Lloc)
    return Problem(n=n, N=N, m=m, X=X, h_ptr=h_ptr, h_idx=h_idx, h_w=h_w, r_var=np.full(m, noise_var), y=y,
                   nz=nz, nx=nx, periodic_z=0, periodic_x=1, bz=bz, bx=bx, table=table, truth=truth, Q=Q, ell=ell,
                   name=f"paper-sec5-{nz}x{nx}-N{N}-d{m}",
                   meta=dict(seed=seed, forcing=F, gamma=gamma, dt=dt, steps_per_cycle=steps_per_cycle))
