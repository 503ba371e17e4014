"""Gaussian-model workloads on a periodic 1-D grid (stand-in for Sec. 4).

Draw order follows one fixed rule for every workload: ensemble members
first, then the truth, then the observation noise, all from one
``numpy.random.Generator(PCG64(seed))`` with
``seed = 250300253 + 1000 * config + trial``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 250300253


def config_seed(config: int, trial: int = 0) -> int:
    return SEED_BASE + 1000 * int(config) + int(trial)


def gaspari_cohn(r):
    """Gaspari & Cohn (1999) fifth-order piecewise rational correlation.

    Argument is distance divided by the half-width c; the function is 1 at
    0 and vanishes for r >= 2 (the localization function named in Sec. 2.3
    and Sec. 5.2 of the paper).
    """
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    a = r <= 1.0
    b = (r > 1.0) & (r < 2.0)
    ra = r[a]
    out[a] = -0.25 * ra**5 + 0.5 * ra**4 + 0.625 * ra**3 - (5.0 / 3.0) * ra**2 + 1.0
    rb = r[b]
    out[b] = (rb**5 / 12.0 - 0.5 * rb**4 + 0.625 * rb**3 + (5.0 / 3.0) * rb**2
              - 5.0 * rb + 4.0 - 2.0 / (3.0 * rb))
    return out


def gc_table_1d(c: float):
    """Stencil table of GC(|dx|/c) over its support; returns (bx, table[1, 2bx+1])."""
    bx = int(np.ceil(2.0 * c)) - 1
    while bx > 0 and gaspari_cohn((bx + 1) / c) > 0.0:
        bx += 1
    dx = np.arange(-bx, bx + 1)
    return bx, gaspari_cohn(dx / c).reshape(1, -1)


def gc_table_2d(c_h: float, c_v: float):
    """Anisotropic 2-D GC stencil: GC(sqrt((dx/c_h)^2 + (dz/c_v)^2)).

    Returns (bz, bx, table[2bz+1, 2bx+1]); entries outside the support are 0.
    """
    bz = int(np.ceil(2.0 * c_v)) - 1
    bx = int(np.ceil(2.0 * c_h)) - 1
    dz = np.arange(-bz, bz + 1)[:, None]
    dx = np.arange(-bx, bx + 1)[None, :]
    rho = np.sqrt((dx / c_h) ** 2 + (dz / c_v) ** 2)
    return bz, bx, gaspari_cohn(rho)


def periodic_distance(n: int):
    k = np.arange(n)
    return np.minimum(k, n - k).astype(np.float64)


def circulant_sqrt_sampler(n: int, length_scale: float):
    """Returns a function drawing k samples of N(0, C), C_ij = exp(-d_ij^2/(2 l^2)).

    C is circulant on the periodic grid, so its eigenvalues are the real DFT
    of its first row; negative round-off eigenvalues are clipped at 0.
    """
    d = periodic_distance(n)
    row = np.exp(-(d**2) / (2.0 * length_scale**2))
    lam = np.clip(np.fft.fft(row).real, 0.0, None)
    sq = np.sqrt(lam)

    def draw(rng, k):
        xi = rng.standard_normal((n, k))
        return np.fft.ifft(sq[:, None] * np.fft.fft(xi, axis=0), axis=0).real

    return draw


def point_obs_csr(n: int, stride: int, offset: int = 0, weight: float = 1.0):
    idx = np.arange(offset, n, stride, dtype=np.int32)
    m = idx.size
    h_ptr = np.arange(m + 1, dtype=np.int32)
    h_w = np.full(m, weight, dtype=np.float64)
    return h_ptr, idx, h_w


@dataclass
class Problem:
    """One filter instance: the arguments of the update, in host memory."""
    n: int
    N: int
    m: int
    X: np.ndarray            # n x N forecast members (column i = member i)
    h_ptr: np.ndarray        # m+1 int32
    h_idx: np.ndarray        # nnz int32 (state indices)
    h_w: np.ndarray          # nnz float64
    r_var: np.ndarray        # m float64 (diagonal of R)
    y: np.ndarray            # m float64 observations
    nz: int
    nx: int
    periodic_z: int
    periodic_x: int
    bz: int
    bx: int
    table: np.ndarray        # (2bz+1) x (2bx+1) float64
    truth: np.ndarray        # n float64
    Q: int = 8
    ell: float = 100.0
    name: str = ""
    meta: dict = field(default_factory=dict)


def gaussian_problem(n, N, length_scale, gc_c, obs_stride, r_var, Q, ell, seed, name=""):
    rng = np.random.Generator(np.random.PCG64(seed))
    draw = circulant_sqrt_sampler(n, length_scale)
    X = np.asfortranarray(draw(rng, N))           # members first
    truth = draw(rng, 1)[:, 0]                    # then the truth
    h_ptr, h_idx, h_w = point_obs_csr(n, obs_stride)
    m = h_idx.size
    noise = rng.standard_normal(m) * np.sqrt(r_var)   # then observation noise
    y = truth[h_idx] + noise
    bx, table = gc_table_1d(gc_c)
    return Problem(n=n, N=N, m=m, X=X, h_ptr=h_ptr, h_idx=h_idx, h_w=h_w,
                   r_var=np.full(m, float(r_var)), y=y, nz=1, nx=n,
                   periodic_z=0, periodic_x=1, bz=0, bx=bx, table=table,
                   truth=truth, Q=Q, ell=ell, name=name,
                   meta=dict(length_scale=length_scale, gc_c=gc_c, obs_stride=obs_stride,
                             seed=seed))


def config1(trial: int = 0) -> Problem:
    """n=256, N=16, length scale 10, GC half-width 20, every 4th point, R=0.25 I, Q=8."""
    return gaussian_problem(256, 16, 10.0, 20.0, 4, 0.25, 8, 100.0,
                            config_seed(1, trial), name="gaussian-n256-N16-m64-Q8")


def config2(trial: int = 0) -> Problem:
    """n=4096, N=40, length scale 40, GC half-width 80, every 4th point, R=0.25 I, Q=16."""
    return gaussian_problem(4096, 40, 40.0, 80.0, 4, 0.25, 16, 1000.0,
                            config_seed(2, trial), name="gaussian-n4096-N40-m1024-Q16")


def config4_instances(count: int = 64, trial: int = 0):
    """Uneven batch of independent Gaussian-model filters.

    n_j = 4*U{128..2048}, N_j in {16,32,48,64}, Q_j = U{8..24}, m_j = n_j/4,
    length scale 40, GC half-width 80, R = 0.25 I.
    """
    rng = np.random.Generator(np.random.PCG64(config_seed(4, trial)))
    specs = []
    for j in range(count):
        n = 4 * int(rng.integers(128, 2049))
        N = int(rng.choice([16, 32, 48, 64]))
        Q = int(rng.integers(8, 25))
        specs.append((n, N, Q))
    probs = []
    for j, (n, N, Q) in enumerate(specs):
        seed = config_seed(4, trial) + 7919 * (j + 1)
        probs.append(gaussian_problem(n, N, 40.0, 80.0, 4, 0.25, Q, 1000.0, seed,
                                      name=f"gaussian-batch-{j}"))
    return probs


def sketch_matrix(m: int, k: int, seed: int):
    """Gaussian test matrix for the randomized range finder (an input, drawn here)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((m, k)))
