"""FP64 reference of the InFo-ESRF update (test infrastructure only).

Notation follows the paper: forecast members x^(i) (columns of X, i=1..N),
normalized perturbations Z and W = HZ (eq. 2.9), localized covariance
P = L o (Z Z^T) (eq. 2.11), normalized observation covariance
S = R^{-1/2} H P H^T R^{-1/2} (the matrix called C in Theorem 3), shifted
normalized matrices C_q = (1+s_q) I + S (Appendix E, eq. E.1), quadrature
nodes/weights (s_q, p_q) (Sec. 3.2 and Appendix D).

Every routine is written for clarity, not speed.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.special as ss

# ---------------------------------------------------------------------------
# Ensemble statistics and covariance (Sec. 2.2, eq. 2.9; Sec. 2.3, eq. 2.11)
# ---------------------------------------------------------------------------


def ensemble_stats(X):
    """Ensemble mean and normalized perturbations Z = (X - mu 1^T)/sqrt(N-1) (eq. 2.9)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[1]
    mu = X.sum(axis=1) / N
    Z = (X - mu[:, None]) / np.sqrt(N - 1.0)
    return mu, Z


def stencil_offset(a, b, n, periodic):
    """Signed offset b - a on a line of n points (wrapped to the nearest image if periodic)."""
    d = b - a
    if periodic:
        d = (d + n // 2) % n - n // 2
    return d


def dense_localization(nz, nx, periodic_z, periodic_x, bz, bx, table):
    """Dense n x n localization matrix L from a symmetric stencil (Sec. 2.3).

    State index = z*nx + x; L[(z1,x1),(z2,x2)] = table[dz+bz, dx+bx] when
    |dz|<=bz and |dx|<=bx (offsets wrapped on periodic axes), else 0.
    """
    table = np.asarray(table, dtype=np.float64).reshape(2 * bz + 1, 2 * bx + 1)
    n = nz * nx
    L = np.zeros((n, n))
    for z1 in range(nz):
        for z2 in range(nz):
            dz = stencil_offset(z1, z2, nz, periodic_z)
            if abs(dz) > bz:
                continue
            for x1 in range(nx):
                for dx in range(-bx, bx + 1):
                    x2 = x1 + dx
                    if periodic_x:
                        x2 %= nx
                    elif x2 < 0 or x2 >= nx:
                        continue
                    L[z1 * nx + x1, z2 * nx + x2] = table[dz + bz, dx + bx]
    return L


def sparse_localization(nz, nx, periodic_z, periodic_x, bz, bx, table):
    """The same L as ``dense_localization`` as a SciPy CSR matrix (for large n)."""
    table = np.asarray(table, dtype=np.float64).reshape(2 * bz + 1, 2 * bx + 1)
    rows, cols, vals = [], [], []
    x1 = np.arange(nx)
    for z1 in range(nz):
        for dz in range(-bz, bz + 1):
            z2 = z1 + dz
            if periodic_z:
                z2 %= nz
            elif z2 < 0 or z2 >= nz:
                continue
            for dx in range(-bx, bx + 1):
                w = table[dz + bz, dx + bx]
                if w == 0.0:
                    continue
                x2 = x1 + dx
                if periodic_x:
                    ok = np.ones(nx, dtype=bool)
                    x2 = x2 % nx
                else:
                    ok = (x2 >= 0) & (x2 < nx)
                rows.append(z1 * nx + x1[ok])
                cols.append(z2 * nx + x2[ok])
                vals.append(np.full(ok.sum(), w))
    n = nz * nx
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def dense_obs_operator(h_ptr, h_idx, h_w, n):
    """Dense m x n linear observation operator H from CSR lists (Sec. 2.3)."""
    m = len(h_ptr) - 1
    H = np.zeros((m, n))
    for k in range(m):
        for e in range(h_ptr[k], h_ptr[k + 1]):
            H[k, h_idx[e]] += h_w[e]
    return H


def localized_covariance(Z, L):
    """P = L o (Z Z^T) (eq. 2.11); PSD by the Schur product theorem."""
    return np.asarray(L) * (Z @ Z.T)


def cov_apply_dense(Z, L, V):
    """P V with the assembled dense P."""
    return localized_covariance(Z, L) @ V


def cov_apply_fb_loops(Z, L, v):
    """Farchi--Bocquet operator form sum_i z_i o (L (z_i o v)) (eq. 2.12), one member at a time."""
    out = np.zeros(Z.shape[0])
    for i in range(Z.shape[1]):
        out += Z[:, i] * (L @ (Z[:, i] * v))
    return out


def normalized_obs_cov(H, P, r_var):
    """S = R^{-1/2} H P H^T R^{-1/2} (the matrix C of Theorem 3), symmetrized."""
    d = 1.0 / np.sqrt(np.asarray(r_var, dtype=np.float64))
    S = d[:, None] * (H @ P @ H.T) * d[None, :]
    return 0.5 * (S + S.T)


# ---------------------------------------------------------------------------
# Quadrature rules (Appendix D)
# ---------------------------------------------------------------------------


def quadrature_elliptic(Q, ell):
    """Hale--Higham--Trefethen elliptic rule (Appendix D, eq. D.1), real-variable reading.

    With k^2 = ell/(1+ell) (k is the paper's g) and K = K(k^2), midpoints
    u_q = (q - 1/2) K / Q, and Jacobi functions at (u_q | k^2):
        s_q = (sn/cn)^2,  r_q = (2K/(pi Q)) dn/cn^2,  p_q = r_q/(1+s_q).
    This is the printed rule after Jacobi's imaginary transformation
    (|sn(i u|k')|^2 = sc^2(u|k), |cn dn(i u|k')| = dn/cn^2 (u|k)), with the
    modulus read so that the integral identity of Theorem 3 holds.
    Returns (s, p, r).
    """
    mpar = ell / (1.0 + ell)
    K = ss.ellipk(mpar)
    u = (np.arange(1, Q + 1) - 0.5) * K / Q
    sn, cn, dn, _ = ss.ellipj(u, mpar)
    s = (sn / cn) ** 2
    r = (2.0 * K / (np.pi * Q)) * dn / cn**2
    p = r / (1.0 + s)
    return s, p, r


def quadrature_gauss_legendre(Q):
    """Trigonometric rule with Gauss--Legendre nodes (Appendix D, eq. D.2).

    s_q = tan^2(pi lambda_q / 2), p_q = v_q / 2 with (lambda_q, v_q) the
    Gauss--Legendre nodes and weights on [-1, 1].  Returns (s, p).
    """
    lam, v = np.polynomial.legendre.leggauss(Q)
    return np.tan(0.5 * np.pi * lam) ** 2, 0.5 * v


def quadrature_invsqrt(s, r, c):
    """sum_q r_q / (s_q + 1 + c): the discretized left side of Theorem 3's hypothesis."""
    c = np.atleast_1d(np.asarray(c, dtype=np.float64))
    return (r[None, :] / (s[None, :] + 1.0 + c[:, None])).sum(axis=1)


# ---------------------------------------------------------------------------
# Exact (dense) updates
# ---------------------------------------------------------------------------


class DenseProblem:
    """Dense pieces of one update: mu, Z, W, P, H, S and its eigendecomposition."""

    def __init__(self, X, H, r_var, L):
        self.X = np.asarray(X, dtype=np.float64)
        self.H = np.asarray(H, dtype=np.float64)
        self.r_var = np.asarray(r_var, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.mu, self.Z = ensemble_stats(self.X)
        self.N = self.X.shape[1]
        self.W = self.H @ self.Z
        self.P = localized_covariance(self.Z, self.L)
        self.dinv = 1.0 / np.sqrt(self.r_var)
        self.S = normalized_obs_cov(self.H, self.P, self.r_var)
        self.lam, self.E = np.linalg.eigh(self.S)
        self.B = self.dinv[:, None] * self.W          # b_i = R^{-1/2} w_i
        self.PHt = self.P @ self.H.T                  # localized Sigma_xh

    @classmethod
    def from_problem(cls, prob):
        H = dense_obs_operator(prob.h_ptr, prob.h_idx, prob.h_w, prob.n)
        L = dense_localization(prob.nz, prob.nx, prob.periodic_z, prob.periodic_x,
                               prob.bz, prob.bx, prob.table)
        return cls(prob.X, H, prob.r_var, L)

    def gain_apply(self, U):
        """P H^T R^{-1/2} U: maps normalized-system solutions to state space."""
        return self.PHt @ (self.dinv[:, None] * U)

    def spectral(self, g, V):
        """E g(Lambda) E^T V."""
        return self.E @ (g(self.lam)[:, None] * (self.E.T @ V))


def mean_update_eig(dp, y):
    """Mean update (Sec. 3.2, eq. 3.4): mu_a = mu + P H^T R^{-1/2} (I+S)^{-1} R^{-1/2}(y - H mu)."""
    d = np.asarray(y) - dp.H @ dp.mu
    u0 = dp.spectral(lambda lam: 1.0 / (1.0 + lam), (dp.dinv * d)[:, None])
    return dp.mu + dp.gain_apply(u0)[:, 0]


def mean_update_cholesky(dp, y):
    """The same mean through a Cholesky solve of (R + H P H^T) v = y - H mu (eq. 2.2)."""
    d = np.asarray(y) - dp.H @ dp.mu
    A = np.diag(dp.r_var) + dp.H @ dp.P @ dp.H.T
    v = sla.cho_solve(sla.cho_factor(0.5 * (A + A.T)), d)
    return dp.mu + dp.PHt @ v


def perturbation_update_nodes(dp, s, p):
    """Finite-Q update, following Sec. 3.2 step by step with one dense solve per (q, i).

    v_q^(i) solves ((s_q+1) R + H P H^T) v = w^(i)  (eq. 3.5);
    z_a^(i) = z^(i) - P H^T sum_q p_q v_q^(i).
    """
    A0 = dp.H @ dp.P @ dp.H.T
    R = np.diag(dp.r_var)
    acc = np.zeros_like(dp.W)
    for q in range(len(s)):
        Aq = (s[q] + 1.0) * R + A0
        for i in range(dp.N):
            acc[:, i] += p[q] * np.linalg.solve(Aq, dp.W[:, i])
    return dp.Z - dp.PHt @ acc


def perturbation_update_quadrature(dp, s, p):
    """Finite-Q update by eigendecomposition (the GPU parity target).

    u_bar_i = E gQ(Lambda) E^T b_i with gQ(lam) = sum_q p_q/(1+s_q+lam), then
    z_a^(i) = z^(i) - P H^T R^{-1/2} u_bar_i (Appendix E, eq. E.1 with Sec. 3.2).
    """
    s = np.asarray(s, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)

    def gQ(lam):
        return (p[None, :] / (1.0 + s[None, :] + lam[:, None])).sum(axis=1)

    Ubar = dp.spectral(gQ, dp.B)
    return dp.Z - dp.gain_apply(Ubar)


def perturbation_update_exact(dp):
    """Q -> infinity limit (Proposition 1): z_a = z - G w with
    G = P H^T R^{-1/2} E g(Lambda) E^T R^{-1/2}, g(lam) = 1/(1+lam+sqrt(1+lam))."""
    Ubar = dp.spectral(lambda lam: 1.0 / (1.0 + lam + np.sqrt(1.0 + lam)), dp.B)
    return dp.Z - dp.gain_apply(Ubar)


def modified_gain_sqrtm(dp):
    """G of eq. 2.6 evaluated literally with a matrix square root (scipy.linalg.sqrtm)."""
    R = np.diag(dp.r_var)
    Shh = dp.H @ dp.P @ dp.H.T
    root = sla.sqrtm(np.eye(len(dp.r_var)) + np.linalg.solve(R, Shh))
    M = R + Shh + R @ np.real(root)
    return np.linalg.solve(M.T, dp.PHt.T).T


def kalman_gain(dp):
    """K = P H^T (R + H P H^T)^{-1} (eq. 2.2 with the localized covariances)."""
    A = np.diag(dp.r_var) + dp.H @ dp.P @ dp.H.T
    return np.linalg.solve(A, dp.PHt.T).T


def analysis_ensemble(mu_a, Za):
    """X_a = mu_a 1^T + sqrt(N-1) Z_a (inverse of eq. 2.9)."""
    N = Za.shape[1]
    return mu_a[:, None] + np.sqrt(N - 1.0) * Za


# ---------------------------------------------------------------------------
# Matrix-free operator, limited-memory preconditioner and PCG (Appendix E)
# ---------------------------------------------------------------------------


class FBOperator:
    """Matrix-free normalized observation covariance S (eq. 2.12 with H and R^{-1/2}).

    S u = R^{-1/2} H sum_i z_i o L (z_i o (H^T R^{-1/2} u)).
    """

    def __init__(self, prob=None, *, Z=None, Hs=None, r_var=None, Ls=None):
        if prob is not None:
            _, Z = ensemble_stats(prob.X)
            m = prob.m
            Hs = sp.csr_matrix((prob.h_w, prob.h_idx, prob.h_ptr), shape=(m, prob.n))
            Ls = sparse_localization(prob.nz, prob.nx, prob.periodic_z, prob.periodic_x,
                                     prob.bz, prob.bx, prob.table)
            r_var = prob.r_var
        self.Z = Z
        self.H = sp.csr_matrix(Hs)
        self.L = sp.csr_matrix(Ls)
        self.dinv = 1.0 / np.sqrt(np.asarray(r_var, dtype=np.float64))
        self.m = self.H.shape[0]
        self.applies = 0

    def cov(self, V):
        """P V for state-space V (n x B): sum_i z_i o L (z_i o V)."""
        V = np.atleast_2d(V.T).T
        out = np.zeros_like(V)
        for i in range(self.Z.shape[1]):
            zi = self.Z[:, i][:, None]
            out += zi * (self.L @ (zi * V))
        return out

    def __call__(self, U):
        U = np.asarray(U, dtype=np.float64)
        one = U.ndim == 1
        U2 = U[:, None] if one else U
        self.applies += U2.shape[1]
        V = self.H.T @ (self.dinv[:, None] * U2)
        out = self.dinv[:, None] * (self.H @ self.cov(V))
        return out[:, 0] if one else out

    def diag(self):
        """diag(S)_k = (1/r_k) sum_i (h_k o z_i)^T L (h_k o z_i)."""
        out = np.zeros(self.m)
        for k in range(self.m):
            hk = self.H.getrow(k).toarray()[0]
            nzs = np.nonzero(hk)[0]
            Lk = self.L[nzs][:, nzs].toarray()
            for i in range(self.Z.shape[1]):
                v = hk[nzs] * self.Z[nzs, i]
                out[k] += v @ Lk @ v
        return out * self.dinv**2


def randomized_eig(apply_S, Omega, p):
    """Randomized symmetric eigendecomposition (Halko et al. range finder + direct eig).

    Y = S Omega; Qb = orth(Y); T = Qb^T (S Qb); T = V diag(theta) V^T.
    Returns the p largest Ritz pairs: Phi = Qb V_p, S Phi = (S Qb) V_p, theta_p.
    """
    Y = apply_S(Omega)
    Qb, _ = np.linalg.qr(Y)
    SQ = apply_S(Qb)
    T = Qb.T @ SQ
    T = 0.5 * (T + T.T)
    th, V = np.linalg.eigh(T)
    order = np.argsort(th)[::-1][:p]
    return Qb @ V[:, order], SQ @ V[:, order], th[order]


class LimitedMemoryPreconditioner:
    """P_q^{-1} of Appendix E for C_q = (1+sigma) I + S with Ritz pairs of S.

    P^{-1} = (I - Phi Theta^{-1} Phi^T C)(I - C Phi Theta^{-1} Phi^T) + beta Phi Theta^{-1} Phi^T,
    Theta = diag(1+sigma+theta_S), C Phi = S Phi + (1+sigma) Phi, beta = min_k C(k,k).
    """

    def __init__(self, Phi, SPhi, theta_S, diagS, sigma):
        self.Phi = Phi
        self.CPhi = SPhi + (1.0 + sigma) * Phi
        self.theta = theta_S + 1.0 + sigma
        self.beta = 1.0 + sigma + float(np.min(diagS))

    def __call__(self, r):
        c1 = (self.Phi.T @ r) / self.theta
        t = r - self.CPhi @ c1
        c2 = (self.CPhi.T @ t) / self.theta
        return t - self.Phi @ c2 + self.beta * (self.Phi @ c1)


def pcg(apply_A, b, precond=None, rtol=1e-8, max_iter=1000, x0=None):
    """Preconditioned conjugate gradients (Golub & Van Loan, Alg. 11.5.1).

    Stops when ||r_k||_2 <= rtol * ||b||_2 (recursive residual).
    Returns (x, iterations, converged).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, True
    if np.linalg.norm(r) <= rtol * bnorm:
        return x, 0, True
    Mi = precond if precond is not None else (lambda v: v)
    z = Mi(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, max_iter + 1):
        Ap = apply_A(p)
        alpha = rz / (p @ Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        if np.linalg.norm(r) <= rtol * bnorm:
            return x, k, True
        z = Mi(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter, False


def info_esrf_pcg(prob, s, p, rtol=1e-8, n_ritz=10, Omega=None, max_iter=1000,
                  members=None, nodes=None):
    """Matrix-free InFo-ESRF perturbation update with PCG + limited-memory preconditioner.

    Follows Sec. 3.2 and Appendix E: b_i = R^{-1/2} w_i; solve C_q u = b_i by
    PCG for each (q, i); u_bar_i = sum_q p_q u_{q,i};
    z_a^(i) = z^(i) - P H^T R^{-1/2} u_bar_i.  ``members``/``nodes`` restrict
    the work to a subset (used for bounded CPU timing samples).
    Returns (Za_subset, iterations[q, i]).
    """
    op = FBOperator(prob)
    mu, Z = ensemble_stats(prob.X)
    W = op.H @ Z
    B = op.dinv[:, None] * W
    members = list(range(prob.N)) if members is None else list(members)
    nodes = list(range(len(s))) if nodes is None else list(nodes)
    if n_ritz > 0:
        Phi, SPhi, th = randomized_eig(op, Omega, n_ritz)
        dS = op.diag()
    iters = np.zeros((len(nodes), len(members)), dtype=np.int64)
    Ubar = np.zeros((prob.m, len(members)))
    for a, q in enumerate(nodes):
        pre = LimitedMemoryPreconditioner(Phi, SPhi, th, dS, s[q]) if n_ritz > 0 else None
        for c, i in enumerate(members):
            u, k, _ = pcg(lambda v, sh=s[q]: (1.0 + sh) * v + op(v), B[:, i], pre, rtol, max_iter)
            iters[a, c] = k
            Ubar[:, c] += p[q] * u
    Vs = op.H.T @ (op.dinv[:, None] * Ubar)
    return Z[:, members] - op.cov(Vs), iters


def info_esrf_mean_pcg(prob, y, rtol=1e-8, n_ritz=10, Omega=None, max_iter=1000):
    """Matrix-free mean update (Sec. 3.2, eq. 3.4) with PCG on (I + S) u0 = R^{-1/2} d,
    d = y - H mu, preconditioned as the perturbation systems are (Appendix E at shift 0),
    then mu_a = mu + P H^T R^{-1/2} u0.  With rtol = 0 the solve runs exactly max_iter
    iterations (the fixed counts of Sec. 4 and Sec. 5).  Returns (mu_a, iterations).
    """
    op = FBOperator(prob)
    mu, _ = ensemble_stats(prob.X)
    d = np.asarray(y, dtype=np.float64) - op.H @ mu
    pre = None
    if n_ritz > 0:
        Phi, SPhi, th = randomized_eig(op, Omega, n_ritz)
        pre = LimitedMemoryPreconditioner(Phi, SPhi, th, op.diag(), 0.0)
    u0, k, _ = pcg(lambda v: v + op(v), op.dinv * d, pre, rtol, max_iter)
    v = op.H.T @ (op.dinv * u0)
    return mu + op.cov(v[:, None])[:, 0], k


# ---------------------------------------------------------------------------
# Sec. 3.2's alternatives to one PCG process per (q, i)
# ---------------------------------------------------------------------------


def multishift_cg(apply_A, b, shifts, rtol=1e-8, max_iter=1000):
    """One CG process for A x = b that also solves (A + sigma I) x = b for every sigma >= 0 in
    `shifts` (Sec. 3.2, first alternative: the Krylov spaces of shifted matrices coincide).

    The shifted residuals stay parallel to the base residual, r_sigma = zeta_sigma r, and the
    shifted iterates follow from the base CG scalars (alpha_k, beta_k) by the coupled recurrences
        zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1}
                     / (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} alpha_{k-1} (1 + sigma alpha_k)),
        alpha^sigma_k = alpha_k zeta_{k+1} / zeta_k,  beta^sigma_k = (zeta_{k+1} / zeta_k)^2 beta_k,
        x^sigma += alpha^sigma_k p^sigma,  p^sigma = zeta_{k+1} r_{k+1} + beta^sigma_k p^sigma,
    with zeta_{-1} = zeta_0 = 1, alpha_{-1} = 1, beta_{-1} = 0, x^sigma_0 = 0, p^sigma_0 = b.  No
    preconditioner (a shift-dependent one would break the shared Krylov space).  A shift stops
    when |zeta| ||r|| <= rtol ||b||; the process stops when every shift has.  With rtol = 0 it runs
    exactly max_iter iterations.  Returns (X with one column per shift, iterations per shift).
    """
    b = np.asarray(b, dtype=np.float64)
    shifts = np.asarray(shifts, dtype=np.float64)
    ns = shifts.size
    X = np.zeros((b.size, ns))
    its = np.zeros(ns, dtype=np.int64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return X, its
    r = b.copy()
    p = b.copy()
    Ps = np.repeat(b[:, None], ns, axis=1)
    z_prev = np.ones(ns)
    z = np.ones(ns)
    alpha_prev, beta_prev = 1.0, 0.0
    rr = r @ r
    live = np.ones(ns, dtype=bool)
    for k in range(1, max_iter + 1):
        Ap = apply_A(p)
        alpha = rr / (p @ Ap)
        r = r - alpha * Ap
        rr_new = r @ r
        beta = rr_new / rr
        for j in np.nonzero(live)[0]:
            den = alpha * beta_prev * (z_prev[j] - z[j]) + z_prev[j] * alpha_prev * (1.0 + shifts[j] * alpha)
            z_new = z[j] * z_prev[j] * alpha_prev / den
            a_j = alpha * z_new / z[j]
            b_j = (z_new / z[j]) ** 2 * beta
            X[:, j] += a_j * Ps[:, j]
            Ps[:, j] = z_new * r + b_j * Ps[:, j]
            z_prev[j], z[j] = z[j], z_new
            its[j] = k
            if abs(z_new) * np.sqrt(rr_new) <= rtol * bnorm:
                live[j] = False
        p = r + beta * p
        alpha_prev, beta_prev, rr = alpha, beta, rr_new
        if not live.any():
            break
    return X, its


def info_esrf_multishift(prob, s, p, rtol=1e-8, max_iter=1000):
    """Perturbation update (Sec. 3.2) with one multi-shift CG process per member: the base
    system is the smallest shift, C_min = (1 + min s) I + S, and every node is a shift of it.
    Returns (Za, iterations[q, i])."""
    op = FBOperator(prob)
    _, Z = ensemble_stats(prob.X)
    B = op.dinv[:, None] * (op.H @ Z)
    s = np.asarray(s, dtype=np.float64)
    q0 = int(np.argmin(s))
    base = 1.0 + s[q0]
    Ubar = np.zeros((prob.m, prob.N))
    iters = np.zeros((len(s), prob.N), dtype=np.int64)
    for i in range(prob.N):
        U, its = multishift_cg(lambda v: base * v + op(v), B[:, i], s - s[q0], rtol, max_iter)
        Ubar[:, i] = U @ np.asarray(p, dtype=np.float64)
        iters[:, i] = its
    Vs = op.H.T @ (op.dinv[:, None] * Ubar)
    return Z - op.cov(Vs), iters


def block_cg(apply_A, B, precond=None, rtol=1e-8, max_iter=1000, drop=1e-12):
    """Block (P)CG for A X = B over all columns of B together (Sec. 3.2, second alternative;
    O'Leary's method): each column's iterate is the A-norm-optimal point of the SUM of the
    columns' (preconditioned) Krylov spaces.

    Every iteration A-orthonormalizes the search block: with G = P^T A P = V diag(lam) V^T,
    directions whose lam <= drop * max(lam) are dropped (a rank-deficient block loses nothing
    of its span), Pt = P V lam^{-1/2}, and then
        X += Pt (Pt^T R),   R -= (A Pt)(Pt^T R),   Zb = M R,   P = Zb - Pt ((A Pt)^T Zb),
    the last step making the next block A-orthogonal to the current one (the block CG short
    recurrence).  Stops when every column has ||r_j|| <= rtol ||b_j||; rtol = 0 runs exactly
    max_iter iterations.  Returns (X, iterations).
    """
    B = np.atleast_2d(np.asarray(B, dtype=np.float64).T).T
    X = np.zeros_like(B)
    R = B.copy()
    bn = np.linalg.norm(B, axis=0)
    Mi = precond if precond is not None else (lambda V: V)
    P = Mi(R)
    if np.all(np.linalg.norm(R, axis=0) <= rtol * bn):
        return X, 0
    k = 0
    for k in range(1, max_iter + 1):
        W = apply_A(P)
        G = P.T @ W
        lam, V = np.linalg.eigh(0.5 * (G + G.T))
        keep = lam > drop * lam.max()
        T = V[:, keep] / np.sqrt(lam[keep])
        Pt, Wt = P @ T, W @ T
        a = Pt.T @ R
        X = X + Pt @ a
        R = R - Wt @ a
        if np.all(np.linalg.norm(R, axis=0) <= rtol * bn):
            break
        Zb = Mi(R)
        P = Zb - Pt @ (Wt.T @ Zb)
    return X, k


def info_esrf_block_cg(prob, s, p, rtol=1e-8, n_ritz=10, Omega=None, max_iter=1000):
    """Perturbation update (Sec. 3.2) with one block PCG per node q over the N members'
    right-hand sides, with the node's limited-memory preconditioner (Appendix E).
    Returns (Za, iterations per node)."""
    op = FBOperator(prob)
    _, Z = ensemble_stats(prob.X)
    B = op.dinv[:, None] * (op.H @ Z)
    if n_ritz > 0:
        Phi, SPhi, th = randomized_eig(op, Omega, n_ritz)
        dS = op.diag()
    Ubar = np.zeros((prob.m, prob.N))
    iters = np.zeros(len(s), dtype=np.int64)
    for q in range(len(s)):
        pre = None
        if n_ritz > 0:
            lmp = LimitedMemoryPreconditioner(Phi, SPhi, th, dS, s[q])
            pre = lambda V, lmp=lmp: np.column_stack([lmp(V[:, j]) for j in range(V.shape[1])])
        U, k = block_cg(lambda V, sh=s[q]: (1.0 + sh) * V + op(V), B, pre, rtol, max_iter)
        Ubar += p[q] * U
        iters[q] = k
    Vs = op.H.T @ (op.dinv[:, None] * Ubar)
    return Z - op.cov(Vs), iters
