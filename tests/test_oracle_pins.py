"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, a
worked example printed in the paper, a textbook special case, an invariant or
a brute-force evaluation on tiny inputs.
"""
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla

import synthetic as syn
from oracle import infoesrf_ref as ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_problem(n=24, N=6, stride=3, seed=1, c=3.0, r=0.3, L_ones=False, dense_H=False):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, N)) + np.linspace(0, 1, n)[:, None]
    if dense_H:
        m = n // stride
        H = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.3)
    else:
        idx = np.arange(0, n, stride)
        m = idx.size
        H = np.zeros((m, n))
        H[np.arange(m), idx] = 1.0 + 0.1 * np.arange(m)
    r_var = r * (1.0 + 0.5 * rng.random(m))
    if L_ones:
        L = np.ones((n, n))
    else:
        d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
        d = np.minimum(d, n - d)
        L = syn.gaspari_cohn(d / c)
    return ref.DenseProblem(X, H, r_var, L), rng


# ----------------------------------------------------------------- quadrature

@pytest.mark.parametrize("ell", [100.0, 1000.0])
def test_elliptic_rule_inverse_sqrt_identity(ell):
    """sum_q r_q/(s_q+1+c) -> 1/sqrt(1+c) for c in [0, ell] (hypothesis of Theorem 3)."""
    c = np.concatenate([[0.0], np.logspace(-3, np.log10(ell), 200)])
    errs = []
    for Q in (4, 8, 12, 16, 24):
        s, p, r = ref.quadrature_elliptic(Q, ell)
        approx = ref.quadrature_invsqrt(s, r, c)
        errs.append(np.max(np.abs(approx * np.sqrt(1.0 + c) - 1.0)))
    # geometric convergence at the Hale-Higham-Trefethen rate exp(-2 pi^2 Q / ln(16(1+ell)))
    rate = np.exp(-2.0 * np.pi**2 / np.log(16.0 * (1.0 + ell)))
    assert errs[-1] < 1e-12
    for Q, e in zip((4, 8, 12), errs[:3]):
        assert e < 20.0 * rate**Q, (Q, e, rate**Q)
        assert e > 0.02 * rate**Q, (Q, e, rate**Q)


def test_elliptic_weights_sum_to_one():
    """c = 0 in Theorem 3 gives sum_q p_q -> 1."""
    for Q, tol in ((8, 1e-5), (16, 1e-12)):
        _, p, _ = ref.quadrature_elliptic(Q, 1000.0)
        assert abs(p.sum() - 1.0) < tol
        assert np.all(p > 0)


def test_theorem2_density_and_identity():
    """p(s) = [pi sqrt(s)(s+1)]^-1 integrates to 1, and the generic form gives 1/sqrt(1+c) (App. B)."""
    val, _ = si.quad(lambda t: 1.0 / (np.pi * np.sqrt(t) * (t + 1.0)), 0, np.inf, limit=400)
    assert abs(val - 1.0) < 1e-8
    for c in (0.5, 7.0, 90.0):
        val, _ = si.quad(lambda t: 1.0 / (np.pi * np.sqrt(t) * (t + 1.0 + c)), 0, np.inf, limit=400)
        assert abs(val - 1.0 / np.sqrt(1.0 + c)) < 1e-8


def test_scalar_gain_worked_example():
    """Appendix D's scalar example: both rules converge to 20/(11+sqrt(11)); elliptic much faster."""
    sxh, shh, G = np.loadtxt(os.path.join(GOLDEN, "scalar_gain.txt"))
    assert abs(G - sxh / (1.0 + shh + np.sqrt(1.0 + shh))) < 1e-15
    def gain(s, p):
        return np.sum(p * sxh / (1.0 + s + shh))
    e_ell = [abs(gain(*ref.quadrature_elliptic(Q, 100.0)[:2]) - G) / G for Q in (8, 16)]
    e_gl = [abs(gain(*ref.quadrature_gauss_legendre(Q)) - G) / G for Q in (8, 16, 128)]
    assert e_ell[0] < 1e-7 and e_ell[1] < 1e-14
    assert e_gl[2] < 1e-10                       # the trig rule converges too
    assert e_ell[0] < 0.01 * e_gl[0] and e_ell[1] < 0.01 * e_gl[1]


def test_gauss_legendre_rule_identity():
    """Trig rule (App. D, eq. D.2): sum_q p_q/(s_q+1+c) (1+c) ... converges to the gain factor."""
    c = np.array([0.0, 1.0, 10.0, 100.0])
    s, p = ref.quadrature_gauss_legendre(200)
    approx = (p[None, :] / (1.0 + s[None, :] + c[:, None])).sum(axis=1)
    exact = 1.0 / (1.0 + c + np.sqrt(1.0 + c))
    assert np.max(np.abs(approx - exact) / exact) < 1e-9
    assert abs(p.sum() - 1.0) < 1e-13


# ----------------------------------------------------------------- covariance

def test_localization_stencil_matches_distance_definition():
    """Stencil-built L equals GC(d_ij/c) from periodic distances (Sec. 2.3, Sec. 4.2 style)."""
    n, c = 50, 4.0
    bx, table = syn.gc_table_1d(c)
    L = ref.dense_localization(1, n, 0, 1, 0, bx, table)
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    d = np.minimum(d, n - d)
    assert np.array_equal(L, syn.gaspari_cohn(d / c))
    Ls = ref.sparse_localization(1, n, 0, 1, 0, bx, table).toarray()
    assert np.array_equal(Ls, L)


def test_localization_2d_matches_definition():
    nz, nx, ch, cv = 4, 30, 3.0, 1.0
    bz, bx, table = syn.gc_table_2d(ch, cv)
    L = ref.dense_localization(nz, nx, 0, 1, bz, bx, table)
    zz, xx = np.divmod(np.arange(nz * nx), nx)
    dx = np.abs(xx[:, None] - xx[None, :]); dx = np.minimum(dx, nx - dx)
    dz = np.abs(zz[:, None] - zz[None, :])
    expect = syn.gaspari_cohn(np.sqrt((dx / ch) ** 2 + (dz / cv) ** 2))
    assert np.allclose(L, expect, atol=0, rtol=1e-15)
    assert np.allclose(ref.sparse_localization(nz, nx, 0, 1, bz, bx, table).toarray(), L)


def test_farchi_bocquet_operator_equals_dense_and_is_psd():
    dp, rng = tiny_problem()
    v = rng.standard_normal(dp.Z.shape[0])
    fb = ref.cov_apply_fb_loops(dp.Z, dp.L, v)
    # brute force: P_jk = L_jk sum_i z_ji z_ki
    n, N = dp.Z.shape
    Pb = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            Pb[j, k] = dp.L[j, k] * sum(dp.Z[j, i] * dp.Z[k, i] for i in range(N))
    assert np.allclose(fb, Pb @ v, rtol=1e-13, atol=1e-13)
    assert np.allclose(dp.P, Pb, rtol=1e-14, atol=1e-15)
    assert np.linalg.eigvalsh(dp.P).min() > -1e-12           # Schur product theorem


def test_matrix_free_operator_matches_dense_S():
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    op = ref.FBOperator(prob)
    U = np.random.default_rng(3).standard_normal((prob.m, 5))
    assert np.allclose(op(U), dp.S @ U, rtol=1e-12, atol=1e-12)
    assert np.allclose(op.diag(), np.diag(dp.S), rtol=1e-13)


def test_ensemble_stats_definition():
    X = np.arange(12.0).reshape(4, 3) ** 1.5
    mu, Z = ref.ensemble_stats(X)
    assert np.allclose(mu, [np.mean(r) for r in X])
    assert np.allclose(Z @ Z.T, np.cov(X), rtol=1e-13)     # ZZ^T is the sample covariance


# ----------------------------------------------------------------- updates

@pytest.mark.parametrize("dense_H", [False, True])
def test_mean_update_eig_matches_cholesky(dense_H):
    dp, rng = tiny_problem(dense_H=dense_H)
    y = rng.standard_normal(dp.H.shape[0])
    a = ref.mean_update_eig(dp, y)
    b = ref.mean_update_cholesky(dp, y)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # residual check of the gain system: (R + H P H^T) v = d with K d = P H^T v
    d = y - dp.H @ dp.mu
    v = np.linalg.lstsq(dp.PHt, a - dp.mu, rcond=None)[0]
    A = np.diag(dp.r_var) + dp.H @ dp.P @ dp.H.T
    assert np.linalg.norm(A @ v - d) < 1e-9 * np.linalg.norm(d)


@pytest.mark.parametrize("dense_H", [False, True])
def test_finite_Q_update_matches_per_node_solves(dense_H):
    dp, _ = tiny_problem(dense_H=dense_H)
    s, p, _ = ref.quadrature_elliptic(8, 100.0)
    a = ref.perturbation_update_nodes(dp, s, p)
    b = ref.perturbation_update_quadrature(dp, s, p)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-13)


def test_finite_Q_converges_to_exact_at_quadrature_rate():
    dp, _ = tiny_problem()
    ell = 10 ** np.ceil(np.log10(2 * dp.lam.max()))
    Zex = ref.perturbation_update_exact(dp)
    errs = []
    for Q in (2, 4, 8, 16):
        s, p, _ = ref.quadrature_elliptic(Q, ell)
        Za = ref.perturbation_update_quadrature(dp, s, p)
        errs.append(np.linalg.norm(Za - Zex) / np.linalg.norm(Zex))
    assert errs[-1] < 1e-13
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_proposition1_modified_gain():
    """Integral form equals G of eq. 2.6, built here with a literal matrix square root."""
    for dense_H in (False, True):
        dp, _ = tiny_problem(dense_H=dense_H)
        G = ref.modified_gain_sqrtm(dp)
        assert np.allclose(ref.perturbation_update_exact(dp), dp.Z - G @ dp.W, rtol=1e-10, atol=1e-12)


def test_operator_covariance_identity():
    """(I - G H) P (I - G H)^T = (I - K H) P (Theorem 3 for the localized operator)."""
    dp, _ = tiny_problem(dense_H=True)
    G = ref.modified_gain_sqrtm(dp)
    K = ref.kalman_gain(dp)
    I = np.eye(dp.P.shape[0])
    lhs = (I - G @ dp.H) @ dp.P @ (I - G @ dp.H).T
    rhs = (I - K @ dp.H) @ dp.P
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(rhs)


def test_unlocalized_ensemble_identities():
    """L = 1: Z_a Z_a^T = (I-KH) Z Z^T and the symmetric ETKF transform Z (I + V^T V)^{-1/2}."""
    dp, _ = tiny_problem(L_ones=True)
    Za = ref.perturbation_update_exact(dp)
    K = ref.kalman_gain(dp)
    I = np.eye(dp.P.shape[0])
    assert np.allclose(Za @ Za.T, (I - K @ dp.H) @ dp.Z @ dp.Z.T, rtol=1e-11, atol=1e-12)
    V = dp.dinv[:, None] * dp.W
    T = sla.fractional_matrix_power(np.eye(dp.N) + V.T @ V, -0.5)
    assert np.allclose(Za, dp.Z @ np.real(T), rtol=1e-11, atol=1e-12)


def test_single_observation_serial_esrf_closed_form():
    """One observation: G = P h^T / (sigma + r + sqrt(r (sigma + r))) (Whitaker-Hamill factor)."""
    dp, rng = tiny_problem()
    h = np.zeros((1, dp.P.shape[0])); h[0, 5] = 1.3; h[0, 6] = -0.4
    r = np.array([0.7])
    one = ref.DenseProblem(dp.X, h, r, dp.L)
    sigma = float(h @ one.P @ h.T)
    G = (one.P @ h.T) / (sigma + r[0] + np.sqrt(r[0] * (sigma + r[0])))
    assert np.allclose(ref.perturbation_update_exact(one), one.Z - G @ one.W, rtol=1e-13, atol=1e-15)


def test_large_R_limit():
    dp, _ = tiny_problem(r=1e12)
    s, p, _ = ref.quadrature_elliptic(8, 100.0)
    Za = ref.perturbation_update_quadrature(dp, s, p)
    assert np.linalg.norm(Za - dp.Z) < 1e-9 * np.linalg.norm(dp.Z)


def test_analysis_ensemble_roundtrip():
    dp, _ = tiny_problem()
    Xa = ref.analysis_ensemble(dp.mu, dp.Z)
    assert np.allclose(Xa, dp.X, rtol=1e-14, atol=1e-14)


# ----------------------------------------------------------------- preconditioner and PCG

def test_lmp_cluster_with_exact_eigenvectors():
    """With exact eigenpairs, P^{-1} C has p eigenvalues at beta, the rest inside [lmin, lmax] (App. E)."""
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    p_r = 10
    Phi = dp.E[:, ::-1][:, :p_r]
    th = dp.lam[::-1][:p_r]
    for sigma in (0.0, 3.7):
        C = (1.0 + sigma) * np.eye(prob.m) + dp.S
        M = ref.LimitedMemoryPreconditioner(Phi, dp.S @ Phi, th, np.diag(dp.S), sigma)
        Pinv = np.column_stack([M(e) for e in np.eye(prob.m)])
        ev = np.sort(np.linalg.eigvals(Pinv @ C).real)
        beta = 1.0 + sigma + np.diag(dp.S).min()
        assert np.sum(np.abs(ev - beta) < 1e-10 * beta) >= p_r
        lo, hi = np.linalg.eigvalsh(C)[[0, -1]]
        assert ev.min() >= lo * (1 - 1e-10) and ev.max() <= hi * (1 + 1e-10)
        assert lo <= beta <= hi


def test_randomized_eig_top_ritz_values():
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    Om = syn.sketch_matrix(prob.m, 30, 5)
    Phi, SPhi, th = ref.randomized_eig(lambda V: dp.S @ V, Om, 5)
    top = dp.lam[::-1][:5]
    assert np.allclose(th, top, rtol=2e-2)
    assert np.allclose(Phi.T @ Phi, np.eye(5), atol=1e-12)
    assert np.allclose(SPhi, dp.S @ Phi, atol=1e-11)


def test_pcg_matches_dense_solve():
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    b = dp.B[:, 3]
    Om = syn.sketch_matrix(prob.m, 20, 9)
    Phi, SPhi, th = ref.randomized_eig(lambda V: dp.S @ V, Om, 10)
    for sigma in (0.01, 2.0):
        C = (1.0 + sigma) * np.eye(prob.m) + dp.S
        M = ref.LimitedMemoryPreconditioner(Phi, SPhi, th, np.diag(dp.S), sigma)
        x, k, ok = ref.pcg(lambda v: C @ v, b, M, rtol=1e-12)
        x0, k0, _ = ref.pcg(lambda v: C @ v, b, None, rtol=1e-12)
        xs = np.linalg.solve(C, b)
        assert ok and np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)
        assert np.linalg.norm(x0 - xs) < 1e-10 * np.linalg.norm(xs)
        assert k <= k0


def test_matrix_free_update_matches_dense_oracle():
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    Om = syn.sketch_matrix(prob.m, 20, 11)
    Za, iters = ref.info_esrf_pcg(prob, s, p, rtol=1e-12, Omega=Om)
    Zd = ref.perturbation_update_quadrature(dp, s, p)
    assert np.linalg.norm(Za - Zd) < 1e-9 * np.linalg.norm(Zd)
    assert iters.min() >= 1


def _galerkin(A, K, b):
    """The A-orthogonal projection of A^{-1} b onto span(K): CG's optimality over a Krylov space."""
    c = np.linalg.solve(K.T @ A @ K, K.T @ b)
    return K @ c


@pytest.mark.parametrize("workload", ["config1", "paper-sec4"])
def test_matrix_free_mean_update_matches_dense(workload):
    prob = syn.config1() if workload == "config1" else syn.experiment1_problem()
    dp = ref.DenseProblem.from_problem(prob)
    Om = syn.sketch_matrix(prob.m, 20, 5)
    mu_a, k = ref.info_esrf_mean_pcg(prob, prob.y, rtol=1e-12, Omega=Om)
    want = ref.mean_update_eig(dp, prob.y)
    assert np.linalg.norm(mu_a - want) < 1e-9 * np.linalg.norm(want - dp.mu)
    assert k >= 1


def test_fixed_count_pcg_is_krylov_galerkin_projection():
    """k PCG iterations from zero give the A-norm-optimal point of the k-dimensional
    preconditioned Krylov space span{M b, (M A) M b, ...} (exact arithmetic; checked at k = 1, 2),
    with M the limited-memory preconditioner (SPD) or the identity."""
    prob = syn.experiment1_problem()
    dp = ref.DenseProblem.from_problem(prob)
    Om = syn.sketch_matrix(prob.m, 30, 8)
    Phi, SPhi, th = ref.randomized_eig(lambda V: dp.S @ V, Om, 20)
    b = dp.B[:, 4]
    for sigma in (0.0, 3.0):
        A = (1.0 + sigma) * np.eye(prob.m) + dp.S
        pre = ref.LimitedMemoryPreconditioner(Phi, SPhi, th, np.diag(dp.S), sigma)
        for M in (None, pre):
            Mi = (lambda v: v) if M is None else M
            z0 = Mi(b)
            K = np.column_stack([z0, Mi(A @ z0)])
            for k in (1, 2):
                x, its, _ = ref.pcg(lambda v: A @ v, b, M, rtol=0.0, max_iter=k)
                want = _galerkin(A, K[:, :k], b)
                assert its == k
                assert np.linalg.norm(x - want) < 1e-10 * np.linalg.norm(want)
    # the one-step mean update is the steepest-descent step along R^{-1/2} d, mapped by P H^T R^{-1/2}
    mu_a, k = ref.info_esrf_mean_pcg(prob, prob.y, rtol=0.0, n_ritz=0, max_iter=1)
    d = dp.dinv * (prob.y - dp.H @ dp.mu)
    A0 = np.eye(prob.m) + dp.S
    step = (d @ d) / (d @ A0 @ d) * d
    assert k == 1
    assert np.linalg.norm(mu_a - dp.mu - dp.gain_apply(step[:, None])[:, 0]) < 1e-10 * np.linalg.norm(mu_a - dp.mu)


def _krylov(A, v, k):
    """Orthonormal basis of span{v, A v, ..., A^{k-1} v} (Gram-Schmidt twice per column)."""
    Q = np.zeros((v.size, 0))
    w = v.copy()
    for _ in range(k):
        for _ in range(2):
            w = w - Q @ (Q.T @ w)
        Q = np.column_stack([Q, w / np.linalg.norm(w)])
        w = A @ Q[:, -1]
    return Q


def test_multishift_cg_iterates_are_shifted_galerkin_projections():
    """k steps of multi-shift CG give, for every shift, the A_sigma-norm-optimal point of the
    common Krylov space K_k(A, b) (k = 1..4, exact arithmetic), and converged runs solve every
    shifted system."""
    prob = syn.experiment1_problem()
    dp = ref.DenseProblem.from_problem(prob)
    base = 1.0 + 0.02
    A = base * np.eye(prob.m) + dp.S
    b = dp.B[:, 3]
    shifts = np.array([0.0, 0.3, 2.0, 40.0, 1e4])
    for k in (1, 2, 3, 4):
        X, its = ref.multishift_cg(lambda v: A @ v, b, shifts, rtol=0.0, max_iter=k)
        K = _krylov(A, b, k)
        assert np.all(its == k)
        for j, sg in enumerate(shifts):
            want = _galerkin(A + sg * np.eye(prob.m), K, b)
            assert np.linalg.norm(X[:, j] - want) < 1e-10 * np.linalg.norm(want), (k, sg)
    X, its = ref.multishift_cg(lambda v: A @ v, b, shifts, rtol=1e-12, max_iter=500)
    for j, sg in enumerate(shifts):
        want = np.linalg.solve(A + sg * np.eye(prob.m), b)
        assert np.linalg.norm(X[:, j] - want) < 1e-10 * np.linalg.norm(want)
    # larger shifts are better conditioned and stop no later; the base runs longest
    assert np.all(np.diff(its) <= 0) and its[0] == its.max()
    # one shift of 0 is plain CG
    x, k0, _ = ref.pcg(lambda v: A @ v, b, None, rtol=1e-12)
    assert its[0] in (k0 - 1, k0, k0 + 1)
    assert np.linalg.norm(X[:, 0] - x) < 1e-11 * np.linalg.norm(x)


def test_block_cg_iterates_are_block_krylov_galerkin_projections():
    """k steps of block PCG give, for every column, the A-norm-optimal point of the sum of the
    columns' preconditioned Krylov spaces span{M B, (M A) M B, ...} (k = 1, 2, 3), with the
    limited-memory preconditioner and without; converged runs solve every column."""
    prob = syn.experiment1_problem()
    dp = ref.DenseProblem.from_problem(prob)
    A = (1.0 + 0.5) * np.eye(prob.m) + dp.S
    B = dp.B[:, :6]
    Om = syn.sketch_matrix(prob.m, 20, 3)
    Phi, SPhi, th = ref.randomized_eig(lambda V: dp.S @ V, Om, 10)
    lmp = ref.LimitedMemoryPreconditioner(Phi, SPhi, th, np.diag(dp.S), 0.5)
    Mblk = lambda V: np.column_stack([lmp(V[:, j]) for j in range(V.shape[1])])
    for M in (None, Mblk):
        Mi = (lambda V: V) if M is None else M
        blocks = [Mi(B)]
        for k in (1, 2, 3):
            X, its = ref.block_cg(lambda V: A @ V, B, M, rtol=0.0, max_iter=k)
            K = np.column_stack(blocks)
            want = K @ np.linalg.solve(K.T @ A @ K, K.T @ B)
            assert its == k
            assert np.linalg.norm(X - want) < 1e-9 * np.linalg.norm(want), (k, M is None)
            blocks.append(Mi(A @ blocks[-1]))
        X, its = ref.block_cg(lambda V: A @ V, B, M, rtol=1e-12, max_iter=500)
        want = np.linalg.solve(A, B)
        assert np.linalg.norm(X - want) < 1e-10 * np.linalg.norm(want)
        # the block method needs no more iterations than single-column CG on its hardest column
        single = max(ref.pcg(lambda v: A @ v, B[:, j], None if M is None else lmp, rtol=1e-12)[1]
                     for j in range(B.shape[1]))
        assert its <= single


def test_multishift_and_block_updates_match_dense_oracle():
    prob = syn.config1()
    dp = ref.DenseProblem.from_problem(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = ref.perturbation_update_quadrature(dp, s, p)
    Za, it_ms = ref.info_esrf_multishift(prob, s, p, rtol=1e-12)
    assert np.linalg.norm(Za - want) < 1e-9 * np.linalg.norm(want)
    q0 = int(np.argmin(s))
    assert np.all(it_ms[q0] == it_ms.max(axis=0))
    Om = syn.sketch_matrix(prob.m, 20, 4)
    Zb, it_b = ref.info_esrf_block_cg(prob, s, p, rtol=1e-12, Omega=Om)
    assert np.linalg.norm(Zb - want) < 1e-9 * np.linalg.norm(want)
    _, it_pcg = ref.info_esrf_pcg(prob, s, p, rtol=1e-12, Omega=Om)
    assert np.all(it_b <= it_pcg.max(axis=1))
