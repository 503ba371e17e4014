"""The paper's own workloads (CPU checks of their reading).

Section 4 prints one number its setting fixes: r^2 ~ 36.3, 10% of the mean
observable variance diag(H Sigma H^T).  Our reading of Sigma (chordal
distance, noise floor) and of H (Gaussian channel weights centred at 20 i)
reproduces it; a wrong lengthscale, a missing factor 2 in either exponent or
a non-chordal distance would not.  Section 5's channel weights are
normalized to unit 2-norm and peak at layer 6 r.
"""
import os

import numpy as np

import synthetic as syn

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    out = {}
    for line in open(os.path.join(HERE, "golden", name)):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            out[k] = [float(x) for x in v]
    return out


def test_sec4_observation_error_variance_matches_paper():
    want, tol = golden("sec4_obs_error_variance.txt")["r2"]
    prob = syn.experiment1_problem()
    assert abs(prob.meta["r2"] - want) < tol, prob.meta["r2"]


def test_sec4_shapes():
    prob = syn.experiment1_problem()
    assert (prob.n, prob.m, prob.N) == (2000, 100, 20)
    # localization and channels are kept down to 1e-17 of their peak
    assert prob.table.min() > 1e-17 and prob.bx > 100
    rows = np.diff(prob.h_ptr)
    assert rows.min() == rows.max() and rows[0] > 150


def test_sec5_channels_normalized():
    prob = syn.experiment2_problem(spinup_time=0.05)
    assert (prob.n, prob.m, prob.N) == (1280, 40, 40)
    nz, nx = prob.nz, prob.nx
    for k in range(prob.m):
        w = prob.h_w[prob.h_ptr[k]:prob.h_ptr[k + 1]]
        assert np.isclose(np.sum(w * w), 1.0)
        r = k % 5 + 1
        assert np.argmax(w) + 1 == min(6 * r, nz)
        cols = prob.h_idx[prob.h_ptr[k]:prob.h_ptr[k + 1]] % nx
        assert len(set(cols.tolist())) == 1
    assert np.allclose(syn.experiment2_forcing(32)[[0, -1]], [8.0, 4.0])


def test_kalman_analysis_variance_matches_dense_formula():
    """The FFT evaluation of the Sec. 4 score's reference variances against the dense Kalman
    analysis covariance Sigma - Sigma H^T (H Sigma H^T + R)^{-1} H Sigma."""
    import scipy.linalg as sla

    from paper_2503_00253_amd import experiments as ex

    prob = syn.experiment1_problem(n=400, d_obs=20)
    row = syn.experiment1_prior_row(400)
    Sig = sla.circulant(row)
    assert np.allclose(Sig, Sig.T)
    Hd = np.zeros((prob.m, prob.n))
    for k in range(prob.m):
        sl = slice(prob.h_ptr[k], prob.h_ptr[k + 1])
        Hd[k, prob.h_idx[sl]] = prob.h_w[sl]
    A = Hd @ Sig @ Hd.T + np.diag(prob.r_var)
    want = np.diag(Sig - Sig @ Hd.T @ np.linalg.solve(A, Hd @ Sig))
    got = ex.kalman_analysis_variance(prob, row)
    assert np.allclose(got, want, rtol=1e-10, atol=1e-12)
    # observations only remove variance; the analysis variance stays positive
    assert np.all(got < row[0]) and np.all(got > 0)
    # E^2 of perturbations whose variances are exact is zero, and scales as the square of a bias
    N = 9
    pert = np.sqrt(want)[:, None] * np.sqrt((N - 1) / N) * np.ones((1, N))
    assert ex.variance_error(pert, want) < 1e-24
    assert np.isclose(ex.variance_error(pert * np.sqrt(1.1), want), 0.01)
