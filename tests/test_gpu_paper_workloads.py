"""The paper's own workloads on the GPU, against the FP64 oracle.

* Section 4: a Gaussian prior on 2000 points of a circle observed through 100
  wide weighted channels (177 weights each), 20 members: mean and
  perturbation updates in the state domain, both covariance forms, the
  limited-memory preconditioner with 10 and 20 Ritz pairs, FP64 and mixed
  FP32 inner solves (bound 1e-6 relative, the FP64-mode target);
* the Gauss--Legendre rule of Appendix D on the same problem (nodes up to
  tan^2 of nearly pi/2, so the shifted systems run from well conditioned to
  nearly the identity): same bound against the oracle with the same nodes;
* Section 5: the 32 x 40 coupled Lorenz-96 atmosphere with 40 members and
  8 columns x 5 vertical channels: the same checks.
"""
import sys

import numpy as np
import pytest

import synthetic as syn
from oracle import infoesrf_ref as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


_CACHE = {}


def workload(name):
    if name not in _CACHE:
        prob = syn.experiment1_problem() if name == "sec4" else syn.experiment2_problem()
        _CACHE[name] = (prob, ref.DenseProblem.from_problem(prob))
    return _CACHE[name]


FORMS = {"operator": ie.COV_OPERATOR, "band": ie.COV_BAND}


@pytest.mark.parametrize("name", ["sec4", "sec5"])
@pytest.mark.parametrize("form", ["operator", "band"])
def test_mean_update(name, form):
    prob, dp = workload(name)
    say("paper mean", name, form)
    want = ref.mean_update_eig(dp, prob.y)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.mean_update(P, prob.y, ie.default_opts(cov_form=FORMS[form]))
    assert st.code == ie.OK and st.converged[0] == 1
    assert rel(got.cpu().numpy() - dp.mu, want - dp.mu) < 1e-6


@pytest.mark.parametrize("name", ["sec4", "sec5"])
@pytest.mark.parametrize("form,precision,n_ritz", [("operator", "fp64", 10), ("band", "fp64", 10),
                                                   ("band", "fp64", 20), ("band", "fp32", 20),
                                                   ("operator", "fp32", 0)])
def test_perturbation_update(name, form, precision, n_ritz):
    prob, dp = workload(name)
    say("paper perturbation", name, form, precision, n_ritz)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    prec = ie.FP64 if precision == "fp64" else ie.MIXED_FP32
    got, st = ie.perturbation_update(P, s, p, ie.default_opts(cov_form=FORMS[form], precision=prec, n_ritz=n_ritz))
    assert st.code == ie.OK
    assert np.all(st.converged == 1) and np.all(st.relres <= 1e-8)
    assert rel(got.cpu().numpy(), want) < 1e-6


@pytest.mark.parametrize("Q", [8, 16])
def test_gauss_legendre_rule(Q):
    prob, dp = workload("sec4")
    say("paper gauss-legendre", Q)
    s, p = ref.quadrature_gauss_legendre(Q)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, ie.default_opts())
    assert st.code == ie.OK and np.all(st.converged == 1)
    assert rel(got.cpu().numpy(), want) < 1e-6
    # the largest nodes make C_q close to a multiple of the identity: those systems converge fastest
    it = st.iters.reshape(Q, prob.N).max(axis=1)
    assert it[np.argmax(s)] <= it[np.argmin(s)]
