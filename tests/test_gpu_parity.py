"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances:
* covariance apply, FP64: 1e-13 relative (rounding order only);
* covariance apply, FP32: 1e-6 relative (stated bound of the FP32 apply);
* mean and perturbation updates at rtol = 1e-8: 1e-6 relative (Frobenius),
  the FP64-mode target; PCG at rtol gives ||u - u*|| <= kappa * rtol, and the
  correction term is a fraction of Z, so the observed error is far smaller;
* at rtol = 1e-12: 1e-9.
"""
import sys

import numpy as np
import pytest

import synthetic as syn
from parity import rel, upd  # noqa: E402
from oracle import infoesrf_ref as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)




def stencil_problem(nz, nx, pz, px, ch, cv, N, stride, seed, r=0.3):
    rng = np.random.default_rng(seed)
    n = nz * nx
    X = rng.standard_normal((n, N)) + 0.5 * np.sin(np.arange(n) / 7.0)[:, None]
    if nz == 1:
        bx, table = syn.gc_table_1d(ch)
        bz = 0
    else:
        bz, bx, table = syn.gc_table_2d(ch, cv)
    idx = np.array([z * nx + x for z in range(nz) for x in range(0, nx, stride)], dtype=np.int32)
    m = idx.size
    h_ptr = np.arange(m + 1, dtype=np.int32)
    h_w = 1.0 + 0.25 * np.cos(np.arange(m))
    r_var = r * (1.0 + 0.5 * rng.random(m))
    y = rng.standard_normal(m)
    return syn.Problem(n=n, N=N, m=m, X=np.asfortranarray(X), h_ptr=h_ptr, h_idx=idx, h_w=h_w, r_var=r_var, y=y,
                       nz=nz, nx=nx, periodic_z=pz, periodic_x=px, bz=bz, bx=bx, table=table,
                       truth=np.zeros(n), Q=8, ell=100.0, name=f"stencil-{nz}x{nx}")


CASES = {
    "gauss-n256-periodic": lambda: syn.config1(),
    "ragged-1d-nonperiodic": lambda: stencil_problem(1, 203, 0, 0, 6.5, 1.0, 7, 3, 11),
    "small-nx-periodic": lambda: stencil_problem(1, 40, 0, 1, 3.0, 1.0, 5, 2, 12),
    "2d-layers": lambda: stencil_problem(4, 50, 0, 1, 3.0, 1.0, 6, 2, 13),
    "2d-periodic-z": lambda: stencil_problem(6, 37, 1, 1, 2.5, 1.0, 5, 1, 14),
    # every point observed, 40 members: a block's lattice window (3 rows of 64 + 11 columns) with
    # the members of its 64 state points needs 92 KiB of LDS, past the 64 KiB the rectangular
    # state x lattice band allows, so the final state-space apply takes the state band instead
    "2d-full-obs-40": lambda: stencil_problem(4, 50, 0, 1, 3.0, 1.0, 40, 1, 15),
}


def dense_of(prob):
    return ref.DenseProblem.from_problem(prob)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("B", [1, 17, 40])
def test_cov_apply_fp64_matches_dense(case, B):
    prob = CASES[case]()
    say("cov_apply fp64", case, "B", B)
    dp = dense_of(prob)
    V = np.random.default_rng(B).standard_normal((prob.n, B))
    want = dp.P @ V
    P = ie.Problem.from_synthetic(prob)
    variants = [dict(cov_form=ie.COV_OPERATOR, tile_rows=r) for r in (16, 64, 128)] + [dict(cov_form=ie.COV_BAND)]
    for kw in variants:
        got = ie.cov_apply(P, torch.from_numpy(V).cuda(), ie.default_opts(**kw)).cpu().numpy()
        assert rel(got, want) < 1e-13, (case, B, kw)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("case", sorted(CASES))
def test_cov_apply_fp32_stated_bound(case):
    prob = CASES[case]()
    say("cov_apply fp32", case)
    dp = dense_of(prob)
    V = np.random.default_rng(3).standard_normal((prob.n, 20))
    want = dp.P @ V
    P = ie.Problem.from_synthetic(prob)
    for form in (ie.COV_OPERATOR, ie.COV_BAND):
        got = ie.cov_apply(P, torch.from_numpy(V).cuda(),
                           ie.default_opts(precision=ie.MIXED_FP32, cov_form=form)).cpu().numpy()
        assert rel(got, want) < 1e-6, form


def test_cov_apply_dense_localization():
    prob = CASES["ragged-1d-nonperiodic"]()
    say("cov_apply dense L")
    dp = dense_of(prob)
    V = np.random.default_rng(5).standard_normal((prob.n, 9))
    P = ie.Problem(prob.X, prob.h_ptr, prob.h_idx, prob.h_w, prob.r_var, dense=dp.L)
    got = ie.cov_apply(P, torch.from_numpy(V).cuda()).cpu().numpy()
    assert rel(got, dp.P @ V) < 1e-13


# operator / band: every PCG apply goes through P in that form; dense-s: S assembled once as an
# m x m matrix (from the band of P when the automatic choice of P's form takes it)
FORMS = {"operator": dict(cov_form=ie.COV_OPERATOR, s_form=ie.S_OPERATOR),
         "band": dict(cov_form=ie.COV_BAND, s_form=ie.S_OPERATOR),
         "dense-s": dict(s_form=ie.S_DENSE)}


def opts_for(prob, P, domain, form=None, **kw):
    if form is not None:
        kw.update(FORMS[form])
    if domain == "lattice":
        lat = P.lattice()
        assert lat is not None
        return ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat, **kw)
    return ie.default_opts(**kw)


@pytest.mark.parametrize("form", ["operator", "band", "dense-s"])
@pytest.mark.parametrize("domain", ["state", "lattice"])
@pytest.mark.parametrize("case", ["gauss-n256-periodic", "ragged-1d-nonperiodic", "2d-layers"])
def test_mean_update_matches_oracle(case, domain, form):
    prob = CASES[case]()
    say("mean_update", case, domain, form)
    dp = dense_of(prob)
    want = ref.mean_update_eig(dp, prob.y)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.mean_update(P, prob.y, opts_for(prob, P, domain, form))
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert upd(got.cpu().numpy() - dp.mu, want - dp.mu) < 1e-6
    assert st.relres[0] <= 1e-8 and st.converged[0] == 1


@pytest.mark.parametrize("form", ["operator", "band", "dense-s"])
@pytest.mark.parametrize("domain", ["state", "lattice"])
@pytest.mark.parametrize("case", ["gauss-n256-periodic", "ragged-1d-nonperiodic", "2d-layers", "2d-periodic-z"])
def test_perturbation_update_matches_oracle(case, domain, form):
    prob = CASES[case]()
    say("perturbation_update", case, domain, form)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, form))
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert np.all(st.relres <= 1e-8) and np.all(st.converged == 1)
    assert st.counter(ie.CNT_NOT_CONVERGED) == 0
    assert st.counter(ie.CNT_ITERATIONS) == int(st.iters.sum())


@pytest.mark.parametrize("precision", ["fp64", "mixed-fp32"])
def test_lattice_update_past_the_rectangular_band(precision):
    prob = CASES["2d-full-obs-40"]()
    say("mean + perturbation update, lattice, state-band final apply", precision)
    dp = dense_of(prob)
    P = ie.Problem.from_synthetic(prob)
    kw = dict(precision=ie.MIXED_FP32) if precision == "mixed-fp32" else {}
    o = opts_for(prob, P, "lattice", "band", **kw)
    got, st = ie.mean_update(P, prob.y, o)
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), ref.mean_update_eig(dp, prob.y)) < 1e-6
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    got, st = ie.perturbation_update(P, s, p, o)
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert np.all(st.relres <= 1e-8) and np.all(st.converged == 1)


def test_perturbation_update_tight_tolerance():
    prob = syn.config1()
    say("perturbation_update rtol 1e-12")
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, ie.default_opts(rtol=1e-12))
    assert upd(got.cpu().numpy(), want) < 1e-9
    assert np.all(st.relres <= 1e-12)


def test_pcg_iterations_match_oracle_pcg():
    """Same sketch -> same preconditioner: per-system iteration counts agree with the CPU PCG (+-1)."""
    prob = syn.config1()
    say("iteration counts vs oracle PCG")
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    Om = syn.sketch_matrix(prob.m, 20, 77)
    _, it_ref = ref.info_esrf_pcg(prob, s, p, rtol=0.5e-8, Omega=Om)
    P = ie.Problem.from_synthetic(prob)
    Omt = torch.from_numpy(np.ascontiguousarray(Om.T)).cuda()  # column-major m x k
    _, st = ie.perturbation_update(P, s, p, ie.default_opts(sketch=Omt))
    got = st.iters.reshape(prob.Q, prob.N)
    assert np.max(np.abs(got - it_ref)) <= 1, (got, it_ref)


@pytest.mark.parametrize("solver", [ie.SOLVER_PLAIN, ie.SOLVER_COMPACT])
def test_solvers_agree_and_are_deterministic(solver):
    prob = syn.config1()
    say("solver", solver)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    P = ie.Problem.from_synthetic(prob)
    # run to run bit-identical, with the persistent kernel (the compacted solver's default) and
    # without it
    for tail in (0, -1):
        a, sa = ie.perturbation_update(P, s, p, ie.default_opts(solver=solver, tail_systems=tail))
        b, sb = ie.perturbation_update(P, s, p, ie.default_opts(solver=solver, tail_systems=tail))
        assert torch.equal(a, b)
        assert np.array_equal(sa.iters, sb.iters)
    # the batched compacted loop runs the same arithmetic as the masked one; the persistent kernel
    # sums its applies and dots in another order
    c, _ = ie.perturbation_update(P, s, p, ie.default_opts(solver=ie.SOLVER_COMPACT, tail_systems=-1))
    assert rel(a.cpu().numpy(), c.cpu().numpy()) < 1e-12
    d, _ = ie.perturbation_update(P, s, p, ie.default_opts(solver=ie.SOLVER_COMPACT))
    assert rel(a.cpu().numpy(), d.cpu().numpy()) < 1e-9


@pytest.mark.parametrize("form", ["operator", "band", "dense-s"])
@pytest.mark.parametrize("domain", ["state", "lattice"])
def test_mixed_fp32_meets_fp64_bound(domain, form):
    prob = syn.config1()
    say("mixed fp32", domain, form)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, form, precision=ie.MIXED_FP32))
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert np.all(st.relres <= 1e-8)
    assert st.counter(ie.CNT_SWEEPS) >= prob.Q * prob.N  # every system had at least one FP64 check


def test_not_converged_is_reported():
    prob = syn.config1()
    say("max_iter=2 -> warning")
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    P = ie.Problem.from_synthetic(prob)
    _, st = ie.perturbation_update(P, s, p, ie.default_opts(max_iter=2))
    assert st.code == ie.WARN_NOT_CONVERGED
    assert st.counter(ie.CNT_NOT_CONVERGED) > 0
    assert np.any(st.converged == 0)
    assert np.all(st.iters <= 2 + 1)


def test_nan_input_is_an_error():
    prob = syn.config1()
    say("NaN in X")
    X = prob.X.copy()
    X[5, 3] = np.nan
    P = ie.Problem(X, prob.h_ptr, prob.h_idx, prob.h_w, prob.r_var, nx=prob.nx, bx=prob.bx, table=prob.table)
    s, p, _ = ref.quadrature_elliptic(4, 100.0)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p)
    assert e.value.code == ie.ERR_NUMERIC


def test_bad_observation_operator_is_an_error():
    prob = syn.config1()
    s, p, _ = ref.quadrature_elliptic(4, 100.0)
    say("out-of-range CSR index")
    idx = prob.h_idx.copy()
    idx[3] = prob.n + 5
    P = ie.Problem(prob.X, prob.h_ptr, idx, prob.h_w, prob.r_var, nx=prob.nx, bx=prob.bx, table=prob.table)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p)
    assert e.value.code == ie.ERR_INVALID_ARG
    say("r_var <= 0")
    rv = prob.r_var.copy()
    rv[0] = 0.0
    P = ie.Problem(prob.X, prob.h_ptr, prob.h_idx, prob.h_w, rv, nx=prob.nx, bx=prob.bx, table=prob.table)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p)
    assert e.value.code == ie.ERR_INVALID_ARG
    say("wrong lattice claim")
    P = ie.Problem.from_synthetic(prob)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p, ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE,
                                                        lattice=(0, 1, 1, 1, 4, 64)))
    assert e.value.code == ie.ERR_INVALID_ARG
    say("out-of-range index under a true lattice claim")
    P = ie.Problem(prob.X, prob.h_ptr, idx, prob.h_w, prob.r_var, nx=prob.nx, bx=prob.bx, table=prob.table)
    lat = ie.Problem.from_synthetic(prob).lattice()
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p, ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat))
    assert e.value.code == ie.ERR_INVALID_ARG


def test_indefinite_localization_is_not_spd():
    """A localization far from PSD makes p^T C p <= 0 at some iteration."""
    prob = syn.config1()
    say("indefinite L -> NOT_SPD")
    n = prob.n
    L = np.zeros((n, n))
    L[np.arange(n), np.arange(n)] = 1.0
    L[np.arange(n), (np.arange(n) + 4) % n] = -40.0
    L[(np.arange(n) + 4) % n, np.arange(n)] = -40.0
    P = ie.Problem(prob.X, prob.h_ptr, prob.h_idx, prob.h_w, prob.r_var, dense=L)
    s, p, _ = ref.quadrature_elliptic(4, 100.0)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p, ie.default_opts(n_ritz=0))
    assert e.value.code in (ie.ERR_NOT_SPD, ie.ERR_NUMERIC)


@pytest.mark.parametrize("form", ["operator", "band"])
@pytest.mark.parametrize("domain", ["lattice", "state"])
def test_full_size_gaussian_n4096(domain, form):
    """n=4096, N=40, m=1024, Q=16 (640 systems) against the eigendecomposition oracle."""
    prob = syn.config2()
    say("full size n4096", domain, form)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, form))
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert np.all(st.relres <= 1e-8)
    mean_want = ref.mean_update_eig(dp, prob.y)
    mean_got, sm = ie.mean_update(P, prob.y, opts_for(prob, P, domain, form))
    assert upd(mean_got.cpu().numpy() - dp.mu, mean_want - dp.mu) < 1e-6


@pytest.mark.parametrize("case", sorted(CASES))
def test_cov_apply_bf16_stated_bound(case):
    """BF16 operands, FP32 accumulation: stated bound 1e-2 relative."""
    prob = CASES[case]()
    say("cov_apply bf16", case)
    dp = dense_of(prob)
    V = np.random.default_rng(4).standard_normal((prob.n, 37))
    want = dp.P @ V
    P = ie.Problem.from_synthetic(prob)
    for tile in (16, 32, 64, 128):
        got = ie.cov_apply(P, torch.from_numpy(V).cuda(),
                           ie.default_opts(precision=ie.MIXED_BF16, tile_rows=tile)).cpu().numpy()
        assert rel(got, want) < 1e-2, (case, tile, rel(got, want))


@pytest.mark.parametrize("domain", ["state", "lattice"])
@pytest.mark.parametrize("case", ["gauss-n256-periodic", "2d-layers"])
def test_mixed_bf16_meets_fp64_bound(case, domain):
    prob = CASES[case]()
    say("mixed bf16", case, domain)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, precision=ie.MIXED_BF16))
    assert st.code == ie.OK
    assert upd(got.cpu().numpy(), want) < 1e-6
    assert np.all(st.relres <= 1e-8)
    assert st.counter(ie.CNT_SWEEPS) >= prob.Q * prob.N


def test_mixed_bf16_full_size_lattice():
    prob = syn.config2()
    say("mixed bf16 n4096 lattice")
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, "lattice", precision=ie.MIXED_BF16))
    assert st.code == ie.OK and np.all(st.relres <= 1e-8)
    assert upd(got.cpu().numpy(), want) < 1e-6


def test_band_form_options():
    """The band form takes FP64 and FP32 only; BF16 asks for the operator form."""
    prob = syn.config1()
    say("band form option checks")
    P = ie.Problem.from_synthetic(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p, ie.default_opts(precision=ie.MIXED_BF16, cov_form=ie.COV_BAND))
    assert e.value.code == ie.ERR_INVALID_ARG
    # AUTO with BF16 runs the operator form; the FP64 forms agree to rounding
    a, _ = ie.perturbation_update(P, s, p, ie.default_opts(cov_form=ie.COV_OPERATOR, s_form=ie.S_OPERATOR))
    b, _ = ie.perturbation_update(P, s, p, ie.default_opts(cov_form=ie.COV_BAND, s_form=ie.S_OPERATOR))
    assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-9


def test_dense_s_options_and_agreement():
    """The dense form of S: not with BF16; AUTO takes it for few observations of a large state
    (same result as the per-iteration applies to rounding), and not for the n = 4096 lattice."""
    prob = syn.config1()
    say("dense S option checks")
    P = ie.Problem.from_synthetic(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.perturbation_update(P, s, p, ie.default_opts(precision=ie.MIXED_BF16, s_form=ie.S_DENSE))
    assert e.value.code == ie.ERR_INVALID_ARG
    a, _ = ie.perturbation_update(P, s, p, ie.default_opts(s_form=ie.S_OPERATOR))
    b, _ = ie.perturbation_update(P, s, p, ie.default_opts(s_form=ie.S_DENSE))
    c, _ = ie.perturbation_update(P, s, p, ie.default_opts())
    assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-9
    assert rel(b.cpu().numpy(), c.cpu().numpy()) < 1e-9
    # the workspace holds the m x m matrix exactly when the form is taken
    Q = prob.Q
    w_op = ie.workspace_bytes(P, Q, ie.default_opts(s_form=ie.S_OPERATOR))
    w_d = ie.workspace_bytes(P, Q, ie.default_opts(s_form=ie.S_DENSE))
    w_auto = ie.workspace_bytes(P, Q, ie.default_opts())
    assert w_d >= w_op + 8 * prob.m * prob.m and w_auto == w_d
    big = syn.config2()
    Pb = ie.Problem.from_synthetic(big)
    lat = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=Pb.lattice())
    lat_op = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=Pb.lattice(), s_form=ie.S_OPERATOR)
    assert ie.workspace_bytes(Pb, big.Q, lat) == ie.workspace_bytes(Pb, big.Q, lat_op)


def test_autotune_records_choices_and_keeps_results():
    """The band form's output does not depend on the tuned block shape; the operator form's
    changes by rounding only; every recorded shape is a valid one."""
    prob = syn.config2()
    say("autotune n4096")
    P = ie.Problem.from_synthetic(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    lat = P.lattice()
    ie.autotune_reset()
    for kw in (dict(), dict(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat),
               dict(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat, precision=ie.MIXED_FP32)):
        o = ie.default_opts(**kw)
        before, _ = ie.perturbation_update(P, s, p, o)
        rep = ie.autotune(P, prob.Q, o)
        say("autotune report", kw.get("precision", 0), rep)
        assert rep and all(r[2] in (8, 16, 32, 64) for r in rep)
        after, st = ie.perturbation_update(P, s, p, o)
        assert st.code == ie.OK
        assert torch.equal(before, after)
    o = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat, precision=ie.MIXED_BF16)
    rep = ie.autotune(P, prob.Q, o)
    say("autotune report bf16", rep)
    assert rep and all(r[2] in (16, 32, 64, 128) for r in rep)
    dp = dense_of(prob)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    got, st = ie.perturbation_update(P, s, p, o)
    assert st.code == ie.OK and upd(got.cpu().numpy(), want) < 1e-6
    ie.autotune_reset()


@pytest.mark.parametrize("form,domain", [("band", "lattice"), ("dense-s", "state"), ("dense-s", "lattice")])
@pytest.mark.parametrize("case", ["gauss-n256-periodic", "ragged-1d-nonperiodic", "small-nx-periodic", "2d-layers",
                                  "2d-periodic-z"])
def test_persistent_finish_matches(case, form, domain):
    """The persistent finish (one workgroup per remaining system, apply in place) against the
    oracle and against the loop without it; tail_systems = S hands every system over at the first
    poll, so the whole solve after four iterations runs in the persistent kernel."""
    prob = CASES[case]()
    say("persistent finish", case, form, domain)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    S = prob.Q * prob.N
    outs = {}
    for tail in (-1, 0, S):
        got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, form, tail_systems=tail))
        assert st.code == ie.OK and np.all(st.relres <= 1e-8)
        assert upd(got.cpu().numpy(), want) < 1e-6, tail
        outs[tail] = (got.cpu().numpy(), st.iters.copy())
    assert upd(outs[S][0], outs[-1][0]) < 1e-9
    assert np.max(np.abs(outs[S][1] - outs[-1][1])) <= 2
    # the default hands every system to the persistent kernel after the first step
    assert upd(outs[0][0], outs[S][0]) < 1e-12


@pytest.mark.parametrize("n_ritz", [0, 4])
@pytest.mark.parametrize("fixed", [0, 5])
def test_persistent_variants(n_ritz, fixed):
    """The persistent kernel without the preconditioner (p = 0) and with a fixed iteration count,
    on an odd number of observations (the last row pair reaches into the column padding)."""
    prob = CASES["ragged-1d-nonperiodic"]()
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    P = ie.Problem.from_synthetic(prob)
    say("persistent variants", n_ritz, fixed, "m", P.m)
    outs = {}
    for tail in (-1, 0):
        o = opts_for(prob, P, "lattice", "band", tail_systems=tail, n_ritz=n_ritz, fixed_iters=fixed)
        got, st = ie.perturbation_update(P, s, p, o)
        assert st.code == ie.OK
        outs[tail] = (got.cpu().numpy(), st.iters.copy())
    if fixed:
        assert np.array_equal(outs[0][1], outs[-1][1])
        assert upd(outs[0][0], outs[-1][0]) < 1e-9
    else:
        want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
        assert upd(outs[0][0], want) < 1e-6
        assert np.max(np.abs(outs[0][1] - outs[-1][1])) <= 2


@pytest.mark.parametrize("n_ritz", [4, 16, 20])
def test_persistent_kernel_variants_at_1024_observations(n_ritz):
    """The persistent kernel at m = 1024 (the n = 4096 workload) with small and large Ritz bases,
    which select different register and LDS layouts (the Ritz bases in registers or in LDS, the
    dots summed through LDS or by wavefront sums): every system converges and the result agrees
    with the batched loop."""
    prob = syn.config2()
    P = ie.Problem.from_synthetic(prob)
    s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
    say("persistent m=1024", n_ritz)
    outs = {}
    for tail in (-1, 0):
        o = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice(), n_ritz=n_ritz,
                            tail_systems=tail)
        got, st = ie.perturbation_update(P, s, p, o)
        assert st.code == ie.OK and np.all(st.relres <= 1e-8)
        outs[tail] = (got.cpu().numpy(), st.iters.copy())
    # two solvers to the same residual, not the oracle: the whole update agrees to 1e-8
    assert rel(outs[0][0], outs[-1][0]) < 1e-8
    assert np.max(np.abs(outs[0][1] - outs[-1][1])) <= 2


@pytest.mark.parametrize("oversample", [4, 3])
def test_fixed_budget_small_sketch_on_the_lattice(oversample):
    """On the observed lattice with at most 8 sketch columns the preconditioner setup applies S
    in place (the sketch written into the apply's input block, S Omega and S Qb read from its
    output block) around the two one-workgroup kernels.  A 2-iteration budget depends on every
    Ritz pair, so it checks the whole preconditioner: each member against the FP64 oracle's PCG
    with the same sketch to 1e-6."""
    prob = syn.config1()
    say("small sketch on the lattice, oversample", oversample)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    Om = syn.sketch_matrix(prob.m, 4 + oversample, 41)
    z64, it = ref.info_esrf_pcg(prob, s, p, rtol=0.0, n_ritz=4, Omega=Om, max_iter=2)
    assert np.all(it == 2)
    P = ie.Problem.from_synthetic(prob)
    Omt = torch.from_numpy(np.ascontiguousarray(Om.T)).cuda()
    got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, "lattice", "band", n_ritz=4, oversample=oversample,
                                                       sketch=Omt, fixed_iters=2))
    assert np.all(st.iters == 2)
    gz = got.cpu().numpy() / np.sqrt(prob.N - 1)
    say("  gpu vs fp64 oracle", upd(gz, z64))
    assert upd(gz, z64) < 1e-6


def test_headline_options_n4096():
    """The n = 4096 workload with exactly the benchmark's options: observed lattice, automatic
    covariance form (the band), 4 Ritz pairs from 4 + 4 sketch columns (the two-launch
    preconditioner setup at m = 1024), every system to the persistent kernel (tail 0).  Each
    member's analysis perturbation and the mean increment against the FP64 eigendecomposition
    oracle to 1e-6, every system to a true FP64 relative residual of 1e-8."""
    prob = syn.config2()
    say("headline options n4096: lattice, band, n_ritz 4, oversample 4, tail 0")
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    o = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice(), cov_form=ie.COV_AUTO,
                        n_ritz=4, oversample=4, tail_systems=0)
    got, st = ie.perturbation_update(P, s, p, o)
    assert st.code == ie.OK
    assert np.all(st.relres <= 1e-8) and np.all(st.converged == 1)
    err = upd(got.cpu().numpy(), want)
    say("  members", err, "iterations max", int(st.iters.max()), "total", int(st.iters.sum()))
    assert err < 1e-6
    mean_want = ref.mean_update_eig(dp, prob.y)
    mean_got, sm = ie.mean_update(P, prob.y, o)
    assert sm.code == ie.OK and upd(mean_got.cpu().numpy() - dp.mu, mean_want - dp.mu) < 1e-6


def ones_localization_problem(N=16, n=128, stride=4, seed=21):
    """L = 1 everywhere, as a stencil on a non-periodic 1-D grid reaching every point: S has rank at
    most N - 1, below the default sketch width of 20 columns."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, N)) + np.cos(np.arange(n) / 9.0)[:, None]
    idx = np.arange(0, n, stride, dtype=np.int32)
    m = idx.size
    table = np.ones(2 * n - 1)
    return syn.Problem(n=n, N=N, m=m, X=np.asfortranarray(X), h_ptr=np.arange(m + 1, dtype=np.int32), h_idx=idx,
                       h_w=np.ones(m), r_var=0.5 * np.ones(m), y=rng.standard_normal(m), nz=1, nx=n,
                       periodic_z=0, periodic_x=0, bz=0, bx=n - 1, table=table, truth=np.zeros(n), Q=8,
                       ell=100.0, name="ones-localization")


@pytest.mark.parametrize("form", ["band", "dense-L"])
def test_rank_deficient_sketch(form):
    """L = 1 and N = 16 with the default 10 Ritz pairs and 10 oversampling columns: the sketch
    S Omega has rank at most 15 < 20, so Cholesky-QR meets dependent columns (zero columns of the
    basis, zero Ritz values).  The update is still computed: to rtol against the dense oracle, and
    at a 2-iteration budget against the oracle's PCG (Householder QR) with the same sketch, which
    checks that the top 10 Ritz pairs are the same."""
    prob = ones_localization_problem()
    say("rank-deficient sketch", form, "N", prob.N, "k", 20)
    dp = dense_of(prob)
    assert np.allclose(dp.L, 1.0) and np.linalg.matrix_rank(dp.S) <= prob.N - 1
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    if form == "band":
        P = ie.Problem.from_synthetic(prob)
        kw = dict(cov_form=ie.COV_BAND)
    else:
        P = ie.Problem(prob.X, prob.h_ptr, prob.h_idx, prob.h_w, prob.r_var, dense=np.ones((prob.n, prob.n)))
        kw = {}
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    got, st = ie.perturbation_update(P, s, p, ie.default_opts(**kw))
    assert st.code == ie.OK and np.all(st.relres <= 1e-8)
    assert upd(got.cpu().numpy(), want) < 1e-6
    Om = syn.sketch_matrix(prob.m, 20, 5)
    z64, it = ref.info_esrf_pcg(prob, s, p, rtol=0.0, n_ritz=10, Omega=Om, max_iter=2)
    assert np.all(it == 2)
    Omt = torch.from_numpy(np.ascontiguousarray(Om.T)).cuda()
    got2, st2 = ie.perturbation_update(P, s, p, ie.default_opts(sketch=Omt, fixed_iters=2, **kw))
    assert st2.code == ie.OK and np.all(st2.iters == 2)
    e2 = upd(got2.cpu().numpy() / np.sqrt(prob.N - 1), z64)
    say("  fixed budget vs oracle", e2)
    assert e2 < 1e-6


def test_headline_options_mixed_fp32_n4096():
    """The benchmark's options with FP32 inner applies: the persistent kernel iterates on the FP32
    band (FP64 vectors, scalars and accumulation) and checks each sweep's true residual with the
    FP64 band; every system to 1e-8, each member against the FP64 oracle to 1e-6."""
    prob = syn.config2()
    say("headline options n4096, mixed fp32")
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    o = ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice(), precision=ie.MIXED_FP32,
                        n_ritz=4, oversample=4, tail_systems=0)
    got, st = ie.perturbation_update(P, s, p, o)
    assert st.code == ie.OK
    assert np.all(st.relres <= 1e-8) and np.all(st.converged == 1)
    assert st.counter(ie.CNT_SWEEPS) >= prob.Q * prob.N
    err = upd(got.cpu().numpy(), want)
    say("  members", err, "iterations max", int(st.iters.max()), "total", int(st.iters.sum()),
        "sweeps", st.counter(ie.CNT_SWEEPS))
    assert err < 1e-6


@pytest.mark.parametrize("form,domain", [("band", "lattice"), ("dense-s", "state")])
@pytest.mark.parametrize("case", ["gauss-n256-periodic", "2d-periodic-z", "ragged-1d-nonperiodic"])
def test_persistent_mixed_fp32(case, form, domain):
    """FP32 inner applies in the persistent kernel (every solve from its start, and the batched
    loop handing its state over), against the oracle and the batched loop."""
    prob = CASES[case]()
    say("persistent mixed fp32", case, form, domain)
    dp = dense_of(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    P = ie.Problem.from_synthetic(prob)
    S = prob.Q * prob.N
    outs = {}
    for tail in (-1, 0, S):
        got, st = ie.perturbation_update(P, s, p, opts_for(prob, P, domain, form, tail_systems=tail,
                                                         precision=ie.MIXED_FP32))
        assert st.code == ie.OK and np.all(st.relres <= 1e-8)
        assert upd(got.cpu().numpy(), want) < 1e-6, tail
        outs[tail] = got.cpu().numpy()
    assert rel(outs[0], outs[-1]) < 1e-8
