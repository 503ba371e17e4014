"""Cycled assimilation pieces and the cycle itself on the GPU, against the oracle.

* forecast: the RK4 integration of the multi-layer Lorenz-96 model against the
  oracle's loop-by-loop integration (FP64; contraction of a*b+c into fused
  multiply-adds changes rounding only: 1e-12 relative after a few steps);
* observations and the RTPS analysis assembly against their definitions;
* every cycle's update is checked on the GPU's own forecast ensemble against
  the FP64 eigendecomposition oracle (1e-6, the FP64-mode bound), at a small
  size over several cycles and at the 8 x 480 size for one cycle;
* a HIP-graph-captured cycle (host_sync 0) replays to the same bits as the
  same cycles run eagerly.
"""
import sys

import numpy as np
import pytest

import synthetic as syn
from parity import rel, upd  # noqa: E402
from oracle import cycle_ref as cr
from oracle import infoesrf_ref as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402
from paper_2503_00253_amd.cycle import CycleRunner  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)




@pytest.mark.parametrize("nz,nx,k,steps,gamma", [(3, 20, 4, 7, 0.5), (8, 480, 21, 5, 0.1), (1, 40, 2, 20, 0.0)])
def test_forecast_matches_oracle(nz, nx, k, steps, gamma):
    say("l96 forecast", nz, nx, k, steps)
    rng = np.random.default_rng(nz * nx + k)
    F = np.linspace(8.0, 6.0, nz)
    X = F.repeat(nx)[:, None] + rng.standard_normal((nz * nx, k))
    want = cr.l96_forecast(X, steps, 0.01, nz, nx, F, gamma)
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    ie.l96_forecast(Xt, nz, nx, torch.from_numpy(F).cuda(), gamma, 0.01, steps)
    assert rel(Xt.cpu().numpy().T, want) < 1e-12


def test_observe_and_rtps_assemble():
    say("observe and rtps")
    prob = syn.lorenz_problem(nz=2, nx=30, N=6, spinup_time=0.5)
    P = ie.Problem.from_synthetic(prob)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(prob.n)
    noise = rng.standard_normal(prob.m)
    y = torch.empty(prob.m, dtype=torch.float64, device="cuda")
    ie.observe(P, torch.from_numpy(x).cuda(), torch.from_numpy(noise).cuda(), y)
    H = ref.dense_obs_operator(prob.h_ptr, prob.h_idx, prob.h_w, prob.n)
    assert np.allclose(y.cpu().numpy(), H @ x + noise, rtol=1e-14, atol=1e-14)
    Xf = rng.standard_normal((prob.n, prob.N)) + 3
    Xa = 0.4 * (Xf - Xf.mean(axis=1, keepdims=True))
    mean_a = rng.standard_normal(prob.n)
    out = torch.empty((prob.N, prob.n), dtype=torch.float64, device="cuda")
    ie.rtps_assemble(torch.from_numpy(np.ascontiguousarray(Xf.T)).cuda(), torch.from_numpy(mean_a).cuda(),
                     torch.from_numpy(np.ascontiguousarray(Xa.T)).cuda(), 0.3, out)
    want = mean_a[:, None] + cr.rtps(Xf - Xf.mean(axis=1, keepdims=True), Xa, 0.3)
    assert rel(out.cpu().numpy().T, want) < 1e-13


def cycle_checks(prob, cycles, Q, tol=1e-6, opts=None, check_every=1):
    """Runs `cycles` cycles on the GPU and checks the update of every `check_every`-th cycle
    (the forecast ensemble and the observations the GPU itself produced) against the dense
    oracle: each member's analysis perturbation and the analysis mean to `tol`."""
    rng = np.random.default_rng(123)
    noise = rng.standard_normal((cycles, prob.m)) * np.sqrt(prob.r_var[0])
    run = CycleRunner(prob, Q=Q, noise=noise)
    if opts is not None:
        run.set_opts(opts(run.P))
    s, p, _ = ref.quadrature_elliptic(Q, prob.ell)
    for t in range(cycles):
        run.load_noise(t)
        run.forecast()
        run.observe()
        check = t % check_every == check_every - 1
        if check:
            torch.cuda.synchronize()
            Xf = run.state[:run.N].cpu().numpy().T.copy()
            y = run.y.cpu().numpy().copy()
        c1, c2 = run.update()
        torch.cuda.synchronize()
        assert c1 == ie.OK and c2 == ie.OK
        if check:
            fc = syn.Problem(n=prob.n, N=prob.N, m=prob.m, X=np.asfortranarray(Xf), h_ptr=prob.h_ptr,
                             h_idx=prob.h_idx, h_w=prob.h_w, r_var=prob.r_var, y=y, nz=prob.nz, nx=prob.nx,
                             periodic_z=prob.periodic_z, periodic_x=prob.periodic_x, bz=prob.bz, bx=prob.bx,
                             table=prob.table, truth=prob.truth, Q=Q, ell=prob.ell, name="cycle")
            dp = ref.DenseProblem.from_problem(fc)
            want_pert = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
            want_mean = ref.mean_update_eig(dp, y)
            got_pert = run.Xa.cpu().numpy().T
            got_mean = run.mean_a.cpu().numpy()
            e1 = upd(got_pert, want_pert)
            e2 = upd(got_mean - dp.mu, want_mean - dp.mu)
            say("cycle", t, "pert", e1, "mean", e2)
            assert e1 < tol and e2 < tol
        run.assemble()
        run.t += 1
    return run


def test_cycles_small_match_oracle():
    prob = syn.lorenz_problem(nz=4, nx=60, N=10, spinup_time=2.0, c_h=4.0, Q=6)
    say("cycles 4x60")
    run = cycle_checks(prob, cycles=4, Q=6)
    mse, var = run.diagnostics()
    assert np.isfinite(mse) and var > 0


def test_cycle_full_size_matches_oracle():
    """The 8 x 480 multi-layer workload (N = 20, m = 1280, Q = 12): two cycles checked in full."""
    prob = syn.lorenz_problem()
    say("cycles 8x480")
    cycle_checks(prob, cycles=2, Q=12)


def test_cycle_full_size_mixed_fp32_100_cycles():
    """The 8 x 480 workload over 100 cycles with FP32 inner applies (FP64 vectors, scalars and
    residual sweeps): every 10th cycle's update against the dense FP64 oracle to 1e-6."""
    prob = syn.lorenz_problem()
    say("cycles 8x480 mixed fp32, 100 cycles")

    def mixed(P):
        return ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice(), precision=ie.MIXED_FP32)

    run = cycle_checks(prob, cycles=100, Q=12, opts=mixed, check_every=10)
    mse, var = run.diagnostics()
    say("  after 100 cycles: forecast mse", mse, "variance", var)
    assert np.isfinite(mse) and var > 0


def test_graph_captured_cycle_matches_eager():
    prob = syn.lorenz_problem(nz=4, nx=60, N=10, spinup_time=2.0, c_h=4.0, Q=6)
    rng = np.random.default_rng(5)
    noise = rng.standard_normal((3, prob.m))
    kw = dict(host_sync=0, max_iter=150)
    say("graph cycle")
    eager = CycleRunner(prob, Q=6, noise=noise)
    P = eager.P
    lat = P.lattice()
    eager.set_opts(ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat, **kw))
    for _ in range(3):
        eager.step()
    torch.cuda.synchronize()
    want = eager.state.clone()

    g_run = CycleRunner(prob, Q=6, noise=noise)
    g_run.set_opts(ie.default_opts(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat, **kw))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    # one eager warm-up cycle on a copy of the state sets kernel attributes before capture
    saved = g_run.state.clone()
    with torch.cuda.stream(side):
        g_run.cycle_body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g_run.state.copy_(saved)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g_run.cycle_body()
    torch.cuda.synchronize()
    g_run.state.copy_(saved)
    for t in range(3):
        g_run.load_noise(t)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
    assert torch.equal(g_run.state, want)


def test_paper_sec5_cycles_match_oracle():
    """Section 5's 32 x 40 atmosphere (forcing 8 -> 4 over the layers, coupling 1, 40 members,
    8 columns x 5 channels): two cycles, each update checked in full."""
    prob = syn.experiment2_problem()
    say("cycles paper sec5")
    assert np.ndim(prob.meta["forcing"]) == 1
    cycle_checks(prob, cycles=2, Q=8)
