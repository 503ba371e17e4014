"""Learned warm start on the GPU (through the C ABI) against the FP64 oracle.

Tolerances: the FP32 network runs with FP32 accumulation over at most
3 x 9 + 2 x (H x 9) terms per output, so forward outputs agree with the FP64
oracle to 1e-5 relative and gradients (a longer chain of FP32 sums over
B x m positions) to 1e-4; one Adam step from a fresh state matches to 1e-6
absolute on unit-scale parameters.  A solve started from the network must
still meet the FP64-mode bound (1e-6 relative to the eigendecomposition
oracle) because the stopping test is the same true FP64 residual.
"""
import sys

import numpy as np
import pytest

import synthetic as syn
from parity import rel, upd  # noqa: E402
from oracle import infoesrf_ref as ref
from oracle import warmstart_ref as wr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)




D = 4  # trunk output channels (terms of the shift head)


def flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflat(v, H, K):
    shapes = [(H, 1, K), (H, H, K), (H, H, K), (D, H, K)]
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        W = v[o:o + n].reshape(sh).astype(np.float64)
        o += n
        b = v[o:o + sh[0]].astype(np.float64)
        o += sh[0]
        out.append((W, b))
    assert o == v.size
    return out


def random_net(H, K, seed):
    rng = np.random.default_rng(seed)
    params = wr.init_params(channels=(1, H, H, H, D), K=K, seed=seed)
    params = [(W, 0.05 * rng.standard_normal(b.shape)) for W, b in params]
    net = ie.Net.create(H, K, seed)
    v = flat(params)
    net.set_params(v)
    return net, unflat(v, H, K)   # the FP32-rounded parameters the GPU uses


def phi_of(cq):
    """The head's basis c_q^(d+1) from the FP32 shift factors the GPU holds."""
    c = np.asarray(cq, dtype=np.float32).astype(np.float64)
    return np.stack([c ** (d + 1) for d in range(D)], axis=1)


@pytest.mark.parametrize("H,K,B,m", [(8, 9, 3, 37), (64, 9, 2, 200), (16, 5, 5, 64), (8, 3, 1, 7)])
def test_forward_matches_oracle(H, K, B, m):
    say("net forward", H, K, B, m)
    net, params = random_net(H, K, 11 + H + K)
    X = np.random.default_rng(1).standard_normal((B, m)).astype(np.float32)
    got = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    want, _ = wr.forward(params, X.astype(np.float64)[:, None, :])
    assert got.shape == (B, D, m)
    assert rel(got, want) < 1e-5


def to_bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16_emulated(params, X):
    """The oracle's layers with BF16 weights, BF16 inputs and BF16 activations between layers
    (the arithmetic itself in FP64): the precision the MFMA inference stores its operands in."""
    a = to_bf16(X)
    for li, (W, b) in enumerate(params):
        z = wr.conv1d_same(a, to_bf16(W), b)
        a = to_bf16(wr.gelu(z)) if li < len(params) - 1 else z
    return a


@pytest.mark.parametrize("H,K,B,m", [(8, 9, 3, 37), (64, 9, 2, 200), (16, 5, 5, 64), (8, 3, 1, 7), (64, 9, 3, 1024)])
def test_forward_bf16_matches_oracle(H, K, B, m):
    """BF16 trunk on MFMA: against the oracle with the same BF16 roundings (operands and
    activations) to 2e-3, the FP32 accumulation order and the few activations whose rounding
    flips being the only differences; against the exact oracle within twice the oracle's own
    change under those roundings."""
    say("net forward bf16", H, K, B, m)
    net, params = random_net(H, K, 11 + H + K)
    X = np.random.default_rng(2).standard_normal((B, m)).astype(np.float32)
    got = net.forward(torch.from_numpy(X).cuda(), bf16=True).cpu().numpy()
    want, _ = wr.forward(params, X.astype(np.float64)[:, None, :])
    emu = forward_bf16_emulated(params, X.astype(np.float64)[:, None, :])
    sens = rel(emu, want)
    say("  bf16 sensitivity", sens, "gpu vs emulated", rel(got, emu))
    assert rel(got, emu) < 2e-3
    assert rel(got, want) < 2 * sens + 1e-3


@pytest.mark.parametrize("H,K,B,Q,m", [(8, 9, 3, 4, 37), (32, 9, 4, 12, 130)])
def test_gradients_match_oracle(H, K, B, Q, m):
    """Loss and gradients through the trunk, the shift head and the relative L2 loss."""
    say("net gradients", H, K, B, Q, m)
    net, params = random_net(H, K, 5)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((B, m)).astype(np.float32)
    cq = (1.0 / (1.0 + rng.uniform(0.0, 30.0, Q))).astype(np.float32)
    T = rng.standard_normal((B, Q, m)).astype(np.float32)
    g, loss = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(cq).cuda(), torch.from_numpy(T).cuda())
    torch.cuda.synchronize()
    phi = phi_of(cq)
    Y, cache = wr.forward(params, X.astype(np.float64)[:, None, :])
    lw, gy = wr.loss_rel_l2(wr.head(Y, phi), T.astype(np.float64))
    want = flat(wr.backward(params, cache, wr.head_grad(gy, phi)))
    assert abs(float(loss.cpu()[0]) - lw) < 1e-5 * max(1.0, lw)
    assert rel(g.cpu().numpy(), want) < 1e-4


def test_adam_step_matches_oracle():
    say("adam step")
    H, K, B, Q, m = 8, 9, 2, 3, 40
    net, params = random_net(H, K, 9)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((B, m)).astype(np.float32)
    cq = np.array([0.9, 0.5, 0.05], dtype=np.float32)
    T = rng.standard_normal((B, Q, m)).astype(np.float32)
    lr = 1e-3
    net.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(cq).cuda(), torch.from_numpy(T).cuda(), lr)
    torch.cuda.synchronize()
    phi = phi_of(cq)
    Y, cache = wr.forward(params, X.astype(np.float64)[:, None, :])
    _, gy = wr.loss_rel_l2(wr.head(Y, phi), T.astype(np.float64))
    grads = wr.backward(params, cache, wr.head_grad(gy, phi))
    want = flat(wr.adam_step(params, grads, {}, lr))
    got = net.params()
    assert np.max(np.abs(got - want)) < 1e-6
    assert np.max(np.abs(got - flat(params))) > 1e-4   # the step moved the parameters


def test_file_round_trip(tmp_path):
    say("net save/load")
    net = ie.Net.create(16, 7, 4)
    path = tmp_path / "w.ienet"
    net.save(path)
    other = ie.Net.load(path)
    assert np.array_equal(net.params(), other.params())
    assert other.param_count == 16 * 1 * 7 + 16 + 2 * (16 * 16 * 7 + 16) + D * 16 * 7 + D
    assert open(path, "rb").read(8) == b"IENET002"


def test_training_pairs_match_oracle():
    prob = syn.config1()
    say("training pairs config1")
    P = ie.Problem.from_synthetic(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    X, cq, T, st = ie.warmstart_pairs(P, s, p, prob.y, ie.default_opts(rtol=1e-12))
    assert st.code == ie.OK
    dp = ref.DenseProblem.from_problem(prob)
    # member i's right-hand side b_i = R^{-1/2} w_i; exact u*_{q,i} from the spectral form
    members = dp.B.T
    assert rel(X.cpu().numpy(), wr.member_features(members)[:, 0, :]) < 1e-6
    assert np.allclose(cq.cpu().numpy(), 1.0 / (1.0 + s), rtol=1e-7)
    U = np.stack([dp.spectral(lambda lam, sq=sq: 1.0 / (1.0 + sq + lam), dp.B).T for sq in s], axis=1)
    assert rel(T.cpu().numpy(), wr.targets(U, members)) < 1e-6


def test_learned_start_solve_meets_bound_and_fallback():
    prob = syn.config1()
    say("learned start solve")
    P = ie.Problem.from_synthetic(prob)
    s, p, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    dp = ref.DenseProblem.from_problem(prob)
    want = np.sqrt(prob.N - 1) * ref.perturbation_update_quadrature(dp, s, p)
    net, _ = random_net(16, 9, 21)
    for fp32 in (0, 1):   # BF16 inference on MFMA (the default), FP32 inference
        got, st = ie.perturbation_update(P, s, p, ie.default_opts(warm_start=ie.START_LEARNED, net=net,
                                                                  warm_fp32=fp32), y=prob.y)
        assert st.code == ie.OK and upd(got.cpu().numpy(), want) < 1e-6
        assert np.all(st.relres <= 1e-8) and st.counter(ie.CNT_FALLBACKS) == 0
    # a network that predicts NaN: every system falls back to the zero start
    bad = ie.Net.create(16, 9, 3)
    v = bad.params()
    v[-1] = np.nan
    bad.set_params(v)
    got2, st2 = ie.perturbation_update(P, s, p, ie.default_opts(warm_start=ie.START_LEARNED, net=bad), y=prob.y)
    assert st2.code == ie.OK and upd(got2.cpu().numpy(), want) < 1e-6
    assert st2.counter(ie.CNT_FALLBACKS) == prob.Q * prob.N
    zero, stz = ie.perturbation_update(P, s, p, ie.default_opts())
    assert np.array_equal(st2.iters, stz.iters)   # the fallback is exactly the zero start


def test_training_lowers_held_out_iterations():
    """Training on the solutions of n = 256 updates from 24 seeds (the library's own solves, the
    library's forward, backward and Adam kernels): on two held-out updates the held-out loss falls
    and the learned start needs fewer PCG iterations in total than the zero start, every system
    still reaching the same true FP64 residual of 1e-8."""
    say("training run, held-out iterations")
    Xs, Ts, cqs = [], [], []
    make = lambda seed: syn.gaussian_problem(256, 16, 10.0, 20.0, 4, 0.25, 8, 100.0, seed)  # noqa: E731
    for seed in range(1, 25):
        prob = make(1000 + seed)
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        X, cq, T, _ = ie.warmstart_pairs(P, s, p)
        Xs.append(X)
        Ts.append(T)
        cqs.append(cq)
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    cq = cqs[0]   # every update here has the same nodes
    net = ie.Net.create(32, 9, 7)
    held = [make(20000 + k) for k in range(2)]
    Hx, Ht = [], []
    for prob in held:
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        x, _, t, _ = ie.warmstart_pairs(P, s, p)
        Hx.append(x)
        Ht.append(t)
    Hx, Ht = torch.cat(Hx), torch.cat(Ht)
    _, l0 = net.gradients(Hx, cq, Ht)
    g = torch.Generator(device="cpu").manual_seed(0)
    for step in range(600):
        idx = torch.randint(0, X.shape[0], (32,), generator=g).cuda()
        net.train_step(X[idx].contiguous(), cq, T[idx].contiguous(), 3e-3 if step < 400 else 1e-3)
    _, l1 = net.gradients(Hx, cq, Ht)
    torch.cuda.synchronize()
    l0, l1 = float(l0.cpu()[0]), float(l1.cpu()[0])
    zero_it = learned_it = 0
    for prob in held:
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        _, sz = ie.perturbation_update(P, s, p, ie.default_opts())
        _, sl = ie.perturbation_update(P, s, p, ie.default_opts(warm_start=ie.START_LEARNED, net=net), y=prob.y)
        assert sz.code == ie.OK and sl.code == ie.OK
        assert np.all(sl.relres <= 1e-8) and np.all(sz.relres <= 1e-8)
        zero_it += int(sz.iters.sum())
        learned_it += int(sl.iters.sum())
    say("held-out loss", l0, "->", l1, "| iterations zero", zero_it, "learned", learned_it)
    assert l1 < 0.5 * l0
    assert learned_it < zero_it


def test_training_lowers_held_out_lorenz_iterations():
    """The multi-layer Lorenz-96 case (8 x 480, N = 20, m = 1280, Q = 12): the network is trained
    on the systems of the forecast ensembles of 40 cycles of two assimilation runs, then, on three
    cycles of a held-out run, the update from the learned start needs fewer PCG iterations in all
    than from the zero start, every system reaching the true FP64 residual 1e-8 either way."""
    from paper_2503_00253_amd.cycle import CycleRunner
    say("training on Lorenz cycles, held-out cycles")

    def cycles(trial, count):
        prob = syn.lorenz_problem(trial=trial)
        noise = np.random.default_rng(7000 + trial).standard_normal((count, prob.m)) * np.sqrt(prob.r_var[0])
        run = CycleRunner(prob, Q=12, noise=noise)
        for t in range(count):
            run.load_noise(t)
            run.forecast()
            run.observe()
            yield run
            run.update()
            run.assemble()
            run.t += 1

    Xs, Ts, cq = [], [], None
    for trial in (1, 2):
        for run in cycles(trial, 20):
            X, cq, T, st = ie.warmstart_pairs(run.P, run.s, run.p, None, run.opts)
            assert st.code == ie.OK
            Xs.append(X)
            Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    net = ie.Net.create(64, 9, 11)
    g = torch.Generator(device="cpu").manual_seed(0)
    for step in range(1200):
        idx = torch.randint(0, X.shape[0], (8,), generator=g).cuda()
        net.train_step(X[idx].contiguous(), cq, T[idx].contiguous(), 2e-3 if step < 800 else 5e-4)
    torch.cuda.synchronize()
    zero_it = learned_it = 0
    for t, run in enumerate(cycles(10000, 11)):
        if t < 8:
            continue
        lo = ie.Opts.from_buffer_copy(run.opts)
        lo.warm_start = ie.START_LEARNED
        lo.net = net.h.value
        _, sz = ie.perturbation_update(run.P, run.s, run.p, run.opts)
        _, sl = ie.perturbation_update(run.P, run.s, run.p, lo)
        assert sz.code == ie.OK and sl.code == ie.OK
        assert np.all(sl.relres <= 1e-8) and np.all(sz.relres <= 1e-8)
        zero_it += int(sz.iters.sum())
        learned_it += int(sl.iters.sum())
    say("held-out Lorenz iterations: zero", zero_it, "learned", learned_it)
    assert learned_it < zero_it
