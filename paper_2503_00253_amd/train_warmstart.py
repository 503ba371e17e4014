"""Train and evaluate the learned warm start on the GPU.

Usage:  python -m paper_2503_00253_amd.train_warmstart --out net.ienet [options]

Training pairs come from the library itself (infoesrf_warmstart_pairs): every
shifted system (q, i) of a perturbation update is solved to rtol and the
members' inputs bh_i, the shift factors c_q and the scaled solutions
sqrt(m) u*/||b_i|| are kept.  Two sources, as the workloads they stand for:
  * the n = 4096 Gaussian update (N = 40, m = 1024, Q = 16), seeds 1..;
  * the 8 x 480 multi-layer Lorenz-96 cycle (N = 20, m = 1280, Q = 12): the
    forecast ensemble of every cycle of a few assimilation runs (trials 1..).
The network (the trunk once per member, the shift head per system) is trained
with the library's Adam step on the mean relative L2 loss, one source per
batch, then evaluated on held-out Lorenz cycles (trial 10000): on each cycle's
forecast ensemble the update runs from the zero start and from the learned
start, to the same true FP64 residual; PCG iterations and wall time of both,
and the network's own inference time, are reported.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def lattice_opts(ie, P, **kw):
    lat = P.lattice()
    if lat is not None:
        kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat)
    return ie.default_opts(**kw)


def gaussian_pairs(ie, syn, seeds, log):
    out = []
    for seed in seeds:
        prob = syn.config2(seed)
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        X, cq, T, st = ie.warmstart_pairs(P, s, p, None, lattice_opts(ie, P))
        assert st.code == ie.OK
        out.append((X, cq, T))
    log(f"gaussian n4096: {len(out)} updates, {sum(t[2].shape[0] * t[2].shape[1] for t in out)} systems")
    return out


def lorenz_pairs(ie, syn, trials, cycles, log, Q=12):
    """Pairs from the forecast ensemble of every cycle of assimilation runs (zero start)."""
    import numpy as np

    from paper_2503_00253_amd.cycle import CycleRunner
    out = []
    for trial in trials:
        prob = syn.lorenz_problem(trial=trial)
        noise = np.random.default_rng(7000 + trial).standard_normal((cycles, prob.m)) * np.sqrt(prob.r_var[0])
        run = CycleRunner(prob, Q=Q, noise=noise)
        s, p = run.s, run.p
        for t in range(cycles):
            run.load_noise(t)
            run.forecast()
            run.observe()
            X, cq, T, st = ie.warmstart_pairs(run.P, s, p, None, run.opts)
            assert st.code == ie.OK
            out.append((X, cq, T))
            run.update()
            run.assemble()
            run.t += 1
    log(f"lorenz 8x480: {len(out)} cycles, {sum(t[2].shape[0] * t[2].shape[1] for t in out)} systems")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gauss-updates", type=int, default=150, help="n = 4096 updates (640 systems each)")
    ap.add_argument("--lorenz-trials", type=int, default=5)
    ap.add_argument("--lorenz-cycles", type=int, default=84, help="cycles per training trial (240 systems each)")
    ap.add_argument("--eval-cycles", type=int, default=20, help="held-out Lorenz cycles evaluated")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8, help="members per batch (each with its Q shifts)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--kernel", type=int, default=9)
    ap.add_argument("--out", default="")
    ap.add_argument("--json", default="", help="also write the JSON record to this file")
    a = ap.parse_args()

    import numpy as np
    import torch

    import synthetic as syn
    from paper_2503_00253_amd import infoesrf as ie
    from paper_2503_00253_amd.cycle import CycleRunner

    log = lambda *x: print("[train]", *x, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    sources = [gaussian_pairs(ie, syn, range(1, 1 + a.gauss_updates), log),
               lorenz_pairs(ie, syn, range(1, 1 + a.lorenz_trials), a.lorenz_cycles, log)]
    # one tensor per source: members (X), shift factors (shared), targets
    data = []
    for src in sources:
        X = torch.cat([t[0] for t in src])
        T = torch.cat([t[2] for t in src])
        data.append((X, src[0][1].contiguous(), T))
    del sources
    pairs = sum(int(T.shape[0] * T.shape[1]) for _, _, T in data)
    gen_s = time.perf_counter() - t0
    log(f"training pairs: {pairs} systems in {gen_s:.1f} s")
    held = lorenz_pairs(ie, syn, [10000], 8, log)
    Hx = torch.cat([t[0] for t in held])
    Hc = held[0][1]
    Ht = torch.cat([t[2] for t in held])

    net = ie.Net.create(a.hidden, a.kernel, 2503)

    def held_loss():
        _, l = net.gradients(Hx, Hc, Ht)
        torch.cuda.synchronize()
        return float(l.cpu()[0])

    l_start = held_loss()
    g = torch.Generator(device="cpu").manual_seed(0)
    t0 = time.perf_counter()
    for step in range(a.steps):
        X, cq, T = data[step % len(data)]
        idx = torch.randint(0, X.shape[0], (a.batch,), generator=g).cuda()
        lr = a.lr * (0.1 + 0.9 * 0.5 * (1 + np.cos(np.pi * step / a.steps)))   # cosine decay to lr/10
        net.train_step(X[idx].contiguous(), cq, T[idx].contiguous(), lr)
        if (step + 1) % max(1, a.steps // 10) == 0:
            log(f"step {step + 1}: held-out loss {held_loss():.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    l_end = held_loss()
    if a.out:
        net.save(a.out)

    # evaluation on held-out Lorenz cycles: the same forecast ensemble from both starts
    prob = syn.lorenz_problem(trial=10000)
    cycles = 8 + a.eval_cycles
    noise = np.random.default_rng(17000).standard_normal((cycles, prob.m)) * np.sqrt(prob.r_var[0])
    run = CycleRunner(prob, Q=12, noise=noise)
    learned_opts = ie.Opts.from_buffer_copy(run.opts)
    learned_opts.warm_start = ie.START_LEARNED
    learned_opts.net = net.h.value
    its = {"zero": [], "learned": []}
    ms = {"zero": [], "learned": []}
    diffs = []
    for t in range(cycles):
        run.load_noise(t)
        run.forecast()
        run.observe()
        if t >= 8:   # the first 8 cycles of this trial were the held-out loss set above
            outs = {}
            for name, o in (("zero", run.opts), ("learned", learned_opts)):
                r = ie.PerturbationRunner(run.P, run.s, run.p, o, y=None)
                r.run()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(3):
                    code = r.run()
                torch.cuda.synchronize()
                ms[name].append((time.perf_counter() - t1) * 1e3 / 3)
                st = r.stats(code)
                assert st.code == ie.OK and st.counter(ie.CNT_NOT_CONVERGED) == 0
                its[name].append(st.iters.astype(np.int64))
                outs[name] = r.result().clone()
            diffs.append(float((outs["learned"] - outs["zero"]).norm() / outs["zero"].norm()))
        run.update()
        run.assemble()
        run.t += 1
    zero_it = np.concatenate(its["zero"])
    learned_it = np.concatenate(its["learned"])
    # the network's own cost per update: the trunk on the N members (BF16 on MFMA, and FP32)
    Xq = torch.randn((prob.N, prob.m), dtype=torch.float32, device="cuda")
    inf = {}
    for bf in (True, False):
        net.forward(Xq, bf16=bf)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(20):
            net.forward(Xq, bf16=bf)
        torch.cuda.synchronize()
        inf["bf16" if bf else "fp32"] = round((time.perf_counter() - t1) * 1e3 / 20, 4)
    out = {"workload": "learned warm start: trained on n=4096 Gaussian updates and 8x480 Lorenz-96 cycles, "
                       "evaluated on held-out 8x480 Lorenz-96 cycles (N=20, m=1280, Q=12)",
           "train_pairs": pairs, "pair_generation_seconds": round(gen_s, 2), "steps": a.steps,
           "batch_members": a.batch, "hidden": a.hidden, "kernel": a.kernel, "out_channels": ie.Net.D,
           "train_seconds": round(train_s, 2),
           "heldout_rel_l2": {"start": round(l_start, 4), "end": round(l_end, 4)},
           "eval_cycles": a.eval_cycles, "systems_per_cycle": int(zero_it.size // max(1, a.eval_cycles)),
           "mean_iterations": {"zero": round(float(zero_it.mean()), 3), "learned": round(float(learned_it.mean()), 3),
                               "saved_fraction": round(1 - float(learned_it.mean()) / float(zero_it.mean()), 4)},
           "max_iterations": {"zero": int(zero_it.max()), "learned": int(learned_it.max())},
           "ms_per_update": {"zero": round(float(np.mean(ms["zero"])), 4),
                             "learned": round(float(np.mean(ms["learned"])), 4)},
           "inference_ms_per_update": inf,
           "max_rel_diff_learned_vs_zero": max(diffs) if diffs else None}
    log(json.dumps(out))
    if a.json:
        with open(a.json, "w") as f:
            f.write(json.dumps(out, indent=1) + "\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
