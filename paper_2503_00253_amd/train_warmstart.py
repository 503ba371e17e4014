"""Train and evaluate the learned warm start on the GPU.

Usage:  python -m paper_2503_00253_amd.train_warmstart --out net.ienet [options]

Training pairs come from the library itself (infoesrf_warmstart_pairs): for
synthetic Gaussian-prior problems of the chosen size, every shifted system
(q, i) of the perturbation update is solved to rtol and its features and
scaled solution u*/||b|| are kept.  The network is trained with the
library's Adam step on the mean relative L2 loss, then evaluated on
held-out problems: PCG iterations and wall time of the update from the zero
start against the learned start, at the same true FP64 residual target.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def problem_for(size, seed):
    import synthetic as syn
    if size == "n4096":
        return syn.gaussian_problem(4096, 40, 40.0, 80.0, 4, 0.25, 16, 1000.0, seed, name=f"gauss4096-{seed}")
    if size == "n1024":
        return syn.gaussian_problem(1024, 24, 20.0, 40.0, 4, 0.25, 12, 300.0, seed, name=f"gauss1024-{seed}")
    return syn.gaussian_problem(256, 16, 10.0, 20.0, 4, 0.25, 8, 100.0, seed, name=f"gauss256-{seed}")


def opts_for(ie, P, precision, **kw):
    lat = P.lattice()
    if lat is not None:
        kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=lat)
    return ie.default_opts(precision=precision, **kw)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", choices=["n256", "n1024", "n4096"], default="n4096")
    ap.add_argument("--train-problems", type=int, default=16)
    ap.add_argument("--val-problems", type=int, default=2)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--kernel", type=int, default=9)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64")
    ap.add_argument("--eval-reps", type=int, default=3)
    ap.add_argument("--out", default="")
    a = ap.parse_args()

    import numpy as np
    import torch

    from paper_2503_00253_amd import infoesrf as ie

    prec = {"fp64": ie.FP64, "fp32": ie.MIXED_FP32, "bf16": ie.MIXED_BF16}[a.precision]
    log = lambda *x: print("[train]", *x, file=sys.stderr, flush=True)  # noqa: E731

    # training pairs (seeds 1.., held-out seeds 10000..)
    t0 = time.perf_counter()
    Xs, Ts = [], []
    for k in range(a.train_problems):
        prob = problem_for(a.size, 1 + k)
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        X, T, st = ie.warmstart_pairs(P, s, p, prob.y, opts_for(ie, P, ie.FP64))
        Xs.append(X)
        Ts.append(T)
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    del Xs, Ts
    val = [problem_for(a.size, 10000 + k) for k in range(a.val_problems)]
    Vx, Vt = [], []
    for prob in val:
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        x, t, _ = ie.warmstart_pairs(P, s, p, prob.y, opts_for(ie, P, ie.FP64))
        Vx.append(x)
        Vt.append(t)
    Vx = torch.cat(Vx)
    Vt = torch.cat(Vt)
    log(f"pairs: {X.shape[0]} train, {Vx.shape[0]} held out, m={X.shape[2]} ({time.perf_counter() - t0:.1f} s)")

    net = ie.Net.create(a.hidden, a.kernel, 2503)
    vb = min(Vx.shape[0], 512)

    def val_loss():
        _, l = net.gradients(Vx[:vb].contiguous(), Vt[:vb].contiguous())
        torch.cuda.synchronize()
        return float(l.cpu()[0])

    l_start = val_loss()
    g = torch.Generator(device="cpu").manual_seed(0)
    t0 = time.perf_counter()
    for step in range(a.steps):
        idx = torch.randint(0, X.shape[0], (a.batch,), generator=g).cuda()
        lr = a.lr * (0.1 + 0.9 * 0.5 * (1 + np.cos(np.pi * step / a.steps)))   # cosine decay to lr/10
        net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr)
        if (step + 1) % max(1, a.steps // 10) == 0:
            log(f"step {step + 1}: held-out loss {val_loss():.4f}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    l_end = val_loss()
    if a.out:
        net.save(a.out)

    # evaluation: zero start against learned start on the held-out problems
    rows = []
    for prob in val:
        P = ie.Problem.from_synthetic(prob)
        s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
        res = {}
        arms = (("zero", {}), ("learned", dict(warm_start=ie.START_LEARNED, net=net)),
                ("learned_fp32_inference", dict(warm_start=ie.START_LEARNED, net=net, warm_fp32=1)))
        for name, kw in arms:
            run = ie.PerturbationRunner(P, s, p, opts_for(ie, P, prec, **kw), y=prob.y)
            code = run.run()
            torch.cuda.synchronize()
            st = run.stats(code)
            t1 = time.perf_counter()
            for _ in range(a.eval_reps):
                run.run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / a.eval_reps
            res[name] = dict(iters_mean=float(st.iters.mean()), iters_max=int(st.iters.max()),
                             fp64_sweeps=st.counter(ie.CNT_SWEEPS), fallbacks=st.counter(ie.CNT_FALLBACKS),
                             ms_per_update=round(ms, 3), solves_per_s=round(prob.Q * prob.N / ms * 1e3, 1),
                             out=run.result().clone())
        diff = float((res["learned"]["out"] - res["zero"]["out"]).norm() / res["zero"]["out"].norm())
        # the network's own cost per update: BF16 inference (the learned start's default) and FP32
        Xq = torch.randn((P.c.N * prob.Q, 3, P.c.m), dtype=torch.float32, device="cuda")
        for bf in (True, False):
            net.forward(Xq[:128], bf16=bf)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for c0 in range(0, Xq.shape[0], 128):
                net.forward(Xq[c0:c0 + 128], bf16=bf)
            torch.cuda.synchronize()
            res[f"inference_ms_{'bf16' if bf else 'fp32'}"] = round((time.perf_counter() - t1) * 1e3, 3)
        for r in res.values():
            if isinstance(r, dict):
                r.pop("out")
        rows.append(dict(problem=prob.name, systems=prob.Q * prob.N, rel_diff_learned_vs_zero=diff, **res))
        log(prob.name, json.dumps(rows[-1]))
    zero_it = float(np.mean([r["zero"]["iters_mean"] for r in rows]))
    learned_it = float(np.mean([r["learned"]["iters_mean"] for r in rows]))
    out = {"workload": f"warm-start {a.size}", "precision": a.precision, "train_pairs": int(X.shape[0]),
           "heldout_pairs": int(Vx.shape[0]), "steps": a.steps, "batch": a.batch, "hidden": a.hidden,
           "kernel": a.kernel, "train_seconds": round(train_s, 2),
           "heldout_rel_l2": {"start": round(l_start, 4), "end": round(l_end, 4)},
           "mean_iterations": {"zero": round(zero_it, 3), "learned": round(learned_it, 3),
                               "saved_fraction": round(1 - learned_it / zero_it, 4)},
           "updates": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
