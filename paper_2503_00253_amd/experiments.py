"""The paper's two experiments, run on the library (Sec. 4 and Sec. 5).

* ``sec4``: one analysis of a Gaussian forecast (n = 2000, 20 members, 100
  wide weighted channels) per trial, with the PCG budget fixed at 2
  iterations, for several Ritz-pair counts p and quadrature sizes Q; the
  score is E^2 of Sec. 4.4, the mean squared relative error of the analysis
  ensemble's variances against the Kalman analysis variances.
* ``sec5``: cycled assimilation of the 32 x 40 coupled Lorenz-96 atmosphere
  (40 members, 8 columns x 5 channels, an analysis every 0.05 time units),
  10 PCG iterations per solve, p = 10, relaxation to prior spread 0.01; the
  scores are the forecast MSE and MSE / variance averaged after burn-in.

The analyses run on the GPU through the C ABI (mean update, perturbation
update, forecast, observation and ensemble assembly kernels).  The scores are
evaluation, not part of the filter: the Kalman analysis variances of Sec. 4
are formed on the host with numpy (the prior is circulant, so its products
go through the FFT), and the forecast statistics of Sec. 5 with torch
reductions on the device, kept there until the run ends.

Run as ``python -m paper_2503_00253_amd.experiments sec4|sec5 [options]``;
prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import infoesrf as ie


def _dense_rows(prob):
    Hd = np.zeros((prob.m, prob.n))
    for k in range(prob.m):
        sl = slice(prob.h_ptr[k], prob.h_ptr[k + 1])
        Hd[k, prob.h_idx[sl]] += prob.h_w[sl]
    return Hd


def kalman_analysis_variance(prob, prior_row):
    """diag(Sigma - Sigma H^T (H Sigma H^T + R)^{-1} H Sigma) for the circulant prior with
    first row prior_row (the analytic analysis variances of Sec. 4)."""
    n = prob.n
    lam = np.fft.rfft(prior_row).real
    Hd = _dense_rows(prob)
    HS = np.fft.irfft(np.fft.rfft(Hd, axis=1) * lam[None, :], n=n, axis=1)   # H Sigma
    A = HS @ Hd.T + np.diag(prob.r_var)
    return prior_row[0] - np.sum(HS * np.linalg.solve(A, HS), axis=0)


def variance_error(pert, var_a):
    """E^2 of Sec. 4.4 from analysis perturbations (n x N, rows are state variables)."""
    N = pert.shape[1]
    emp = np.sum(pert * pert, axis=1) / (N - 1)
    return float(np.mean(((emp - var_a) / var_a) ** 2))


def sec4_experiment(trials=10, ps=(0, 4, 10, 20), Qs=(2, 4, 8), iters=2, ell=None, seed=7, log=None):
    """E^2 per (p, Q), averaged over trials, with every Krylov solve stopped at `iters`."""
    import synthetic as syn

    torch = ie._torch()
    E = {(p, Q): [] for p in ps for Q in Qs}
    runs, t_update = 0, 0.0
    for t in range(trials):
        prob = syn.experiment1_problem(trial=t)
        var_a = kalman_analysis_variance(prob, syn.experiment1_prior_row(prob.n))
        P = ie.Problem.from_synthetic(prob)
        for Q in Qs:
            s, w = ie.quadrature_elliptic(Q, ell or prob.ell)
            for p in ps:
                o = ie.default_opts(n_ritz=p, fixed_iters=iters, seed=seed + t)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, sm = ie.mean_update(P, prob.y, o)
                pert, sp = ie.perturbation_update(P, s, w, o)
                t_update += time.perf_counter() - t0
                runs += 1
                if sm.code != ie.OK or sp.code != ie.OK:
                    raise ie.InfoEsrfError(sp.code or sm.code, "analysis failed")
                E[(p, Q)].append(variance_error(pert.cpu().numpy(), var_a))
        if log:
            log(f"trial {t}: " + " ".join(f"p{p}/Q{Q}={E[(p, Q)][-1]:.4f}" for p in ps for Q in Qs))
    table = [{"p": p, "Q": Q, "E2_mean": float(np.mean(v)),
              "E2_ci95": float(1.96 * np.std(v, ddof=1) / np.sqrt(len(v))) if len(v) > 1 else None}
             for (p, Q), v in E.items()]
    return {"experiment": "sec4-variance-error", "trials": trials, "iterations": iters,
            "mean_ms_per_analysis": 1e3 * t_update / max(runs, 1), "results": table}


def sec5_experiment(cycles=5000, burn=1000, Q=8, iters=10, n_ritz=10, alpha=0.01, trial=0, log=None):
    """Forecast MSE and MSE / variance of the cycled experiment, averaged over cycles after burn-in.

    MSE_T = ||mean_T - truth_T||^2 / n and the ratio MSE_T / sigma_T^2 with sigma_T^2 the forecast
    variance averaged over the state (the 1/n of the MSE is read into the ratio as well, so that a
    calibrated ensemble scores near 1)."""
    import synthetic as syn

    from .cycle import CycleRunner

    torch = ie._torch()
    prob = syn.experiment2_problem(trial=trial, Q=Q)
    noise = syn.experiment2_noise(cycles, prob.m, trial=trial)
    opts = ie.default_opts(n_ritz=n_ritz, fixed_iters=iters, host_sync=0)
    run = CycleRunner(prob, Q=Q, noise=noise, alpha=alpha, opts=opts, lattice=False)
    mse = torch.zeros(cycles, dtype=torch.float64, device="cuda")
    var = torch.zeros(cycles, dtype=torch.float64, device="cuda")
    ens, truth = run.state[:run.N], run.state[run.N]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(cycles):
        run.load_noise(t)
        run.forecast()
        mu = ens.mean(dim=0)
        mse[t] = ((mu - truth) ** 2).mean()
        var[t] = ens.var(dim=0, unbiased=True).mean()
        run.observe()
        c1, c2 = run.update()
        run.assemble()
        run.t += 1
        if log and (t + 1) % 500 == 0:
            torch.cuda.synchronize()
            log(f"cycle {t + 1}: mse {float(mse[t]):.4f} var {float(var[t]):.4f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    m, v = mse.cpu().numpy(), var.cpu().numpy()
    keep = slice(burn, cycles)
    sm, sp = run.stats()
    return {"experiment": "sec5-cycled", "cycles": cycles, "burn_in": burn, "Q": Q, "iterations": iters,
            "n_ritz": n_ritz, "rtps_alpha": alpha, "ms_per_cycle": 1e3 * elapsed / cycles,
            "forecast_mse": float(np.mean(m[keep])), "forecast_mse_over_variance": float(np.mean(m[keep] / v[keep])),
            "finite": bool(np.all(np.isfinite(m)) and np.all(np.isfinite(v))),
            "last_status": [int(sm.counters[ie.CNT_STATUS]), int(sp.counters[ie.CNT_STATUS])]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="which", required=True)
    a4 = sub.add_parser("sec4")
    a4.add_argument("--trials", type=int, default=10)
    a4.add_argument("--p", type=int, nargs="+", default=[0, 4, 10, 20])
    a4.add_argument("--Q", type=int, nargs="+", default=[2, 4, 8])
    a4.add_argument("--iters", type=int, default=2)
    a5 = sub.add_parser("sec5")
    a5.add_argument("--cycles", type=int, default=5000)
    a5.add_argument("--burn", type=int, default=1000)
    a5.add_argument("--Q", type=int, default=8)
    a5.add_argument("--iters", type=int, default=10)
    a5.add_argument("--n-ritz", type=int, default=10)
    a5.add_argument("--alpha", type=float, default=0.01)
    a = ap.parse_args(argv)

    def log(msg):
        print("[experiment]", msg, file=sys.stderr, flush=True)

    if a.which == "sec4":
        out = sec4_experiment(a.trials, tuple(a.p), tuple(a.Q), a.iters, log=log)
    else:
        out = sec5_experiment(a.cycles, a.burn, a.Q, a.iters, a.n_ritz, a.alpha, log=log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
