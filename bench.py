#!/usr/bin/env python
"""Benchmark of the InFo-ESRF perturbation update on one MI355X.

One step = one call of infoesrf_perturbation_update on the n=4096 Gaussian
workload (N=40 members, m=1024 point observations, Q=16 elliptic nodes: 640
shifted SPD systems solved to a true FP64 relative residual of 1e-8),
including ensemble statistics, preconditioner setup, all PCG solves, the
quadrature combine and the final state-space apply.  Inputs are resident in
HBM before the timed region.

Printed: one JSON line with the solve rate, the roofline position of the
dominant kernel (the instrumented kernel with the most time: a covariance
apply or the fused PCG step, timed live with HIP events on its stream), the
rate of plain GPU PCG (FP64, operator-form state-space applies, masked
systems, no compaction) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {0: 78.6, 1: 157.3, 2: 2500.0}   # MI355X dense matrix peaks: FP64, FP32, BF16
# FP64 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
PEAK_ALU_FP64 = 78.6
PEAK_HBM_GBS = 8000.0                            # MI355X HBM3E
# L2 -> CU reads: each CU's vector L1 fills at 64 B/clk from its XCD's L2 (16 channels x 128 B/clk
# per XCD serve its 32 CUs): 256 CUs x 64 B x 2.4 GHz
PEAK_L2_GBS = 256 * 64 * 2.4
DTYPE = {0: "f64", 1: "f32/f64", 2: "bf16/f64"}
# profile slots of the covariance applies: (kernel, bound, MFMA peak key)
SLOTS = {0: ("k_cov_stencil<fp64>", "mfma", 0), 1: ("k_cov_stencil<fp32>", "mfma", 1),
         2: ("k_cov_bf16", "mfma", 2), 3: ("k_band_apply<fp64>", "hbm", None),
         4: ("k_band_apply<fp32>", "hbm", None), 5: ("k_pcg_fused", "hbm", None),
         6: ("k_pcg_tail", "alu", None)}
SOLVERS = {"plain": 0, "compact": 1, "multishift": 3, "block": 4}
SRC = {0: "cov_apply.hip", 1: "cov_apply.hip", 2: "cov_apply.hip", 3: "band.hip", 4: "band.hip", 5: "pcg.hip",
       6: "pcg_tail.hip"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default=None,
                    help="inner applies: fp64, or fp32/bf16 with FP64 residual sweeps (default: fp32 for the "
                         "n4096 and batched64 workloads, fp64 for the cycles)")
    ap.add_argument("--domain", choices=["state", "lattice"], default="lattice")
    ap.add_argument("--solver", choices=["plain", "compact", "multishift", "block"], default="compact",
                    help="compact: batched PCG with the limited-memory preconditioner (default); plain: the "
                         "same with converged systems masked; multishift: one unpreconditioned CG process "
                         "per member serving every node; block: one block PCG per node over the members")
    ap.add_argument("--form", choices=["auto", "operator", "band"], default="auto",
                    help="covariance form: explicit band of P, or the operator form sum_i z_i o L(z_i o v)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing Sec. 3.2's two alternatives (block PCG, multi-shift CG) beside the line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["n4096", "batched64", "lorenz-cycle", "paper-sec5-cycle"],
                    default="n4096",
                    help="n4096: one update of the n=4096 case (the headline line); batched64: the uneven "
                         "batch of 64 independent instances in one batched call; lorenz-cycle: cycled "
                         "assimilation of the 8 x 480 multi-layer Lorenz-96 model (steps = cycles); "
                         "paper-sec5-cycle: the cycled experiment of Sec. 5 (32 x 40 atmosphere, 40 "
                         "members, 40 vertical channels, 10 fixed PCG iterations, p = 10)")
    ap.add_argument("--graph", action="store_true", help="lorenz-cycle: replay a HIP graph of one cycle")
    ap.add_argument("--eager", action="store_true",
                    help="n4096: time host-synchronized calls instead of replays of a captured update")
    ap.add_argument("--no-fp64-line", action="store_true", help="n4096: skip the FP64 line beside a mixed one")
    ap.add_argument("--no-learned", action="store_true", help="n4096: skip the learned+mixed line")
    ap.add_argument("--learn-updates", type=int, default=24,
                    help="n4096 learned line: n = 4096 updates (other seeds) whose 640 systems each train the net")
    ap.add_argument("--learn-steps", type=int, default=1500, help="n4096 learned line: Adam steps of 8 members")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in block-shape rules")
    ap.add_argument("--inner-rtol", type=float, default=None,
                    help="mixed precision: the first sweep's inner target relative to the residual "
                         "(default: the library's)")
    ap.add_argument("--n-ritz", type=int, default=None,
                    help="Ritz pairs of the limited-memory preconditioner (default: 4 for the n = 4096 workload, "
                         "the library's 10 for the cycles and the batch)")
    ap.add_argument("--oversample", type=int, default=None,
                    help="extra sketch columns of the randomized eigensolver (default: 4 for the n = 4096 "
                         "workload, the library's 10 otherwise)")
    ap.add_argument("--tail", type=int, default=0,
                    help="live systems at which one persistent launch finishes the PCG loop (0: the library's "
                         "default, -1: never)")
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="largest number of host cores the CPU oracle baseline may use")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device copy before the timed region (scale for HBM counters)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_record(src_path, kernel):
    """HBM traffic per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/traffic.json, one record per kernel family), if its source is unchanged since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    recs = json.load(open(path))
    rec = recs.get(kernel.split("<")[0])
    if not rec:
        return None
    sha = hashlib.sha256(open(src_path, "rb").read()).hexdigest()
    return rec if rec.get("source_sha256") == sha else None


def band_shape(prob, P, domain):
    """(stencil planes, rows) of the band the persistent kernel applies: the sub-sampled stencil
    on the observed lattice (rows = m), or the state grid's stencil (rows = n)."""
    if domain == "lattice":
        z0, sz, nzo, x0, sx, nxo = P.lattice()
        return (2 * (prob.bz // sz) + 1) * (2 * (prob.bx // sx) + 1), nzo * nxo
    return (2 * prob.bz + 1) * (2 * prob.bx + 1), prob.n


def cpu_baseline(a):
    """The CPU oracle timed on the host, in a child process that never touches the GPU (the
    parent has initialised it): the result of cpu_baseline_child."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--n-ritz", str(a.n_ritz),
           "--oversample", str(a.oversample), "--cpu-cores", str(a.cpu_cores)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"error": f"cpu baseline child exited with {r.returncode}: {r.stderr[-400:]}"}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _pcg_member(args):
    """One member x all nodes of the n = 4096 workload by the oracle's matrix-free PCG on one
    thread (a worker of the all-cores sample)."""
    member, n_ritz, oversample = args
    from threadpoolctl import threadpool_limits

    import synthetic as syn
    from oracle import infoesrf_ref as ref
    prob = syn.config2()
    s0, p0, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
    Om = syn.sketch_matrix(prob.m, n_ritz + oversample, 1) if n_ritz > 0 else None
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, it = ref.info_esrf_pcg(prob, s0, p0, rtol=1e-8, n_ritz=n_ritz, Omega=Om, members=[member])
        t1 = time.perf_counter()
    return prob.Q, int(it.sum()), t1 - t0


def cpu_baseline_child(a):
    """Times the oracle as it stands on the n = 4096 workload, on the host's cores:

    * dense: the eigendecomposition oracle (dense P, S and its eigenvectors, the finite-Q update
      of all Q N systems at once), BLAS on all the cores it may use;
    * pcg: the matrix-free FP64 PCG with the limited-memory preconditioner to rel-res 1e-8, one
      member x all Q nodes per worker process, one worker per core, and the same on one core.
    Prints one JSON line; value is the faster of the all-core paths."""
    import concurrent.futures as cf
    import multiprocessing as mp

    from threadpoolctl import threadpool_info, threadpool_limits

    import synthetic as syn
    from oracle import infoesrf_ref as ref
    cores = max(1, min(len(os.sched_getaffinity(0)), a.cpu_cores))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    prob = syn.config2()
    systems = prob.Q * prob.N
    with threadpool_limits(limits=cores):
        blas = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
        t0 = time.perf_counter()
        dp = ref.DenseProblem.from_problem(prob)
        s0, p0, _ = ref.quadrature_elliptic(prob.Q, prob.ell)
        ref.perturbation_update_quadrature(dp, s0, p0)
        t1 = time.perf_counter()
    dense = {"value": round(systems / (t1 - t0), 3), "seconds": round(t1 - t0, 3), "systems": systems,
             "blas_threads": cores}
    # matrix-free PCG: one member per worker, every worker on its own core
    ctx = mp.get_context("fork")
    members = list(range(min(cores, prob.N)))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=len(members), mp_context=ctx) as ex:
        res = list(ex.map(_pcg_member, [(i, a.n_ritz, a.oversample) for i in members]))
    t1 = time.perf_counter()
    nsys = sum(r[0] for r in res)
    pcg_all = {"value": round(nsys / (t1 - t0), 3), "seconds": round(t1 - t0, 3), "systems": nsys,
               "workers": len(members), "iterations": sum(r[1] for r in res)}
    q1, it1, sec1 = _pcg_member((0, a.n_ritz, a.oversample))
    pcg_one = {"value": round(q1 / sec1, 3), "seconds": round(sec1, 3), "systems": q1, "iterations": it1,
               "cores": 1}
    best = max((dense, "dense"), (pcg_all, "pcg"), key=lambda t: t[0]["value"])
    return {"value": best[0]["value"], "unit": "solves/s",
            "cores": cores if best[1] == "dense" else len(members), "kind": "oracle",
            "sample": (f"value = the {best[1]} path. dense: one whole update ({systems} systems) by the "
                       f"eigendecomposition oracle, BLAS on {cores} threads, {dense['seconds']} s; pcg: "
                       f"{nsys} systems ({len(members)} members x {prob.Q} nodes), matrix-free FP64 PCG with "
                       f"{a.n_ritz} Ritz pairs to rel-res 1e-8 in the state space, one worker process per "
                       f"member on its own core, {pcg_all['seconds']} s; one core: {q1} systems in {sec1:.1f} s"),
            "cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)), "cores_used_max": cores,
            "blas": blas, "paths": {"dense_all_cores": dense, "pcg_all_cores": pcg_all, "pcg_one_core": pcg_one}}


def main():
    a = parse()
    if a.cpu_baseline_child:
        if a.n_ritz is None:
            a.n_ritz = 4
        if a.oversample is None:
            a.oversample = 4
        print(json.dumps(cpu_baseline_child(a)), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                          "(sharding by ensemble member is designed but not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import synthetic as syn
    from paper_2503_00253_amd import infoesrf as ie

    if a.precision is None:
        a.precision = "fp32" if a.workload in ("n4096", "batched64") else "fp64"
    prec = {"fp64": ie.FP64, "fp32": ie.MIXED_FP32, "bf16": ie.MIXED_BF16}[a.precision]
    if a.workload == "batched64":
        return bench_batched(a, prec)
    if a.workload in ("lorenz-cycle", "paper-sec5-cycle"):
        return bench_cycle(a, prec)
    prob = syn.config2()
    # at this workload a small Ritz basis costs least per solve (n_ritz 0/4/8/10/12: 554k/527k/465k/
    # 462k/394k solves/s measured with oversample 4 or 10); the default keeps a preconditioner
    if a.n_ritz is None:
        a.n_ritz = 4
    if a.oversample is None:
        a.oversample = 4
    log("workload", prob.name, "precision", a.precision, "domain", a.domain, "solver", a.solver)
    P = ie.Problem.from_synthetic(prob)
    s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
    kw = dict(precision=prec, solver=SOLVERS[a.solver],
              cov_form={"auto": ie.COV_AUTO, "operator": ie.COV_OPERATOR, "band": ie.COV_BAND}[a.form],
              n_ritz=a.n_ritz, oversample=a.oversample, tail_systems=a.tail)
    if a.inner_rtol is not None:
        kw.update(inner_rtol=a.inner_rtol)
    if a.domain == "lattice":
        kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice())
    opts = ie.default_opts(**kw)
    # block shapes measured on this problem (outside the timed region)
    tuned = ie.autotune(P, prob.Q, opts) if not a.no_autotune else []
    log("autotune", tuned)
    run = ie.PerturbationRunner(P, s, p, opts)
    systems = prob.Q * prob.N
    if a.copy_calibration:
        src_buf = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del src_buf, dst_buf

    for w in range(a.warmup):
        code = run.run()
        torch.cuda.synchronize()
        log("warmup", w, "code", code)
        st = run.stats(code)
        log("iterations: total", int(st.iters.sum()), "max", int(st.iters.max()), "mean", float(st.iters.mean()),
            "sweeps", st.counter(ie.CNT_SWEEPS), "not converged", st.counter(ie.CNT_NOT_CONVERGED))

    # one profiled step finds the dominant kernel; the timed steps then carry events around that
    # kernel only, so the measurement perturbs the timeline as little as possible
    ie.profile_enable(True)
    run.run()
    torch.cuda.synchronize()
    ms0 = ie.profile_read()[0]
    dom = max(range(len(ms0)), key=lambda i: ms0[i])
    ie.profile_enable(True)
    ie.profile_select([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        code = run.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches, vectors, flops, nbytes = ie.profile_read()   # one entry per profile slot
    ie.profile_enable(False)
    st = run.stats(code)
    assert st.counter(ie.CNT_NOT_CONVERGED) == 0, "systems missed rtol"
    ms_step = (t1 - t0) * 1e3 / a.steps
    value = systems * a.steps / (t1 - t0)
    log(f"{value:.1f} solves/s, {ms_step:.3f} ms/step")

    kname, bound, pk = SLOTS[dom]
    secs = ms[dom] * 1e-3
    avg_ms = ms[dom] / max(launches[dom], 1)
    src = os.path.join(ROOT, "paper_2503_00253_amd", "csrc", SRC[dom])
    tr = traffic_record(src, kname)
    extra = {}
    if bound == "mfma":
        achieved = flops[dom] / secs / 1e12 if secs > 0 else 0.0
        peak, unit = PEAK_TFLOPS[pk], "TFLOP/s"
    elif bound == "alu":
        # the persistent PCG kernel streams the band of S from L2 once per iteration: bound by the
        # L2 -> CU path, with the FP64 ALU fraction beside it
        # the kernel counts each system-iteration (vectors) and adds the flops of every apply,
        # the residual checks' included, at 2 nnz(L) + m (12 + 8 p) each (periodic lattice: every
        # stencil point of every row is a nonzero)
        planes, m_rows = band_shape(prob, P, a.domain)
        per_apply = 2.0 * planes * m_rows + m_rows * (12.0 + 8.0 * a.n_ritz)
        checks = max(flops[dom] / per_apply - vectors[dom], 0.0)
        it_bytes = planes * m_rows * (4.0 if a.precision == "fp32" else 8.0)
        l2_bytes = vectors[dom] * it_bytes + checks * planes * m_rows * 8.0
        alu = flops[dom] / secs / 1e12 if secs > 0 else 0.0
        achieved = l2_bytes / secs / 1e9 if secs > 0 else 0.0
        peak, unit, bound = PEAK_L2_GBS, "GB/s", "l2"
        extra = {"alu_achieved_tflops": round(alu, 3), "alu_peak_tflops": PEAK_ALU_FP64,
                 "alu_frac": round(alu / PEAK_ALU_FP64, 4),
                 "l2_bytes_per_launch": l2_bytes / max(launches[dom], 1),
                 "l2_bytes_per_iteration_apply": it_bytes, "band_planes": planes, "band_rows": m_rows}
    else:
        achieved = nbytes[dom] / secs / 1e9 if secs > 0 else 0.0
        peak, unit = PEAK_HBM_GBS, "GB/s"
    roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": (tr or {}).get("bytes_per_launch"), **extra,
            "kernel": kname, "launches": launches[dom], "avg_launch_ms": round(avg_ms, 4), "vectors": vectors[dom],
            "flops_per_launch": flops[dom] / max(launches[dom], 1),
            "flops_per_vector": flops[dom] / max(vectors[dom], 1),
            "bytes_per_launch": nbytes[dom] / max(launches[dom], 1),
            "time_share": round(ms[dom] / (ms_step * a.steps), 4)}
    log("roofline", roof)
    log("profile slots ms", [round(x, 3) for x in ms], "launches", launches)
    roof["first_step_ms_by_kernel"] = {SLOTS[i][0]: round(ms0[i], 3) for i in range(len(ms0)) if ms0[i] > 0}

    out = {"metric": "shifted SPD solves/s at rel-res 1e-8", "value": round(value, 2), "unit": "solves/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
           "data": "synthetic",
           "config": {"workload": prob.name, "n": prob.n, "N": prob.N, "m": prob.m, "Q": prob.Q,
                      "systems_per_step": systems, "rtol": 1e-8, "precision": a.precision,
                      "apply_domain": a.domain, "solver": a.solver, "cov_form": a.form, "n_ritz": a.n_ritz,
                      "oversample": a.oversample,
                      "tail_systems": a.tail,
                      "autotuned": [list(t) for t in tuned]},
           "iterations": {"total": int(st.iters.sum()), "max": int(st.iters.max()),
                          "fp64_sweeps": st.counter(ie.CNT_SWEEPS)},
           "roofline": roof}

    if not a.eager:
        # the same update captured once without host synchronization and replayed: the setup's
        # launches cost no host time.  The roofline above comes from the eager steps (the graph
        # holds the same kernels with the same arguments); every replay must reproduce the eager
        # result, and the device statistics after the replays must show every system converged.
        gvalue, gms, gres, gst = time_replays(ie, torch, P, s, p, kw, a.steps, systems)
        gdiff = float((gres - run.result()).norm() / run.result().norm())
        assert gdiff <= 1e-12, f"graph replay differs from the eager update: {gdiff}"
        out["eager"] = {"value": out["value"], "ms_per_step": out["ms_per_step"]}
        out["value"] = round(gvalue, 2)
        out["ms_per_step"] = round(gms, 4)
        out["config"]["graph"] = True
        out["roofline"]["time_share"] = round(roof["avg_launch_ms"] / gms, 4)
        value = gvalue
        log(f"graph replay: {gvalue:.1f} solves/s, {gms:.3f} ms/step, rel diff vs eager {gdiff:.2e}")
    else:
        out["config"]["graph"] = False

    if prec != ie.FP64 and not a.no_fp64_line:
        # the same options with FP64 inner applies: the mixed line's error against it, per member
        fkw = dict(kw, precision=ie.FP64)
        if a.eager:
            frun = ie.PerturbationRunner(P, s, p, ie.default_opts(**fkw))
            frun.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                fcode = frun.run()
            torch.cuda.synchronize()
            fms = (time.perf_counter() - t0) * 1e3 / a.steps
            fst, fres = frun.stats(fcode), frun.result()
            fvalue = systems * 1e3 / fms
        else:
            fvalue, fms, fres, fst = time_replays(ie, torch, P, s, p, fkw, a.steps, systems)
        assert fst.counter(ie.CNT_NOT_CONVERGED) == 0, "FP64 line: systems missed rtol"
        col = ((run.result() - fres).norm(dim=0) / fres.norm(dim=0)).max()
        out["fp64_line"] = {"value": round(fvalue, 2), "unit": "solves/s", "ms_per_step": round(fms, 4),
                            "max_iterations": int(fst.iters.max()),
                            "mixed_vs_fp64_rel_err": float((run.result() - fres).norm() / fres.norm()),
                            "mixed_vs_fp64_max_member_rel_err": float(col),
                            "mixed_speedup": round(value / fvalue, 3)}
        log("FP64 line", out["fp64_line"])

    if not a.no_learned:
        out["learned_mixed"] = learned_line(a, ie, torch, syn, P, s, p, kw, run, st, systems)
        log("learned line", out["learned_mixed"])

    if not a.no_compare and a.solver == "compact":
        # Sec. 3.2's alternatives on the same workload and options, to the same true FP64 residual
        comp = {}
        for name in ("block", "multishift"):
            okw = dict(kw, solver=SOLVERS[name], precision=ie.FP64)   # both run FP64 inner solves
            if name == "multishift":
                okw.pop("n_ritz", None)
                okw.pop("oversample", None)
            arun = ie.PerturbationRunner(P, s, p, ie.default_opts(**okw))
            arun.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                acode = arun.run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ast = arun.stats(acode)
            assert ast.counter(ie.CNT_NOT_CONVERGED) == 0, f"{name}: systems missed rtol"
            diff = float((arun.result() - run.result()).norm() / run.result().norm())
            comp[name] = {"value": round(systems * 3 / (t1 - t0), 2), "ms_per_step": round((t1 - t0) * 1e3 / 3, 4),
                          "max_iterations": int(ast.iters.max()), "rel_diff_vs_line": diff}
            log("alternative", name, comp[name])
        out["solver_comparison"] = comp

    if not a.no_plain:
        # the plain baseline: FP64 operator-form applies of P in the state space every iteration
        # (no band, no dense S), masked systems
        popts = ie.default_opts(precision=ie.FP64, solver=ie.SOLVER_PLAIN, cov_form=ie.COV_OPERATOR,
                                s_form=ie.S_OPERATOR, n_ritz=a.n_ritz, oversample=a.oversample)
        prun = ie.PerturbationRunner(P, s, p, popts)
        prun.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.plain_steps):
            prun.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pv = systems * a.plain_steps / (t1 - t0)
        diff = float((run.result() - prun.result()).norm() / prun.result().norm())
        if "learned_mixed" in out:
            out["learned_mixed"]["speedup_vs_plain"] = round(out["learned_mixed"]["value"] / pv, 3)
        out["plain_gpu_pcg"] = {"value": round(pv, 2), "unit": "solves/s", "steps": a.plain_steps,
                                "speedup": round(value / pv, 3), "rel_diff_vs_plain": diff,
                                "options": f"FP64, operator form sum_i z_i o L(z_i o v) in the state space, masked "
                                           f"systems, one launch per iteration, zero start, {a.n_ritz} Ritz pairs "
                                           f"+ {a.oversample} oversampling (the line's preconditioner)"}
        log("plain GPU PCG", pv, "speedup", value / pv, "diff", diff)
        if a.domain == "lattice":
            # the same solver and options in the state space (general H), beside the lattice line
            skw = dict(kw)
            skw.pop("apply_domain", None)
            skw.pop("lattice", None)
            srun = ie.PerturbationRunner(P, s, p, ie.default_opts(**skw))
            srun.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.plain_steps):
                scode = srun.run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sst = srun.stats(scode)
            assert sst.counter(ie.CNT_NOT_CONVERGED) == 0, "state-domain line: systems missed rtol"
            sv = systems * a.plain_steps / (t1 - t0)
            out["state_domain_line"] = {"value": round(sv, 2), "unit": "solves/s",
                                        "ms_per_step": round((t1 - t0) * 1e3 / a.plain_steps, 4),
                                        "max_iterations": int(sst.iters.max()),
                                        "rel_diff_vs_line": float((srun.result() - run.result()).norm()
                                                                  / run.result().norm())}
            log("state-domain line", out["state_domain_line"])

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a)
        log("cpu baseline", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


def time_replays(ie, torch, P, s, p, kw, steps, systems):
    """One update with these options captured without host synchronization, replayed twice, then
    timed over `steps` replays: (solves/s, ms per update, result, device statistics)."""
    grun = ie.PerturbationRunner(P, s, p, ie.default_opts(host_sync=0, **kw))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        grun.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        grun.run()
    torch.cuda.synchronize()
    for _ in range(2):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gst = grun.stats(0)
    assert gst.counter(ie.CNT_NOT_CONVERGED) == 0, "graph replay: systems missed rtol"
    ms = (t1 - t0) * 1e3 / steps
    return systems * 1e3 / ms, ms, grun.result().clone(), gst


def learned_line(a, ie, torch, syn, P, s, p, kw, run, st, systems):
    """The learned start on the line's options: a network trained here, on the GPU by the
    library's kernels, on the systems of other n = 4096 updates (seeds 1..k), then the update run
    from its start (host-synchronized, eager) against the zero start timed the same way."""
    import numpy as np

    t0 = time.perf_counter()
    Xs, Ts, cq = [], [], None
    for seed in range(1, 1 + a.learn_updates):
        pr = syn.config2(seed)
        Pj = ie.Problem.from_synthetic(pr)
        okw = dict(kw)
        if "lattice" in okw:
            okw["lattice"] = Pj.lattice()
        X, cq, T, wst = ie.warmstart_pairs(Pj, s, p, None, ie.default_opts(**okw))
        assert wst.code == ie.OK
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    gen_s = time.perf_counter() - t0
    net = ie.Net.create(64, 9, 2503)
    g = torch.Generator(device="cpu").manual_seed(0)
    t0 = time.perf_counter()
    for step in range(a.learn_steps):
        idx = torch.randint(0, X.shape[0], (8,), generator=g).cuda()
        lr = 2e-3 * (0.1 + 0.9 * 0.5 * (1 + np.cos(np.pi * step / a.learn_steps)))
        net.train_step(X[idx].contiguous(), cq, T[idx].contiguous(), lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def eager(opts):
        r = ie.PerturbationRunner(P, s, p, opts)
        r.run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(a.steps):
            code = r.run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / a.steps
        rst = r.stats(code)
        assert rst.counter(ie.CNT_NOT_CONVERGED) == 0, "learned line: systems missed rtol"
        return systems * 1e3 / ms, ms, rst, r.result()

    lv, lms, lst, lres = eager(ie.default_opts(warm_start=ie.START_LEARNED, net=net, **kw))
    zv, zms, zst, _ = eager(ie.default_opts(**kw))
    return {"value": round(lv, 2), "unit": "solves/s", "ms_per_step": round(lms, 4),
            "zero_start_value": round(zv, 2), "zero_start_ms_per_step": round(zms, 4),
            "mean_iterations": {"zero": round(float(zst.iters.mean()), 3), "learned": round(float(lst.iters.mean()), 3)},
            "max_iterations": {"zero": int(zst.iters.max()), "learned": int(lst.iters.max())},
            "rel_diff_vs_line": float((lres - run.result()).norm() / run.result().norm()),
            "train": {"pairs": int(T.shape[0] * T.shape[1]), "updates": a.learn_updates, "steps": a.learn_steps,
                      "pair_seconds": round(gen_s, 2), "train_seconds": round(train_s, 2)},
            "timing": "both host-synchronized calls (no graph), same options as the line"}


def bench_cycle(a, prec):
    """Forecast-analysis cycles: the 8 x 480 multi-layer Lorenz-96 assimilation (N = 20, m = 1280
    point observations, Q = 12, solves to rel-res 1e-8), or the experiment of Sec. 5 (32 x 40,
    N = 40, 40 vertical channels, Q = 8, 10 fixed PCG iterations per solve)."""
    import numpy as np
    import torch

    import synthetic as syn
    from paper_2503_00253_amd import infoesrf as ie
    from paper_2503_00253_amd.cycle import CycleRunner

    paper = a.workload == "paper-sec5-cycle"
    cycles = a.warmup + a.steps
    form = {"auto": ie.COV_AUTO, "operator": ie.COV_OPERATOR, "band": ie.COV_BAND}[a.form]
    if paper:
        if prec != ie.FP64:
            raise SystemExit("paper-sec5-cycle runs its fixed iteration count in FP64 (--precision fp64)")
        prob = syn.experiment2_problem()
        noise = syn.experiment2_noise(cycles, prob.m)
        kw = dict(precision=prec, cov_form=form, n_ritz=10 if a.n_ritz is None else a.n_ritz, fixed_iters=10,
                  solver=SOLVERS[a.solver], tail_systems=a.tail)
        if a.oversample is not None:
            kw.update(oversample=a.oversample)
        run = CycleRunner(prob, noise=noise, opts=ie.default_opts(**kw), lattice=False)
        name = f"paper-sec5-lorenz96-32x40-N40-m40-Q{run.Q}-fixed10-cycle"
        metric = "shifted SPD solves/s at 10 fixed PCG iterations"
    else:
        prob = syn.lorenz_problem()
        noise = np.random.default_rng(4242).standard_normal((cycles, prob.m)) * np.sqrt(prob.r_var[0])
        run = CycleRunner(prob, noise=noise)
        # a small Ritz basis, as on the n4096 line (4 pairs + 4 oversampling unless given)
        kw = dict(precision=prec, apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=run.P.lattice(), cov_form=form,
                  solver=SOLVERS[a.solver], tail_systems=a.tail, n_ritz=4 if a.n_ritz is None else a.n_ritz,
                  oversample=4 if a.oversample is None else a.oversample)
        if a.inner_rtol is not None:
            kw.update(inner_rtol=a.inner_rtol)
        run.set_opts(ie.default_opts(**kw))
        name = "lorenz96-8x480-N20-m1280-Q12-cycle"
        metric = "shifted SPD solves/s at rel-res 1e-8"
    for _ in range(a.warmup):
        run.step()
    torch.cuda.synchronize()
    graph = None
    if a.graph:
        # without host synchronization every launch of the iteration loop is in the graph: cap the
        # loop at twice the largest count the eager warm-up cycles needed
        most = int(max(run.stats()[1].iters.max(), run.stats()[0].iters.max()))
        run.set_opts(ie.default_opts(host_sync=0, max_iter=2 * most + 4, **kw))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        saved = run.state.clone()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            run.cycle_body()
        torch.cuda.synchronize()
        run.state.copy_(saved)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        if graph is not None:
            run.load_noise(run.t)
            graph.replay()
            run.t += 1
        else:
            run.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mse, var = run.diagnostics()
    sm, sp = run.stats()
    systems = prob.N * run.Q + 1
    value = systems * a.steps / (t1 - t0)
    out = {"metric": metric, "value": round(value, 2), "unit": "solves/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round((t1 - t0) * 1e3 / a.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
           "data": "synthetic",
           "config": {"workload": name, "n": prob.n, "N": prob.N, "m": prob.m,
                      "Q": run.Q, "systems_per_step": systems, "step": "one forecast-analysis cycle",
                      "graph": bool(a.graph), "precision": a.precision, "rtps_alpha": run.alpha,
                      "solver": a.solver, "n_ritz": run.opts.n_ritz, "oversample": run.opts.oversample},
           "final_analysis": {"mse": mse, "variance": var},
           "last_cycle_iterations": {"mean": float(sp.iters.mean()), "max": int(sp.iters.max())}}
    log(f"{value:.1f} solves/s, {(t1 - t0) * 1e3 / a.steps:.3f} ms/cycle, mse {mse:.4f} var {var:.4f}")
    print(json.dumps(out), flush=True)


def bench_batched(a, prec):
    """64 independent instances (n = 4*U{128..2048}, N in {16..64}, Q = U{8..24}) in one batched call."""
    import torch

    import synthetic as syn
    from paper_2503_00253_amd import infoesrf as ie

    probs = syn.config4_instances()
    Ps = [ie.Problem.from_synthetic(pr) for pr in probs]
    nodes = [ie.quadrature_elliptic(pr.Q, pr.ell) for pr in probs]
    systems = sum(pr.Q * pr.N for pr in probs)
    kw = dict(precision=prec, solver=SOLVERS[a.solver],
              cov_form={"auto": ie.COV_AUTO, "operator": ie.COV_OPERATOR, "band": ie.COV_BAND}[a.form],
              tail_systems=a.tail)
    # a small Ritz basis, as on the n4096 line (4 pairs + 4 oversampling unless given): 474k against
    # 344k solves/s with the library's 10 + 10 (mixed FP32)
    if a.n_ritz is None:
        a.n_ritz = 4
    if a.oversample is None:
        a.oversample = 4
    kw.update(n_ritz=a.n_ritz, oversample=a.oversample)
    if a.inner_rtol is not None:
        kw.update(inner_rtol=a.inner_rtol)
    lats = None
    if a.domain == "lattice":
        kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE)
        lats = [P.lattice() for P in Ps]
    run = ie.BatchedRunner(Ps, nodes, ie.default_opts(**kw), ys=[pr.y for pr in probs], want_mean=False,
                           lattices=lats)
    log("batched64:", len(probs), "instances,", systems, "systems, workspace", run.ws.numel() >> 20, "MiB")
    for w in range(a.warmup):
        code = run.run()
        torch.cuda.synchronize()
        log("warmup", w, "code", code)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        code = run.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = run.stats(code)
    assert st.counter(ie.CNT_NOT_CONVERGED) == 0, "systems missed rtol"
    value = systems * a.steps / (t1 - t0)
    out = {"metric": "shifted SPD solves/s at rel-res 1e-8", "value": round(value, 2), "unit": "solves/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round((t1 - t0) * 1e3 / a.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
           "data": "synthetic",
           "config": {"workload": "gaussian-batch64-uneven", "instances": len(probs), "systems_per_step": systems,
                      "n_range": [min(pr.n for pr in probs), max(pr.n for pr in probs)],
                      "N_range": [min(pr.N for pr in probs), max(pr.N for pr in probs)],
                      "Q_range": [min(pr.Q for pr in probs), max(pr.Q for pr in probs)], "rtol": 1e-8,
                      "precision": a.precision, "apply_domain": a.domain, "solver": a.solver,
                      "n_ritz": a.n_ritz, "oversample": a.oversample, "one_launch": run.one_launch()},
           "iterations": {"total": int(st.iters.sum()), "max": int(st.iters.max())}}
    log(f"{value:.1f} solves/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
