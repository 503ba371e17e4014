"""HIP graph capture of one update (host_sync = 0).

With host_sync 0 the mean and perturbation updates make no host
synchronization and no host read-back, so torch.cuda.graph can capture them.
The captured graph is replayed several times with eager work and
synchronizations in between; every replay must reproduce the eager result
bit for bit (the graph holds the same kernels with the same arguments, and
clears its flags and counters with fill kernels, not memset nodes).
"""
import sys

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("precision,domain", [(ie.FP64, "state"), (ie.MIXED_BF16, "lattice")])
def test_graph_replays_match_eager(precision, domain):
    prob = syn.config1()
    P = ie.Problem.from_synthetic(prob)
    s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
    kw = dict(precision=precision, host_sync=0, max_iter=120)
    if domain == "lattice":
        kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice())
    opts = ie.default_opts(**kw)
    say("graph", precision, domain)
    run = ie.PerturbationRunner(P, s, p, opts)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert run.run() == ie.OK     # eager run (also sets kernel attributes before capture)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = run.result().clone()
    st = run.stats()
    assert st.counter(ie.CNT_STATUS) == 0 and st.counter(ie.CNT_NOT_CONVERGED) == 0
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run.run()
    torch.cuda.synchronize()
    for rep in range(3):
        run.out.fill_(float("nan"))        # eager work between replays
        run.keep[3].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("replay", rep)
        assert torch.equal(run.result(), eager), rep
        st = run.stats()
        assert st.counter(ie.CNT_STATUS) == 0 and st.counter(ie.CNT_NOT_CONVERGED) == 0
    # the graph also matches a host-synchronized call
    ref_opts = ie.default_opts(**{k: v for k, v in kw.items() if k != "host_sync"})
    want, _ = ie.perturbation_update(P, s, p, ref_opts)
    assert torch.equal(want, eager)


@pytest.mark.parametrize("precision", [ie.FP64, ie.MIXED_FP32])
def test_graph_replays_persistent_headline(precision):
    """The n = 4096 update with the bench's options (observed-lattice band, every system in
    the persistent kernel from its zero start, p = 4 + 4): one persistent launch per update
    runs every sweep, so the captured graph holds no host-decided launch count; each replay
    must equal the eager result bit for bit and the host-synchronized call too."""
    prob = syn.config2()
    P = ie.Problem.from_synthetic(prob)
    s, p = ie.quadrature_elliptic(prob.Q, prob.ell)
    kw = dict(precision=precision, apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=P.lattice(), n_ritz=4,
              oversample=4, tail_systems=0)
    say("graph headline", precision)
    run = ie.PerturbationRunner(P, s, p, ie.default_opts(host_sync=0, **kw))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert run.run() == ie.OK
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = run.result().clone()
    st = run.stats()
    assert st.counter(ie.CNT_STATUS) == 0 and st.counter(ie.CNT_NOT_CONVERGED) == 0
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run.run()
    torch.cuda.synchronize()
    for rep in range(3):
        run.out.fill_(float("nan"))
        run.keep[3].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("replay", rep)
        assert torch.equal(run.result(), eager), rep
        st = run.stats()
        assert st.counter(ie.CNT_STATUS) == 0 and st.counter(ie.CNT_NOT_CONVERGED) == 0
    want, _ = ie.perturbation_update(P, s, p, ie.default_opts(**kw))
    assert torch.equal(want, eager)
