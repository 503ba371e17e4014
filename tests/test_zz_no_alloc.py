"""The no-allocation covariance apply (infoesrf_cov_apply_noalloc) against the workspace entry
point infoesrf_cov_apply, through the C ABI: bit-identical results (same kernels, same inputs) on
two calls in a row, the second with a smaller input, which runs on the scratch the first call left
behind; FP64 also against the dense oracle P V to 1e-13; a call past the fixed scratch is refused
before any work."""
import sys

import numpy as np
import pytest

import synthetic as syn
from oracle import infoesrf_ref as ref
from parity import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2503_00253_amd import infoesrf as ie  # noqa: E402


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def workspace_apply(P, V, opts):
    """infoesrf_cov_apply on a workspace filled with NaN: nothing it reads may be stale."""
    import ctypes as C
    lib = ie.library()
    Vt = V.t().contiguous()
    B = Vt.shape[0]
    out = torch.empty_like(Vt)
    nbytes = lib.infoesrf_cov_apply_workspace_bytes(C.byref(P.c), B, C.byref(opts))
    ws = torch.full((nbytes // 8 + 1,), float("nan"), dtype=torch.float64, device=V.device)
    code = lib.infoesrf_cov_apply(C.byref(P.c), Vt.data_ptr(), P.n, B, out.data_ptr(), P.n, C.byref(opts),
                                  ws.data_ptr(), nbytes, ie._stream())
    assert code == ie.OK, ie.library().infoesrf_last_error()
    return out.t()


CASES = [("n4096-band-fp64", syn.config2, dict(cov_form=ie.COV_BAND), 300, 37),
         ("n4096-operator-fp32", syn.config2, dict(cov_form=ie.COV_OPERATOR, precision=ie.MIXED_FP32), 64, 5),
         ("n256-operator-bf16", syn.config1, dict(cov_form=ie.COV_OPERATOR, precision=ie.MIXED_BF16), 129, 17),
         ("n256-band-fp64", syn.config1, dict(cov_form=ie.COV_BAND), 640, 3)]


@pytest.mark.parametrize("name,make,kw,B1,B2", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_workspace_entry_point(name, make, kw, B1, B2):
    prob = make()
    P = ie.Problem.from_synthetic(prob)
    opts = ie.default_opts(**kw)
    dp = ref.DenseProblem.from_problem(prob) if kw.get("precision", ie.FP64) == ie.FP64 else None
    rng = np.random.default_rng(B1)
    for call, B in enumerate((B1, B2)):
        say("noalloc", name, "call", call, "B", B)
        Vh = rng.standard_normal((prob.n, B))
        V = torch.from_numpy(Vh).cuda()
        got = ie.cov_apply_noalloc(P, V, opts)
        want = workspace_apply(P, V, opts)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (name, call, float((got - want).abs().max()))
        if dp is not None:
            assert rel(got.cpu().numpy(), dp.P @ Vh) < 1e-13


def test_noalloc_refuses_past_its_scratch():
    prob = syn.config2()
    P = ie.Problem.from_synthetic(prob)
    opts = ie.default_opts(cov_form=ie.COV_BAND)
    import ctypes as C
    lib = ie.library()
    per = (lib.infoesrf_cov_apply_workspace_bytes(C.byref(P.c), 2, C.byref(opts))
           - lib.infoesrf_cov_apply_workspace_bytes(C.byref(P.c), 1, C.byref(opts)))
    base = lib.infoesrf_cov_apply_workspace_bytes(C.byref(P.c), 1, C.byref(opts)) - per
    Bmax = ((64 << 20) - base) // per
    say("noalloc limit: largest B", Bmax)
    V = torch.zeros((prob.n, Bmax + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(ie.InfoEsrfError) as e:
        ie.cov_apply_noalloc(P, V, opts)
    assert e.value.code == ie.ERR_WORKSPACE and "scratch" in str(e.value)
    # the largest call that fits runs
    V = torch.from_numpy(np.random.default_rng(1).standard_normal((prob.n, Bmax))).cuda()
    assert torch.equal(ie.cov_apply_noalloc(P, V, opts), workspace_apply(P, V, opts))
