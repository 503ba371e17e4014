"""ctypes binding of libinfoesrf.so (include/infoesrf.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  torch supplies device memory (tensors, workspaces) and the current
HIP stream.  If the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinfoesrf.so")

# ---- constants mirrored from the header
OK, WARN_NOT_CONVERGED = 0, 1
ERR_INVALID_ARG, ERR_NOT_SPD, ERR_NUMERIC, ERR_WORKSPACE, ERR_HIP = -1, -2, -3, -4, -5
LOC_DENSE, LOC_STENCIL = 0, 1
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
SOLVER_PLAIN, SOLVER_COMPACT, SOLVER_PERSISTENT, SOLVER_MULTISHIFT, SOLVER_BLOCK = 0, 1, 2, 3, 4
DOMAIN_STATE, DOMAIN_OBS_LATTICE = 0, 1
START_ZERO, START_LEARNED = 0, 1
COV_AUTO, COV_OPERATOR, COV_BAND = 0, 1, 2
S_AUTO, S_OPERATOR, S_DENSE = 0, 1, 2
PROF_OP_FP64, PROF_OP_FP32, PROF_OP_BF16, PROF_BAND_FP64, PROF_BAND_FP32, PROF_PCG, PROF_TAIL = 0, 1, 2, 3, 4, 5, 6
PROF_SLOTS = 7
CNT_APPLIES, CNT_APPLIES_FP64, CNT_ITERATIONS, CNT_SWEEPS = 0, 1, 2, 3
CNT_FALLBACKS, CNT_NOT_CONVERGED, CNT_MAX_ITERS, CNT_STATUS = 4, 5, 6, 7
NUM_COUNTERS = 8


class Loc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nz", C.c_int32), ("nx", C.c_int32),
                ("periodic_z", C.c_int32), ("periodic_x", C.c_int32),
                ("bz", C.c_int32), ("bx", C.c_int32), ("reserved", C.c_int32),
                ("table", C.c_void_p), ("dense", C.c_void_p)]


class ProblemC(C.Structure):
    _fields_ = [("n", C.c_int64), ("N", C.c_int64), ("m", C.c_int64),
                ("X", C.c_void_p), ("h_ptr", C.c_void_p), ("h_idx", C.c_void_p),
                ("h_w", C.c_void_p), ("r_var", C.c_void_p), ("loc", Loc)]


class Lattice(C.Structure):
    _fields_ = [("z0", C.c_int32), ("sz", C.c_int32), ("nzo", C.c_int32),
                ("x0", C.c_int32), ("sx", C.c_int32), ("nxo", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("inner_rtol", C.c_double),
                ("max_iter", C.c_int32), ("n_ritz", C.c_int32), ("oversample", C.c_int32),
                ("precision", C.c_int32), ("solver", C.c_int32), ("warm_start", C.c_int32),
                ("host_sync", C.c_int32), ("apply_domain", C.c_int32), ("lattice", Lattice),
                ("seed", C.c_uint64), ("sketch", C.c_void_p), ("net", C.c_void_p),
                ("tile_rows", C.c_int32), ("cov_form", C.c_int32), ("fixed_iters", C.c_int32),
                ("s_form", C.c_int32), ("tail_systems", C.c_int32),
                ("warm_fp32", C.c_int32), ("reserved", C.c_int32 * 2)]


class StatsC(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("relres", C.c_void_p), ("converged", C.c_void_p),
                ("counters", C.c_void_p)]


class InfoEsrfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"infoesrf error {code}: {msg}")
        self.code = code


_lib = None


def library():
    """Load libinfoesrf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise InfoEsrfError(ERR_HIP, f"{LIB_PATH} not found: run python -m paper_2503_00253_amd.build")
    lib = C.CDLL(LIB_PATH)
    P, VP = C.POINTER, C.c_void_p
    lib.infoesrf_default_opts.argtypes = [P(Opts)]
    lib.infoesrf_default_opts.restype = None
    lib.infoesrf_workspace_bytes.argtypes = [P(ProblemC), C.c_int32, P(Opts)]
    lib.infoesrf_workspace_bytes.restype = C.c_size_t
    lib.infoesrf_cov_apply_workspace_bytes.argtypes = [P(ProblemC), C.c_int64, P(Opts)]
    lib.infoesrf_cov_apply_workspace_bytes.restype = C.c_size_t
    lib.infoesrf_cov_apply.argtypes = [P(ProblemC), VP, C.c_int64, C.c_int64, VP, C.c_int64, P(Opts),
                                       VP, C.c_size_t, VP]
    lib.infoesrf_cov_apply.restype = C.c_int
    lib.infoesrf_cov_apply_noalloc.argtypes = [P(ProblemC), VP, C.c_int64, C.c_int64, VP, C.c_int64, P(Opts), VP]
    lib.infoesrf_cov_apply_noalloc.restype = C.c_int
    lib.infoesrf_mean_update.argtypes = [P(ProblemC), VP, VP, P(Opts), P(StatsC), VP, C.c_size_t, VP]
    lib.infoesrf_mean_update.restype = C.c_int
    lib.infoesrf_perturbation_update.argtypes = [P(ProblemC), C.c_int32, P(C.c_double), P(C.c_double), VP, VP,
                                                 P(Opts), P(StatsC), VP, C.c_size_t, VP]
    lib.infoesrf_perturbation_update.restype = C.c_int
    lib.infoesrf_batched_workspace_bytes.argtypes = [P(ProblemC), C.c_int32, P(C.c_int32), P(Opts), P(Lattice)]
    lib.infoesrf_batched_workspace_bytes.restype = C.c_size_t
    PD = P(C.c_double)
    lib.infoesrf_update_batched.argtypes = [P(ProblemC), C.c_int32, P(C.c_int32), P(PD), P(PD), P(VP), P(VP),
                                            P(VP), P(Opts), P(Lattice), P(StatsC), VP, C.c_size_t, VP]
    lib.infoesrf_update_batched.restype = C.c_int
    lib.infoesrf_batched_one_launch.argtypes = [P(ProblemC), C.c_int32, P(C.c_int32), P(Opts), P(Lattice)]
    lib.infoesrf_batched_one_launch.restype = C.c_int
    FP = P(C.c_float)
    lib.infoesrf_net_create.argtypes = [C.c_int32, C.c_int32, C.c_uint64, P(VP)]
    lib.infoesrf_net_create.restype = C.c_int
    lib.infoesrf_net_load.argtypes = [C.c_char_p, P(VP)]
    lib.infoesrf_net_load.restype = C.c_int
    lib.infoesrf_net_save.argtypes = [VP, C.c_char_p]
    lib.infoesrf_net_save.restype = C.c_int
    lib.infoesrf_net_free.argtypes = [VP]
    lib.infoesrf_net_free.restype = None
    lib.infoesrf_net_param_count.argtypes = [VP]
    lib.infoesrf_net_param_count.restype = C.c_int64
    lib.infoesrf_net_get_params.argtypes = [VP, FP]
    lib.infoesrf_net_get_params.restype = C.c_int
    lib.infoesrf_net_set_params.argtypes = [VP, FP]
    lib.infoesrf_net_set_params.restype = C.c_int
    lib.infoesrf_net_workspace_bytes.argtypes = [VP, C.c_int64, C.c_int64, C.c_int64, C.c_int32]
    lib.infoesrf_net_workspace_bytes.restype = C.c_size_t
    lib.infoesrf_net_forward.argtypes = [VP, VP, C.c_int64, C.c_int64, VP, VP, C.c_size_t, VP]
    lib.infoesrf_net_forward.restype = C.c_int
    lib.infoesrf_net_forward_bf16.argtypes = [VP, VP, C.c_int64, C.c_int64, VP, VP, C.c_size_t, VP]
    lib.infoesrf_net_forward_bf16.restype = C.c_int
    lib.infoesrf_net_gradients.argtypes = [VP, VP, VP, VP, C.c_int64, C.c_int64, C.c_int64, VP, VP, VP, C.c_size_t,
                                           VP]
    lib.infoesrf_net_gradients.restype = C.c_int
    lib.infoesrf_net_train_step.argtypes = [VP, VP, VP, VP, C.c_int64, C.c_int64, C.c_int64, C.c_float, VP, VP,
                                            C.c_size_t, VP]
    lib.infoesrf_net_train_step.restype = C.c_int
    lib.infoesrf_warmstart_pairs.argtypes = [P(ProblemC), C.c_int32, P(C.c_double), P(C.c_double), VP, VP, VP, VP,
                                             P(Opts), P(StatsC), VP, C.c_size_t, VP]
    lib.infoesrf_warmstart_pairs.restype = C.c_int
    lib.infoesrf_l96_forecast.argtypes = [VP, C.c_int64, C.c_int64, C.c_int32, C.c_int32, VP, C.c_double,
                                          C.c_double, C.c_int32, VP]
    lib.infoesrf_l96_forecast.restype = C.c_int
    lib.infoesrf_observe.argtypes = [P(ProblemC), VP, VP, VP, VP]
    lib.infoesrf_observe.restype = C.c_int
    lib.infoesrf_rtps_assemble.argtypes = [VP, C.c_int64, VP, VP, C.c_int64, C.c_int64, C.c_int64, C.c_double, VP,
                                           C.c_int64, VP]
    lib.infoesrf_rtps_assemble.restype = C.c_int
    lib.infoesrf_autotune.argtypes = [P(ProblemC), C.c_int32, P(Opts), VP, C.c_size_t, VP, P(C.c_int32)]
    lib.infoesrf_autotune.restype = C.c_int
    lib.infoesrf_autotune_reset.argtypes = []
    lib.infoesrf_autotune_reset.restype = None
    lib.infoesrf_quadrature_elliptic.argtypes = [C.c_int32, C.c_double, P(C.c_double), P(C.c_double)]
    lib.infoesrf_quadrature_elliptic.restype = C.c_int
    lib.infoesrf_quadrature_gauss_legendre.argtypes = [C.c_int32, P(C.c_double), P(C.c_double)]
    lib.infoesrf_quadrature_gauss_legendre.restype = C.c_int
    lib.infoesrf_error_string.argtypes = [C.c_int]
    lib.infoesrf_error_string.restype = C.c_char_p
    lib.infoesrf_last_error.argtypes = []
    lib.infoesrf_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(code, allow_warn=True):
    if code == OK or (allow_warn and code == WARN_NOT_CONVERGED):
        return code
    lib = library()
    raise InfoEsrfError(code, lib.infoesrf_last_error().decode() or lib.infoesrf_error_string(code).decode())


def default_opts(**kw) -> Opts:
    o = Opts()
    library().infoesrf_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "lattice":
            o.lattice = Lattice(*v)
        elif k == "sketch":
            o.sketch = 0 if v is None else v.data_ptr()
        elif k == "net":
            o.net = None if v is None else (v.h.value if isinstance(v, Net) else v)
        else:
            setattr(o, k, v)
    return o


def quadrature_elliptic(Q: int, ell: float):
    s = np.zeros(Q)
    p = np.zeros(Q)
    _check(library().infoesrf_quadrature_elliptic(Q, ell, s.ctypes.data_as(C.POINTER(C.c_double)),
                                                   p.ctypes.data_as(C.POINTER(C.c_double))))
    return s, p


def quadrature_gauss_legendre(Q: int):
    s = np.zeros(Q)
    p = np.zeros(Q)
    _check(library().infoesrf_quadrature_gauss_legendre(Q, s.ctypes.data_as(C.POINTER(C.c_double)),
                                                         p.ctypes.data_as(C.POINTER(C.c_double))))
    return s, p


def lattice_of(h_ptr, h_idx, nz, nx):
    """Detect whether host CSR arrays describe point observations on a regular
    sub-lattice of the nz x nx grid; returns (z0, sz, nzo, x0, sx, nxo) or None."""
    h_ptr = np.asarray(h_ptr)
    h_idx = np.asarray(h_idx)
    m = len(h_ptr) - 1
    if not np.array_equal(h_ptr, np.arange(m + 1)):
        return None
    z, x = np.divmod(h_idx.astype(np.int64), nx)
    xs = np.unique(x)
    zs = np.unique(z)
    nxo, nzo = len(xs), len(zs)
    if nxo * nzo != m:
        return None
    sx = int(xs[1] - xs[0]) if nxo > 1 else 1
    sz = int(zs[1] - zs[0]) if nzo > 1 else 1
    a, b = np.divmod(np.arange(m), nxo)
    want = (zs[0] + a * sz) * nx + (xs[0] + b * sx)
    if not np.array_equal(want, h_idx):
        return None
    return (int(zs[0]), sz, nzo, int(xs[0]), sx, nxo)


def _torch():
    import torch
    return torch


class Problem:
    """Device-resident arguments of one filter instance (keeps the tensors alive)."""

    def __init__(self, X, h_ptr, h_idx, h_w, r_var, *, nz=1, nx=None, periodic_z=0, periodic_x=1, bz=0, bx=0,
                 table=None, dense=None, device="cuda"):
        torch = _torch()
        # column-major n x N on the device: a contiguous (N, n) tensor whose row i is member i
        if isinstance(X, np.ndarray):
            self.X = torch.from_numpy(np.ascontiguousarray(np.asarray(X, dtype=np.float64).T)).to(device)
        else:
            self.X = X.t().contiguous().to(device)
        N, n = self.X.shape
        self.n, self.N = int(n), int(N)
        self.h_ptr = torch.as_tensor(np.asarray(h_ptr, dtype=np.int32)).to(device)
        self.h_idx = torch.as_tensor(np.asarray(h_idx, dtype=np.int32)).to(device)
        self.h_w = torch.as_tensor(np.asarray(h_w, dtype=np.float64)).to(device)
        self.r_var = torch.as_tensor(np.asarray(r_var, dtype=np.float64)).to(device)
        self.m = int(len(h_ptr) - 1)
        self.host_h_ptr = np.asarray(h_ptr)
        self.host_h_idx = np.asarray(h_idx)
        loc = Loc()
        if dense is not None:
            # column-major n x n: a contiguous tensor holding L^T row by row
            self.dense = torch.from_numpy(np.ascontiguousarray(np.asarray(dense, dtype=np.float64).T)).to(device)
            loc.kind = LOC_DENSE
            loc.dense = self.dense.data_ptr()
            loc.nz, loc.nx = 1, self.n
        else:
            nx = self.n if nx is None else nx
            self.table = torch.as_tensor(np.ascontiguousarray(table, dtype=np.float64).reshape(-1)).to(device)
            loc.kind = LOC_STENCIL
            loc.nz, loc.nx = int(nz), int(nx)
            loc.periodic_z, loc.periodic_x = int(periodic_z), int(periodic_x)
            loc.bz, loc.bx = int(bz), int(bx)
            loc.table = self.table.data_ptr()
        self.loc = loc
        self.c = ProblemC(self.n, self.N, self.m, self.X.data_ptr(), self.h_ptr.data_ptr(), self.h_idx.data_ptr(),
                          self.h_w.data_ptr(), self.r_var.data_ptr(), loc)

    @classmethod
    def from_synthetic(cls, prob, device="cuda"):
        return cls(prob.X, prob.h_ptr, prob.h_idx, prob.h_w, prob.r_var, nz=prob.nz, nx=prob.nx,
                   periodic_z=prob.periodic_z, periodic_x=prob.periodic_x, bz=prob.bz, bx=prob.bx,
                   table=prob.table, device=device)

    def lattice(self):
        return lattice_of(self.host_h_ptr, self.host_h_idx, self.loc.nz, self.loc.nx)


@dataclass
class Stats:
    code: int
    iters: object
    relres: object
    converged: object
    counters: object

    def counter(self, i):
        return int(self.counters[i])


_ws_cache = {}


def _workspace(nbytes, device):
    torch = _torch()
    key = str(device)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _stats(nsys, device):
    torch = _torch()
    it = torch.zeros(nsys, dtype=torch.int32, device=device)
    rr = torch.zeros(nsys, dtype=torch.float64, device=device)
    cv = torch.zeros(nsys, dtype=torch.uint8, device=device)
    cn = torch.zeros(NUM_COUNTERS, dtype=torch.int64, device=device)
    sc = StatsC(it.data_ptr(), rr.data_ptr(), cv.data_ptr(), cn.data_ptr())
    return sc, (it, rr, cv, cn)


def workspace_bytes(problem: Problem, Q: int, opts: Opts) -> int:
    b = library().infoesrf_workspace_bytes(C.byref(problem.c), Q, C.byref(opts))
    if b == 0:
        raise InfoEsrfError(ERR_INVALID_ARG, library().infoesrf_last_error().decode())
    return int(b)


def cov_apply(problem: Problem, V, opts: Opts | None = None):
    """P V for state-space vectors V (torch, n x B, column-major: pass V with V.t() contiguous)."""
    torch = _torch()
    lib = library()
    opts = opts or default_opts()
    Vt = V.t().contiguous()  # B x n row-major == n x B column-major
    B = Vt.shape[0]
    out = torch.empty_like(Vt)
    nbytes = lib.infoesrf_cov_apply_workspace_bytes(C.byref(problem.c), B, C.byref(opts))
    ws = _workspace(nbytes, Vt.device)
    _check(lib.infoesrf_cov_apply(C.byref(problem.c), Vt.data_ptr(), problem.n, B, out.data_ptr(), problem.n,
                                  C.byref(opts), ws.data_ptr(), ws.numel(), _stream()), allow_warn=False)
    return out.t()


def cov_apply_noalloc(problem: Problem, V, opts: Opts | None = None, out=None):
    """P V through infoesrf_cov_apply_noalloc: no workspace (the library's fixed per-device
    scratch); the caller passes V (n x B, as for cov_apply) and may pass the output buffer
    (B x n contiguous, i.e. n x B column-major)."""
    torch = _torch()
    lib = library()
    opts = opts or default_opts()
    Vt = V.t().contiguous()
    B = Vt.shape[0]
    if out is None:
        out = torch.empty_like(Vt)
    _check(lib.infoesrf_cov_apply_noalloc(C.byref(problem.c), Vt.data_ptr(), problem.n, B, out.data_ptr(),
                                          problem.n, C.byref(opts), _stream()), allow_warn=False)
    return out.t()


def mean_update(problem: Problem, y, opts: Opts | None = None):
    torch = _torch()
    lib = library()
    opts = opts or default_opts()
    dev = problem.X.device
    y = torch.as_tensor(np.asarray(y, dtype=np.float64) if not torch.is_tensor(y) else y).to(dev)
    out = torch.empty(problem.n, dtype=torch.float64, device=dev)
    ws = _workspace(workspace_bytes(problem, 0, opts), dev)
    sc, keep = _stats(1, dev)
    code = _check(lib.infoesrf_mean_update(C.byref(problem.c), y.data_ptr(), out.data_ptr(), C.byref(opts),
                                           C.byref(sc), ws.data_ptr(), ws.numel(), _stream()))
    torch.cuda.synchronize()
    return out, Stats(code, *(t.cpu().numpy() for t in keep))


def perturbation_update(problem: Problem, s_nodes, p_weights, opts: Opts | None = None, y=None):
    """Returns (Xa_pert as an n x N torch view, Stats)."""
    torch = _torch()
    lib = library()
    opts = opts or default_opts()
    dev = problem.X.device
    s_nodes = np.ascontiguousarray(s_nodes, dtype=np.float64)
    p_weights = np.ascontiguousarray(p_weights, dtype=np.float64)
    Q = len(s_nodes)
    out = torch.empty((problem.N, problem.n), dtype=torch.float64, device=dev)  # column-major n x N
    ws = _workspace(workspace_bytes(problem, Q, opts), dev)
    sc, keep = _stats(Q * problem.N, dev)
    yp = 0
    if y is not None:
        yt = torch.as_tensor(np.asarray(y, dtype=np.float64)).to(dev)
        yp = yt.data_ptr()
    dp = C.POINTER(C.c_double)
    code = _check(lib.infoesrf_perturbation_update(
        C.byref(problem.c), Q, s_nodes.ctypes.data_as(dp), p_weights.ctypes.data_as(dp), C.c_void_p(yp),
        out.data_ptr(), C.byref(opts), C.byref(sc), ws.data_ptr(), ws.numel(), _stream()))
    torch.cuda.synchronize()
    return out.t(), Stats(code, *(t.cpu().numpy() for t in keep))


def batched_workspace_bytes(problems, Qs, opts: Opts, lattices=None) -> int:
    arr = (ProblemC * len(problems))(*[pb.c for pb in problems])
    qa = (C.c_int32 * len(Qs))(*Qs)
    lat = None
    if lattices is not None:
        lat = lattices if isinstance(lattices, C.Array) else (Lattice * len(lattices))(*[Lattice(*t) for t in lattices])
    b = library().infoesrf_batched_workspace_bytes(arr, len(problems), qa, C.byref(opts), lat)
    if b == 0:
        raise InfoEsrfError(ERR_INVALID_ARG, library().infoesrf_last_error().decode())
    return int(b)


def batched_one_launch(problems, Qs, opts: Opts, lattices=None) -> bool:
    """Whether infoesrf_update_batched runs these instances in one persistent launch per sweep."""
    arr = (ProblemC * len(problems))(*[pb.c for pb in problems])
    qa = (C.c_int32 * len(Qs))(*Qs)
    lat = None
    if lattices is not None:
        lat = lattices if isinstance(lattices, C.Array) else (Lattice * len(lattices))(*[Lattice(*t) for t in lattices])
    return bool(library().infoesrf_batched_one_launch(arr, len(problems), qa, C.byref(opts), lat))


class BatchedRunner:
    """Many independent instances in one infoesrf_update_batched call (buffers preallocated).

    problems: list of Problem; nodes: list of (s, p) host arrays; ys: list of observation
    vectors (needed when means are wanted).  run() only enqueues the call.
    """

    def __init__(self, problems, nodes, opts: Opts, ys=None, want_mean=True, lattices=None):
        torch = _torch()
        self.lib = library()
        self.problems = list(problems)
        self.opts = opts
        k = len(self.problems)
        dev = self.problems[0].X.device
        self.s = [np.ascontiguousarray(sn, dtype=np.float64) for sn, _ in nodes]
        self.p = [np.ascontiguousarray(pw, dtype=np.float64) for _, pw in nodes]
        self.Qs = [len(x) for x in self.s]
        self.outs = [torch.empty((pb.N, pb.n), dtype=torch.float64, device=dev) for pb in self.problems]
        self.means = [torch.empty(pb.n, dtype=torch.float64, device=dev) for pb in self.problems] if want_mean \
            else None
        self.ys = None
        if ys is not None:
            self.ys = [torch.as_tensor(np.asarray(y, dtype=np.float64)).to(dev) if not torch.is_tensor(y)
                       else y.to(dev, torch.float64) for y in ys]
        self.nsys = sum(q * pb.N + 1 for q, pb in zip(self.Qs, self.problems))
        self.sc, self.keep = _stats(self.nsys, dev)
        self._probs = (ProblemC * k)(*[pb.c for pb in self.problems])
        self._qa = (C.c_int32 * k)(*self.Qs)
        PD = C.POINTER(C.c_double)
        self._sp = (PD * k)(*[x.ctypes.data_as(PD) for x in self.s])
        self._pp = (PD * k)(*[x.ctypes.data_as(PD) for x in self.p])
        self._yp = (C.c_void_p * k)(*[y.data_ptr() for y in self.ys]) if self.ys is not None else None
        self._mp = (C.c_void_p * k)(*[mm.data_ptr() for mm in self.means]) if self.means is not None else None
        self._xp = (C.c_void_p * k)(*[o.data_ptr() for o in self.outs])
        self._lat = (Lattice * k)(*[Lattice(*t) for t in lattices]) if lattices is not None else None
        nbytes = batched_workspace_bytes(self.problems, self.Qs, opts, self._lat)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def run(self):
        return _check(self.lib.infoesrf_update_batched(
            self._probs, len(self.problems), self._qa, self._sp, self._pp, self._yp, self._mp, self._xp,
            C.byref(self.opts), self._lat, C.byref(self.sc), self.ws.data_ptr(), self.ws.numel(), _stream()))

    def one_launch(self):
        return bool(self.lib.infoesrf_batched_one_launch(self._probs, len(self.problems), self._qa,
                                                         C.byref(self.opts), self._lat))

    def results(self):
        """(list of n_j x N_j analysis deviations, list of analysis means or None)."""
        return [o.t() for o in self.outs], self.means

    def stats(self, code=0):
        """Per-system arrays over all instances (instance order, node-major, the mean system last)."""
        return Stats(code, *(t.cpu().numpy() for t in self.keep))


class Net:
    """Warm-start network handle (device parameters, Adam state); see infoesrf_net_* in the header."""

    def __init__(self, handle):
        self.h = C.c_void_p(handle) if not isinstance(handle, C.c_void_p) else handle
        self._ws = {}

    @classmethod
    def create(cls, hidden=64, kernel=9, seed=0):
        h = C.c_void_p()
        _check(library().infoesrf_net_create(hidden, kernel, seed, C.byref(h)), allow_warn=False)
        return cls(h)

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        _check(library().infoesrf_net_load(str(path).encode(), C.byref(h)), allow_warn=False)
        return cls(h)

    def save(self, path):
        _check(library().infoesrf_net_save(self.h, str(path).encode()), allow_warn=False)

    def free(self):
        if self.h:
            library().infoesrf_net_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def param_count(self):
        return int(library().infoesrf_net_param_count(self.h))

    def params(self):
        out = np.zeros(self.param_count, dtype=np.float32)
        _check(library().infoesrf_net_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))), allow_warn=False)
        return out

    def set_params(self, values):
        v = np.ascontiguousarray(values, dtype=np.float32)
        assert v.size == self.param_count
        _check(library().infoesrf_net_set_params(self.h, v.ctypes.data_as(C.POINTER(C.c_float))), allow_warn=False)

    D = 4  # trunk output channels (terms of the shift head)

    def _workspace(self, B, Q, m, training):
        torch = _torch()
        key = (B, Q if training else 1, m, bool(training))
        if key not in self._ws:
            nbytes = library().infoesrf_net_workspace_bytes(self.h, B, Q, m, 1 if training else 0)
            if nbytes == 0:
                raise InfoEsrfError(ERR_INVALID_ARG, library().infoesrf_last_error().decode())
            self._ws = {key: torch.empty(nbytes, dtype=torch.float32, device="cuda")}
        return self._ws[key]

    def forward(self, X, bf16=False):
        """Trunk: X (B, m) float32 CUDA tensor of the members' bh -> Y (B, D, m); bf16: BF16 weights
        and activations on MFMA."""
        torch = _torch()
        X = X.contiguous()
        B, m = X.shape
        Y = torch.empty((B, self.D, m), dtype=torch.float32, device=X.device)
        ws = self._workspace(B, 1, m, False)
        fn = library().infoesrf_net_forward_bf16 if bf16 else library().infoesrf_net_forward
        _check(fn(self.h, X.data_ptr(), B, m, Y.data_ptr(), ws.data_ptr(), ws.numel() * 4, _stream()),
               allow_warn=False)
        return Y

    @staticmethod
    def head(Y, cq):
        """The shift head: y (B, Q, m) = sum_d c_q^(d+1) Y[b, d] for cq (Q,) (torch, on Y's device)."""
        D = Y.shape[1]
        phi = torch_stack_pow(cq, D)
        return _torch().einsum("qd,bdt->bqt", phi, Y)

    def gradients(self, X, cq, T):
        """(gradient in the parameter layout, loss) of the mean relative L2 loss of the B x Q
        systems: X (B, m), cq (Q,), T (B, Q, m)."""
        torch = _torch()
        X, cq, T = X.contiguous(), cq.contiguous(), T.contiguous()
        B, m = X.shape
        Q = cq.shape[0]
        g = torch.empty(self.param_count, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        ws = self._workspace(B, Q, m, True)
        _check(library().infoesrf_net_gradients(self.h, X.data_ptr(), cq.data_ptr(), T.data_ptr(), B, Q, m,
                                                g.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel() * 4,
                                                _stream()), allow_warn=False)
        return g, loss

    def train_step(self, X, cq, T, lr):
        """One Adam step on a batch X (B, m), cq (Q,), T (B, Q, m); returns the batch loss before the
        step (device tensor)."""
        torch = _torch()
        B, m = X.shape
        Q = cq.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        ws = self._workspace(B, Q, m, True)
        _check(library().infoesrf_net_train_step(self.h, X.data_ptr(), cq.data_ptr(), T.data_ptr(), B, Q, m,
                                                 float(lr), loss.data_ptr(), ws.data_ptr(), ws.numel() * 4,
                                                 _stream()), allow_warn=False)
        return loss


def torch_stack_pow(cq, D):
    """(Q, D) powers c_q^(d+1)."""
    torch = _torch()
    return torch.stack([cq ** (d + 1) for d in range(D)], dim=1)


def warmstart_pairs(problem: Problem, s_nodes, p_weights, y=None, opts: Opts | None = None):
    """Training batch of the perturbation update's systems: X (N, m) the members' bh, cq (Q,) the
    shift factors, T (N, Q, m) the scaled solutions, and the solve's Stats."""
    torch = _torch()
    lib = library()
    opts = opts or default_opts()
    dev = problem.X.device
    s_nodes = np.ascontiguousarray(s_nodes, dtype=np.float64)
    p_weights = np.ascontiguousarray(p_weights, dtype=np.float64)
    Q = len(s_nodes)
    S = Q * problem.N
    X = torch.empty((problem.N, problem.m), dtype=torch.float32, device=dev)
    cq = torch.empty(Q, dtype=torch.float32, device=dev)
    T = torch.empty((problem.N, Q, problem.m), dtype=torch.float32, device=dev)
    yp = 0
    if y is not None:
        yt = torch.as_tensor(np.asarray(y, dtype=np.float64)).to(dev)
        yp = yt.data_ptr()
    ws = _workspace(workspace_bytes(problem, Q, opts), dev)
    sc, keep = _stats(S, dev)
    dp = C.POINTER(C.c_double)
    code = _check(lib.infoesrf_warmstart_pairs(C.byref(problem.c), Q, s_nodes.ctypes.data_as(dp),
                                               p_weights.ctypes.data_as(dp), C.c_void_p(yp), X.data_ptr(),
                                               cq.data_ptr(), T.data_ptr(), C.byref(opts), C.byref(sc),
                                               ws.data_ptr(), ws.numel(), _stream()))
    torch.cuda.synchronize()
    return X, cq, T, Stats(code, *(t.cpu().numpy() for t in keep))


def l96_forecast(X, nz, nx, forcing, gamma, dt, steps):
    """Advance the rows of X (k, n) (each row one state, i.e. a column-major n x k array) in place."""
    k, n = X.shape
    _check(library().infoesrf_l96_forecast(X.data_ptr(), n, k, nz, nx, forcing.data_ptr(), float(gamma), float(dt),
                                           int(steps), _stream()), allow_warn=False)
    return X


def observe(problem: Problem, x, noise, y):
    """y = H x + noise (device vectors; noise may be None)."""
    _check(library().infoesrf_observe(C.byref(problem.c), x.data_ptr(), None if noise is None else noise.data_ptr(),
                                      y.data_ptr(), _stream()), allow_warn=False)
    return y


def rtps_assemble(Xf, mean_a, Xa, alpha, out):
    """Analysis members out (N, n) = mean_a + RTPS-relaxed deviations Xa (N, n); Xf the forecast members."""
    N, n = Xf.shape
    _check(library().infoesrf_rtps_assemble(Xf.data_ptr(), n, mean_a.data_ptr(), Xa.data_ptr(), n, n, N,
                                            float(alpha), out.data_ptr(), n, _stream()), allow_warn=False)
    return out


def autotune(problem: Problem, Q: int, opts: Opts | None = None):
    """Measure and record the fastest apply block shapes for this problem's grid; returns
    [(precision, batch, choice, microseconds per launch), ...]."""
    lib = library()
    opts = opts or default_opts()
    dev = problem.X.device
    ws = _workspace(workspace_bytes(problem, Q, opts), dev)
    rep = (C.c_int32 * 24)(*([-1] * 24))
    _check(lib.infoesrf_autotune(C.byref(problem.c), Q, C.byref(opts), ws.data_ptr(), ws.numel(), _stream(), rep),
           allow_warn=False)
    return [tuple(rep[4 * i:4 * i + 4]) for i in range(6) if rep[4 * i] >= 0]


def autotune_reset():
    library().infoesrf_autotune_reset()


class PerturbationRunner:
    """Preallocated perturbation update: run() only enqueues the C call (no allocation)."""

    def __init__(self, problem: Problem, s_nodes, p_weights, opts: Opts, y=None):
        torch = _torch()
        self.lib = library()
        self.y = None if y is None else torch.as_tensor(np.asarray(y, dtype=np.float64)).to(problem.X.device)
        self.problem = problem
        self.opts = opts
        self.s = np.ascontiguousarray(s_nodes, dtype=np.float64)
        self.p = np.ascontiguousarray(p_weights, dtype=np.float64)
        self.Q = len(self.s)
        dev = problem.X.device
        self.out = torch.empty((problem.N, problem.n), dtype=torch.float64, device=dev)
        nbytes = workspace_bytes(problem, self.Q, opts)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.sc, self.keep = _stats(self.Q * problem.N, dev)
        dp = C.POINTER(C.c_double)
        self._sp = self.s.ctypes.data_as(dp)
        self._pp = self.p.ctypes.data_as(dp)

    def run(self):
        return _check(self.lib.infoesrf_perturbation_update(
            C.byref(self.problem.c), self.Q, self._sp, self._pp,
            None if self.y is None else C.c_void_p(self.y.data_ptr()), self.out.data_ptr(), C.byref(self.opts),
            C.byref(self.sc), self.ws.data_ptr(), self.ws.numel(), _stream()))

    def result(self):
        return self.out.t()

    def stats(self, code=0):
        return Stats(code, *(t.cpu().numpy() for t in self.keep))


def profile_enable(on: bool):
    lib = library()
    lib.infoesrf_profile_enable.argtypes = [C.c_int]
    lib.infoesrf_profile_enable.restype = C.c_int
    _check(lib.infoesrf_profile_enable(1 if on else 0), allow_warn=False)


def profile_select(slots):
    """Measure only the listed profile slots (PROF_*) until the next profile_enable."""
    lib = library()
    lib.infoesrf_profile_select.argtypes = [C.c_uint32]
    lib.infoesrf_profile_select.restype = C.c_int
    mask = 0
    for s in slots:
        mask |= 1 << int(s)
    _check(lib.infoesrf_profile_select(mask), allow_warn=False)


def profile_read():
    """Per slot (PROF_*: operator FP64/FP32/BF16, band FP64/FP32, the fused PCG step, the persistent
    PCG kernel): kernel ms, launches, vectors, algorithmic FLOPs and algorithmic bytes."""
    lib = library()
    D, I = C.c_double * PROF_SLOTS, C.c_int64 * PROF_SLOTS
    lib.infoesrf_profile_read.argtypes = [D, I, I, D, D]
    lib.infoesrf_profile_read.restype = C.c_int
    ms, la, ve, fl, by = D(), I(), I(), D(), D()
    _check(lib.infoesrf_profile_read(ms, la, ve, fl, by), allow_warn=False)
    return list(ms), list(la), list(ve), list(fl), list(by)
