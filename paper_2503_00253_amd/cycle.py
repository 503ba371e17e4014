"""Cycled assimilation driver (the experiment of Sec. 5) on the library's kernels.

One cycle: forecast every member and the truth with the multi-layer
Lorenz-96 model (infoesrf_l96_forecast), observe the truth
(infoesrf_observe, noise drawn beforehand and passed in), update the mean
and the perturbations (infoesrf_mean_update, infoesrf_perturbation_update),
and form the analysis members with relaxation to prior spread
(infoesrf_rtps_assemble).  All buffers are allocated once; a cycle only
enqueues library calls on the current stream, so with host_sync = 0 a cycle
can be captured in a HIP graph and replayed (the noise of cycle t is copied
into the fixed noise buffer before each replay).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import infoesrf as ie


class CycleRunner:
    def __init__(self, prob, Q=None, ell=None, opts=None, alpha=0.01, noise=None, lattice=True):
        """prob: a synthetic multi-layer problem (synthetic.lorenz.lorenz_problem); noise: (cycles, m)."""
        torch = ie._torch()
        self.lib = ie.library()
        meta = prob.meta
        self.nz, self.nx = prob.nz, prob.nx
        self.n, self.N, self.m = prob.n, prob.N, prob.m
        self.gamma, self.dt, self.steps = meta["gamma"], meta["dt"], meta["steps_per_cycle"]
        self.alpha = alpha
        dev = "cuda"
        # members and truth in one (N + 1, n) buffer: rows 0..N-1 are the ensemble the update sees
        self.state = torch.empty((self.N + 1, self.n), dtype=torch.float64, device=dev)
        self.state[:self.N] = torch.from_numpy(np.ascontiguousarray(prob.X.T))
        self.state[self.N] = torch.from_numpy(prob.truth)
        self.P = ie.Problem.from_synthetic(prob)
        self.P.X = self.state[:self.N]          # the update reads the live ensemble
        self.P.c.X = self.P.X.data_ptr()
        forcing = np.broadcast_to(np.asarray(meta["forcing"], dtype=np.float64), (self.nz,))
        self.forcing = torch.from_numpy(np.array(forcing)).to(dev)   # per layer
        Q = Q or prob.Q
        ell = ell or prob.ell
        s, p = ie.quadrature_elliptic(Q, ell)
        self.s = np.ascontiguousarray(s)
        self.p = np.ascontiguousarray(p)
        self.Q = Q
        kw = {}
        if lattice and self.P.lattice() is not None:
            kw.update(apply_domain=ie.DOMAIN_OBS_LATTICE, lattice=self.P.lattice())
        self.y = torch.empty(self.m, dtype=torch.float64, device=dev)
        self.noise_buf = torch.zeros(self.m, dtype=torch.float64, device=dev)
        self.noise = None if noise is None else torch.as_tensor(np.asarray(noise, dtype=np.float64)).to(dev)
        self.mean_a = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.Xa = torch.empty((self.N, self.n), dtype=torch.float64, device=dev)
        self.ws = None
        self.set_opts(opts if opts is not None else ie.default_opts(**kw))
        self.sc_m, self.keep_m = ie._stats(1, dev)
        self.sc_p, self.keep_p = ie._stats(Q * self.N, dev)
        dp = C.POINTER(C.c_double)
        self._sp, self._pp = self.s.ctypes.data_as(dp), self.p.ctypes.data_as(dp)
        self.t = 0

    def set_opts(self, opts):
        """Options of the mean and perturbation updates; the workspace grows when they need more
        (set options before capturing a cycle in a graph)."""
        torch = ie._torch()
        nbytes = max(ie.workspace_bytes(self.P, self.Q, opts), ie.workspace_bytes(self.P, 0, opts))
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.state.device)
        self.opts = opts

    # --- the pieces of one cycle (each only enqueues library calls)
    def forecast(self):
        ie.l96_forecast(self.state, self.nz, self.nx, self.forcing, self.gamma, self.dt, self.steps)

    def observe(self):
        ie.observe(self.P, self.state[self.N], self.noise_buf, self.y)

    def update(self):
        st = ie._stream()
        c1 = self.lib.infoesrf_mean_update(C.byref(self.P.c), self.y.data_ptr(), self.mean_a.data_ptr(),
                                           C.byref(self.opts), C.byref(self.sc_m), self.ws.data_ptr(),
                                           self.ws.numel(), st)
        c2 = self.lib.infoesrf_perturbation_update(C.byref(self.P.c), self.Q, self._sp, self._pp, None,
                                                   self.Xa.data_ptr(), C.byref(self.opts), C.byref(self.sc_p),
                                                   self.ws.data_ptr(), self.ws.numel(), st)
        return ie._check(c1), ie._check(c2)

    def assemble(self):
        ens = self.state[:self.N]
        ie.rtps_assemble(ens, self.mean_a, self.Xa, self.alpha, ens)

    def cycle_body(self):
        self.forecast()
        self.observe()
        self.update()
        self.assemble()

    def load_noise(self, t):
        if self.noise is not None:
            self.noise_buf.copy_(self.noise[t % self.noise.shape[0]])

    def step(self):
        self.load_noise(self.t)
        self.cycle_body()
        self.t += 1

    def diagnostics(self):
        """Forecast-space diagnostics of the current ensemble: (mse of the mean vs truth, mean variance)."""
        ens = self.state[:self.N]
        mu = ens.mean(dim=0)
        mse = float(((mu - self.state[self.N]) ** 2).mean())
        var = float(ens.var(dim=0, unbiased=True).mean())
        return mse, var

    def stats(self):
        return (ie.Stats(0, *(t.cpu().numpy() for t in self.keep_m)),
                ie.Stats(0, *(t.cpu().numpy() for t in self.keep_p)))
