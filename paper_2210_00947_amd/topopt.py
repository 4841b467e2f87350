"""Optimisation-loop driver over the libmgar C ABI (Fig. 5 flow, Sec. 3.1).

One cycle: density filter (Eq 6) -> solve (MGCG while the cycle index is below
N_on = 2/15 of the maximum cycle count, MGAR afterwards; Sec. 3.1-3.2) ->
compliance and filtered sensitivities (Eq 5, 9-11) -> optimality-criteria
update. Every step is a library call; this module only keeps the buffers and
the cycle counter.
"""
from __future__ import annotations

import dataclasses

import torch

from . import mgar as M


@dataclasses.dataclass
class Cycle:
    cycle: int
    compliance: float
    path: int
    cg_iters: int
    res_ca: float
    res_final: float
    solve_ms: float
    lam: float
    refinements: int = 0


class TopOpt:
    def __init__(self, prob, qelem, use_mgar=True, n_basis=2, cg_max=200, x_init=None,
                 eps_accept=None, basis_x0_zero=False, precision=M.PREC_FP64, inner_tol=None,
                 autotune=True, device="cuda"):
        self.prob = prob
        self.use_mgar = use_mgar
        self.params = M.params_for(prob, n_basis=n_basis, eps_accept=eps_accept, cg_max=cg_max,
                                   basis_x0_zero=basis_x0_zero, precision=precision,
                                   inner_tol=inner_tol)
        self.h = M.Handle(self.params)
        self.tune_source = None
        if autotune:
            from . import tune
            _, self.tune_source = tune.autotune(self.h, self.params, tune.device_arch())
        N, E = self.h.N, self.h.E
        f64 = dict(dtype=torch.float64, device=device)
        self.Qe = torch.as_tensor(qelem, **f64).contiguous()
        self.q = torch.empty(N, **f64)
        self.h.mgar_load_vector(self.Qe, self.q)
        if x_init is None:
            self.x = torch.full((E,), prob.x_init, **f64)
        else:
            self.x = torch.as_tensor(x_init, **f64).clone()
        self.xnew = torch.empty(E, **f64)
        self.xphys = torch.empty(E, **f64)
        self.T = torch.zeros(N, **f64)
        self.T_prev = torch.zeros(N, **f64)
        self.dc = torch.empty(E, **f64)
        self.dv = torch.empty(E, **f64)
        self.k = 0
        self.non = M.n_on(prob.maxit)

    def step(self) -> Cycle:
        self.k += 1
        h, p = self.h, self.prob
        h.mgar_density_filter(self.x, self.xphys)
        if (not self.use_mgar) or self.k < self.non:
            st = h.mgcg_solve(self.xphys, self.q, self.T_prev, p.tol, self.T)
        else:
            st = h.mgar_solve(self.xphys, self.q, self.T_prev, p.tol, self.T)
        f = h.sens_filter(self.xphys, self.T, self.q, self.dc, self.dv)
        lam = h.oc_update(self.x, self.dc, self.dv, p.volfrac, p.move, self.xnew)
        self.x, self.xnew = self.xnew, self.x
        self.T, self.T_prev = self.T_prev, self.T
        return Cycle(self.k, f, st["path"], st["cg_iters"], st["res_ca"], st["res_final"],
                     st["ms"], lam, st["refinements"])

    def run(self, ncycles=None):
        n = self.prob.maxit if ncycles is None else ncycles
        return [self.step() for _ in range(n)]

    @property
    def temperature(self):
        """Temperature of the last cycle."""
        return self.T_prev
