"""Optimisation-loop driver over the libmgar C ABI (Fig. 5 flow, Sec. 3.1).

One cycle: density filter (Eq 6) -> solve (MGCG while the cycle index is below
N_on = 2/15 of the maximum cycle count, MGAR afterwards; Sec. 3.1-3.2) ->
compliance and filtered sensitivities (Eq 5, 9-11) -> optimality-criteria
update. Every step is a library call; this module only keeps the buffers, the
cycle counter and the filter-radius schedule of continuous density filtering
(Eq 22-23), whose radius it hands to the library when it changes.
"""
from __future__ import annotations

import dataclasses
import math

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
    seed_used: bool = False       # the learned guess replaced the previous temperature as T0
    res_seed: float = float("nan")
    res_prev: float = float("nan")
    radius: float = float("nan")  # density-filter radius of the cycle


def filter_radii(prob, ncycles, continuous=None):
    """Filter radius of cycles 1..ncycles. Fixed: prob.filter_r. Continuous
    (Eq 22-23), continuous = dict(r_min, alpha = 1.4/50, lp = 5/6 of
    prob.maxit): r^(0) = max(alpha L, r_min) with L the longest side in
    element edges, r^(k) = max(r_min, eta r^(k-1)), eta = exp((ln r_min -
    ln r^(0)) / lp); cycle k filters with r^(k-1)."""
    if not continuous:
        return [float(prob.filter_r)] * ncycles
    L = max(prob.nelx, prob.nely, prob.nelz if prob.dim == 3 else 0)
    r_min = float(continuous["r_min"])
    r = max(float(continuous.get("alpha", 1.4 / 50)) * L, r_min)
    lp = float(continuous.get("lp", 5.0 * prob.maxit / 6.0))
    eta = math.exp((math.log(r_min) - math.log(r)) / lp)
    out = []
    for _ in range(ncycles):
        out.append(r)
        r = max(r_min, eta * r)
    return out


class GuessSchedule:
    """When the learned guess is evaluated (inference plus two true residuals
    per evaluation). Every cycle while it wins; after a loss the next `gap`
    cycles start from the previous temperature (the fallback) without
    evaluating it, and the gap doubles with each further loss up to `cap`; a
    win resets it to 1. Disabled: every cycle."""

    def __init__(self, enabled=True, cap=16):
        self.enabled, self.cap = bool(enabled), int(cap)
        self.skip, self.gap = 0, 1

    def want(self) -> bool:
        if self.skip > 0:
            self.skip -= 1
            return False
        return True

    def record(self, won: bool):
        if not self.enabled:
            return
        if won:
            self.gap = 1
        else:
            self.skip = self.gap
            self.gap = min(2 * self.gap, self.cap)


class TopOpt:
    def __init__(self, prob, qelem, use_mgar=True, n_basis=2, cg_max=200, x_init=None,
                 eps_accept=None, basis_x0_zero=False, precision=M.PREC_FP64, inner_tol=None,
                 autotune=True, seed=None, timing=False, continuous=None, device="cuda"):
        """timing: per-solve device time in Cycle.solve_ms (one more host
        synchronisation per solve). continuous: None (fixed filter radius
        prob.filter_r) or the continuous-filtering schedule (filter_radii).
        seed: None, or a dict enabling the learned
        initial guess with keys
        channels (per level of the element-grid U-Net; default 16, 32, 64,
        64), train_until (cycles whose pairs train it; it is
        used from the next cycle on), steps (Adam steps after cycle
        train_until), lr, init_seed, backoff (GuessSchedule on; default True),
        backoff_cap, lag (default 0: training runs when cycle train_until
        ends and the guess is used from the next cycle; lag > 0: training
        runs in the background on the network's own stream, beside the
        solves of the next lag cycles, and the guess is used from cycle
        train_until + 1 + lag, whose solver stream first waits for it)."""
        self.prob = prob
        self.use_mgar = use_mgar
        self.params = M.params_for(prob, n_basis=n_basis, eps_accept=eps_accept, cg_max=cg_max,
                                   basis_x0_zero=basis_x0_zero, precision=precision,
                                   inner_tol=inner_tol)
        self.h = M.Handle(self.params)
        # per-solve device timing costs a host synchronisation per solve; off,
        # Cycle.solve_ms is -1
        self.h.mgar_set_timing(timing)
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
        self.radii = filter_radii(prob, prob.maxit, continuous) if continuous else None
        self.radius = float(prob.filter_r)
        self.seed = None
        if seed is not None:
            import workloads as W
            cfg = dict(channels=(16, 32, 64, 64), train_until=20, steps=120, lr=1e-3, init_seed=0,
                       backoff=True, backoff_cap=16, lag=0)
            cfg.update(seed)
            self.seed = cfg
            self.sched = GuessSchedule(cfg["backoff"], cfg["backoff_cap"])
            # lag > 0: the network works on a stream of its own (default priority)
            self.net_stream = torch.cuda.Stream() if int(cfg["lag"]) > 0 else None
            self.train_done = None
            self.net = M.Net(self.params, channels=cfg["channels"],
                             stream=self.net_stream.cuda_stream if self.net_stream is not None else None)
            self.net.mgar_net_set_params(W.unet_init(cfg["channels"], seed=cfg["init_seed"]))
            self.net.mgar_net_set_source(self.Qe)
            self.pairs = []
            self.Tseed = torch.zeros(N, **f64)
            self.train_losses = []

    def _seed_guess(self):
        """Learned guess for this cycle, kept only when its true residual is
        below that of the previous temperature (which stays the fallback)."""
        h = self.h
        scale = float(self.T_prev.abs().max())
        if scale <= 0.0:
            return self.T_prev, False, float("nan"), float("nan")
        cur = torch.cuda.current_stream()
        if self.net_stream is not None:
            if self.train_done is not None:     # first use: the background training ends first
                cur.wait_event(self.train_done)
                self.train_done = None
                self.pairs = []                 # later work on this stream comes after the wait
            self.net_stream.wait_stream(cur)    # this cycle's densities
        self.net.mgar_net_infer(self.xphys, scale, self.Tseed)
        if self.net_stream is not None:
            cur.wait_stream(self.net_stream)
        r_seed = h.mgar_residual(self.xphys, self.q, self.Tseed)
        r_prev = h.mgar_residual(self.xphys, self.q, self.T_prev)
        if r_seed < r_prev:
            return self.Tseed, True, r_seed, r_prev
        return self.T_prev, False, r_seed, r_prev

    def _seed_train(self):
        """Adam steps over the collected pairs in a seeded random order. The
        loss is read back (a host synchronisation) after the first step and,
        when training runs in the foreground, after the last."""
        cfg = self.seed
        n = len(self.pairs)
        if n == 0:
            return
        order = torch.Generator().manual_seed(int(cfg["init_seed"]))
        if self.net_stream is not None:
            self.net_stream.wait_stream(torch.cuda.current_stream())   # the pairs are ready
        steps = int(cfg["steps"])
        for s in range(steps):
            if s % n == 0:
                perm = torch.randperm(n, generator=order).tolist()
            xp, tp, sc = self.pairs[perm[s % n]]
            want = s == 0 or (s == steps - 1 and self.net_stream is None)
            loss = self.net.mgar_net_train_step(xp, tp, sc, cfg["lr"], want_loss=want)
            if want:
                self.train_losses.append(loss)
        if self.net_stream is not None:
            self.train_done = torch.cuda.Event()
            self.train_done.record(self.net_stream)   # the pairs stay alive until it is waited on
        else:
            self.pairs = []   # training data is not needed once the guess is in use

    def step(self) -> Cycle:
        self.k += 1
        h, p = self.h, self.prob
        if self.radii is not None:
            r = self.radii[min(self.k, len(self.radii)) - 1]
            if r != self.radius:
                h.mgar_set_filter_radius(r)
                self.radius = r
        h.mgar_density_filter(self.x, self.xphys)
        T0, used, r_seed, r_prev = self.T_prev, False, float("nan"), float("nan")
        if (self.seed is not None and self.k > self.seed["train_until"] + int(self.seed["lag"])
                and self.sched.want()):
            T0, used, r_seed, r_prev = self._seed_guess()
            self.sched.record(used)
        if (not self.use_mgar) or self.k < self.non:
            st = h.mgcg_solve(self.xphys, self.q, T0, p.tol, self.T)
        else:
            st = h.mgar_solve(self.xphys, self.q, T0, p.tol, self.T)
        if self.seed is not None and self.k <= self.seed["train_until"]:
            if self.k >= 2:
                scale = float(self.T_prev.abs().max())
                if scale > 0.0:
                    self.pairs.append((self.xphys.clone(), self.T.clone(), scale))
            if self.k == self.seed["train_until"]:
                self._seed_train()
        f, lam = h.mgar_sens_oc(self.xphys, self.T, self.q, self.x, p.volfrac, p.move, self.dc, self.dv,
                                self.xnew)
        self.x, self.xnew = self.xnew, self.x
        self.T, self.T_prev = self.T_prev, self.T
        return Cycle(self.k, f, st["path"], st["cg_iters"], st["res_ca"], st["res_final"],
                     st["ms"], lam, st["refinements"], used, r_seed, r_prev, self.radius)

    def postprocess(self, r_proj=None, nsub=4):
        """Boundary smoothing after the loop (Sec. 2.3, Eq 24-27; Fig. 5): filter
        the final design (the last cycle's radius), solve, sensitivities,
        mgar_smooth_boundary with projection radius r_proj (default: that
        filter radius), and one more solve on the smoothed densities. Returns
        (rho, level, volume, compliance before, compliance after)."""
        h, p = self.h, self.prob
        E = self.h.E
        f64 = dict(dtype=torch.float64, device=self.x.device)
        h.mgar_density_filter(self.x, self.xphys)
        st = h.mgcg_solve(self.xphys, self.q, self.T_prev, p.tol, self.T)
        f0 = h.sens_filter(self.xphys, self.T, self.q, self.dc, self.dv)
        rho = torch.empty(E, **f64)
        level, vol = h.mgar_smooth_boundary(self.dc, p.volfrac, self.radius if r_proj is None else r_proj, rho,
                                            nsub=nsub)
        h.mgcg_solve(rho, self.q, self.T, p.tol, self.T_prev)
        f1 = h.sens_filter(rho, self.T_prev, self.q, self.dc, self.dv)
        del st
        return rho, level, vol, f0, f1

    def run(self, ncycles=None):
        n = self.prob.maxit if ncycles is None else ncycles
        return [self.step() for _ in range(n)]

    @property
    def temperature(self):
        """Temperature of the last cycle."""
        return self.T_prev
