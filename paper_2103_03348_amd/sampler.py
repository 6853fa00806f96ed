"""Adaptively preconditioned HMC on the free log-rates (Sec. 2.3.2).

The driver keeps all state on the device and calls the library's hmc_step once
per iteration.  Between iterations it adapts:
  * the step size, by dual averaging towards a target acceptance rate during
    warm-up (Hoffman & Gelman 2014, Algorithm 5's schedule), then frozen; each
    iteration uses the step size times a uniform jitter in [1 - j, 1 + j] (Neal
    2011, Sec. 5.4.2.2), so that a well-preconditioned target, whose coordinates
    all oscillate at one frequency, is not sampled at a fixed fraction of its
    period;
  * the diagonal mass matrix, as the running average of preconditioner
    estimates computed at a fixed interval (the paper's adaptation, which keeps
    Monte Carlo estimates asymptotically unbiased).  The estimate is either the
    exact z-space curvature theta^2 H - theta g + P (Eq. 4 and Eq. 5 by the O(N
    M) subset path, floored at the prior's precision P), or theta^2 exp(y) + P
    with y a small network's prediction of log H (preconditioner.py), or the
    prior's precision alone (no preconditioning).
Only the scalar control (step size, iteration counters) lives on the host; every
quantity of the method is computed by the library.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from . import _lib
from .hawkes import Plan


class DualAveraging:
    """Nesterov dual averaging of log(eps) (Hoffman & Gelman 2014)."""

    def __init__(self, eps0, target=0.8, gamma=0.05, t0=10.0, kappa=0.75):
        self.mu = math.log(10.0 * eps0)
        self.target, self.gamma, self.t0, self.kappa = target, gamma, t0, kappa
        self.hbar = 0.0
        self.log_eps_bar = 0.0
        self.t = 0
        self.eps = eps0

    def update(self, accept_prob):
        self.t += 1
        w = 1.0 / (self.t + self.t0)
        self.hbar = (1.0 - w) * self.hbar + w * (self.target - accept_prob)
        log_eps = self.mu - math.sqrt(self.t) / self.gamma * self.hbar
        eta = self.t ** (-self.kappa)
        self.log_eps_bar = eta * log_eps + (1.0 - eta) * self.log_eps_bar
        self.eps = math.exp(log_eps)
        return self.eps

    def final(self):
        return math.exp(self.log_eps_bar)


class HmcSampler:
    """HMC over z = log theta on the subset `idx` of a plan's events."""

    def __init__(self, plan: Plan, theta: torch.Tensor, idx: torch.Tensor, hyper, sigma_z=0.5, L=20, seed=1,
                 jitter=0.5, beta=0.0):
        self.plan = plan
        self.dev = theta.device
        self.theta = theta.clone().contiguous()
        self.idx = idx.to(device=self.dev, dtype=torch.int64).contiguous()
        self.m = int(self.idx.numel())
        _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, self.m, _lib.ptr(self.idx),
                                                     _lib.stream_handle()), "hawkes_plan_set_subset")
        self.hyper = _lib.Hyper.of(hyper)
        self.sigma_z = float(sigma_z)
        self.L = int(L)
        self.seed = int(seed)
        self.counter = 0
        self.jitter = float(jitter)
        self.beta = float(beta)  # temporal trend: theta_k = exp(z_k + beta t_k) (Sec. 2.2)
        self.prior = 0           # 0: z ~ N(0, sigma_z^2 I); 1: phylogenetic prior (set_tree)
        self._jrng = np.random.default_rng(seed)
        self.z = torch.empty(self.m, dtype=torch.float64, device=self.dev)
        _lib.check(_lib.lib().hawkes_subset_z(plan.handle, _lib.ptr(self.theta), self.beta, _lib.ptr(self.z),
                                              _lib.stream_handle()), "hawkes_subset_z")
        # the prior's precision 1/sigma_z^2 until the first estimate is folded in
        self.mass = torch.full((self.m,), 1.0 / self.sigma_z ** 2, dtype=torch.float64, device=self.dev)
        self.mass_count = 0
        self.out = torch.zeros(8, dtype=torch.float64, device=self.dev)

    # ---- preconditioner estimates ----------------------------------------------------------
    def curvature(self, curv: torch.Tensor = None, log_h: torch.Tensor = None):
        """The library's hawkes_subset_curvature at the current state, into the
        given device buffers (slot order): the exact z-space curvature
        theta^2 H - theta g + P (FP64) and log max(H, 1e-6) (FP32)."""
        _lib.check(_lib.lib().hawkes_subset_curvature(self.plan.handle, ctypes.byref(self.hyper),
                                                      _lib.ptr(self.theta), self.sigma_z, self.prior,
                                                      _lib.ptr(curv), _lib.ptr(log_h), _lib.stream_handle()),
                   "hawkes_subset_curvature")

    def exact_curvature(self) -> torch.Tensor:
        """-d2 log pi / dz^2 on the subset at the current state (a new FP64 tensor)."""
        out = torch.empty(self.m, dtype=torch.float64, device=self.dev)
        self.curvature(curv=out)
        return out

    def fold_exact(self):
        """Fold the exact curvature at the current state into the running-average mass."""
        _lib.check(_lib.lib().hawkes_mass_update(self.plan.handle, ctypes.byref(self.hyper), _lib.ptr(self.theta),
                                                 None, self.sigma_z, self.prior, self.mass_count,
                                                 _lib.ptr(self.mass), _lib.stream_handle()), "hawkes_mass_update")
        self.mass_count += 1

    def set_tree(self, parent, length, tau0):
        """Use the phylogenetic Brownian prior of Eq. 2 on z (tips = subset slots):
        parent [2m - 1] (-1 at the root), branch lengths [2m - 1], root factor tau0.
        The prior's variance scale is sigma_z."""
        import numpy as np
        par = np.ascontiguousarray(parent, dtype=np.int64)
        ln = np.ascontiguousarray(length, dtype=np.float64)
        if par.shape[0] != 2 * self.m - 1 or ln.shape[0] != par.shape[0]:
            raise ValueError("the tree must have 2m - 1 nodes for m subset slots")
        _lib.check(_lib.lib().hawkes_plan_set_tree(self.plan.handle, par.shape[0], par.ctypes.data_as(ctypes.c_void_p),
                                                   ln.ctypes.data_as(ctypes.c_void_p), float(tau0)),
                   "hawkes_plan_set_tree")
        self.prior = 1

    def trend_grad(self, beta=None):
        """hawkes_subset_trend_grad at the current z: (loglik, d/dz [m], d/dbeta) as
        device tensors; also writes theta on the subset for that beta."""
        b = self.beta if beta is None else float(beta)
        ll = torch.empty(1, dtype=torch.float64, device=self.dev)
        gz = torch.empty(self.m, dtype=torch.float64, device=self.dev)
        gb = torch.empty(1, dtype=torch.float64, device=self.dev)
        _lib.check(_lib.lib().hawkes_subset_trend_grad(self.plan.handle, ctypes.byref(self.hyper),
                                                       _lib.ptr(self.z), b, _lib.ptr(self.theta), _lib.ptr(ll),
                                                       _lib.ptr(gz), _lib.ptr(gb), _lib.stream_handle()),
                   "hawkes_subset_trend_grad")
        return ll, gz, gb

    # ---- one iteration ------------------------------------------------------------------------
    def step(self, eps):
        if self.jitter > 0:
            eps = eps * self._jrng.uniform(1.0 - self.jitter, 1.0 + self.jitter)
        args = _lib.HmcArgs(self.z.data_ptr(), self.theta.data_ptr(), self.mass.data_ptr(), float(eps), self.L,
                            self.sigma_z, self.seed, self.counter, 0, self.out.data_ptr(), self.beta, self.prior,
                            None)
        _lib.check(_lib.lib().hmc_step(self.plan.handle, ctypes.byref(self.hyper), ctypes.byref(args),
                                       _lib.stream_handle()), "hmc_step")
        self.counter += 1

    def run(self, n_iter, warmup, eps0=0.02, mass="exact", refresh=50, learned=None, exact_every=None,
            record=True, target_accept=0.8):
        """Run warmup + n_iter iterations.  mass in {"identity", "exact", "learned"}.
        With "learned", `learned` (a LearnedPreconditioner) supplies the estimate and
        the exact estimate is still folded in every `exact_every` iterations (the
        exact kernel stays the judge).  Returns dict(draws [n_iter, m] host array, eps, accept,
        seconds of the sampling phase, seconds of the warm-up)."""
        da = DualAveraging(eps0, target=target_accept)
        eps = eps0
        draws = torch.empty((n_iter if record else 0, self.m), dtype=torch.float64, device=self.dev)
        acc = torch.zeros((), dtype=torch.float64, device=self.dev)

        def refresh_mass(it):
            if mass == "identity":
                return
            if it % refresh != 0:
                return
            if mass == "exact" or (exact_every and it % exact_every == 0):
                self.fold_exact()
            else:
                learned.fold_into_mass(self)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(warmup):
            refresh_mass(it)
            self.step(eps)
            eps = da.update(float(self.out[4].item()))
        eps = da.final() if warmup > 0 else eps0
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        t0 = time.perf_counter()
        for it in range(n_iter):
            refresh_mass(warmup + it)
            self.step(eps)
            acc += self.out[0]
            if record:
                draws[it].copy_(self.z)
        torch.cuda.synchronize()
        t_samp = time.perf_counter() - t0
        return {"draws": draws.cpu().numpy() if record else None, "eps": eps,
                "accept": float(acc.item()) / max(n_iter, 1), "seconds": t_samp, "warmup_seconds": t_warm}
