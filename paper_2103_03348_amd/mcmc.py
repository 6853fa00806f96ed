"""Random-scan Metropolis-within-Gibbs over the Hawkes hyperparameters and the
temporal-trend coefficient, around the HMC update of the log-rates (Sec. 2.3).

The paper samples (mu0, tau_x, theta0, omega, h, beta) with univariate,
adaptive Metropolis-Hastings proposals, each evaluating the log-likelihood of
Eq. 1 through the massively parallel library, and the log-rates z by HMC.
Here one Gibbs iteration is: one HMC step on z (hmc_step), then `n_mh`
univariate MH updates, each of a parameter drawn uniformly at random.

* Positive parameters move on the log scale, x' = x exp(s u), u ~ N(0, 1),
  whose acceptance ratio carries the Jacobian x'/x; beta moves additively.
* Each parameter's scale s adapts towards acceptance 0.44 (the optimum for
  univariate random-walk proposals) by the diminishing rule of Roberts &
  Rosenthal (2009): after every batch of 50 proposals, log s moves by
  +-min(delta_max, n_batch^(-1/2)), with delta_max = 0.05 (their example uses
  0.01; a larger first step reaches a good scale in fewer batches).
* Priors follow the paper's families (Sec. 3.2): tau_x ~ InvGamma(1, 10);
  h and 1/omega ~ InvGamma(2, 0.5); theta0 ~ Gamma(1, scale 0.001); mu0 ~
  Gamma(2, scale 2); beta ~ N(0, 10^2).  tau_t is this library's extension
  (the paper's background has no time factor); it gets InvGamma(2, 5).  The
  paper's values are in its data's units (degrees, years); they are defaults
  to be replaced for other units.

Every likelihood evaluation runs on the device; the host holds only the
scalar chain state and draws the proposals and uniforms (numpy PCG64).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

HYPER_NAMES = ("mu0", "tau_x", "tau_t", "theta0", "omega", "h")


@dataclass
class Gamma:
    shape: float
    scale: float

    def logpdf(self, x):
        if x <= 0:
            return -math.inf
        return (self.shape - 1) * math.log(x) - x / self.scale - self.shape * math.log(self.scale) - math.lgamma(
            self.shape)


@dataclass
class InvGamma:
    shape: float
    scale: float

    def logpdf(self, x):
        if x <= 0:
            return -math.inf
        return self.shape * math.log(self.scale) - math.lgamma(self.shape) - (self.shape + 1) * math.log(x) - \
            self.scale / x


@dataclass
class InvGammaOfReciprocal:
    """Density of x when 1/x ~ InvGamma(shape, scale) (the paper's prior on omega)."""
    shape: float
    scale: float

    def logpdf(self, x):
        if x <= 0:
            return -math.inf
        return InvGamma(self.shape, self.scale).logpdf(1.0 / x) - 2.0 * math.log(x)


@dataclass
class Normal:
    mean: float
    sd: float

    def logpdf(self, x):
        return -0.5 * ((x - self.mean) / self.sd) ** 2 - math.log(self.sd) - 0.5 * math.log(2 * math.pi)


def paper_priors():
    return {"mu0": Gamma(2.0, 2.0), "tau_x": InvGamma(1.0, 10.0), "tau_t": InvGamma(2.0, 5.0),
            "theta0": Gamma(1.0, 0.001), "omega": InvGammaOfReciprocal(2.0, 0.5), "h": InvGamma(2.0, 0.5),
            "beta": Normal(0.0, 10.0)}


class AdaptiveMH:
    """Univariate random-walk MH with Roberts-Rosenthal scale adaptation, over
    named parameters with a caller-supplied log target (any callable)."""

    def __init__(self, names, positive, scales=None, seed=0, target_accept=0.44, batch=50, delta_max=0.05):
        self.names = list(names)
        self.positive = dict(positive)
        self.log_s = {n: math.log((scales or {}).get(n, 0.05)) for n in self.names}
        self.rng = np.random.default_rng(seed)
        self.target = target_accept
        self.batch = batch
        self.tried = {n: 0 for n in self.names}
        self.acc = {n: 0 for n in self.names}
        self.batch_acc = {n: 0 for n in self.names}
        self.nbatch = {n: 0 for n in self.names}
        self.adapt = True
        self.delta_max = delta_max

    def update(self, state: dict, logp_state: float, log_target, name=None):
        """One MH update of one parameter (uniformly chosen unless `name`).
        Returns (state, logp, accepted)."""
        n = self.names[self.rng.integers(len(self.names))] if name is None else name
        s = math.exp(self.log_s[n])
        u = self.rng.standard_normal()
        prop = dict(state)
        if self.positive[n]:
            prop[n] = state[n] * math.exp(s * u)
            log_jac = math.log(prop[n]) - math.log(state[n])
        else:
            prop[n] = state[n] + s * u
            log_jac = 0.0
        lp = log_target(prop)
        log_ratio = lp - logp_state + log_jac
        accepted = math.isfinite(lp) and math.log(self.rng.uniform()) < log_ratio
        self.tried[n] += 1
        if accepted:
            self.acc[n] += 1
            self.batch_acc[n] += 1
            state, logp_state = prop, lp
        if self.adapt and self.tried[n] % self.batch == 0:
            self.nbatch[n] += 1
            delta = min(self.delta_max, self.nbatch[n] ** -0.5)
            rate = self.batch_acc[n] / self.batch
            self.log_s[n] += delta if rate > self.target else -delta
            self.batch_acc[n] = 0
        return state, logp_state, accepted

    def acceptance(self):
        return {n: (self.acc[n] / self.tried[n] if self.tried[n] else None) for n in self.names}


class HawkesGibbs:
    """Random-scan Metropolis-within-Gibbs: HMC on z, univariate MH on the
    hyperparameters and beta.  `sampler` is an HmcSampler (its plan, subset and
    fixed rates); the likelihood of a proposal is the library's subset
    evaluation at the current z (O(N M) with the static part cached; a new
    hyperparameter setting refreshes the static part, one O(N^2) row pass)."""

    def __init__(self, sampler, priors=None, sample=("mu0", "tau_x", "tau_t", "theta0", "omega", "h", "beta"),
                 n_mh=4, seed=0):
        from . import _lib
        self._lib = _lib
        self.s = sampler
        self.priors = paper_priors() if priors is None else priors
        h = sampler.hyper
        self.state = {n: float(getattr(h, n)) for n in HYPER_NAMES}
        self.state["beta"] = float(sampler.beta)
        self.mh = AdaptiveMH(sample, {n: n != "beta" for n in sample}, seed=seed,
                             scales={n: (0.02 if n != "beta" else 1e-3) for n in sample})
        self.n_mh = n_mh
        self.logp = self.log_target(self.state)

    def loglik(self, state) -> float:
        hy = self._lib.Hyper(*[state[n] for n in HYPER_NAMES])
        if not self._lib_hyper_ok(hy):
            return -math.inf
        ll = torch.empty(1, dtype=torch.float64, device=self.s.dev)
        code = self._lib.lib().hawkes_subset_trend_grad(self.s.plan.handle, ctypes.byref(hy), self._lib.ptr(self.s.z),
                                                        float(state["beta"]), self._lib.ptr(self.s.theta),
                                                        self._lib.ptr(ll), None, None, self._lib.stream_handle())
        self._lib.check(code, "hawkes_subset_trend_grad")
        v = float(ll.item())
        return v if math.isfinite(v) else -math.inf

    @staticmethod
    def _lib_hyper_ok(hy):
        vals = (hy.mu0, hy.tau_x, hy.tau_t, hy.theta0, hy.omega, hy.h)
        return all(math.isfinite(v) for v in vals) and hy.tau_x > 0 and hy.tau_t > 0 and hy.omega > 0 and \
            hy.h > 0 and hy.mu0 >= 0 and hy.theta0 >= 0

    def log_prior(self, state) -> float:
        return sum(self.priors[n].logpdf(state[n]) for n in self.mh.names)

    def log_target(self, state) -> float:
        lp = self.log_prior(state)
        if not math.isfinite(lp):
            return -math.inf
        return lp + self.loglik(state)

    def _sync_sampler(self):
        self.s.hyper = self._lib.Hyper(*[self.state[n] for n in HYPER_NAMES])
        self.s.beta = self.state["beta"]

    def iteration(self, eps):
        """One Gibbs iteration: HMC on z at the current parameters, then n_mh
        univariate MH updates.  Returns the accept flags of the MH updates."""
        self._sync_sampler()
        self.s.step(eps)
        # z (and theta on the subset) changed: the current log target moves with it
        self.logp = self.log_target(self.state)
        flags = []
        for _ in range(self.n_mh):
            self.state, self.logp, a = self.mh.update(self.state, self.logp, self.log_target)
            flags.append(a)
        # leave theta on the subset at the current state's beta
        self.loglik(self.state)
        self._sync_sampler()
        return flags

