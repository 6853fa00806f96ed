"""Seeded synthetic event sets shaped like the paper's workloads.

This module draws inputs only.  It evaluates nothing of the likelihood, its
derivatives or the sampler, so both the FP64 oracle and the GPU library can be
fed from it without sharing any of the method's arithmetic.

Workloads (all 2-D, hyperparameters (mu0, tau_x, tau_t, theta0, omega, h) =
(0.7, 2, 5, 0.3, 0.5, 0.3)):

* ``uniform_mixture``: times sorted U[0, T], locations from a K-component
  equal-weight Gaussian mixture (sigma = 1, centres U[-10, 10]^2).
* ``branching``: a Hawkes cluster process simulated forward in time
  (Sec. 2.1's model with theta = 1): immigrants arrive as a Poisson process with
  locations from the mixture; each event has Poisson(theta0) children, delayed by
  Exp(omega) and displaced by N(0, h^2 I).  The process is simulated on a
  generous window and the earliest N events are kept, so exactly N come out.

The paper's own benchmark uses 25,000 random points (Sec. 3.1) and its
application 23,422 geolocated cases of which 1,610 are sequenced (Sec. 3.2);
these generators stand in for both.
"""
from __future__ import annotations

import dataclasses

import numpy as np

HYPER_DEFAULT = (0.7, 2.0, 5.0, 0.3, 0.5, 0.3)


@dataclasses.dataclass
class EventSet:
    t: np.ndarray          # [N] float64, caller order (not necessarily sorted)
    x: np.ndarray          # [N] float64
    y: np.ndarray          # [N] float64
    theta: np.ndarray      # [N] float64, per-event rates
    subset: np.ndarray     # [M] int64, indices whose rates are free (exp(z))
    z: np.ndarray          # [M] float64, log-rates on the subset
    hyper: tuple           # (mu0, tau_x, tau_t, theta0, omega, h)
    t0: float = 0.0        # window start
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    @property
    def xy(self) -> np.ndarray:
        return np.stack([self.x, self.y], axis=1)


def _mixture_centres(rng, k):
    return rng.uniform(-10.0, 10.0, size=(k, 2))


def _draw_mixture(rng, centres, n, sigma=1.0):
    comp = rng.integers(0, centres.shape[0], size=n)
    return centres[comp] + sigma * rng.standard_normal((n, 2))


def uniform_mixture(n, t_end=100.0, k=5, seed=1000, z_sd=0.5, hyper=HYPER_DEFAULT,
                    all_free=True, name="uniform_mixture"):
    """Times sorted U[0, t_end]; locations from a k-component mixture; every
    event's rate free, theta = exp(z), z ~ N(0, z_sd^2)."""
    rng = np.random.default_rng(seed)
    centres = _mixture_centres(rng, k)
    t = np.sort(rng.uniform(0.0, t_end, size=n))
    xy = _draw_mixture(rng, centres, n)
    if all_free:
        subset = np.arange(n, dtype=np.int64)
    else:
        subset = np.sort(rng.choice(n, size=max(1, n // 15), replace=False)).astype(np.int64)
    z = z_sd * rng.standard_normal(subset.shape[0])
    theta = np.ones(n)
    theta[subset] = np.exp(z)
    return EventSet(t, xy[:, 0].copy(), xy[:, 1].copy(), theta, subset, z, tuple(hyper), 0.0, name)


def branching(n, immigrant_rate, k=5, seed=1001, m_free=None, z_sd=0.5,
              theta0=0.3, omega=0.5, h=0.3, hyper=HYPER_DEFAULT, name="branching"):
    """Cluster-process simulation, earliest n events kept.

    ``m_free`` events (a uniformly random subset) get theta = exp(z),
    z ~ N(0, z_sd^2); all others keep theta = 1.
    """
    rng = np.random.default_rng(seed)
    centres = _mixture_centres(rng, k)
    # expected total rate = immigrant_rate / (1 - theta0); simulate on a window
    # long enough that at least n events fall inside it with margin
    horizon = 1.3 * n * (1.0 - theta0) / immigrant_rate + 10.0 / omega
    while True:
        n_imm = rng.poisson(immigrant_rate * horizon)
        t_gen = rng.uniform(0.0, horizon, size=n_imm)
        xy_gen = _draw_mixture(rng, centres, n_imm)
        ts, xys = [t_gen], [xy_gen]
        while t_gen.shape[0] > 0:
            kids = rng.poisson(theta0, size=t_gen.shape[0])
            parent = np.repeat(np.arange(t_gen.shape[0]), kids)
            if parent.shape[0] == 0:
                break
            t_new = t_gen[parent] + rng.exponential(1.0 / omega, size=parent.shape[0])
            xy_new = xy_gen[parent] + h * rng.standard_normal((parent.shape[0], 2))
            keep = t_new < horizon
            t_gen, xy_gen = t_new[keep], xy_new[keep]
            ts.append(t_gen)
            xys.append(xy_gen)
        t_all = np.concatenate(ts)
        xy_all = np.concatenate(xys)
        if t_all.shape[0] >= n:
            break
        horizon *= 1.5
    order = np.argsort(t_all, kind="stable")[:n]
    t = t_all[order]
    xy = xy_all[order]
    # present the events in a shuffled caller order: the library sorts internally
    shuffle = rng.permutation(n)
    t, xy = t[shuffle], xy[shuffle]
    m = n if m_free is None else int(m_free)
    subset = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)
    z = z_sd * rng.standard_normal(m)
    theta = np.ones(n)
    theta[subset] = np.exp(z)
    return EventSet(t, xy[:, 0].copy(), xy[:, 1].copy(), theta, subset, z, tuple(hyper), 0.0, name)


# The five workloads.  Index 0 is the small case the oracle finishes in
# seconds; index 1 is the paper-sized one (N = 23,422, M = 1,610).
def config(k: int) -> EventSet:
    if k == 0:
        return uniform_mixture(1000, t_end=100.0, k=5, seed=1000, name="N1000_uniform_mix5")
    if k == 1:
        return branching(23422, immigrant_rate=1e-3 * 23422, k=5, seed=1001, m_free=1610,
                         name="N23422_branching_M1610")
    if k == 2:
        return branching(100000, immigrant_rate=70.0, k=5, seed=1002, m_free=6874,
                         name="N100000_branching_M6874")
    if k == 3:
        return branching(23422, immigrant_rate=1e-3 * 23422, k=5, seed=1001, m_free=1610,
                         name="N23422_branching_M1610_hmc")
    if k == 4:
        return branching(250000, immigrant_rate=70.0, k=20, seed=1004, m_free=17185,
                         name="N250000_branching_mix20_M17185")
    raise ValueError(f"no workload {k}")


def coalescent_tree(m, seed=0, scale=1.0):
    """A random bifurcating tree over m tips by Kingman's coalescent: with k
    lineages left, the next merger comes after Exp(k (k - 1) / 2) time (times
    `scale`) and joins two lineages drawn uniformly.  Returns (parent [2m - 1],
    length [2m - 1]) with the tips first and the root last (parent -1)."""
    rng = np.random.default_rng(seed)
    n = 2 * m - 1
    parent = np.full(n, -1, dtype=np.int64)
    length = np.zeros(n)
    height = np.zeros(n)
    live = list(range(m))
    t = 0.0
    nxt = m
    while len(live) > 1:
        k = len(live)
        t += scale * rng.exponential(2.0 / (k * (k - 1)))
        i, j = rng.choice(k, size=2, replace=False)
        a, b = live[i], live[j]
        for c in (a, b):
            parent[c] = nxt
            length[c] = t - height[c]
        height[nxt] = t
        live = [v for q, v in enumerate(live) if q not in (i, j)] + [nxt]
        nxt += 1
    return parent, length


def small(n, seed=7, t_end=None, k=3, all_free=True, ties=0, dup_xy=0):
    """Small ragged test sets.  ``ties`` events copy another event's time and
    ``dup_xy`` copy another event's location (edge cases of the indicators)."""
    rng = np.random.default_rng(seed)
    if t_end is None:
        t_end = max(1.0, n / 10.0)
    es = uniform_mixture(n, t_end=t_end, k=k, seed=seed, all_free=all_free, name=f"small{n}")
    if ties and n > 1:
        src = rng.integers(0, n, size=ties)
        dst = rng.integers(0, n, size=ties)
        es.t[dst] = es.t[src]
    if dup_xy and n > 1:
        src = rng.integers(0, n, size=dup_xy)
        dst = rng.integers(0, n, size=dup_xy)
        es.x[dst] = es.x[src]
        es.y[dst] = es.y[src]
    perm = rng.permutation(n)
    theta_full = es.theta[perm]
    # remap the free subset through the shuffle
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    subset = np.sort(inv[es.subset])
    z = np.log(theta_full[subset])
    return EventSet(es.t[perm], es.x[perm], es.y[perm], theta_full, subset, z, es.hyper, 0.0, es.name)
