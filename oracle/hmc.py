"""One Hamiltonian Monte Carlo iteration on the log-rates z of the free events,
in FP64 on the CPU (Sec. 2.3.2).  Test infrastructure only.

Target: log pi(z) = loglik(theta(z)) - sum_k z_k^2 / (2 sigma_z^2), with
theta_{idx_k} = exp(z_k + beta t_{idx_k}) and every other rate held fixed
(Sec. 2.2 with f(t) = t; the phylogenetic prior of Eq. 2 with V = I, or a dense
V when one is given).  Energy H(z, p) = -log pi(z) + p^T M^{-1} p / 2 with a
diagonal mass M.  The leapfrog integrator uses dz/dt = M^{-1} p (the paper
prints a factor 1/2 there, read here as a typo).  Momenta and the Metropolis
uniform come from Philox-4x32-10 (oracle.philox) so that a GPU run with the
same seed and counter can be replayed exactly.
"""
from __future__ import annotations

import numpy as np

from . import evaluate, philox


def rates(es_t, theta_full, idx, z, beta=0.0):
    """theta with the subset entries exp(z_k + beta t_k) (Sec. 2.2, f(t) = t)."""
    th = np.array(theta_full, dtype=np.float64, copy=True)
    th[idx] = np.exp(np.asarray(z) + beta * np.asarray(es_t)[idx])
    return th


def trend_grad(es_t, es_x, es_y, theta_full, idx, z, beta, hyper, t0):
    """loglik and its gradients in z and beta by the chain rule through
    theta_k = exp(z_k + beta t_k):  d/dz_k = theta_k g_k,
    d/dbeta = sum_k t_k theta_k g_k, with g = Eq. 4 on the subset."""
    th = rates(es_t, theta_full, idx, z, beta)
    r = evaluate(es_t, es_x, es_y, th, hyper, t0, want=("loglik", "grad_theta"))
    gz = th[idx] * r["grad_theta"][idx]
    return r["loglik"], gz, float(np.sum(np.asarray(es_t)[idx] * gz))


def log_post(es_t, es_x, es_y, theta_full, idx, z, hyper, t0, sigma_z, beta=0.0, prior_v=None):
    """prior_v: None for z ~ N(0, sigma_z^2 I), else the dense covariance V of
    the phylogenetic prior (Eq. 2), z ~ N(0, sigma_z^2 V).  Constants of the
    prior are dropped (they cancel in the energy difference)."""
    th = rates(es_t, theta_full, idx, z, beta)
    r = evaluate(es_t, es_x, es_y, th, hyper, t0, want=("loglik", "grad_theta"))
    ll = r["loglik"]
    g = r["grad_theta"][idx]
    vz = z if prior_v is None else np.linalg.solve(prior_v, z)
    lp = ll - float(z @ vz) / (2.0 * sigma_z ** 2)
    grad_z = th[idx] * g - vz / sigma_z ** 2
    return lp, grad_z, ll, r


def leapfrog(es_t, es_x, es_y, theta_full, idx, z, p, mass, hyper, t0, eps, L, sigma_z, beta=0.0, prior_v=None,
             grad0=None):
    """L leapfrog steps of size eps from (z, p): a half kick, then L drifts with
    full kicks between them and a closing half kick.  grad0, when given, is the
    log-posterior gradient at the starting z.  Returns (z, p, log pi(z),
    loglik(z)) at the end of the path."""
    z = np.array(z, dtype=np.float64, copy=True)
    mass = np.asarray(mass, dtype=np.float64)
    g = grad0
    if g is None:
        _, g, _, _ = log_post(es_t, es_x, es_y, theta_full, idx, z, hyper, t0, sigma_z, beta, prior_v)
    p = np.asarray(p, dtype=np.float64) + 0.5 * eps * g
    lp = ll = None
    for step in range(L):
        z = z + eps * p / mass
        lp, g, ll, _ = log_post(es_t, es_x, es_y, theta_full, idx, z, hyper, t0, sigma_z, beta, prior_v)
        p = p + (eps if step < L - 1 else 0.5 * eps) * g
    return z, p, lp, ll


def hmc_iteration(es_t, es_x, es_y, theta_full, idx, z0, mass, hyper, t0, eps, L, sigma_z, seed, counter,
                  beta=0.0, prior_v=None):
    """Returns dict(z, accepted, dH, loglik, logpost, z_proposal, H0, H1, u, p0,
    loglik_proposal)."""
    z0 = np.asarray(z0, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    p0 = np.sqrt(mass) * philox.normals(seed, counter, z0.shape[0])
    lp0, g0, ll0, _ = log_post(es_t, es_x, es_y, theta_full, idx, z0, hyper, t0, sigma_z, beta, prior_v)
    z, p, lp, ll = leapfrog(es_t, es_x, es_y, theta_full, idx, z0, p0, mass, hyper, t0, eps, L, sigma_z, beta,
                            prior_v, grad0=g0)
    H0 = -lp0 + 0.5 * float(np.sum(p0 * p0 / mass))
    H1 = -lp + 0.5 * float(np.sum(p * p / mass))
    dH = H1 - H0
    u = philox.accept_uniform(seed, counter)
    accepted = bool(np.isfinite(dH) and np.log(u) < -dH)
    return {"z": z if accepted else z0, "z_proposal": z, "accepted": accepted, "dH": dH, "H0": H0, "H1": H1,
            "loglik": ll if accepted else ll0, "logpost": lp if accepted else lp0, "u": u, "p0": p0,
            "loglik_proposal": ll}


def prior_precision_diag(m, sigma_z, prior_v=None):
    """Diagonal of the prior's precision, -d2 log p(z) / dz_k^2: 1/sigma_z^2 for
    z ~ N(0, sigma_z^2 I), (V^{-1})_kk / sigma_z^2 for the dense V of Eq. 2."""
    if prior_v is None:
        return np.full(m, 1.0 / sigma_z ** 2)
    return np.diag(np.linalg.inv(prior_v)) / sigma_z ** 2


def z_hessian_diag(es_t, es_x, es_y, theta_full, idx, z, hyper, t0, sigma_z, beta=0.0, prior_v=None):
    """-d2 log pi / dz_k^2 = theta_k^2 H_k - theta_k g_k + (prior precision)_kk,
    theta_k = exp(z_k + beta t_k) (chain rule through d theta_k / d z_k = theta_k
    with Eq. 4 and Eq. 5)."""
    th = rates(es_t, theta_full, idx, z, beta)
    r = evaluate(es_t, es_x, es_y, th, hyper, t0, want=("grad_theta", "negH_theta"))
    tk = th[idx]
    return (tk * tk * r["negH_theta"][idx] - tk * r["grad_theta"][idx]
            + prior_precision_diag(len(idx), sigma_z, prior_v))
