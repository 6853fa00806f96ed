"""Effective sample size of MCMC output: Geyer's initial monotone sequence
estimator (Geyer 1992, "Practical Markov chain Monte Carlo"), the diagnostic
the paper reports for its 1,377 parameters (Sec. 3.2).  A host-side diagnostic
of sampler output, not part of the likelihood path."""
from __future__ import annotations

import numpy as np


def autocov(x: np.ndarray) -> np.ndarray:
    """Autocovariances of a 1-D chain at lags 0..n-1 (biased, divisor n), by FFT."""
    n = x.shape[0]
    xc = x - x.mean()
    nfft = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(xc, nfft)
    ac = np.fft.irfft(f * np.conj(f), nfft)[:n]
    return ac / n


def ess_1d(x: np.ndarray) -> float:
    """ESS = n / (1 + 2 sum_k rho_k), with the sum truncated by Geyer's initial
    positive sequence of pair sums Gamma_m = rho_2m + rho_2m+1 made monotone."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if n < 4:
        return float(n)
    ac = autocov(x)
    if ac[0] <= 0:
        return float(n)
    rho = ac / ac[0]
    npairs = (n - 1) // 2
    gam = rho[0:2 * npairs:2] + rho[1:2 * npairs:2]
    # initial positive sequence
    m = 0
    while m < gam.shape[0] and gam[m] > 0:
        m += 1
    gam = gam[:m]
    # initial monotone sequence
    for k in range(1, gam.shape[0]):
        if gam[k] > gam[k - 1]:
            gam[k] = gam[k - 1]
    tau = -1.0 + 2.0 * float(np.sum(gam))
    tau = max(tau, 1.0 / np.log10(max(n, 10)))  # guard against antithetic blow-up
    return float(n / tau)


def ess(draws: np.ndarray) -> np.ndarray:
    """Per-coordinate ESS of draws [n_iter, dim]."""
    draws = np.asarray(draws, dtype=np.float64)
    return np.array([ess_1d(draws[:, j]) for j in range(draws.shape[1])])
