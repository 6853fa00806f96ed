"""Host logic of the Metropolis-within-Gibbs layer: prior densities against
scipy, and the adaptive univariate MH sampling a known target."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2103_03348_amd.mcmc import AdaptiveMH, Gamma, InvGamma, InvGammaOfReciprocal, Normal


def test_prior_densities_match_scipy():
    for x in (0.05, 0.3, 1.7, 12.0):
        assert Gamma(2.0, 2.0).logpdf(x) == pytest.approx(stats.gamma(a=2.0, scale=2.0).logpdf(x), rel=1e-12)
        assert InvGamma(1.0, 10.0).logpdf(x) == pytest.approx(stats.invgamma(a=1.0, scale=10.0).logpdf(x),
                                                               rel=1e-12)
        # omega with 1/omega ~ InvGamma(2, 0.5): change of variables
        ref = stats.invgamma(a=2.0, scale=0.5).logpdf(1.0 / x) - 2.0 * math.log(x)
        assert InvGammaOfReciprocal(2.0, 0.5).logpdf(x) == pytest.approx(ref, rel=1e-12)
        assert Normal(0.0, 10.0).logpdf(x) == pytest.approx(stats.norm(0.0, 10.0).logpdf(x), rel=1e-12)
    assert Gamma(1.0, 0.001).logpdf(-1.0) == -math.inf
    # the reciprocal density integrates to one
    from scipy import integrate
    val, _ = integrate.quad(lambda w: math.exp(InvGammaOfReciprocal(2.0, 0.5).logpdf(w)), 0, np.inf)
    assert val == pytest.approx(1.0, rel=1e-8)


def test_adaptive_mh_samples_known_target():
    """x ~ Gamma(3, scale 2) (log-scale moves with the Jacobian) and y ~ N(1, 0.5^2)."""
    gx, ny = stats.gamma(a=3.0, scale=2.0), stats.norm(1.0, 0.5)

    def logp(s):
        return gx.logpdf(s["x"]) + ny.logpdf(s["y"]) if s["x"] > 0 else -math.inf

    mh = AdaptiveMH(["x", "y"], {"x": True, "y": False}, scales={"x": 2.0, "y": 0.01}, seed=5)
    state = {"x": 1.0, "y": 0.0}
    lp = logp(state)
    xs, ys = [], []
    for it in range(60000):
        state, lp, _ = mh.update(state, lp, logp)
        if it >= 10000:
            xs.append(state["x"])
            ys.append(state["y"])
    xs, ys = np.array(xs), np.array(ys)
    acc = {n: (mh.acc[n] / mh.tried[n]) for n in ("x", "y")}
    assert np.mean(xs) == pytest.approx(6.0, rel=0.05)
    assert np.var(xs) == pytest.approx(12.0, rel=0.15)
    assert np.mean(ys) == pytest.approx(1.0, abs=0.03)
    assert np.std(ys) == pytest.approx(0.5, rel=0.05)
    assert 0.3 < acc["x"] < 0.6 and 0.3 < acc["y"] < 0.6
