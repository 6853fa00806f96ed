"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage it follows and the mistake it would catch:
  * golden N=2 case (independent 40-digit evaluation)  -> sign, index, normaliser
  * intensity at events vs scipy's normal densities     -> c_b, c_e, indicators
  * integral term vs numerical quadrature (App. A)      -> dropped/extra Lambda terms
  * background-only closed form (theta0 = 0)            -> mu0 derivative, C
  * Euler homogeneity and row/column consistency        -> hyper/rate gradients
  * central finite differences of loglik and gradient   -> every derivative formula
  * permutation / translation / rotation / rescaling    -> index and scaling mistakes
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

import oracle
from paper_2103_03348_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HY = (0.7, 2.0, 5.0, 0.3, 0.5, 0.3)


def _es(n, seed, ties=0, dup_xy=0, t_end=None):
    return synth.small(n, seed=seed, ties=ties, dup_xy=dup_xy, t_end=t_end)


def test_n2_golden_case():
    """Sec. 2.1 / Eq. 1, 3, 4 on the two-event case (tests/golden/n2_case.json)."""
    g = json.load(open(os.path.join(GOLDEN, "n2_case.json")))
    r = oracle.evaluate(g["t"], g["x"], g["y"], g["theta"], g["hyper"], g["t0"])
    np.testing.assert_allclose(r["lam"], g["lam"], rtol=1e-14)
    assert r["Lam_n"].sum() == pytest.approx(g["Lambda"], rel=1e-14)
    assert r["loglik"] == pytest.approx(g["loglik"], rel=1e-14)
    np.testing.assert_allclose(r["grad_theta"], g["grad_theta"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(r["negH_theta"], g["negH_theta"], rtol=1e-13, atol=1e-15)


def test_single_event_has_zero_intensity():
    """Sec. 2.1: the background excludes the event itself, and nothing precedes
    a lone event, so lambda_1 = 0 and the log-likelihood is -inf."""
    r = oracle.evaluate([2.0], [0.1], [0.2], [1.0], HY, 0.0)
    assert r["lam"][0] == 0.0
    assert r["loglik"] == -math.inf


def _intensity_at(px, py, pt, es, theta, hyper, exclude=None):
    """lambda(x, t) of Sec. 2.1 built from scipy's normal densities: background
    mu0 * N2(x; x_n, tau_x^2) * N1(t; t_n, tau_t^2) over all n (except `exclude`),
    excitation theta0 * theta_n * omega * exp(-omega (t - t_n)) * N2(x; x_n, h^2)
    over t_n < t."""
    mu0, tau_x, tau_t, theta0, omega, h = hyper
    tot = 0.0
    for n in range(es.n):
        if n == exclude:
            continue
        tot += mu0 * norm.pdf(px, es.x[n], tau_x) * norm.pdf(py, es.y[n], tau_x) * norm.pdf(pt, es.t[n], tau_t)
        if es.t[n] < pt:
            tot += (theta0 * theta[n] * omega * math.exp(-omega * (pt - es.t[n]))
                    * norm.pdf(px, es.x[n], h) * norm.pdf(py, es.y[n], h))
    return tot


def test_intensity_matches_density_construction():
    """lambda_i of the oracle equals the Sec. 2.1 intensity, assembled from
    library normal densities, at each event with the event itself excluded."""
    es = _es(9, seed=3, t_end=4.0)
    r = oracle.evaluate_es(es)
    for i in range(es.n):
        ref = _intensity_at(es.x[i], es.y[i], es.t[i], es, es.theta, es.hyper, exclude=i)
        assert r["lam"][i] == pytest.approx(ref, rel=1e-12)


def test_integral_term_by_quadrature():
    """App. A (Claim 1) for the excitation part and the exact background
    integral: Lambda equals the time quadrature of the spatially integrated
    intensity.  Over R^2 each normal density integrates to one, so the spatial
    integral of lambda(., t) is
      sum_n mu0 N1(t; t_n, tau_t^2) + sum_{t_n < t} theta0 theta_n omega e^{-omega (t - t_n)}."""
    es = _es(6, seed=11, t_end=5.0)
    t0 = -0.5
    r = oracle.evaluate(es.t, es.x, es.y, es.theta, es.hyper, t0)
    mu0, tau_x, tau_t, theta0, omega, h = es.hyper
    T1 = es.t.max()

    def spatial_total(tt):
        s = 0.0
        for n in range(es.n):
            s += mu0 * norm.pdf(tt, es.t[n], tau_t)
            if es.t[n] < tt:
                s += theta0 * es.theta[n] * omega * math.exp(-omega * (tt - es.t[n]))
        return s

    pts = sorted(set(float(v) for v in es.t))
    val, err = integrate.quad(spatial_total, t0, T1, points=pts, limit=400, epsabs=1e-13, epsrel=1e-13)
    assert r["Lam_n"].sum() == pytest.approx(val, rel=1e-10)


def test_spatial_density_integrates_to_one():
    """The 2-D normaliser used for both kernels: (2 pi s^2)^-1 exp(-r^2/(2 s^2))
    integrates to one over R^2 (checked numerically on a fine grid for the
    background and excitation lengthscales)."""
    for s in (HY[1], HY[5]):
        g = np.linspace(-12 * s, 12 * s, 2401)
        dx = g[1] - g[0]
        X, Y = np.meshgrid(g, g)
        val = (np.exp(-(X ** 2 + Y ** 2) / (2 * s * s)) / (2 * np.pi * s * s)).sum() * dx * dx
        assert val == pytest.approx(1.0, rel=1e-9)


def test_background_only_closed_form():
    """theta0 = 0: lambda_i = c_b B0_i, so loglik(mu0) = N log mu0 + const - mu0 C,
    d loglik/d mu0 = N/mu0 - C with C = sum_n [Phi(u1_n) - Phi(u0_n)], and the rate
    gradient and Hessian vanish identically (Eq. 3, 4 carry a factor theta0)."""
    es = _es(40, seed=5)
    hy = (0.7, 2.0, 5.0, 0.0, 0.5, 0.3)
    r = oracle.evaluate_es(es, hyper=hy)
    T1 = es.t.max()
    C = float(np.sum(norm.cdf((T1 - es.t) / hy[2]) - norm.cdf((0.0 - es.t) / hy[2])))
    assert r["grad_hyper"][0] == pytest.approx(es.n / hy[0] - C, rel=1e-12)
    assert np.all(r["grad_theta"] == 0.0)
    assert np.all(r["negH_theta"] == 0.0)
    hy2 = (1.9, 2.0, 5.0, 0.0, 0.5, 0.3)
    r2 = oracle.evaluate_es(es, hyper=hy2)
    expect = es.n * math.log(hy2[0] / hy[0]) - (hy2[0] - hy[0]) * C
    assert r2["loglik"] - r["loglik"] == pytest.approx(expect, rel=1e-11)
    # the MLE of mu0 is N / C
    assert (es.n / C) > 0
    assert r["negH_hyper"][0] == pytest.approx(es.n / hy[0] ** 2, rel=1e-12)


def test_euler_homogeneity():
    """lambda_i is homogeneous of degree one in (mu0, theta0) and so is Lambda, hence
    mu0 dl/dmu0 + theta0 dl/dtheta0 = N - Lambda."""
    es = _es(60, seed=8, ties=3)
    r = oracle.evaluate_es(es)
    g = r["grad_hyper"]
    lhs = es.hyper[0] * g[0] + es.hyper[3] * g[3]
    assert lhs == pytest.approx(es.n - r["Lam_n"].sum(), rel=1e-11)


def test_row_column_consistency():
    """theta0 dl/dtheta0 (row sums) equals sum_m theta_m dl/dtheta_m (column sums of Eq. 3):
    both are sum_i c_e X0_i / lambda_i - theta0 sum_n theta_n (1 - e^{-omega (T1 - t_n)})."""
    es = _es(80, seed=9, ties=4)
    r = oracle.evaluate_es(es)
    lhs = es.hyper[3] * r["grad_hyper"][3]
    rhs = float(np.dot(es.theta, r["grad_theta"]))
    assert lhs == pytest.approx(rhs, rel=1e-11)


def _fd_loglik(fn, p0, step):
    """Central difference of sum_n ell_n, summing per-event differences."""
    lp = fn(p0 + step)
    lm = fn(p0 - step)
    return float(np.sum(lp - lm)) / (2 * step)


@pytest.mark.parametrize("seed", [21, 22])
def test_fd_rate_gradient_and_hessian(seed):
    """Eq. 3 and Eq. 4 against central finite differences of Eq. 1 (step 1e-6 for
    the gradient, 1e-4 on the gradient for the Hessian)."""
    es = _es(50, seed=seed, ties=2)
    r = oracle.evaluate_es(es)
    rng = np.random.default_rng(seed)
    for j in rng.choice(es.n, size=8, replace=False):
        def ell_n(v, j=j):
            th = es.theta.copy()
            th[j] = v
            return oracle.evaluate_es(es, theta=th, want=("ell_n",))["ell_n"]

        def grad_j(v, j=j):
            th = es.theta.copy()
            th[j] = v
            return oracle.evaluate_es(es, theta=th, want=("grad_theta",))["grad_theta"][j]

        fd = _fd_loglik(ell_n, es.theta[j], 1e-6)
        scale = abs(r["grad_theta"][j]) + es.hyper[3]
        assert r["grad_theta"][j] == pytest.approx(fd, abs=1e-7 * scale + 1e-9)
        fdh = -(grad_j(es.theta[j] + 1e-4) - grad_j(es.theta[j] - 1e-4)) / 2e-4
        assert r["negH_theta"][j] == pytest.approx(fdh, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("p", range(6))
def test_fd_hyper_gradient_and_hessian(p):
    """The hyperparameter derivatives (differentiated from the Sec. 2.1
    definitions) against central finite differences of Eq. 1."""
    es = _es(40, seed=31, ties=2)
    hy0 = np.array(es.hyper, dtype=np.float64)
    r = oracle.evaluate_es(es)

    def ell_n(v):
        hy = hy0.copy()
        hy[p] = v
        return oracle.evaluate_es(es, hyper=hy, want=("ell_n",))["ell_n"]

    def grad_p(v):
        hy = hy0.copy()
        hy[p] = v
        return oracle.evaluate_es(es, hyper=hy, want=("grad_hyper",))["grad_hyper"][p]

    step = 1e-6 * hy0[p]
    fd = _fd_loglik(ell_n, hy0[p], step)
    assert r["grad_hyper"][p] == pytest.approx(fd, rel=1e-6, abs=1e-6)
    hs = 1e-4 * hy0[p]
    fdh = -(grad_p(hy0[p] + hs) - grad_p(hy0[p] - hs)) / (2 * hs)
    assert r["negH_hyper"][p] == pytest.approx(fdh, rel=1e-5, abs=1e-5)


def test_permutation_invariance_with_ties():
    """Eq. 1 sums over events: reordering the input leaves loglik unchanged and
    permutes the gradient and Hessian."""
    es = _es(70, seed=41, ties=6, dup_xy=3)
    r = oracle.evaluate_es(es)
    perm = np.random.default_rng(1).permutation(es.n)
    r2 = oracle.evaluate(es.t[perm], es.x[perm], es.y[perm], es.theta[perm], es.hyper, es.t0)
    assert r2["loglik"] == pytest.approx(r["loglik"], rel=1e-13)
    np.testing.assert_allclose(r2["grad_theta"], r["grad_theta"][perm], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(r2["negH_theta"], r["negH_theta"][perm], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(r2["grad_hyper"], r["grad_hyper"], rtol=1e-11)


def test_translation_and_rotation_invariance():
    """The kernels depend on |x_i - x_j| and t_i - t_j only; the window moves with time."""
    es = _es(50, seed=42)
    r = oracle.evaluate_es(es)
    rs = oracle.evaluate(es.t, es.x + 3.25, es.y - 1.5, es.theta, es.hyper, es.t0)
    rr = oracle.evaluate(es.t, -es.y, es.x, es.theta, es.hyper, es.t0)
    rt = oracle.evaluate(es.t + 17.0, es.x, es.y, es.theta, es.hyper, es.t0 + 17.0)
    for o in (rs, rr, rt):
        assert o["loglik"] == pytest.approx(r["loglik"], rel=1e-12)
        np.testing.assert_allclose(o["grad_theta"], r["grad_theta"], rtol=1e-9, atol=1e-13)


def test_exact_rescaling():
    """x, tau_x, h doubled: both normalisers carry s^-2 in 2-D, so every lambda_i
    halves twice and loglik drops by 2 N ln 2 (Lambda unchanged).  t, T0, tau_t doubled
    and omega halved: lambda_i halves, loglik drops by N ln 2."""
    es = _es(45, seed=43)
    mu0, tau_x, tau_t, theta0, omega, h = es.hyper
    r = oracle.evaluate_es(es)
    r_s = oracle.evaluate(es.t, 2 * es.x, 2 * es.y, es.theta, (mu0, 2 * tau_x, tau_t, theta0, omega, 2 * h), es.t0)
    r_t = oracle.evaluate(2 * es.t, es.x, es.y, es.theta, (mu0, tau_x, 2 * tau_t, theta0, omega / 2, h), 2 * es.t0)
    assert r_s["loglik"] == pytest.approx(r["loglik"] - 2 * es.n * math.log(2), rel=1e-12)
    assert r_t["loglik"] == pytest.approx(r["loglik"] - es.n * math.log(2), rel=1e-12)


def test_tied_times_do_not_excite():
    """Strict causality of the excitation indicator (Sec. 2.1): two events at the
    same time contribute background to each other but no excitation."""
    t = [1.0, 1.0, 2.0]
    x = [0.0, 0.1, 0.2]
    y = [0.0, 0.0, 0.1]
    th = [2.0, 3.0, 1.0]
    r = oracle.evaluate(t, x, y, th, HY, 0.0)
    acc = oracle.row_sums(t, x, y, th, HY)
    assert acc[0, 5] == 0.0 and acc[1, 5] == 0.0
    assert acc[2, 5] > 0.0
    assert acc[0, 0] > 0.0 and acc[1, 0] > 0.0
    assert r["negH_theta"][2] == 0.0
