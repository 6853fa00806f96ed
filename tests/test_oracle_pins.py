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
    """Sec. 2.1 / Eq. 1, 4, 5 on the two-event case (tests/golden/n2_case.json)."""
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
    gradient and Hessian vanish identically (Eq. 4, 5 carry a factor theta0)."""
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
    """theta0 dl/dtheta0 (row sums) equals sum_m theta_m dl/dtheta_m (column sums of Eq. 4):
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
    """Eq. 4 and Eq. 5 against central finite differences of Eq. 1 (step 1e-6 for
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


def test_philox_known_answers():
    """Philox-4x32-10 against the published known-answer vectors (Salmon et al. 2011)."""
    from oracle import philox
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))

    def v(x):
        return int(x, 16) if isinstance(x, str) else int(x)

    for vec in kat["vectors"]:
        out = philox.philox4x32_10(np.array([v(c) for c in vec["ctr"]]), np.array([v(k) for k in vec["key"]]))
        assert [int(o) for o in out] == [v(o) for o in vec["out"]]


def test_philox_normals_are_standard():
    """Box-Muller on Philox uniforms: mean 0, variance 1, normal quantiles (KS test)."""
    from scipy import stats

    from oracle import philox
    z = philox.normals(seed=12345, counter=7, m=200000)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_hmc_samples_prior_when_no_excitation():
    """theta0 = 0: the likelihood does not depend on the rates, so the HMC chain
    targets the N(0, sigma_z^2) prior exactly; check its first two moments over
    a short chain of the oracle sampler (Sec. 2.3.2 special case)."""
    from oracle import hmc
    es = _es(30, seed=51)
    hy = (0.7, 2.0, 5.0, 0.0, 0.5, 0.3)
    idx = np.arange(10)
    z = np.zeros(10)
    sig = 0.5
    mass = np.full(10, 1.0 / sig ** 2)
    draws = []
    acc = 0
    for it in range(400):
        r = hmc.hmc_iteration(es.t, es.x, es.y, es.theta, idx, z, mass, hy, 0.0, 0.9, 3, sig, seed=3, counter=it)
        z = r["z"]
        acc += r["accepted"]
        draws.append(z.copy())
    d = np.array(draws[50:])
    assert acc > 300
    assert abs(d.mean()) < 0.06
    assert abs(d.var() - sig ** 2) < 0.04


def test_hmc_leapfrog_reversible():
    """Leapfrog is time-reversible: L steps forward, the momentum negated, L steps
    back return to the starting point (z0, -p0) up to FP64 rounding (Sec. 2.3.2;
    Neal 2011, Sec. 2.3).  Catches a kick or drift taken with the wrong step, a
    missing half kick or a gradient evaluated at the wrong point -- each breaks
    the symmetry of the integrator.  Checked with the iid prior, with the temporal
    trend and with a dense Eq. 2 covariance."""
    from oracle import hmc, tree as otree
    es = _es(25, seed=52)
    idx = np.arange(0, 25, 3)
    m = idx.shape[0]
    z0 = np.log(es.theta[idx]) + 0.1
    mass = np.linspace(3.0, 9.0, m)
    p0 = np.random.default_rng(52).standard_normal(m) * np.sqrt(mass)
    par, ln = synth.coalescent_tree(m, seed=5, scale=float(m))
    for beta, V in ((0.0, None), (-0.02, None), (0.0, otree.covariance(par, ln, 0.7))):
        z1, p1, _, _ = hmc.leapfrog(es.t, es.x, es.y, es.theta, idx, z0, p0, mass, es.hyper, 0.0, 0.05, 12, 0.5,
                                    beta, V)
        assert np.max(np.abs(z1 - z0)) > 1e-3          # the path went somewhere
        z2, p2, _, _ = hmc.leapfrog(es.t, es.x, es.y, es.theta, idx, z1, -p1, mass, es.hyper, 0.0, 0.05, 12, 0.5,
                                    beta, V)
        np.testing.assert_allclose(z2, z0, rtol=0, atol=1e-10)
        np.testing.assert_allclose(-p2, p0, rtol=0, atol=1e-10)


def test_hmc_leapfrog_second_order():
    """The leapfrog's energy error over a fixed trajectory length shrinks as eps^2."""
    from oracle import hmc
    es = _es(25, seed=52)
    idx = np.arange(0, 25, 3)
    z0 = np.log(es.theta[idx])
    mass = np.full(idx.shape[0], 4.0)
    errs = []
    for eps, L in ((0.04, 5), (0.02, 10), (0.01, 20)):
        r = hmc.hmc_iteration(es.t, es.x, es.y, es.theta, idx, z0, mass, es.hyper, 0.0, eps, L, 0.5, 9, 0)
        errs.append(abs(r["dH"]))
    assert errs[1] == pytest.approx(errs[0] / 4.0, rel=0.1)
    assert errs[2] == pytest.approx(errs[1] / 4.0, rel=0.1)


def _z_grad(es, idx, z, beta, sigma, V):
    """d log pi / dz from the oracle: the chain-rule gradient of Eq. 1 (itself
    pinned by finite differences in test_fd_temporal_trend_gradient) plus the
    prior's gradient (pinned against scipy in test_tree_prior_closed_form_and_scipy)."""
    from oracle import hmc, tree as otree
    _, gz, _ = hmc.trend_grad(es.t, es.x, es.y, es.theta, idx, z, beta, es.hyper, es.t0)
    if V is None:
        return gz - z / sigma ** 2
    return gz + otree.logpdf_and_grad(z, V, sigma)[1]


@pytest.mark.parametrize("case", ["iid", "trend", "tree"])
def test_z_hessian_diag_by_finite_differences(case):
    """The exact z-space curvature -d2 log pi / dz_k^2 = theta^2 H - theta g + P_kk
    (Eq. 4, Eq. 5 through theta_k = exp(z_k + beta t_k), P the prior precision)
    against central differences of the log-posterior gradient in z_k (step 1e-5).
    A sign slip in the -theta g term, a missing square on theta, a rate taken
    as exp(z) while beta != 0 or the wrong prior precision each fail here."""
    from oracle import hmc, tree as otree
    es = _es(70, seed=61, ties=2)
    idx = np.arange(1, es.n, 4)
    m = idx.shape[0]
    z = 0.3 * np.random.default_rng(61).standard_normal(m)
    sigma = 0.7
    beta = -0.03 if case == "trend" else 0.0
    V = None
    if case == "tree":
        par, ln = synth.coalescent_tree(m, seed=7, scale=float(m))
        V = otree.covariance(par, ln, 0.6)
    ref = hmc.z_hessian_diag(es.t, es.x, es.y, es.theta, idx, z, es.hyper, es.t0, sigma, beta=beta, prior_v=V)
    step = 1e-5
    checked = 0
    for k in range(0, m, 3):
        zp, zm = z.copy(), z.copy()
        zp[k] += step
        zm[k] -= step
        fd = -(_z_grad(es, idx, zp, beta, sigma, V)[k] - _z_grad(es, idx, zm, beta, sigma, V)[k]) / (2 * step)
        assert ref[k] == pytest.approx(fd, rel=1e-6, abs=1e-8), (case, k)
        checked += 1
    assert checked >= 5
    # the likelihood part is not negligible here: the check sees the -theta g and theta^2 H terms
    lik = ref - hmc.prior_precision_diag(m, sigma, V)
    assert np.max(np.abs(lik)) > 0.05 * np.median(hmc.prior_precision_diag(m, sigma, V))


def test_prior_precision_diag_is_conditional_precision():
    """(V^{-1})_kk is the inverse of the conditional variance of tip k given the
    other tips.  On the three-tip tree ((0, 1), 2) with root factor tau0, the
    conditional variance of tip 0 follows by hand from the Brownian motion of
    Eq. 2: the root given tip 2, then the parent of tips 0 and 1 given tip 1 and
    the root side, then tip 0's own branch.  The oracle's dense inverse must
    agree; an inverse taken of the wrong matrix or a missing 1/sigma^2 fails."""
    from oracle import hmc
    w0, w1, w2, w3, tau0 = 0.4, 0.9, 1.3, 0.5, 0.8
    # nodes 0, 1, 2 tips; 3 = parent of (0, 1), branch w3 to the root 4; tip 2 hangs off the root
    V = np.array([[tau0 + w3 + w0, tau0 + w3, tau0],
                  [tau0 + w3, tau0 + w3 + w1, tau0],
                  [tau0, tau0, tau0 + w2]])
    P = hmc.prior_precision_diag(3, 1.0, V)
    # conditional variance of tip 0: the ancestor node 3 given tips 1 and 2 combines
    # the message from tip 1 (variance w1) and from the root side (w3 + (tau0 given tip 2))
    root_given_2 = 1.0 / (1.0 / tau0 + 1.0 / w2)
    node3 = 1.0 / (1.0 / w1 + 1.0 / (w3 + root_given_2))
    assert P[0] == pytest.approx(1.0 / (w0 + node3), rel=1e-13)
    assert np.all(hmc.prior_precision_diag(4, 0.5) == 4.0)


def test_mlp_gradient_by_finite_differences():
    """Back-propagation of the preconditioner network against central differences
    of its loss (step 1e-6) on random parameters."""
    from oracle import mlp
    rng = np.random.default_rng(3)
    p = mlp.init(seed=1) + 0.05 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((37, 12))
    tgt = rng.standard_normal(37)
    loss, g = mlp.loss_and_grad(p, X, tgt)
    for j in rng.choice(mlp.N_PARAMS, size=25, replace=False).tolist() + [mlp.N_PARAMS - 1, 0, 768, 900]:
        e = np.zeros(mlp.N_PARAMS)
        e[j] = 1e-6
        fd = (mlp.loss_and_grad(p + e, X, tgt)[0] - mlp.loss_and_grad(p - e, X, tgt)[0]) / 2e-6
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mlp_forward_closed_form_and_adam_first_step():
    """With W2 = 0 the output is w3 . tanh(b2) + b3 whatever the input; Adam's first
    bias-corrected step moves every parameter by -lr g / (|g| + eps)."""
    from oracle import mlp
    p = mlp.unpack(mlp.init(seed=2))
    p["W2"][:] = 0.0
    p["b2"][:] = np.linspace(-1, 1, 64)
    flat = mlp.pack(p)
    X = np.random.default_rng(0).standard_normal((5, 12))
    y, _ = mlp.forward(flat, X)
    np.testing.assert_allclose(y, np.dot(p["w3"], np.tanh(p["b2"])) + p["b3"][0], rtol=1e-14)
    g = np.random.default_rng(1).standard_normal(mlp.N_PARAMS)
    new, m, v = mlp.adam_step(flat, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    np.testing.assert_allclose(new - flat, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_later_steps_closed_forms():
    """Adam (Kingma & Ba 2015) over several steps, against closed forms of its
    moment recursions rather than the recursions themselves:
      * a constant gradient g: the bias-corrected moments are g and g^2 at every
        step, so after k steps each parameter has moved by -k lr g / (|g| + eps);
      * an alternating gradient (-1)^t g: the first moment is the geometric sum
        m_t = (1 - b1) g (-1)^t (1 - (-b1)^t) / (1 + b1) and the second is still
        (1 - b2^t) g^2, so step t moves by
        -lr (-1)^t (1 - b1) (1 - (-b1)^t) / ((1 + b1)(1 - b1^t)) g / (|g| + eps).
    A wrong decay exponent in the bias correction, or moments not carried from
    step to step, fail these."""
    from oracle import mlp
    rng = np.random.default_rng(9)
    g = rng.standard_normal(mlp.N_PARAMS)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    p = np.zeros(mlp.N_PARAMS)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 8):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-9)
    p = np.zeros(mlp.N_PARAMS)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 8):
        prev = p.copy()
        p, m, v = mlp.adam_step(p, (-1.0) ** t * g, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mhat_over_g = (-1.0) ** t * (1 - b1) * (1 - (-b1) ** t) / ((1 + b1) * (1 - b1 ** t))
        np.testing.assert_allclose(p - prev, -lr * mhat_over_g * g / (np.abs(g) + eps), rtol=1e-8)


def test_features_small_hand_case():
    """Disc and time-window count features on a hand-built set (h = 0.3,
    tau_x = 2, omega = 0.5: windows of 2 and 6 time units), counted by hand:
    the counts, the self-exclusion, the strict and closed window ends and the
    rank / window-end features follow their definitions."""
    from oracle import features
    hy = (0.7, 2.0, 5.0, 0.3, 0.5, 0.3)
    #             e0    e1    e2    e3    e4    e5
    t = np.array([0.5, 1.0, 2.5, 2.6, 7.0, 2.5])
    x = np.array([0.0, 0.1, 0.0, 5.0, 0.5, 1.5])
    y = np.array([0.0, 0.1, 0.25, 5.0, 0.0, 0.0])
    # distances from e0: e1 0.141, e2 0.25, e3 7.07, e4 0.5, e5 1.5
    # distances from e2: e0 0.25, e1 0.180, e3 6.9, e4 0.559, e5 1.52
    F = features.features(t, x, y, np.array([0, 2]), np.array([0.1, -0.2]), hy, 0.0, -1.0, -1.0)
    L = np.log1p
    # e0: within h = 0.3: e1, e2; within 0.9: + e4; later within 0.9 and 12 time units: e1, e2, e4
    assert F[0, 0] == L(2) and F[0, 1] == L(3) and F[0, 2] == L(3)
    # e0, r = h: no earlier event; later within 2 time units: e1 (dt 0.5), e2 (dt 2.0, closed end)
    assert F[0, 3] == L(0) and F[0, 4] == L(2) and F[0, 5] == L(2)
    # e0, r = 3h: no earlier event, e1 and e2 within 2 time units
    assert F[0, 6] == L(0) and F[0, 7] == L(2)
    # feature 8, the forward squared-kernel sum over r < 3h, 0 < dt <= 12:
    # e1 (dt 0.5, r^2 0.02), e2 (dt 2.0, r^2 0.0625), e4 (dt 6.5, r^2 0.25), by hand
    # exp(-0.7222) = 0.485672, exp(-2.6944) = 0.067580, exp(-9.2778) = 0.0000935
    assert 2.0 ** (8.0 * F[0, 8]) == pytest.approx(0.485672 + 0.067580 + 0.0000935, rel=2e-6)
    # e2: within h: e0, e1; within 3h: + e4; later within 3h and 12 time units: e4 (e5 ties)
    assert F[1, 0] == L(2) and F[1, 1] == L(3) and F[1, 2] == L(1)
    # e2, r = h: earlier within [-2, 0): e1 (dt -1.5); e0 (dt -2.0, closed end) too
    assert F[1, 3] == L(2) and F[1, 4] == L(0) and F[1, 5] == L(0)
    # e2, r = 3h: e0, e1 earlier; no later event within 2 time units
    assert F[1, 6] == L(2) and F[1, 7] == L(0)
    # feature 8: e4 alone (dt 4.5, r^2 0.3125); e5 ties (dt 0) and is far, by hand
    # exp(-4.5 - 3.47222) = 0.000344912
    assert 2.0 ** (8.0 * F[1, 8]) == pytest.approx(0.000344912, rel=2e-6)
    assert F[1, 9] == -0.2
    assert F[1, 10] == pytest.approx(2 / 6) and F[1, 11] == pytest.approx((7.0 - 2.5) / 7.0)


def test_kernel_sum_feature_special_cases():
    """Feature 8 (forward sum of the squared excitation kernel) in cases with a
    closed form: one later event at dt = 1/omega and distance h gives
    exp(-3); no later event gives the floor; the window's ends (dt = 6/omega
    included, distance 3h excluded); the sum of two neighbours is the sum of
    their single-neighbour values; and it is invariant to translations and to
    scaling space with h and time with 1/omega."""
    import math

    from oracle import features
    hy = (0.7, 2.0, 5.0, 0.3, 0.5, 0.3)  # omega = 0.5, h = 0.3

    def f8(t, x, y, hyper=hy):
        return features.features(np.asarray(t, float), np.asarray(x, float), np.asarray(y, float),
                                 np.array([0]), np.array([0.0]), hyper, 0.0, -1.0, -1.0)[0, 8]

    assert f8([1.0, 3.0], [0.0, 0.3], [0.0, 0.0]) == pytest.approx(-3.0 / math.log(2.0) / 8.0, rel=1e-12)
    assert f8([1.0, 0.5], [0.0, 0.1], [0.0, 0.0]) == -4.0          # only an earlier event
    assert f8([1.0, 1.0], [0.0, 0.1], [0.0, 0.0]) == -4.0          # a tie (dt = 0)
    assert f8([1.0, 13.0], [0.0, 0.0], [0.0, 0.0]) == pytest.approx(-12.0 / math.log(2.0) / 8.0, rel=1e-12)
    assert f8([1.0, 13.0 + 1e-9], [0.0, 0.0], [0.0, 0.0]) == -4.0  # past 6/omega
    assert f8([1.0, 2.0], [0.0, 0.9], [0.0, 0.0]) == -4.0          # at 3h: outside
    a = f8([1.0, 1.7], [0.0, 0.2], [0.0, 0.1])
    b = f8([1.0, 4.2], [0.0, -0.4], [0.0, 0.3])
    ab = f8([1.0, 1.7, 4.2], [0.0, 0.2, -0.4], [0.0, 0.1, 0.3])
    assert 2.0 ** (8.0 * ab) == pytest.approx(2.0 ** (8.0 * a) + 2.0 ** (8.0 * b), rel=1e-12)
    t, x, y = [1.0, 1.7, 4.2], [0.0, 0.2, -0.4], [0.0, 0.1, 0.3]
    shifted = f8([v + 10.0 for v in t], [v - 3.0 for v in x], [v + 5.0 for v in y])
    assert shifted == pytest.approx(ab, abs=1e-12)
    scaled_hy = (0.7, 4.0, 5.0, 0.3, 0.25, 0.6)  # h doubled, omega halved
    scaled = f8([2.0 * v for v in t], [2.0 * v for v in x], [2.0 * v for v in y], scaled_hy)
    assert scaled == pytest.approx(ab, abs=1e-12)


def test_ess_of_ar1_chain():
    """Geyer's estimator on AR(1) chains, whose ESS is n (1 - rho) / (1 + rho)."""
    from paper_2103_03348_amd import ess
    rng = np.random.default_rng(11)
    n = 200000
    for rho in (0.0, 0.5, 0.9):
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0]
        for k in range(1, n):
            x[k] = rho * x[k - 1] + np.sqrt(1 - rho * rho) * e[k]
        expect = n * (1 - rho) / (1 + rho)
        assert ess.ess_1d(x) == pytest.approx(expect, rel=0.1)


def test_fd_temporal_trend_gradient():
    """Sec. 2.2's rates theta_k = exp(z_k + beta t_k): the chain-rule gradients
    d/dz_k = theta_k (Eq. 4)_k and d/dbeta = sum_k t_k theta_k (Eq. 4)_k against
    central finite differences of Eq. 1 in beta and in two z_k."""
    from oracle import hmc as ohmc

    es = _es(60, seed=41, ties=2)
    idx = np.arange(0, es.n, 3)
    z = 0.3 * np.random.default_rng(41).standard_normal(idx.shape[0])
    beta = -0.04
    ll, gz, gb = ohmc.trend_grad(es.t, es.x, es.y, es.theta, idx, z, beta, es.hyper, es.t0)

    def ell_beta(b):
        th = ohmc.rates(es.t, es.theta, idx, z, b)
        return oracle.evaluate_es(es, theta=th, want=("ell_n",))["ell_n"]

    fd = _fd_loglik(ell_beta, beta, 1e-6)
    assert gb == pytest.approx(fd, rel=1e-7, abs=1e-9)
    for k in (0, idx.shape[0] // 2):
        def ell_z(v, k=k):
            zz = z.copy()
            zz[k] = v
            return oracle.evaluate_es(es, theta=ohmc.rates(es.t, es.theta, idx, zz, beta), want=("ell_n",))["ell_n"]

        assert gz[k] == pytest.approx(_fd_loglik(ell_z, z[k], 1e-6), rel=1e-7, abs=1e-9)
    # beta = 0 reduces to theta_k = exp(z_k)
    _, gz0, _ = ohmc.trend_grad(es.t, es.x, es.y, es.theta, idx, z, 0.0, es.hyper, es.t0)
    th = es.theta.copy()
    th[idx] = np.exp(z)
    r = oracle.evaluate_es(es, theta=th, want=("grad_theta",))
    np.testing.assert_allclose(gz0, np.exp(z) * r["grad_theta"][idx], rtol=1e-15)


def test_tree_prior_closed_form_and_scipy():
    """Eq. 2's covariance from a tree: a two-tip tree by hand, and the oracle's
    log density and gradient against scipy's multivariate normal and central
    differences on a coalescent tree."""
    from scipy.stats import multivariate_normal

    from oracle import tree as otree

    # two tips joined at the root: V = [[tau0 + w0, tau0], [tau0, tau0 + w1]]
    V2 = otree.covariance([2, 2, -1], [0.3, 0.7, 0.0], 1.5)
    np.testing.assert_allclose(V2, [[1.8, 1.5], [1.5, 2.2]], rtol=1e-15)
    parent, length = synth.coalescent_tree(40, seed=3)
    V = otree.covariance(parent, length, 0.8)
    assert np.allclose(V, V.T) and np.all(np.linalg.eigvalsh(V) > 0)
    z = np.random.default_rng(3).standard_normal(40)
    sigma = 0.6
    logp, grad, quad = otree.logpdf_and_grad(z, V, sigma)
    assert logp == pytest.approx(multivariate_normal(np.zeros(40), sigma ** 2 * V).logpdf(z), rel=1e-10)
    for k in (0, 17, 39):
        e = np.zeros(40)
        e[k] = 1e-6
        fd = (otree.logpdf_and_grad(z + e, V, sigma)[0] - otree.logpdf_and_grad(z - e, V, sigma)[0]) / 2e-6
        assert grad[k] == pytest.approx(fd, rel=1e-6)
    # tip variances: tau0 + root-to-tip path length
    k = 5
    d, v = 0.0, k
    while parent[v] >= 0:
        d += length[v]
        v = parent[v]
    assert V[k, k] == pytest.approx(0.8 + d, rel=1e-14)
