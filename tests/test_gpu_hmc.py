"""Free-rate subset path and HMC step on the GPU vs the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import hmc as ohmc
from paper_2103_03348_amd import synth

from gpu_helpers import h_rel_all

pytestmark = pytest.mark.gpu


def _setup(es):
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    idx = torch.as_tensor(es.subset, dtype=torch.int64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle()),
               "set_subset")
    return plan, idx


def _subset_grad(plan, es, theta, refresh=0, want_h=True):
    import torch

    from paper_2103_03348_amd import _lib

    m = es.subset.shape[0]
    th = torch.as_tensor(theta, device="cuda:0")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    h = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    hy = _lib.Hyper.of(es.hyper)
    _lib.check(_lib.lib().hawkes_subset_grad(plan.handle, ctypes.byref(hy), _lib.ptr(th), refresh, _lib.ptr(ll),
                                             _lib.ptr(g), _lib.ptr(h) if want_h else None, _lib.stream_handle()),
               "subset_grad")
    torch.cuda.synchronize()
    return float(ll.item()), g.cpu().numpy(), (h.cpu().numpy() if want_h else None)


@pytest.mark.parametrize("cfg", ["small", "allfree", "dense", "isolated", "n23422"])
def test_subset_grad_matches_oracle(gpu, cfg):
    """Eq. 1, 4, 5 restricted to the free rates, by the cached-static O(N M) path
    (allfree: every rate free, so the static part holds the background only;
    dense: the latest 2,500 of 3,000 events free, so that late row chunks have
    up to 40 row items each and their finalisation takes more than one round of
    batched reads; isolated: 2,500 events over 1e5 time units, 60 of whose
    intensities lie below 1e-38, down to 6e-110, recomputed in FP64 by the
    static part and the row finalisation)."""
    if cfg == "isolated":
        es = synth.small(2500, seed=9, t_end=1e5, all_free=False)
    elif cfg == "small":
        es = synth.small(1500, seed=21, ties=6, all_free=False)
    elif cfg == "allfree":
        es = synth.small(333, seed=22, ties=5, all_free=True)
    elif cfg == "dense":
        import dataclasses

        es = synth.small(3000, seed=23, ties=4, all_free=False)
        sub = np.sort(np.argsort(es.t, kind="stable")[500:]).astype(np.int64)
        es = dataclasses.replace(es, subset=sub, z=np.log(es.theta[sub]))
    else:
        es = synth.config(1)
    plan, idx = _setup(es)
    ll, g, h = _subset_grad(plan, es, es.theta)
    assert plan.status() == 0
    ref = oracle.evaluate_es(es)
    gi = ref["grad_theta"][es.subset]
    hi = ref["negH_theta"][es.subset]
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t[es.subset])))
    rel_l = abs(ll - ref["loglik"]) / abs(ref["loglik"])
    rel_g = np.max(np.abs(g - gi) / np.maximum(gi + 2 * a, 1e-300))
    rel_h = h_rel_all(h, hi)
    print(f"\nsubset {cfg}: n={es.n} m={es.subset.shape[0]} loglik rel {rel_l:.2e} g {rel_g:.2e} H {rel_h:.2e}")
    assert rel_l < (1e-9 if cfg == "n23422" else 2e-6 * es.n / abs(ref["loglik"]))
    assert rel_g < 1e-6
    assert rel_h < 1e-6
    # a second call at new rates reuses the cached static part
    rng = np.random.default_rng(4)
    th2 = es.theta.copy()
    th2[es.subset] = np.exp(rng.normal(0, 0.5, es.subset.shape[0]))
    ll2, g2, _ = _subset_grad(plan, es, th2)
    ref2 = oracle.evaluate_es(es, theta=th2, want=("loglik", "grad_theta"))
    assert abs(ll2 - ref2["loglik"]) / abs(ref2["loglik"]) < (1e-9 if cfg == "n23422" else 1e-6)
    gi2 = ref2["grad_theta"][es.subset]
    assert np.max(np.abs(g2 - gi2) / np.maximum(np.abs(gi2) + 2 * a, 1e-300)) < 1e-6


@pytest.mark.parametrize("cfg", ["small", "dense", "sparse", "isolated", "n23422"])
def test_subset_grad_only_matches_oracle(gpu, cfg):
    """Eq. 4 alone on the subset (the leapfrog's gradient): its column pass
    applies the row weight's integer part exactly and rounds the rest of each
    exponent to FP32; held to the same bound as with Eq. 5, against the oracle
    (sparse: 2,000 events over 2,400 time units, most terms tiny)."""
    import dataclasses

    if cfg == "small":
        es = synth.small(1500, seed=21, ties=6, all_free=False)
    elif cfg == "dense":
        es = synth.small(3000, seed=23, ties=4, all_free=False)
        sub = np.sort(np.argsort(es.t, kind="stable")[500:]).astype(np.int64)
        es = dataclasses.replace(es, subset=sub, z=np.log(es.theta[sub]))
    elif cfg == "sparse":
        es = synth.small(2000, seed=33, t_end=2400.0, ties=2, all_free=False)
    elif cfg == "isolated":
        es = synth.small(2500, seed=9, t_end=1e5, all_free=False)
    else:
        es = synth.config(1)
    plan, idx = _setup(es)
    ll, g, _ = _subset_grad(plan, es, es.theta, want_h=False)
    assert plan.status() == 0
    ref = oracle.evaluate_es(es, want=("loglik", "grad_theta"))
    gi = ref["grad_theta"][es.subset]
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t[es.subset])))
    rel_g = np.max(np.abs(g - gi) / np.maximum(gi + 2 * a, 1e-300))
    print(f"\nsubset grad only {cfg}: n={es.n} m={es.subset.shape[0]} g {rel_g:.2e}")
    assert rel_g < 1e-6
    plan.close()


def test_subset_rejects_bad_indices(gpu):
    """A repeated or out-of-range free-rate index is an argument error, and the
    plan keeps working for a valid subset afterwards."""
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es = synth.small(300, seed=23, ties=4, all_free=False)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    for bad in ([3, 7, 3], [0, 299, 300], [-1, 5]):
        idx = torch.as_tensor(bad, dtype=torch.int64, device="cuda:0")
        code = _lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle())
        assert code == _lib.E_INVALID, (bad, code)
    # an empty subset, and one larger than the event set
    idx = torch.arange(301, dtype=torch.int64, device="cuda:0")
    assert _lib.lib().hawkes_plan_set_subset(plan.handle, 0, _lib.ptr(idx), _lib.stream_handle()) == _lib.E_INVALID
    assert _lib.lib().hawkes_plan_set_subset(plan.handle, 301, _lib.ptr(idx), _lib.stream_handle()) == _lib.E_INVALID
    idx = torch.as_tensor(es.subset, dtype=torch.int64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle()),
               "set_subset")
    ll, g, _ = _subset_grad(plan, es, es.theta)
    ref = oracle.evaluate_es(es, want=("loglik", "grad_theta"))
    assert abs(ll - ref["loglik"]) / abs(ref["loglik"]) < 1e-6
    plan.close()


def _hmc_gpu(plan, es, z0, mass, eps, L, sigma, seed, counter, theta=None):
    import torch

    from paper_2103_03348_amd import _lib

    dev = "cuda:0"
    z = torch.as_tensor(np.asarray(z0, dtype=np.float64).copy(), device=dev)
    th = torch.as_tensor((es.theta if theta is None else theta).copy(), device=dev)
    ms = torch.as_tensor(np.asarray(mass, dtype=np.float64), device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    args = _lib.HmcArgs(z.data_ptr(), th.data_ptr(), ms.data_ptr(), eps, L, sigma, seed, counter, 0, out.data_ptr())
    hy = _lib.Hyper.of(es.hyper)
    _lib.check(_lib.lib().hmc_step(plan.handle, ctypes.byref(hy), ctypes.byref(args), _lib.stream_handle()), "hmc")
    torch.cuda.synchronize()
    return z.cpu().numpy(), th.cpu().numpy(), out.cpu().numpy()


def test_hmc_step_replays_oracle(gpu):
    """One HMC iteration with the same Philox seed/counter on both sides: same
    momenta, same leapfrog path (to FP32 gradient error), same energy change and
    the same accept decision."""
    es = synth.small(400, seed=23, ties=3, all_free=False)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    z0 = np.log(es.theta[es.subset])
    mass = np.full(m, 6.0)
    for counter in range(3):
        zg, thg, out = _hmc_gpu(plan, es, z0, mass, 0.05, 8, 0.5, 77, counter)
        r = ohmc.hmc_iteration(es.t, es.x, es.y, es.theta, es.subset, z0, mass, es.hyper, 0.0, 0.05, 8, 0.5,
                               77, counter)
        print(f"\ncounter {counter}: gpu dH {out[1]:.9f} acc {out[0]} | oracle dH {r['dH']:.9f} acc {r['accepted']}")
        assert abs(out[1] - r["dH"]) < 1e-5
        margin = abs(np.log(r["u"]) + r["dH"])
        if margin > 1e-4:
            assert bool(out[0]) == r["accepted"]
        if r["accepted"]:
            np.testing.assert_allclose(zg, r["z_proposal"], atol=1e-6)
            np.testing.assert_allclose(thg[es.subset], np.exp(zg), rtol=1e-15)
        else:
            np.testing.assert_array_equal(zg, z0)
        assert abs(out[6] - r["H0"]) < 1e-6 * max(1.0, abs(r["H0"]))


def test_hmc_step_replays_oracle_isolated(gpu):
    """hmc_step against the oracle's iteration on 2,500 events over 1e5 time
    units (166 free rates): 60 intensities lie below FP32's range and wide
    subset batches take the unsplit exponent; same momenta, path, energy change
    and accept decision as the FP64 oracle.  dH and H0 to 2e-9 and 1e-9 of
    |loglik| (its 1e-9 target at each end), the path's end to 1e-6."""
    es = synth.small(2500, seed=9, t_end=1e5, all_free=False)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    z0 = np.log(es.theta[es.subset])
    mass = np.full(m, 6.0)
    for counter in range(2):
        zg, thg, out = _hmc_gpu(plan, es, z0, mass, 0.05, 8, 0.5, 91, counter)
        assert plan.status() == 0
        r = ohmc.hmc_iteration(es.t, es.x, es.y, es.theta, es.subset, z0, mass, es.hyper, 0.0, 0.05, 8, 0.5,
                               91, counter)
        print(f"\ncounter {counter}: gpu dH {out[1]:.9f} acc {out[0]} | oracle dH {r['dH']:.9f} acc {r['accepted']}")
        assert abs(out[1] - r["dH"]) < 2e-9 * abs(r["H0"])
        margin = abs(np.log(r["u"]) + r["dH"])
        if margin > 1e-4:
            assert bool(out[0]) == r["accepted"]
        if r["accepted"]:
            np.testing.assert_allclose(zg, r["z_proposal"], atol=1e-6)
        else:
            np.testing.assert_array_equal(zg, z0)
        assert abs(out[6] - r["H0"]) < 1e-9 * abs(r["H0"])
    plan.close()


def test_hmc_deterministic(gpu):
    es = synth.small(300, seed=24, all_free=False)
    plan, _ = _setup(es)
    m = es.subset.shape[0]
    z0 = np.log(es.theta[es.subset])
    a = _hmc_gpu(plan, es, z0, np.full(m, 5.0), 0.1, 5, 0.5, 1, 9)
    b = _hmc_gpu(plan, es, z0, np.full(m, 5.0), 0.1, 5, 0.5, 1, 9)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_hmc_samples_prior_without_excitation(gpu):
    """theta0 = 0 makes the likelihood independent of the rates: the GPU chain
    must sample N(0, sigma_z^2) (mean, variance and a KS test of the pooled draws)."""
    import torch
    from scipy import stats

    from paper_2103_03348_amd import _lib

    es = synth.small(500, seed=25, all_free=False)
    es.hyper = (0.7, 2.0, 5.0, 0.0, 0.5, 0.3)
    plan, _ = _setup(es)
    m = es.subset.shape[0]
    sig = 0.5
    dev = "cuda:0"
    z = torch.zeros(m, dtype=torch.float64, device=dev)
    th = torch.as_tensor(es.theta.copy(), device=dev)
    ms = torch.full((m,), 1.0 / sig ** 2, dtype=torch.float64, device=dev)
    out = torch.zeros(8, dtype=torch.float64, device=dev)
    hy = _lib.Hyper.of(es.hyper)
    draws = []
    acc = 0.0
    for it in range(1500):
        args = _lib.HmcArgs(z.data_ptr(), th.data_ptr(), ms.data_ptr(), 0.9, 3, sig, 11, it, 0, out.data_ptr())
        _lib.check(_lib.lib().hmc_step(plan.handle, ctypes.byref(hy), ctypes.byref(args), _lib.stream_handle()),
                   "hmc")
        if it >= 100:
            draws.append(z.clone())
        acc += 0  # accept flags are read once at the end
    torch.cuda.synchronize()
    d = torch.stack(draws).cpu().numpy()
    print(f"\nprior check: mean {d.mean():.4f} var {d.var():.4f} (target 0, {sig ** 2})")
    assert abs(d.mean()) < 0.03
    assert abs(d.var() - sig ** 2) < 0.02
    assert stats.kstest(d[::7, 0] / sig, "norm").pvalue > 1e-3


def test_trend_gradient_matches_oracle(gpu):
    """Sec. 2.2's temporal trend theta_k = exp(z_k + beta t_k): loglik, d/dz and
    d/dbeta of the subset path against the oracle's chain rule (itself pinned
    by finite differences in test_oracle_pins)."""
    import torch

    from paper_2103_03348_amd import _lib

    es = synth.small(1500, seed=43, ties=4, all_free=False)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    rng = np.random.default_rng(43)
    z = 0.4 * rng.standard_normal(m)
    beta = -0.006   # times span [0, 150]
    dz = torch.as_tensor(z, device="cuda:0")
    th = torch.as_tensor(es.theta.copy(), device="cuda:0")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    gz = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    gb = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    hy = _lib.Hyper.of(es.hyper)
    _lib.check(_lib.lib().hawkes_subset_trend_grad(plan.handle, ctypes.byref(hy), _lib.ptr(dz), beta, _lib.ptr(th),
                                                   _lib.ptr(ll), _lib.ptr(gz), _lib.ptr(gb), _lib.stream_handle()),
               "trend")
    torch.cuda.synchronize()
    assert plan.status() == 0
    ll_o, gz_o, gb_o = ohmc.trend_grad(es.t, es.x, es.y, es.theta, es.subset, z, beta, es.hyper, es.t0)
    th_o = ohmc.rates(es.t, es.theta, es.subset, z, beta)
    np.testing.assert_allclose(th.cpu().numpy(), th_o, rtol=1e-15)
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t[es.subset])))
    r = oracle.evaluate_es(es, theta=th_o, want=("grad_theta",))
    scale_z = th_o[es.subset] * (np.abs(r["grad_theta"][es.subset]) + 2 * a)   # C11 scale through the chain rule
    rel_l = abs(float(ll.item()) - ll_o) / abs(ll_o)
    rel_z = np.max(np.abs(gz.cpu().numpy() - gz_o) / scale_z)
    rel_b = abs(float(gb.item()) - gb_o) / float(np.sum(es.t[es.subset] * scale_z))
    print(f"\ntrend: loglik {rel_l:.2e} d/dz {rel_z:.2e} d/dbeta {rel_b:.2e}")
    assert rel_l < 2e-6 * es.n / abs(ll_o)
    assert rel_z < 1e-6
    assert rel_b < 1e-6


def test_hmc_step_with_trend_replays_oracle(gpu):
    es = synth.small(400, seed=44, ties=3, all_free=False)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    z0 = np.log(es.theta[es.subset]) + 0.05
    mass = np.full(m, 6.0)
    beta = -0.01

    import torch

    from paper_2103_03348_amd import _lib

    for counter in range(2):
        z = torch.as_tensor(z0.copy(), device="cuda:0")
        th = torch.as_tensor(es.theta.copy(), device="cuda:0")
        ms = torch.as_tensor(mass, device="cuda:0")
        out = torch.zeros(8, dtype=torch.float64, device="cuda:0")
        args = _lib.HmcArgs(z.data_ptr(), th.data_ptr(), ms.data_ptr(), 0.05, 8, 0.5, 91, counter, 0,
                            out.data_ptr(), beta)
        hy = _lib.Hyper.of(es.hyper)
        _lib.check(_lib.lib().hmc_step(plan.handle, ctypes.byref(hy), ctypes.byref(args), _lib.stream_handle()),
                   "hmc")
        torch.cuda.synchronize()
        r = ohmc.hmc_iteration(es.t, es.x, es.y, es.theta, es.subset, z0, mass, es.hyper, 0.0, 0.05, 8, 0.5, 91,
                               counter, beta=beta)
        o = out.cpu().numpy()
        print(f"\ntrend counter {counter}: gpu dH {o[1]:.9f} | oracle dH {r['dH']:.9f}")
        assert abs(o[1] - r["dH"]) < 1e-5
        if abs(np.log(r["u"]) + r["dH"]) > 1e-4:
            assert bool(o[0]) == r["accepted"]
        if r["accepted"]:
            np.testing.assert_allclose(z.cpu().numpy(), r["z_proposal"], atol=1e-6)


def test_gibbs_log_target_and_iterations(gpu):
    """The Metropolis-within-Gibbs layer: its log target at a state is the
    oracle's log-likelihood (rates exp(z + beta t) on the subset) plus the log
    prior; a few Gibbs iterations (HMC on z + univariate MH on the
    hyperparameters and beta) keep a finite target and move the parameters."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan
    from paper_2103_03348_amd.mcmc import HawkesGibbs
    from paper_2103_03348_amd.sampler import HmcSampler

    es = synth.small(800, seed=45, all_free=False)
    dev = "cuda:0"
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    smp = HmcSampler(plan, torch.as_tensor(es.theta, device=dev), torch.as_tensor(es.subset, device=dev),
                     es.hyper, sigma_z=0.5, L=5, seed=4, beta=-0.002)
    gibbs = HawkesGibbs(smp, n_mh=6, seed=4)
    z = smp.z.cpu().numpy()
    th = ohmc.rates(es.t, es.theta, es.subset, z, -0.002)
    ll_o = oracle.evaluate_es(es, theta=th, want=("loglik",))["loglik"]
    lp_o = ll_o + gibbs.log_prior(gibbs.state)
    print(f"\ngibbs: log target {gibbs.logp:.9f} oracle {lp_o:.9f}")
    assert abs(gibbs.logp - lp_o) < 2e-6 * es.n
    start = dict(gibbs.state)
    for _ in range(25):
        gibbs.iteration(0.1)
        assert np.isfinite(gibbs.logp)
    moved = [k for k in start if gibbs.state[k] != start[k]]
    acc = gibbs.mh.acceptance()
    print("gibbs acceptance", acc, "moved", moved)
    assert len(moved) >= 3
    assert plan.status() == 0
    plan.close()


def test_tree_prior_matches_oracle(gpu):
    """Eq. 2 by O(M) message passing on the device against the dense-V oracle
    (Cholesky), on coalescent trees of 1, 2, 57 and 1,610 tips."""
    import torch

    from oracle import tree as otree
    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es = synth.small(300, seed=46)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    for m in (1, 2, 57, 1610):
        par, ln = synth.coalescent_tree(m, seed=m, scale=float(m))
        par, ln = np.ascontiguousarray(par), np.ascontiguousarray(ln)
        _lib.check(_lib.lib().hawkes_plan_set_tree(plan.handle, 2 * m - 1, par.ctypes.data_as(ctypes.c_void_p),
                                                   ln.ctypes.data_as(ctypes.c_void_p), 0.9), "set_tree")
        z = np.random.default_rng(m).standard_normal(m)
        dz = torch.as_tensor(z, device="cuda:0")
        lp = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        g = torch.zeros(m, dtype=torch.float64, device="cuda:0")
        q = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        _lib.check(_lib.lib().hawkes_tree_prior(plan.handle, _lib.ptr(dz), 0.5, _lib.ptr(lp), _lib.ptr(g),
                                                _lib.ptr(q), _lib.stream_handle()), "tree_prior")
        torch.cuda.synchronize()
        lpo, go, qo = otree.logpdf_and_grad(z, otree.covariance(par, ln, 0.9), 0.5)
        rel_l = abs(float(lp.item()) - lpo) / abs(lpo)
        rel_g = np.max(np.abs(g.cpu().numpy() - go)) / np.max(np.abs(go))
        print(f"\ntree M={m}: logp {rel_l:.2e} grad {rel_g:.2e}")
        assert rel_l < 1e-10 and rel_g < 1e-9
    # a malformed tree is rejected
    bad = np.ascontiguousarray(np.array([2, 2, 3, -1, 3], dtype=np.int64))
    ln = np.ascontiguousarray(np.ones(5))
    assert _lib.lib().hawkes_plan_set_tree(plan.handle, 5, bad.ctypes.data_as(ctypes.c_void_p),
                                           ln.ctypes.data_as(ctypes.c_void_p), 0.9) == _lib.E_INVALID
    plan.close()


def test_hmc_step_with_tree_prior_replays_oracle(gpu):
    """hmc_step with the phylogenetic prior (prior = 1) against the oracle's
    iteration with the dense V, same Philox seed and counter."""
    import torch

    from oracle import tree as otree
    from paper_2103_03348_amd import _lib

    es = synth.small(400, seed=47, ties=2, all_free=False)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    par, ln = synth.coalescent_tree(m, seed=47, scale=float(m))
    par, ln = np.ascontiguousarray(par), np.ascontiguousarray(ln)
    _lib.check(_lib.lib().hawkes_plan_set_tree(plan.handle, 2 * m - 1, par.ctypes.data_as(ctypes.c_void_p),
                                               ln.ctypes.data_as(ctypes.c_void_p), 1.0), "set_tree")
    V = otree.covariance(par, ln, 1.0)
    z0 = np.log(es.theta[es.subset])
    mass = np.full(m, 8.0)
    for counter in range(2):
        z = torch.as_tensor(z0.copy(), device="cuda:0")
        th = torch.as_tensor(es.theta.copy(), device="cuda:0")
        ms = torch.as_tensor(mass, device="cuda:0")
        out = torch.zeros(8, dtype=torch.float64, device="cuda:0")
        args = _lib.HmcArgs(z.data_ptr(), th.data_ptr(), ms.data_ptr(), 0.05, 6, 0.5, 93, counter, 0,
                            out.data_ptr(), 0.0, 1)
        hy = _lib.Hyper.of(es.hyper)
        _lib.check(_lib.lib().hmc_step(plan.handle, ctypes.byref(hy), ctypes.byref(args), _lib.stream_handle()),
                   "hmc")
        torch.cuda.synchronize()
        r = ohmc.hmc_iteration(es.t, es.x, es.y, es.theta, es.subset, z0, mass, es.hyper, 0.0, 0.05, 6, 0.5, 93,
                               counter, prior_v=V)
        o = out.cpu().numpy()
        print(f"\ntree prior counter {counter}: gpu dH {o[1]:.9f} | oracle dH {r['dH']:.9f}")
        assert abs(o[1] - r["dH"]) < 1e-5
        if abs(np.log(r["u"]) + r["dH"]) > 1e-4:
            assert bool(o[0]) == r["accepted"]
        if r["accepted"]:
            np.testing.assert_allclose(z.cpu().numpy(), r["z_proposal"], atol=1e-6)


def test_hmc_step_replays_oracle_n23422(gpu):
    """Whole hmc_step iterations on the N = 23,422 workload (1,610 free rates:
    26 subset chunks, so the fused kick/drift, the per-chunk staging of the
    updated rates and the batched energy gather all run over many chunks), L =
    20, two Philox counters each, for the iid prior, the temporal trend and the
    phylogenetic prior, against the FP64 oracle's iterations stored by
    tests/golden/make_hmc_replay.py.  Compared on every counter, accepted or
    not: the end of the leapfrog path, H0, the energy change and the
    log-likelihood at the proposal; the accept decision wherever the oracle's
    log u is not within 1e-4 of -dH.

    Tolerances: the log-likelihood's target of 1e-9 relative at each end, so
    2e-9 |loglik| on dH and 1e-9 |H0| on H0; the path's end to 1e-6 (the FP32
    gradient's ~1e-7 relative error carried through 20 steps of size 0.03)."""
    import os

    import torch

    from oracle import tree as otree  # noqa: F401  (the stored file was written with it)
    from paper_2103_03348_amd import _lib

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hmc_replay_N23422.npz")
    gold = np.load(path)
    es = synth.config(3)
    plan, idx = _setup(es)
    m = es.subset.shape[0]
    eps, L, sigma = float(gold["eps"]), int(gold["L"]), float(gold["sigma"])
    mass = gold["mass"]
    z0 = gold["z0"]
    np.testing.assert_array_equal(z0, np.log(es.theta[es.subset]))
    par, ln = synth.coalescent_tree(m, seed=int(gold["tree_seed"]), scale=float(m))
    par, ln = np.ascontiguousarray(par), np.ascontiguousarray(ln)
    _lib.check(_lib.lib().hawkes_plan_set_tree(plan.handle, 2 * m - 1, par.ctypes.data_as(ctypes.c_void_p),
                                               ln.ctypes.data_as(ctypes.c_void_p), float(gold["tree_tau0"])),
               "set_tree")
    dev = "cuda:0"
    for name in ("iid", "trend", "tree"):
        for counter in (0, 1):
            key = f"{name}_{counter}"
            beta, seed = float(gold[f"{key}_beta"]), int(gold[f"{key}_seed"])
            z = torch.as_tensor(z0.copy(), device=dev)
            th = torch.as_tensor(es.theta.copy(), device=dev)
            ms = torch.as_tensor(mass, device=dev)
            out = torch.zeros(8, dtype=torch.float64, device=dev)
            zp = torch.zeros(m, dtype=torch.float64, device=dev)
            args = _lib.HmcArgs(z.data_ptr(), th.data_ptr(), ms.data_ptr(), eps, L, sigma, seed, counter, 0,
                                out.data_ptr(), beta, 1 if name == "tree" else 0, zp.data_ptr())
            hy = _lib.Hyper.of(es.hyper)
            _lib.check(_lib.lib().hmc_step(plan.handle, ctypes.byref(hy), ctypes.byref(args), _lib.stream_handle()),
                       "hmc_step")
            torch.cuda.synchronize()
            assert plan.status() == 0
            o = out.cpu().numpy()
            zpg = zp.cpu().numpy()
            dH, H0, llp = float(gold[f"{key}_dH"]), float(gold[f"{key}_H0"]), float(gold[f"{key}_loglik_proposal"])
            acc = bool(gold[f"{key}_accepted"])
            dz = float(np.max(np.abs(zpg - gold[f"{key}_z_proposal"])))
            print(f"\n{key}: dH gpu {o[1]:.9f} oracle {dH:.9f} | H0 rel {abs(o[6] - H0) / abs(H0):.2e} | "
                  f"loglik(prop) rel {abs(o[5] - llp) / abs(llp):.2e} | z_prop max abs {dz:.2e} | "
                  f"accepted gpu {int(o[0])} oracle {int(acc)}", flush=True)
            assert abs(o[1] - dH) <= 2e-9 * abs(llp)
            assert abs(o[6] - H0) <= 1e-9 * abs(H0)
            assert abs(o[5] - llp) <= 1e-9 * abs(llp)
            assert dz < 1e-6
            if abs(np.log(float(gold[f"{key}_u"])) + dH) > 1e-4:
                assert bool(o[0]) == acc
            zg = z.cpu().numpy()
            if bool(o[0]):
                np.testing.assert_array_equal(zg, zpg)
            else:
                np.testing.assert_array_equal(zg, z0)
    plan.close()
