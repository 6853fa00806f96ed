"""Seeded random configurations against the FP64 oracle (Eq. 1, 4, 5 and the
hyperparameter derivatives): event counts, time spans, cluster counts and all
six hyperparameters drawn over wide ranges, so that the pair passes' forms
(split or precise, expanded or difference spatial exponent), the subset
path's split and unsplit batches, and the finalisation's FP64 recomputation of
low intensities are all met in combinations the fixed cases do not pin down.

Bounds as in the other parity tests: lambda 2e-6 relative, loglik 2e-6 N
absolute (on the larger sets 1e-9 of sum_i |log lambda_i| + Lambda, the
magnitude of its terms), Eq. 4 1e-6 of its two terms' magnitude, Eq. 5 1e-6 relative on every entry (floor 1e-30) and norm-wise;
the hyperparameter derivatives 1e-6 of the larger of the usual scale and the
summed magnitudes of their per-event terms (which cancel on sparse sets)."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_2103_03348_amd import synth

from gpu_helpers import errors, h_rel_all, hyper_magnitudes, run_gpu

pytestmark = pytest.mark.gpu


def _config(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(200, 3000))
    per_event = float(np.exp(rng.uniform(np.log(0.01), np.log(50.0))))
    k = int(rng.integers(1, 9))
    lo = np.log([0.1, 0.1, 0.1, 0.01, 0.01, 0.05])
    hi = np.log([5.0, 10.0, 50.0, 2.0, 10.0, 5.0])
    hyper = tuple(float(v) for v in np.exp(rng.uniform(lo, hi)))
    es = synth.uniform_mixture(n, t_end=per_event * n, k=k, seed=2000 + seed, hyper=hyper, all_free=False,
                               name=f"random{seed}")
    return es


@pytest.mark.parametrize("seed", range(12))
def test_random_configuration_matches_oracle(gpu, seed):
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es = _config(seed)
    ref = oracle.evaluate_es(es)
    print(f"\n[random {seed}] n={es.n} t_end={es.t.max():.3g} hyper={np.round(es.hyper, 4)} "
          f"min lambda={ref['lam'].min():.3e}", flush=True)
    g = run_gpu(es)
    if not np.isfinite(ref["loglik"]):
        # some lambda_i is 0 in FP64 as well: flagged, loglik -inf
        assert g["status"] == 2 and g["loglik"] == -np.inf
        return
    e = errors(es, g, ref)
    print(" ".join(f"{k}={np.max(v):.3e}" for k, v in e.items()), flush=True)
    assert g["status"] == 0
    if es.n >= 1000 and ref["lam"].min() > 1e-30:
        # relative to the magnitude of loglik's terms: on some draws
        # sum_i log lambda_i and the integral nearly cancel (config 4: loglik
        # -1,310 from terms of magnitude ~2,800)
        assert e["loglik_mag"] < 1e-9
    else:
        assert abs(g["loglik"] - ref["loglik"]) <= 2e-6 * es.n
    assert e["lam_rel"] < 2e-6
    assert e["g_rel"] < 1e-6
    assert e["h_rel_all"] < 1e-6
    assert e["h_rel_norm"] < 1e-6
    hy = np.asarray(es.hyper)
    g_mag, h_mag = hyper_magnitudes(es)
    gscale = np.maximum(np.maximum(np.abs(ref["grad_hyper"]), es.n / hy), g_mag)
    hscale = np.maximum(np.maximum(np.abs(ref["negH_hyper"]), es.n / hy ** 2), h_mag)
    assert np.all(e["gh_abs"] / gscale < 1e-6), e["gh_abs"] / gscale
    assert np.all(e["Hh_abs"] / hscale < 1e-6), e["Hh_abs"] / hscale

    # Eq. 4 alone, and the subset path (Eq. 1, 4, 5 on the free rates)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    out = plan.eval(th, es.hyper, loglik=True, grad_theta=True)
    g_only = out["grad_theta"].cpu().numpy()
    theta0, omega = es.hyper[3], es.hyper[4]
    a = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t)))
    scale = np.maximum(a + (ref["grad_theta"] + a), 1e-300)
    assert np.max(np.abs(g_only - ref["grad_theta"]) / scale) < 1e-6
    idx = torch.as_tensor(es.subset, dtype=torch.int64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle()),
               "set_subset")
    m = es.subset.shape[0]
    ll = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    gs = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    hs = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    hyc = _lib.Hyper.of(es.hyper)
    _lib.check(_lib.lib().hawkes_subset_grad(plan.handle, ctypes.byref(hyc), _lib.ptr(th), 0, _lib.ptr(ll),
                                             _lib.ptr(gs), _lib.ptr(hs), _lib.stream_handle()), "subset_grad")
    torch.cuda.synchronize()
    assert plan.status() == 0
    plan.close()
    sub = es.subset
    assert abs(float(ll.item()) - ref["loglik"]) <= 2e-6 * es.n
    assert np.max(np.abs(gs.cpu().numpy() - ref["grad_theta"][sub]) / scale[sub]) < 1e-6
    assert h_rel_all(hs.cpu().numpy(), ref["negH_theta"][sub]) < 1e-6
