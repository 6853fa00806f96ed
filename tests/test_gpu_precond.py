"""Learned-preconditioner kernels vs the FP64 oracle: network forward,
back-propagation, Adam; grid-count features; the exact mass update."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import features as ofeat
from oracle import hmc as ohmc
from oracle import mlp as omlp
from paper_2103_03348_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0") if dtype is None else \
        torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def test_mlp_forward_grad_adam_match_oracle(gpu):
    import torch

    from paper_2103_03348_amd import _lib

    L = _lib.lib()
    rng = np.random.default_rng(5)
    p = (omlp.init(seed=3) + 0.1 * rng.standard_normal(omlp.N_PARAMS)).astype(np.float32)
    B = 777
    X = rng.standard_normal((B, 12)).astype(np.float32)
    T = rng.standard_normal(B).astype(np.float32)
    dp, dX, dT = _t(p), _t(X), _t(T)
    y = torch.empty(B, dtype=torch.float32, device="cuda:0")
    _lib.check(L.hawkes_mlp_forward(_lib.ptr(dp), _lib.ptr(dX), B, _lib.ptr(y), _lib.stream_handle()), "fwd")
    yref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(y.cpu().numpy(), yref, rtol=1e-5, atol=1e-5)
    work = torch.empty(int(L.hawkes_mlp_workspace_floats(B)), dtype=torch.float32, device="cuda:0")
    grad = torch.empty(omlp.N_PARAMS, dtype=torch.float64, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
    _lib.check(L.hawkes_mlp_grad(_lib.ptr(dp), _lib.ptr(dX), B, None, _lib.ptr(dT), B, _lib.ptr(work),
                                 _lib.ptr(grad), _lib.ptr(loss), None, _lib.stream_handle()), "grad")
    lref, gref = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    torch.cuda.synchronize()
    assert loss.item() == pytest.approx(lref, rel=1e-5)
    g = grad.cpu().numpy()
    scale = np.abs(gref) + 1e-3 * np.abs(gref).max()
    assert np.max(np.abs(g - gref) / scale) < 1e-4
    # one Adam step from zero moments (bias-corrected first step)
    m = torch.zeros(omlp.N_PARAMS, dtype=torch.float32, device="cuda:0")
    v = torch.zeros_like(m)
    _lib.check(L.hawkes_mlp_train_step(_lib.ptr(dp), _lib.ptr(m), _lib.ptr(v), 1, ctypes.c_float(1e-3),
                                       _lib.ptr(dX), B, None, _lib.ptr(dT), B, _lib.ptr(work), _lib.ptr(grad),
                                       _lib.ptr(loss), None, _lib.stream_handle()), "train")
    pnew, _, _ = omlp.adam_step(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    np.testing.assert_allclose(dp.cpu().numpy(), pnew, rtol=1e-6, atol=2e-7)


def test_mlp_batch_rows(gpu):
    """A batch given by row indices equals the same rows passed contiguously; an
    out-of-range row index is reported, not read."""
    import torch

    from paper_2103_03348_amd import _lib

    L = _lib.lib()
    rng = np.random.default_rng(6)
    p = omlp.init(seed=4).astype(np.float32)
    X = rng.standard_normal((1000, 12)).astype(np.float32)
    T = rng.standard_normal(1000).astype(np.float32)
    rows = rng.integers(0, 1000, size=300).astype(np.int32)
    B = rows.shape[0]
    # every argument tensor stays referenced until the GPU work is done
    dp, dX, dT, drows = _t(p), _t(X), _t(T), _t(rows)
    dXr, dTr = _t(X[rows]), _t(T[rows])
    work = torch.empty(int(L.hawkes_mlp_workspace_floats(B)), dtype=torch.float32, device="cuda:0")
    g1 = torch.empty(omlp.N_PARAMS, dtype=torch.float64, device="cuda:0")
    g2 = torch.empty_like(g1)
    err = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    _lib.check(L.hawkes_mlp_grad(_lib.ptr(dp), _lib.ptr(dX), 1000, _lib.ptr(drows), _lib.ptr(dT), B,
                                 _lib.ptr(work), _lib.ptr(g1), None, _lib.ptr(err), _lib.stream_handle()), "g1")
    _lib.check(L.hawkes_mlp_grad(_lib.ptr(dp), _lib.ptr(dXr), B, None, _lib.ptr(dTr), B,
                                 _lib.ptr(work), _lib.ptr(g2), None, _lib.ptr(err), _lib.stream_handle()), "g2")
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    assert int(err.item()) == 0
    bad = rows.copy()
    bad[7] = 1000
    bad[9] = -1
    dbad = _t(bad)
    _lib.check(L.hawkes_mlp_grad(_lib.ptr(dp), _lib.ptr(dX), 1000, _lib.ptr(dbad), _lib.ptr(dT), B,
                                 _lib.ptr(work), _lib.ptr(g1), None, _lib.ptr(err), _lib.stream_handle()), "g3")
    torch.cuda.synchronize()
    assert int(err.item()) == 1


def _plan_with_subset(es):
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    idx = torch.as_tensor(es.subset, dtype=torch.int64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle()),
               "subset")
    return plan


@pytest.mark.parametrize("cfg", ["small", "n23422"])
def test_features_match_oracle(gpu, cfg):
    import torch

    from paper_2103_03348_amd import _lib

    es = synth.small(3000, seed=31, all_free=False) if cfg == "small" else synth.config(1)
    plan = _plan_with_subset(es)
    z = np.log(es.theta[es.subset])
    gx0, gy0 = float(es.x.min()) - 1e-9, float(es.y.min()) - 1e-9
    feat = torch.empty((es.subset.shape[0], 12), dtype=torch.float32, device="cuda:0")
    hy = _lib.Hyper.of(es.hyper)
    dt, dxy, dz = _t(es.t), _t(np.stack([es.x, es.y], 1)), _t(z)
    _lib.check(_lib.lib().hawkes_features(plan.handle, ctypes.byref(hy), _lib.ptr(dt), _lib.ptr(dxy), _lib.ptr(dz),
                                          gx0, gy0, _lib.ptr(feat), _lib.stream_handle()), "features")
    torch.cuda.synchronize()
    F = feat.cpu().numpy()
    sub = slice(None) if cfg == "small" else slice(0, 300)
    ref = ofeat.features(es.t, es.x, es.y, es.subset[sub], z[sub], es.hyper, es.t0, gx0, gy0)
    np.testing.assert_allclose(F[sub], ref, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("variant", ["iid", "trend", "tree"])
def test_curvature_and_mass_update_match_oracle(gpu, variant):
    """hawkes_subset_curvature: the z-space curvature theta^2 H - theta g + P
    (Eq. 4, Eq. 5 and the chain rule through theta_k = exp(z_k + beta t_k)) and
    log H, against the oracle's z_hessian_diag (itself pinned by central
    differences of the log-posterior gradient) at beta = 0, at beta != 0 and
    with the tree prior of Eq. 2 (P = diag(V^{-1}) / sigma^2 there); then the
    exact and the learned mass estimates folded by hawkes_mass_update."""
    import torch

    from oracle import tree as otree
    from paper_2103_03348_amd import _lib

    es = synth.small(1200, seed=32, all_free=False)
    plan = _plan_with_subset(es)
    m = es.subset.shape[0]
    sig = 0.5
    beta = -0.004 if variant == "trend" else 0.0
    prior = 1 if variant == "tree" else 0
    V = None
    if prior:
        par, ln = synth.coalescent_tree(m, seed=32, scale=float(m))
        par, ln = np.ascontiguousarray(par), np.ascontiguousarray(ln)
        _lib.check(_lib.lib().hawkes_plan_set_tree(plan.handle, 2 * m - 1, par.ctypes.data_as(ctypes.c_void_p),
                                                   ln.ctypes.data_as(ctypes.c_void_p), 0.8), "set_tree")
        V = otree.covariance(par, ln, 0.8)
    z = np.log(es.theta[es.subset]) + 0.1
    th = ohmc.rates(es.t, es.theta, es.subset, z, beta)
    hy = _lib.Hyper.of(es.hyper)
    dth = _t(th)
    # z recovered from the rates by the library
    dz = torch.empty(m, dtype=torch.float64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_subset_z(plan.handle, _lib.ptr(dth), beta, _lib.ptr(dz), _lib.stream_handle()),
               "subset_z")
    curv = torch.empty(m, dtype=torch.float64, device="cuda:0")
    logh = torch.empty(m, dtype=torch.float32, device="cuda:0")
    _lib.check(_lib.lib().hawkes_subset_curvature(plan.handle, ctypes.byref(hy), _lib.ptr(dth), sig, prior,
                                                  _lib.ptr(curv), _lib.ptr(logh), _lib.stream_handle()),
               "curvature")
    torch.cuda.synchronize()
    np.testing.assert_allclose(dz.cpu().numpy(), z, rtol=0, atol=1e-13)
    ref = ohmc.z_hessian_diag(es.t, es.x, es.y, es.theta, es.subset, z, es.hyper, 0.0, sig, beta=beta, prior_v=V)
    prec = ohmc.prior_precision_diag(m, sig, V)
    r = oracle.evaluate_es(es, theta=th, want=("grad_theta", "negH_theta"))
    H, g = r["negH_theta"][es.subset], r["grad_theta"][es.subset]
    tk = th[es.subset]
    # C11 scale of the chain rule's terms: theta^2 H + theta (|g| + 2 a) + P
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t[es.subset])))
    scale = tk * tk * H + tk * (np.abs(g) + 2 * a) + prec
    c = curv.cpu().numpy()
    rel = float(np.max(np.abs(c - ref) / scale))
    lh = logh.cpu().numpy().astype(np.float64)
    lh_ref = np.log(np.maximum(H, 1e-6))
    print(f"\n[{variant}] curvature rel {rel:.2e}  log H max abs {np.max(np.abs(lh - lh_ref)):.2e}", flush=True)
    assert rel < 1e-6
    # FP32 output of log H: its rounding (|log H| <= 69, 2^-24 relative) plus Eq. 5's 1e-6
    np.testing.assert_allclose(lh, lh_ref, rtol=2e-7, atol=2e-6)
    # exact estimate, floored at the prior's precision (count 0: the mass becomes it)
    mass = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_mass_update(plan.handle, ctypes.byref(hy), _lib.ptr(dth), None, sig, prior, 0,
                                             _lib.ptr(mass), _lib.stream_handle()), "mass")
    torch.cuda.synchronize()
    want = np.maximum(ref - prec, 0.0) + prec
    assert float(np.max(np.abs(mass.cpu().numpy() - want) / scale)) < 1e-6
    # learned estimate theta^2 exp(pred) + P, folded with weight 1/2 (count 1)
    pred = np.linspace(-6.0, 1.0, m).astype(np.float32)
    dpred = torch.as_tensor(pred, device="cuda:0")
    mass0 = mass.clone()
    _lib.check(_lib.lib().hawkes_mass_update(plan.handle, ctypes.byref(hy), _lib.ptr(dth), _lib.ptr(dpred), sig,
                                             prior, 1, _lib.ptr(mass), _lib.stream_handle()), "mass learned")
    torch.cuda.synchronize()
    est = tk * tk * np.exp(pred.astype(np.float64)) + prec
    np.testing.assert_allclose(mass.cpu().numpy(), 0.5 * (mass0.cpu().numpy() + est), rtol=1e-13)
    plan.close()


def test_learned_preconditioner_gain(gpu):
    """What the trained network gains over the method without it.  On Eq. 5
    diagonals (log H) collected along an HMC chain (N = 23,422, 1,610 free
    rates) and held out from training, the network's prediction must beat
    (a) its untrained self by a wide margin and (b) the best constant
    predictor (the targets' mean); and (c) at the chain's last state the
    learned mass theta^2 exp(y) + 1/sigma_z^2 must be closer to the exact mass
    theta^2 H + 1/sigma_z^2 than the unpreconditioned 1/sigma_z^2 is."""
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan
    from paper_2103_03348_amd.preconditioner import LearnedPreconditioner
    from paper_2103_03348_amd.sampler import HmcSampler

    es = synth.config(3)
    dev = "cuda:0"
    sig = 2.0
    t = torch.as_tensor(es.t, device=dev)
    xy = torch.as_tensor(np.stack([es.x, es.y], 1), device=dev).contiguous()
    plan = Plan(t, xy, es.t0)
    smp = HmcSampler(plan, torch.as_tensor(es.theta, device=dev), torch.as_tensor(es.subset, device=dev),
                     es.hyper, sigma_z=sig, L=20, seed=3)
    r = smp.run(0, 150, eps0=0.05, mass="exact", refresh=25, record=False)
    pre = LearnedPreconditioner(smp, t, xy, seed=3)
    X, T = pre.collect(60, r["eps"], thin=2)
    m = smp.m
    ntr = 48 * m                              # the last 12 states are held out
    Xtr, Ttr, Xva, Tva = X[:ntr], T[:ntr], X[ntr:], T[ntr:]
    loss0 = pre.evaluate(Xva, Tva)
    pre.train(Xtr, Ttr, steps=800, batch=4096, lr=2e-3, seed=3)
    loss1 = pre.evaluate(Xva, Tva)
    var = float(Tva.double().var().item())
    # masses at the last state (its features and targets are the last m rows)
    y = pre.predict().double().cpu().numpy()
    th = smp.theta[smp.idx].double().cpu().numpy()
    H = np.exp(T[-m:].double().cpu().numpy())
    prec = 1.0 / sig ** 2
    exact = th * th * H + prec
    err_learned = float(np.mean(np.abs(th * th * np.exp(y) + prec - exact) / exact))
    err_identity = float(np.mean(np.abs(prec - exact) / exact))
    plan.close()
    print(f"\nheld-out MSE (log H): untrained {loss0:.3e} trained {loss1:.3e} constant {var:.3e}; "
          f"mean relative mass error at the last state: learned {err_learned:.3e}, identity {err_identity:.3e}",
          flush=True)
    # log H spans about 14 units (a long tail of small entries, down to the
    # 1e-6 floor), so the untrained network's error is mostly the targets'
    # offset; the decisive checks are the constant predictor and the mass
    assert loss1 < 0.2 * loss0
    assert loss1 < 0.8 * var
    assert err_learned < err_identity
