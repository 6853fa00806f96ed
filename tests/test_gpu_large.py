"""Large workloads on the GPU: the full N = 100,000 parity, the differentiable
log-likelihood (torch.autograd.Function with the hand-written backward) checked
against the oracle and against central finite differences, and sampled parity
at N = 250,000.

Finite differences: for a rate theta_m the log-likelihood restricted to that
coordinate is
    f(s) = sum_n log(lambda_n + (s - theta_m) c_e E_nm [t_m < t_n])
           - Lambda - theta0 (s - theta_m)(1 - exp(-omega (T1 - t_m))),
exact because lambda and Lambda are linear in theta_m.  Its central difference
(step 1e-6, FP64) is formed term by term from the oracle's lambda_n and FP64
pair terms, so the difference does not drown in the rounding of the total.
"""
import numpy as np
import pytest

import oracle
from paper_2103_03348_amd import synth

from gpu_helpers import errors, h_rel_all, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def n100k():
    es = synth.config(2)
    print(f"\n[N=100,000] oracle evaluation ({oracle.max_threads()} threads) ...", flush=True)
    ref = oracle.evaluate_es(es)
    return es, ref


def test_n100k_parity(gpu, n100k):
    es, ref = n100k
    g = run_gpu(es)
    e = errors(es, g, ref)
    print("\n[N=100,000] " + " ".join(f"{k}={np.max(v):.3e}" for k, v in e.items()), flush=True)
    assert g["status"] == 0
    assert e["loglik_rel"] < 1e-9
    assert e["lam_rel"] < 2e-6
    assert e["g_rel"] < 1e-6
    assert e["h_rel_all"] < 1e-6
    assert e["h_rel_norm"] < 1e-6
    hy = np.asarray(es.hyper)
    assert np.all(e["gh_abs"] / np.maximum(np.abs(ref["grad_hyper"]), es.n / hy) < 1e-6)
    assert np.all(e["Hh_abs"] / np.maximum(np.abs(ref["negH_hyper"]), es.n / hy ** 2) < 1e-6)


def test_subset_path_n100k(gpu, n100k):
    """The O(N M) free-rate path at N = 100,000 (6,874 free rates): here its
    schedules split the subset passes into multi-batch items (column items of
    the maximum 16 row chunks, row items of several 64-entry batches); Eq. 1,
    4 and 5 on the subset against the oracle's full evaluation."""
    import ctypes

    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es, ref = n100k
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    idx = torch.as_tensor(es.subset, dtype=torch.int64, device="cuda:0")
    _lib.check(_lib.lib().hawkes_plan_set_subset(plan.handle, idx.numel(), _lib.ptr(idx), _lib.stream_handle()),
               "set_subset")
    m = es.subset.shape[0]
    th = torch.as_tensor(es.theta, device="cuda:0")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    h = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    hy = _lib.Hyper.of(es.hyper)
    _lib.check(_lib.lib().hawkes_subset_grad(plan.handle, ctypes.byref(hy), _lib.ptr(th), 0, _lib.ptr(ll),
                                             _lib.ptr(g), _lib.ptr(h), _lib.stream_handle()), "subset_grad")
    torch.cuda.synchronize()
    assert plan.status() == 0
    g, h = g.cpu().numpy(), h.cpu().numpy()
    gi = ref["grad_theta"][es.subset]
    hi = ref["negH_theta"][es.subset]
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t[es.subset])))
    rel_l = abs(float(ll.item()) - ref["loglik"]) / abs(ref["loglik"])
    rel_g = np.max(np.abs(g - gi) / np.maximum(gi + 2 * a, 1e-300))
    rel_h = h_rel_all(h, hi)
    print(f"\n[subset N=100,000 m={m}] loglik {rel_l:.2e} g {rel_g:.2e} H {rel_h:.2e}", flush=True)
    assert rel_l < 1e-9
    assert rel_g < 1e-6
    assert rel_h < 1e-6
    plan.close()


def _fd_rate(es, lam, m, step=1e-6):
    """Central difference of f(s) above at s = theta_m, term by term."""
    mu0, tau_x, tau_t, theta0, omega, h = es.hyper
    c_e = theta0 * omega / (2.0 * np.pi * h * h)
    later = es.t > es.t[m]
    dt = es.t[later] - es.t[m]
    r2 = (es.x[later] - es.x[m]) ** 2 + (es.y[later] - es.y[m]) ** 2
    q = c_e * np.exp(-omega * dt - r2 / (2.0 * h * h)) / lam[later]
    d_sum = np.sum(np.log1p(step * q) - np.log1p(-step * q))
    d_int = 2.0 * step * theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t[m])))
    return (d_sum - d_int) / (2.0 * step)


def test_autograd_backward_n100k(gpu, n100k):
    import torch

    from paper_2103_03348_amd import autograd
    from paper_2103_03348_amd.hawkes import Plan

    es, ref = n100k
    dev = "cuda:0"
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0, device=dev)
    theta = torch.as_tensor(es.theta, device=dev).requires_grad_(True)
    hyper = torch.tensor(es.hyper, dtype=torch.float64, requires_grad=True)
    ll = autograd.loglik(theta, hyper, plan)
    ll.backward()
    torch.cuda.synchronize()
    assert plan.status() == 0
    gt = theta.grad.cpu().numpy()
    gh = hyper.grad.numpy()
    a = es.hyper[3] * (1.0 - np.exp(-es.hyper[4] * (es.t.max() - es.t)))
    scale = np.maximum(a + (ref["grad_theta"] + a), 1e-300)  # 0 for the last event (no later event)
    rel_l = abs(float(ll.item()) - ref["loglik"]) / abs(ref["loglik"])
    rel_g = np.max(np.abs(gt - ref["grad_theta"]) / scale)
    rel_h = np.max(np.abs(gh - ref["grad_hyper"]) / np.maximum(np.abs(ref["grad_hyper"]), es.n / np.asarray(es.hyper)))
    # central finite differences on 50 random rate coordinates (FP64, step 1e-6)
    rng = np.random.default_rng(2024)
    coords = rng.choice(es.n, size=50, replace=False)
    fd = np.array([_fd_rate(es, ref["lam"], m) for m in coords])
    rel_fd_oracle = np.max(np.abs(fd - ref["grad_theta"][coords]) / scale[coords])
    rel_fd_gpu = np.max(np.abs(fd - gt[coords]) / scale[coords])
    print(f"\n[autograd N=100,000] loglik {rel_l:.2e} grad_theta {rel_g:.2e} grad_hyper {rel_h:.2e} "
          f"FD vs oracle {rel_fd_oracle:.2e} FD vs GPU {rel_fd_gpu:.2e}", flush=True)
    assert rel_l < 1e-9
    assert rel_g < 1e-6
    assert rel_h < 1e-6
    assert rel_fd_oracle < 1e-8   # pins the oracle's Eq. 4 at this size
    assert rel_fd_gpu < 1e-6

    # a backward after the plan has evaluated something else recomputes the
    # intensities (stale forward).  That evaluation asks for the rate gradient
    # alone and so takes the log-likelihood-only row pass, whose intensities
    # are rounded differently from the forward's (its FP32 exponent constants
    # are completed inside the pair loop rather than through the first
    # moments): the gradient is held to the oracle at the same bar.
    theta2 = torch.as_tensor(es.theta, device=dev).requires_grad_(True)
    ll2 = autograd.loglik(theta2, hyper.detach(), plan)
    plan.eval(torch.ones(es.n, dtype=torch.float64, device=dev), es.hyper, loglik=True)
    ll2.backward()
    torch.cuda.synchronize()
    g2 = theta2.grad.cpu().numpy()
    rel_g2 = np.max(np.abs(g2 - ref["grad_theta"]) / scale)
    print(f"[autograd N=100,000] stale-forward backward: grad_theta {rel_g2:.2e}", flush=True)
    assert rel_g2 < 1e-6
    assert np.max(np.abs(g2 - gt) / scale) < 2e-6
    plan.close()


def test_sampled_parity_n250k(gpu):
    """N = 250,000: the GPU's lambda on a block of rows and its Eq. 4 / Eq. 5 on
    the columns of a time window, against the oracle row sums for those rows.
    Columns only need the intensities of events within 80 time units after
    them: exp(-omega * 80) = 4e-18 at omega = 0.5."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    es = synth.config(4)
    n = es.n
    dev = "cuda:0"
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0, device=dev)
    th = torch.as_tensor(es.theta, device=dev)
    out = plan.eval(th, es.hyper, loglik=True, grad_theta=True, grad_hyper=True, negH_theta=True,
                    negH_hyper=True)
    lam_g = plan.lam().cpu().numpy()
    g_g = out["grad_theta"].cpu().numpy()
    h_g = out["negH_theta"].cpu().numpy()
    ll_g = float(out["loglik"].item())
    assert plan.status() == 0 and np.isfinite(ll_g)
    plan.close()

    order = np.argsort(es.t, kind="stable")
    mu0, tau_x, tau_t, theta0, omega, h = es.hyper
    c_b, c_e = oracle.constants(es.hyper)
    start = n // 3
    cols = order[start:start + 256]                       # 256 consecutive events in time
    t_hi = es.t[cols].max() + 80.0
    rows = order[start:np.searchsorted(es.t[order], t_hi, side="right")]
    print(f"\n[N=250,000] oracle row sums for {rows.size} rows ...", flush=True)
    acc = oracle.row_sums(es.t, es.x, es.y, es.theta, es.hyper, rows=rows)
    lam_o = c_b * acc[:, 0] + c_e * acc[:, 5]
    lam_rel = np.max(np.abs(lam_g[rows] - lam_o) / lam_o)
    lam_full = np.full(n, np.inf)
    lam_full[rows] = lam_o
    G = np.zeros(cols.size)
    H = np.zeros(cols.size)
    for k, j in enumerate(cols):
        sel = rows[es.t[rows] > es.t[j]]
        dt = es.t[sel] - es.t[j]
        r2 = (es.x[sel] - es.x[j]) ** 2 + (es.y[sel] - es.y[j]) ** 2
        q = c_e * np.exp(-omega * dt - r2 / (2.0 * h * h)) / lam_full[sel]
        G[k] = q.sum()
        H[k] = (q * q).sum()
    a = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t[cols])))
    g_rel = np.max(np.abs(g_g[cols] - (G - a)) / (G + a))
    h_rel = h_rel_all(h_g[cols], H)
    print(f"[N=250,000] lambda {lam_rel:.2e} (rows {rows.size}) g {g_rel:.2e} H {h_rel:.2e} (cols {cols.size})",
          flush=True)
    assert lam_rel < 2e-6
    assert g_rel < 1e-6
    assert h_rel < 1e-6


def test_full_parity_n250k(gpu):
    """N = 250,000: every output of one full evaluation -- loglik, lambda,
    Eq. 4, Eq. 5 and the hyperparameter gradient and Hessian -- against one
    full FP64 oracle evaluation of the same workload, stored by
    tests/golden/make_n250k.py (the oracle needs minutes at this size)."""
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_N250000.npz")
    ref = dict(np.load(path))
    es = synth.config(4)
    assert int(ref["n"]) == es.n
    assert float(ref["t_checksum"]) == float(np.sum(es.t)) and float(ref["x_checksum"]) == float(np.sum(es.x))
    ref["loglik"] = float(ref["loglik"])
    # the integral term per event is not stored; errors() needs it only for a report
    ref["Lam_n"] = np.zeros(es.n)
    g = run_gpu(es)
    e = errors(es, g, ref)
    print("\n[N=250,000 full] " + " ".join(f"{k}={np.max(v):.3e}" for k, v in e.items() if k != "loglik_mag"),
          flush=True)
    assert g["status"] == 0
    assert e["loglik_rel"] < 1e-9
    assert e["lam_rel"] < 2e-6
    assert e["g_rel"] < 1e-6
    assert e["h_rel_all"] < 1e-6
    assert e["h_rel_norm"] < 1e-6
    hy = np.asarray(es.hyper)
    assert np.all(e["gh_abs"] / np.maximum(np.abs(ref["grad_hyper"]), es.n / hy) < 1e-6)
    assert np.all(e["Hh_abs"] / np.maximum(np.abs(ref["negH_hyper"]), es.n / hy ** 2) < 1e-6)
