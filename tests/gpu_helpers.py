"""Shared helpers of the GPU parity tests: run the library and the oracle on the
same seeded event set and report errors in the metrics the tolerances use."""
from __future__ import annotations

import numpy as np


def run_gpu(es, want_all=True, theta=None, hyper=None):
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    dev = "cuda:0"
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0, device=dev)
    th = torch.as_tensor(es.theta if theta is None else theta, device=dev)
    hy = es.hyper if hyper is None else hyper
    out = plan.eval(th, hy, loglik=True, grad_theta=want_all, grad_hyper=want_all, negH_theta=want_all,
                    negH_hyper=want_all)
    lam = plan.lam()
    torch.cuda.synchronize()
    st = plan.status()
    res = {k: (v.cpu().numpy() if v.numel() > 1 else float(v.item())) for k, v in out.items()}
    res["lam"] = lam.cpu().numpy()
    res["status"] = st
    plan.close()
    return res


# Eq. 5's terms are squared in FP32: a square below ~1e-45 is zero there and
# one below ~1e-38 keeps few bits, so entries are compared relative to
# H_j + H_FLOOR (an entry below the floor only needs to be tiny in absolute terms).
H_FLOOR = 1e-30


def h_rel_all(h_gpu, h_ref):
    """max_j |dH_j| / (H_j + H_FLOOR): Eq. 5's terms are all positive, so every
    entry is held to a plain relative bound down to the FP32 underflow floor."""
    h_gpu = np.asarray(h_gpu)
    h_ref = np.asarray(h_ref)
    if h_ref.size == 0:
        return 0.0
    return float(np.max(np.abs(h_gpu - h_ref) / (h_ref + H_FLOOR)))


def errors(es, gpu, ref):
    """Error metrics:
      loglik_rel : |dl| / |l|
      loglik_mag : |dl| / (sum_i |log lambda_i| + Lambda)
      lam_rel    : max_i |dlambda_i| / lambda_i
      g_rel      : max_j |dg_j| / (a_j + sum_i c_e E_ij / lambda_i)   (Eq. 4's two terms)
      h_rel_all  : max_j |dH_j| / (H_j + H_FLOOR) over every entry (see h_rel_all)
      gh_rel     : per hyperparameter |dg_p| / max(|g_p|, scale_p)
    """
    out = {}
    l_ref = ref["loglik"]
    out["loglik_rel"] = abs(gpu["loglik"] - l_ref) / abs(l_ref)
    mag = np.sum(np.abs(np.log(ref["lam"]))) + np.sum(ref["Lam_n"])
    out["loglik_mag"] = abs(gpu["loglik"] - l_ref) / mag
    rel = (gpu["lam"] - ref["lam"]) / ref["lam"]
    out["lam_rel"] = float(np.max(np.abs(rel)))
    out["lam_bias"] = float(np.mean(rel))
    if "grad_theta" in gpu:
        theta0, omega = es.hyper[3], es.hyper[4]
        a = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t)))
        scale = a + (ref["grad_theta"] + a)
        out["g_rel"] = float(np.max(np.abs(gpu["grad_theta"] - ref["grad_theta"]) / np.maximum(scale, 1e-300)))
        H = ref["negH_theta"]
        pos = H > 0
        out["h_rel_all"] = h_rel_all(gpu["negH_theta"], H)
        out["h_rel_norm"] = float(np.linalg.norm(gpu["negH_theta"] - H) / max(np.linalg.norm(H), 1e-300))
        out["h_zero_abs"] = float(np.max(np.abs(gpu["negH_theta"][~pos]))) if (~pos).any() else 0.0
        out["gh_abs"] = np.abs(gpu["grad_hyper"] - ref["grad_hyper"])
        out["Hh_abs"] = np.abs(gpu["negH_hyper"] - ref["negH_hyper"])
    return out


def hyper_magnitudes(es):
    """Per hyperparameter, sum_i |lambda'_i| / lambda_i and
    sum_i |lambda''_i| / lambda_i + (lambda'_i / lambda_i)^2: the magnitudes of
    the per-event terms whose sums are the likelihood parts of the
    hyperparameter gradient and Hessian diagonal, from the oracle's per-event
    pair sums and the derivatives of lambda_i in the six hyperparameters."""
    import oracle

    mu0, tx, tt, th0, om, h = [float(v) for v in es.hyper]
    cb, ce = oracle.constants(es.hyper)
    S = oracle.row_sums(es.t, es.x, es.y, es.theta, es.hyper)
    B0, B1, B2, B11, B22, X0, X1, X2, X11, X22 = S.T
    lam = cb * B0 + ce * X0
    d1 = [cb * B0 / mu0, cb * (-2 * B0 / tx + B1 / tx ** 3), cb * (-B0 / tt + B2 / tt ** 3),
          ce * X0 / th0, ce * (X0 / om - X1), ce * (-2 * X0 / h + X2 / h ** 3)]
    d2 = [0.0 * B0, cb * (6 * B0 / tx ** 2 - 7 * B1 / tx ** 4 + B11 / tx ** 6),
          cb * (2 * B0 / tt ** 2 - 5 * B2 / tt ** 4 + B22 / tt ** 6), 0.0 * X0, ce * (X11 - 2 * X1 / om),
          ce * (6 * X0 / h ** 2 - 7 * X2 / h ** 4 + X22 / h ** 6)]
    g_mag = np.array([np.sum(np.abs(d1[p]) / lam) for p in range(6)])
    h_mag = np.array([np.sum(np.abs(d2[p]) / lam + (d1[p] / lam) ** 2) for p in range(6)])
    return g_mag, h_mag


def hyper_hessian_magnitude(es):
    """The Hessian part of hyper_magnitudes."""
    return hyper_magnitudes(es)[1]
