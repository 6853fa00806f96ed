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
