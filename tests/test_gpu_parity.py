"""GPU library vs FP64 oracle, element by element, on seeded inputs.

Tolerances (FP32 pair arithmetic, compensated sums, FP64 finals):
  * log-likelihood: 1e-9 relative (the stated target) on the workloads; on
    sets of a few hundred events the FP32 errors of the individual lambda_i do
    not average out, so there the bound is the sum of the per-event bounds:
    |dl| <= 2e-6 * N (the lambda tolerance below, summed).
  * lambda_i: 2e-6 relative (a sum of FP32 terms with ~1e-7 error each, bounded
    with margin for sets where one term dominates).
  * rate gradient: 1e-6 relative to the magnitude of Eq. 4's two terms.
  * Hessian diagonal: 1e-6 relative (all terms positive) on every entry, with
    an absolute floor of 1e-30 where Eq. 5's squared FP32 terms underflow, and
    1e-6 norm-wise.  The column pass forms each term's whole exponent in FP64
    and rounds only its fractional part to FP32, so a term's relative error
    does not grow with the size of its exponent.
  * sparse data (chunks of 64 events spanning more than tau_t/2 in time), where
    the row pass takes its precise form (FP64 time differences, whole
    exponents in FP64 with an exact power of two): the same bounds.
  * hyperparameter derivatives on sets below 256 events: 1e-5 instead of 1e-6
    (a handful of FP32 terms carry each sum without averaging, and the second
    derivatives in tau_x and h cancel three such sums).
  * hyperparameter gradient / Hessian: 1e-6 relative to max(|value|, N/p) --
    their per-event terms are O(1/p), so N/p is the size of the sums that cancel.
"""
import numpy as np
import pytest

import oracle
from paper_2103_03348_amd import synth

from gpu_helpers import errors, hyper_hessian_magnitude, run_gpu

pytestmark = pytest.mark.gpu

SMALL = [
    (2, 1, 0, 0), (3, 2, 0, 0), (5, 3, 1, 0), (63, 4, 2, 1), (64, 5, 0, 0), (65, 6, 3, 2),
    (255, 7, 4, 0), (256, 8, 0, 3), (257, 9, 6, 0), (700, 10, 5, 5), (1111, 11, 9, 4),
]


def _check(es, gpu, ref, l_tol=1e-9, tiny=False, hh_mag=None):
    e = errors(es, gpu, ref)
    print(f"\n[{es.name} n={es.n}] " + " ".join(
        f"{k}={v:.3e}" if np.isscalar(v) else f"{k}={np.max(v):.3e}" for k, v in e.items()), flush=True)
    assert gpu["status"] == 0
    if tiny:
        assert abs(gpu["loglik"] - ref["loglik"]) <= 2e-6 * es.n
    else:
        assert e["loglik_rel"] < l_tol
    assert e["lam_rel"] < 2e-6
    assert e["g_rel"] < 1e-6
    assert e["h_rel_all"] < 1e-6
    assert e["h_rel_norm"] < 1e-6
    n = es.n
    hy = np.asarray(es.hyper)
    gscale = np.maximum(np.abs(ref["grad_hyper"]), n / hy)
    hscale = np.maximum(np.abs(ref["negH_hyper"]), n / hy ** 2)
    if hh_mag is not None:
        hscale = np.maximum(hscale, hh_mag)
    htol = 1e-6 if n >= 256 else 1e-5
    assert np.all(e["gh_abs"] / gscale < htol), e["gh_abs"] / gscale
    assert np.all(e["Hh_abs"] / hscale < htol), e["Hh_abs"] / hscale


@pytest.mark.parametrize("n,seed,ties,dup", SMALL)
def test_small_ragged(gpu, n, seed, ties, dup):
    es = synth.small(n, seed=seed, ties=ties, dup_xy=dup)
    gpu_r = run_gpu(es)
    ref = oracle.evaluate_es(es)
    _check(es, gpu_r, ref, tiny=True)


@pytest.mark.parametrize("n,seed,per_event", [(300, 31, 3.0), (700, 32, 3.0), (2000, 33, 1.2)])
def test_sparse_fallback(gpu, n, seed, per_event):
    """Chunks that span more than tau_t/2 in time take the row pass's precise
    form (every chunk of these sets); at 3 time units per event every chunk
    also spans more than the split limit 40/omega, at 1.2 about a third of
    them, where the split factors carried by step factors restart."""
    es = synth.small(n, seed=seed, t_end=per_event * n, ties=2)
    g = run_gpu(es)
    ref = oracle.evaluate_es(es)
    e = errors(es, g, ref)
    print(f"\n[sparse n={n}] " + " ".join(f"{k}={np.max(v):.3e}" for k, v in e.items()), flush=True)
    assert g["status"] == 0
    assert abs(g["loglik"] - ref["loglik"]) <= 2e-6 * es.n
    assert e["lam_rel"] < 2e-6
    assert e["g_rel"] < 1e-6
    assert e["h_rel_norm"] < 1e-6
    # every entry, also the tiny ones of events whose later events are all far
    assert e["h_rel_all"] < 1e-6


@pytest.mark.parametrize("shift", [800.0, 3000.0])
def test_wide_domain_difference_form(gpu, shift):
    """A domain thousands of bandwidths wide.  The column passes expand
    -|u_i - u_j|^2 as 2 u_i.u_j - |u_i|^2 - |u_j|^2 only while every |u|^2 is
    small enough for the cancellation to be harmless (|u| <= 512 with
    u = x / (h sqrt(2 ln 2)), i.e. half the domain's side at most ~603 h);
    here they form the differences.  Half of the events are moved `shift`
    units away, so that the half side W is about 1,400 h and 5,000 h: the
    coordinates must keep their FP64 resolution (a term's relative error from
    rounding them to a grid of spacing W 2^-30 would be ~(d/h)(W/h) 2^-31)."""
    base = synth.small(1500, seed=41)
    rng = np.random.default_rng(41)
    far = rng.random(base.n) < 0.5
    x = base.x + np.where(far, shift, 0.0)
    es = synth.EventSet(base.t, x, base.y, base.theta, base.subset, base.z, base.hyper, base.t0, "wide")
    half = 0.5 * max(np.ptp(es.x), np.ptp(es.y))
    h = es.hyper[5]
    assert half > 512.0 * np.sqrt(2.0 * np.log(2.0)) * h
    _check(es, run_gpu(es), oracle.evaluate_es(es), tiny=True)


def test_workload_n1000(gpu):
    es = synth.config(0)
    _check(es, run_gpu(es), oracle.evaluate_es(es))


def test_workload_n23422(gpu):
    es = synth.config(1)
    _check(es, run_gpu(es), oracle.evaluate_es(es))


def test_single_event_zero_intensity(gpu):
    """A lone event has no other event to excite it or to carry background: lambda = 0,
    loglik = -inf and the sticky status says so."""
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    plan = Plan.from_numpy([1.5], [0.25], [-0.5], 0.0)
    th = torch.ones(1, dtype=torch.float64, device="cuda:0")
    out = plan.eval(th, synth.HYPER_DEFAULT)
    torch.cuda.synchronize()
    assert out["loglik"].item() == -np.inf
    assert plan.status() == _lib.E_ZERO_INTENSITY
    assert plan.status() == 0  # cleared


def test_invalid_arguments(gpu):
    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es = synth.small(50, seed=3)
    plan = Plan.from_numpy(es.t, es.x, es.y, 0.0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    with pytest.raises(_lib.HawkesError):
        plan.eval(th, (0.7, -2.0, 5.0, 0.3, 0.5, 0.3))
    with pytest.raises(_lib.HawkesError):
        Plan.from_numpy(es.t, es.x, es.y, t_start=es.t.min() + 1.0)
    # an empty event set and non-finite inputs are argument errors
    with pytest.raises(_lib.HawkesError):
        Plan.from_numpy(np.zeros(0), np.zeros(0), np.zeros(0), 0.0)
    x_nan = es.x.copy()
    x_nan[7] = np.nan
    with pytest.raises(_lib.HawkesError):
        Plan.from_numpy(es.t, x_nan, es.y, 0.0)
    t_inf = es.t.copy()
    t_inf[11] = np.inf
    with pytest.raises(_lib.HawkesError):
        Plan.from_numpy(t_inf, es.x, es.y, 0.0)
    bad = th.clone()
    bad[3] = -1.0
    plan.eval(bad, es.hyper)
    assert plan.status() == _lib.E_INVALID


def test_determinism(gpu):
    """Fixed-order reductions: two evaluations are bitwise equal."""
    es = synth.small(3000, seed=12, ties=7)
    a = run_gpu(es)
    b = run_gpu(es)
    for k in ("loglik", "grad_theta", "negH_theta", "grad_hyper", "negH_hyper", "lam"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_pass_timing_samples_evaluations(gpu):
    """hawkes_profile_enable(p, k) records HIP events around the passes of the
    first evaluation and every k-th after it only; 0 discards."""
    import ctypes

    import torch

    from paper_2103_03348_amd import _lib
    from paper_2103_03348_amd.hawkes import Plan

    es = synth.small(500, seed=13)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    lib = _lib.lib()
    assert lib.hawkes_profile_enable(plan.handle, -1) == _lib.E_INVALID
    _lib.check(lib.hawkes_profile_enable(plan.handle, 3), "profile_enable")
    for _ in range(7):
        plan.eval(th, es.hyper, loglik=True, grad_theta=True)
    out = (ctypes.c_double * 6)()
    _lib.check(lib.hawkes_profile_read(plan.handle, out), "profile_read")
    # evaluations 1, 4 and 7 of seven: row pass, column pass, whole evaluation
    assert [out[1], out[3], out[5]] == [3.0, 3.0, 3.0]
    assert all(out[2 * k] > 0.0 for k in range(3))
    _lib.check(lib.hawkes_profile_enable(plan.handle, 0), "profile_disable")
    plan.eval(th, es.hyper, loglik=True)
    _lib.check(lib.hawkes_profile_read(plan.handle, out), "profile_read")
    assert [out[1], out[3], out[5]] == [0.0, 0.0, 0.0]
    torch.cuda.synchronize()
    plan.close()


def test_permutation_invariance(gpu):
    """Inputs are re-sorted inside the library: a permuted caller order gives the same
    loglik and permuted outputs."""
    es = synth.small(2000, seed=13, ties=10)
    perm = np.random.default_rng(0).permutation(es.n)
    es2 = synth.EventSet(es.t[perm], es.x[perm], es.y[perm], es.theta[perm], es.subset, es.z, es.hyper)
    a = run_gpu(es)
    b = run_gpu(es2)
    # tied events keep the caller's order, so a permutation can reorder ties and
    # with them the FP32 summation order: equal to rounding, not bitwise
    assert b["loglik"] == pytest.approx(a["loglik"], rel=1e-11)
    # Eq. 4 is a difference of two positive terms: held, as in the oracle
    # comparisons, relative to their magnitude (an entry where they nearly cancel
    # moves by an FP32 rounding of the terms, not of the difference)
    theta0, omega = es.hyper[3], es.hyper[4]
    a_int = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t)))
    g_scale = np.maximum(a_int + (a["grad_theta"] + a_int), 1e-300)
    assert np.max(np.abs(b["grad_theta"] - a["grad_theta"][perm]) / g_scale[perm]) < 1e-6
    np.testing.assert_allclose(b["negH_theta"], a["negH_theta"][perm], rtol=1e-6, atol=1e-12)


def test_exact_power_of_two_rescaling(gpu):
    """x, tau_x, h doubled: the pre-scaled coordinates and every FP32 exponent
    argument are bit-identical, so loglik drops by exactly 2 N ln 2 (to FP64 rounding)."""
    es = synth.small(1500, seed=14)
    mu0, tau_x, tau_t, theta0, omega, h = es.hyper
    a = run_gpu(es)
    es2 = synth.EventSet(es.t, 2 * es.x, 2 * es.y, es.theta, es.subset, es.z,
                         (mu0, 2 * tau_x, tau_t, theta0, omega, 2 * h))
    b = run_gpu(es2)
    assert b["loglik"] == pytest.approx(a["loglik"] - 2 * es.n * np.log(2.0), rel=1e-13, abs=1e-9)


def test_exp2_bias_matches_library_constant(gpu):
    """The library divides its FP64 normalisers by (1 + b) with b the mean relative
    error of the hardware exp2.  Re-measure b on this GPU over 2^27 arguments spread
    over the exponent range the pair terms use and check the constant."""
    import ctypes

    import torch

    from paper_2103_03348_amd import _lib

    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    for lo, hi in ((-1.0, 0.0), (-40.0, 0.0), (-126.0, 0.0)):
        _lib.check(_lib.lib().hawkes_exp2_bias(1 << 27, lo, hi, _lib.ptr(out), _lib.stream_handle()), "exp2_bias")
        torch.cuda.synchronize()
        mean, mean_abs, _ = out.cpu().numpy()
        const = _lib.lib().hawkes_exp2_bias_constant()
        print(f"\nexp2 over [{lo},{hi}): mean rel {mean:.4e}, mean |rel| {mean_abs:.4e}, library {const:.4e}")
        assert abs(mean - const) < 4e-10


def test_loglik_only_n23422(gpu):
    """The log-likelihood-only row pass (no moments; scaled times, so the
    background exponent carries no rounded constant, and the excitation ratio
    completed by its low part inside an FMA)."""
    es = synth.config(1)
    g = run_gpu(es, want_all=False)
    ref = oracle.evaluate_es(es, want=("loglik", "lam", "Lam_n"))
    rel = abs(g["loglik"] - ref["loglik"]) / abs(ref["loglik"])
    print(f"\nloglik-only n={es.n}: rel {rel:.3e}")
    assert g["status"] == 0
    assert rel < 1e-9
    assert np.max(np.abs(g["lam"] - ref["lam"]) / ref["lam"]) < 2e-6


@pytest.mark.parametrize("n,seed,per_event", [(700, 32, 3.0), (2000, 33, 1.2)])
def test_loglik_only_sparse(gpu, n, seed, per_event):
    """The log-likelihood-only row pass on sparse data, where chunks take the
    precise form (FP64 time differences, whole exponents with the exact
    excitation ratio kex / kbx in FP64): lambda to the same bound, loglik to
    the per-event bound of small sets."""
    es = synth.small(n, seed=seed, t_end=per_event * n, ties=2)
    g = run_gpu(es, want_all=False)
    ref = oracle.evaluate_es(es, want=("loglik", "lam", "Lam_n"))
    lam_rel = np.max(np.abs(g["lam"] - ref["lam"]) / ref["lam"])
    print(f"\nloglik-only sparse n={es.n}: dl {abs(g['loglik'] - ref['loglik']):.3e} lam {lam_rel:.3e}")
    assert g["status"] == 0
    assert abs(g["loglik"] - ref["loglik"]) <= 2e-6 * es.n
    assert lam_rel < 2e-6


@pytest.mark.parametrize("cfg", [1, 4])
def test_underflow_cutoff_changes_nothing(gpu, cfg):
    """The optional cutoff skips pair blocks whose terms are all below 2^-160;
    every output must agree with the full evaluation to 1e-12 relative
    (bit-identical in practice: the skipped background terms are exact FP32
    zeros and the skipped excitation terms vanish against the FP64 sums)."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    es = synth.config(cfg)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    outs = []
    for cut in (False, True):
        plan.set_cutoff(cut)
        o = plan.eval(th, es.hyper, loglik=True, grad_theta=True, grad_hyper=True, negH_theta=True,
                      negH_hyper=True)
        outs.append({k: v.cpu().numpy().copy() for k, v in o.items()})
    assert plan.status() == 0
    plan.close()
    a, b = outs
    for k in a:
        rel = np.max(np.abs(a[k] - b[k]) / np.maximum(np.abs(a[k]), 1e-300))
        print(f"\ncutoff N={es.n} {k}: max rel diff {rel:.2e}", flush=True)
        assert rel <= 1e-12, k


@pytest.mark.parametrize("case", ["n23422", "sparse", "isolated"])
def test_underflow_cutoff_matches_oracle(gpu, case):
    """The cutoff path against the FP64 oracle (which sums every pair), at the
    parity tolerances: on the N = 23,422 workload and on a sparse set (3,000
    events over 3,000 time units, so that chunk pairs more than the cutoff's
    ~222 time units apart are skipped whole); isolated: 2,500 events over 1e5
    time units, whose rows with every term below the cutoff get lambda_i from
    the finalisation's FP64 recomputation."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    if case == "n23422":
        es = synth.config(1)
    elif case == "sparse":
        es = synth.small(3000, seed=35, t_end=3000.0, ties=3)
    else:
        es = _isolated_set("sparse_range")
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    plan.set_cutoff(True)
    th = torch.as_tensor(es.theta, device="cuda:0")
    out = plan.eval(th, es.hyper, loglik=True, grad_theta=True, grad_hyper=True, negH_theta=True, negH_hyper=True)
    lam = plan.lam()
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if v.numel() > 1 else float(v.item())) for k, v in out.items()}
    g["lam"] = lam.cpu().numpy()
    g["status"] = plan.status()
    plan.close()
    if case == "isolated":
        _check(es, g, oracle.evaluate_es(es), tiny=True, hh_mag=hyper_hessian_magnitude(es))
    else:
        _check(es, g, oracle.evaluate_es(es))


@pytest.mark.parametrize("case", ["n23422", "sparse"])
def test_underflow_cutoff_loglik_only_matches_oracle(gpu, case):
    """The log-likelihood-only row pass (the Metropolis proposals' evaluation)
    with the cutoff on, against the oracle: loglik and lambda."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    es = synth.config(1) if case == "n23422" else synth.small(3000, seed=35, t_end=3000.0, ties=3)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    plan.set_cutoff(True)
    th = torch.as_tensor(es.theta, device="cuda:0")
    out = plan.eval(th, es.hyper, loglik=True)
    lam = plan.lam().cpu().numpy()
    ll = float(out["loglik"].item())
    st = plan.status()
    plan.close()
    ref = oracle.evaluate_es(es, want=("loglik", "lam", "Lam_n"))
    lam_rel = np.max(np.abs(lam - ref["lam"]) / ref["lam"])
    print(f"\ncutoff loglik-only {case}: dl {abs(ll - ref['loglik']):.3e} lam {lam_rel:.3e}")
    assert st == 0
    if case == "n23422":
        assert abs(ll - ref["loglik"]) / abs(ref["loglik"]) < 1e-9
    else:
        assert abs(ll - ref["loglik"]) <= 2e-6 * es.n
    assert lam_rel < 2e-6


@pytest.mark.parametrize("case", ["n23422", "sparse", "wide"])
def test_grad_only_matches_oracle(gpu, case):
    """Eq. 4 without Eq. 5: the column pass applies the row weight's integer
    part exactly and rounds the rest of each exponent to FP32; the rate
    gradient is held to the same bound as with the Hessian (sparse: most terms
    tiny; wide: a domain thousands of bandwidths wide)."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    if case == "n23422":
        es = synth.config(1)
    elif case == "sparse":
        es = synth.small(2000, seed=33, t_end=2400.0, ties=2)
    else:
        base = synth.small(1500, seed=41)
        far = np.random.default_rng(41).random(base.n) < 0.5
        es = synth.EventSet(base.t, base.x + np.where(far, 3000.0, 0.0), base.y, base.theta, base.subset, base.z,
                            base.hyper, base.t0, "wide")
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    out = plan.eval(th, es.hyper, loglik=True, grad_theta=True)
    g = out["grad_theta"].cpu().numpy()
    st = plan.status()
    plan.close()
    ref = oracle.evaluate_es(es, want=("loglik", "grad_theta"))
    theta0, omega = es.hyper[3], es.hyper[4]
    a = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t)))
    g_rel = float(np.max(np.abs(g - ref["grad_theta"]) / np.maximum(a + (ref["grad_theta"] + a), 1e-300)))
    print(f"\ngrad only {case}: g {g_rel:.3e}")
    assert st == 0
    assert g_rel < 1e-6


def _isolated_set(case):
    """Event sets in which some events are so far from every other one that all
    of their pair terms lie below FP32's range (the oracle's lambda of those
    events is ~1e-110 and ~1e-50, finite in FP64)."""
    if case == "sparse_range":
        # 2,500 events over 1e5 time units: the smallest intensity is ~4e-110
        return synth.small(2500, seed=9, t_end=1e5)
    base = synth.small(1000, seed=44)
    tau_x = base.hyper[1]
    # three events 15 tau_x outside the set, each beyond a different extreme
    # event and at its time: their largest background term is exp(-112.5)
    # (1.4e-49, below FP32's range), their excitation terms underflow in FP64
    # as well (h < tau_x)
    e_xmax, e_xmin, e_ymax = np.argmax(base.x), np.argmin(base.x), np.argmax(base.y)
    d = 15.0 * tau_x
    x_far = np.array([base.x[e_xmax] + d, base.x[e_xmin] - d, base.x[e_ymax]])
    y_far = np.array([base.y[e_xmax], base.y[e_xmin], base.y[e_ymax] + d])
    t_far = base.t[[e_xmax, e_xmin, e_ymax]]
    t = np.concatenate([base.t, t_far])
    x = np.concatenate([base.x, x_far])
    y = np.concatenate([base.y, y_far])
    theta = np.concatenate([base.theta, np.ones(3)])
    return synth.EventSet(t, x, y, theta, base.subset, base.z, base.hyper, base.t0, "far")


@pytest.mark.parametrize("case", ["sparse_range", "far"])
def test_isolated_events_match_oracle(gpu, case):
    """Rows whose intensity from the FP32 pair terms falls below
    (c_b + c_e) n 2^-96 are recomputed in FP64 by the row finalisation: every
    output matches the oracle, where the FP32 terms alone would give
    lambda_i = 0 and loglik = -inf.  On the sparse set the hyperparameter
    Hessian's per-event terms cancel about 40-fold (their magnitudes sum to
    ~1e6 against a diagonal of ~8e4 for omega), so its entries are held to
    1e-6 of that magnitude, the scale of the FP32 terms' rounding."""
    es = _isolated_set(case)
    ref = oracle.evaluate_es(es)
    assert np.isfinite(ref["loglik"]) and ref["lam"].min() < 1e-38
    gpu_r = run_gpu(es)
    _check(es, gpu_r, ref, tiny=True, hh_mag=hyper_hessian_magnitude(es))


@pytest.mark.parametrize("case", ["sparse_range", "far"])
def test_isolated_events_grad_only_matches_oracle(gpu, case):
    """Eq. 4 alone on the same sets: the chunks that hold a row of large weight
    log2(c_e / lambda_i) split every exponent exactly."""
    import torch

    from paper_2103_03348_amd.hawkes import Plan

    es = _isolated_set(case)
    plan = Plan.from_numpy(es.t, es.x, es.y, es.t0)
    th = torch.as_tensor(es.theta, device="cuda:0")
    out = plan.eval(th, es.hyper, loglik=True, grad_theta=True)
    g = out["grad_theta"].cpu().numpy()
    ll = float(out["loglik"].item())
    st = plan.status()
    plan.close()
    ref = oracle.evaluate_es(es, want=("loglik", "grad_theta"))
    theta0, omega = es.hyper[3], es.hyper[4]
    a = theta0 * (1.0 - np.exp(-omega * (es.t.max() - es.t)))
    g_rel = float(np.max(np.abs(g - ref["grad_theta"]) / np.maximum(a + (ref["grad_theta"] + a), 1e-300)))
    print(f"\nisolated grad only {case}: dl {abs(ll - ref['loglik']):.3e} g {g_rel:.3e}")
    assert st == 0
    assert abs(ll - ref["loglik"]) <= 2e-6 * es.n
    assert g_rel < 1e-6
