"""Writes hmc_replay_N23422.npz: whole HMC iterations of the FP64 oracle on the
N = 23,422 workload (1,610 free rates, 26 subset chunks of 64), L = 20
leapfrog steps, two Philox counters each, for three targets -- the iid prior
(beta = 0), the temporal trend theta_k = exp(z_k + beta t_k) of Sec. 2.2 and
the phylogenetic prior of Eq. 2 on a coalescent tree -- for the GPU replay test
(tests/test_gpu_hmc.py).  Calls only oracle/ (inputs from the seeded
generator).  About 10 minutes on 8 cores:

    python tests/golden/make_hmc_replay.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import hmc as ohmc  # noqa: E402
from oracle import tree as otree  # noqa: E402
from paper_2103_03348_amd import synth  # noqa: E402

# the replay's settings (the GPU test reads them back from the file)
EPS, L, SIGMA = 0.03, 20, 0.5
VARIANTS = (("iid", 0.0, False, 501), ("trend", -4e-4, False, 502), ("tree", 0.0, True, 503))
COUNTERS = (0, 1)
TREE_SEED, TREE_TAU0 = 1610, 1.0


def mass_of(m):
    """A diagonal mass with distinct entries (4 ... 7), slot order."""
    return 4.0 + 0.5 * (np.arange(m) % 7)


def main():
    es = synth.config(3)
    m = es.subset.shape[0]
    z0 = np.log(es.theta[es.subset])
    mass = mass_of(m)
    par, ln = synth.coalescent_tree(m, seed=TREE_SEED, scale=float(m))
    V = otree.covariance(par, ln, TREE_TAU0)
    out = {"eps": EPS, "L": L, "sigma": SIGMA, "mass": mass, "z0": z0, "tree_seed": TREE_SEED,
           "tree_tau0": TREE_TAU0}
    for name, beta, tree, seed in VARIANTS:
        for counter in COUNTERS:
            r = ohmc.hmc_iteration(es.t, es.x, es.y, es.theta, es.subset, z0, mass, es.hyper, es.t0, EPS, L, SIGMA,
                                   seed, counter, beta=beta, prior_v=V if tree else None)
            key = f"{name}_{counter}"
            for f in ("dH", "H0", "H1", "u", "loglik_proposal"):
                out[f"{key}_{f}"] = np.float64(r[f])
            out[f"{key}_accepted"] = np.int64(r["accepted"])
            out[f"{key}_z_proposal"] = r["z_proposal"]
            out[f"{key}_beta"] = np.float64(beta)
            out[f"{key}_seed"] = np.int64(seed)
            print(f"{key}: dH {r['dH']:.9f} accepted {r['accepted']} H0 {r['H0']:.6f}", flush=True)
    np.savez_compressed(os.path.join(HERE, "hmc_replay_N23422.npz"), **out)


if __name__ == "__main__":
    print(f"oracle threads: {oracle.max_threads()}", flush=True)
    main()
