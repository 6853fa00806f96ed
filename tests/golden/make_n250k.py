"""Writes oracle_N250000.npz: one full FP64 oracle evaluation of the
N = 250,000 workload (20-component mixture, branching process, 17,185 free
rates; ~3.1e10 pairs) -- log-likelihood (Eq. 1), intensities, rate gradient
(Eq. 4), Hessian diagonal (Eq. 5) and the hyperparameter derivatives -- for
the GPU parity test of every output at that size (tests/test_gpu_large.py).
Calls only oracle/ (inputs from the seeded generator).  About 8 minutes on 8
cores:

    python tests/golden/make_n250k.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2103_03348_amd import synth  # noqa: E402


def main():
    es = synth.config(4)
    t0 = time.time()
    r = oracle.evaluate_es(es, want=("loglik", "lam", "grad_theta", "negH_theta", "grad_hyper", "negH_hyper"))
    print(f"N={es.n}: oracle evaluation {time.time() - t0:.0f} s, loglik {r['loglik']:.12f}", flush=True)
    np.savez_compressed(os.path.join(HERE, "oracle_N250000.npz"), n=np.int64(es.n), loglik=np.float64(r["loglik"]),
                        lam=r["lam"], grad_theta=r["grad_theta"], negH_theta=r["negH_theta"],
                        grad_hyper=r["grad_hyper"], negH_hyper=r["negH_hyper"],
                        t_checksum=np.float64(np.sum(es.t)), x_checksum=np.float64(np.sum(es.x)))


if __name__ == "__main__":
    print(f"oracle threads: {oracle.max_threads()}", flush=True)
    main()
