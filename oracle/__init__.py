"""FP64 CPU oracle for the Hawkes path: TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never imports, links or calls it, and
it shares no code with the GPU library: the only common module is the seeded
input generator, which holds none of the method's arithmetic.

Contents:
  * ``hawkes_oracle.c`` (compiled to ``liboracle.so``): the log-likelihood of
    Eq. 1, the rate gradient of Eq. 4 and the Hessian diagonal of Eq. 5, plus
    the hyperparameter derivatives, as plain FP64 double loops;
  * ``philox.py``: the Philox-4x32-10 counter-based generator;
  * ``mlp.py``: FP64 forward/backward of the small preconditioner network;
  * ``hmc.py``: the leapfrog integrator and Metropolis step in FP64;
  * ``features.py``: the per-event grid-count features of the preconditioner.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "hawkes_oracle.c")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build_oracle(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_eval.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double,
                                    dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_row_sums.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int64, lp, dp,
                                        ctypes.c_int]
        lib.oracle_row_sums.restype = ctypes.c_int
        lib.oracle_col_sums.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int64, lp, dp, dp,
                                        ctypes.c_int]
        lib.oracle_col_sums.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def evaluate(t, x, y, theta, hyper, t0=0.0, nthreads=0, want=("loglik", "lam", "ell_n", "Lam_n",
                                                               "grad_theta", "negH_theta",
                                                               "grad_hyper", "negH_hyper")):
    """Full FP64 evaluation.  Returns a dict with the requested outputs:
    loglik (float), lam[n], ell_n[n], Lam_n[n], grad_theta[n], negH_theta[n],
    grad_hyper[6], negH_hyper[6] (hyper order mu0, tau_x, tau_t, theta0, omega, h)."""
    lib = _load()
    t, x, y, theta = _c(t), _c(x), _c(y), _c(theta)
    hy = _c(hyper)
    n = t.shape[0]
    out = {}
    bufs = {}
    for k, sz in (("lam", n), ("ell_n", n), ("Lam_n", n), ("grad_theta", n), ("negH_theta", n),
                  ("grad_hyper", 6), ("negH_hyper", 6), ("loglik", 1)):
        bufs[k] = np.zeros(sz) if k in want else None
    rc = lib.oracle_eval(n, _p(t), _p(x), _p(y), _p(theta), _p(hy), float(t0),
                         _p(bufs["lam"]), _p(bufs["ell_n"]), _p(bufs["Lam_n"]),
                         _p(bufs["grad_theta"]), _p(bufs["negH_theta"]),
                         _p(bufs["grad_hyper"]), _p(bufs["negH_hyper"]), _p(bufs["loglik"]),
                         int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_eval rejected its arguments (code {rc})")
    for k, v in bufs.items():
        if v is not None:
            out[k] = float(v[0]) if k == "loglik" else v
    return out


def row_sums(t, x, y, theta, hyper, rows=None, nthreads=0):
    """Pair sums [len(rows)][10] (B0, B1, B2, B11, B22, X0, X1, X2, X11, X22) for the given rows."""
    lib = _load()
    t, x, y, theta, hy = _c(t), _c(x), _c(y), _c(theta), _c(hyper)
    n = t.shape[0]
    if rows is None:
        rows_a = np.arange(n, dtype=np.int64)
    else:
        rows_a = np.ascontiguousarray(rows, dtype=np.int64)
    acc = np.zeros((rows_a.shape[0], 10))
    lib.oracle_row_sums(n, _p(t), _p(x), _p(y), _p(theta), _p(hy), rows_a.shape[0],
                        rows_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(acc), int(nthreads))
    return acc


def col_sums(t, x, y, hyper, lam, cols=None, nthreads=0):
    """Eq. 4 / Eq. 5 column sums (G_j, H_j) for the given columns, given lambda for all events."""
    lib = _load()
    t, x, y, hy, lam = _c(t), _c(x), _c(y), _c(hyper), _c(lam)
    n = t.shape[0]
    cols_a = np.arange(n, dtype=np.int64) if cols is None else np.ascontiguousarray(cols, dtype=np.int64)
    G = np.zeros(cols_a.shape[0])
    H = np.zeros(cols_a.shape[0])
    lib.oracle_col_sums(n, _p(t), _p(x), _p(y), _p(hy), _p(lam), cols_a.shape[0],
                        cols_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(G), _p(H), int(nthreads))
    return G, H


def constants(hyper):
    """(c_b, c_e): the background and excitation normalisers of Sec. 2.1 (D = 2,
    with the temporal background factor)."""
    mu0, tau_x, tau_t, theta0, omega, h = [float(v) for v in hyper]
    c_b = mu0 / ((2.0 * np.pi) ** 1.5 * tau_x ** 2 * tau_t)
    c_e = theta0 * omega / (2.0 * np.pi * h ** 2)
    return c_b, c_e


def evaluate_es(es, theta=None, hyper=None, **kw):
    """evaluate() on an EventSet from the synthetic generator."""
    return evaluate(es.t, es.x, es.y, es.theta if theta is None else theta,
                    es.hyper if hyper is None else hyper, es.t0, **kw)
