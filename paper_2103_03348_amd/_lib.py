"""ctypes binding of libhawkes.so (argument marshalling only).

Every computation of the Hawkes path runs in the library's HIP kernels; this
module converts torch tensors to device pointers and the current torch stream
to a hipStream_t.  There is no fallback: if the library is missing the import
of this module fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhawkes.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -m paper_2103_03348_amd.build "
        "or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

STATUS = {
    0: "HAWKES_OK",
    1: "HAWKES_E_INVALID",
    2: "HAWKES_E_ZERO_INTENSITY",
    3: "HAWKES_E_NONFINITE",
    4: "HAWKES_E_DEVICE",
    5: "HAWKES_E_NOMEM",
    6: "HAWKES_E_UNSUPPORTED",
    7: "HAWKES_E_STALE",
    8: "HAWKES_E_CAPACITY",
}
OK, E_INVALID, E_ZERO_INTENSITY, E_NONFINITE, E_DEVICE, E_NOMEM, E_UNSUPPORTED, E_STALE, E_CAPACITY = range(9)


class HawkesError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class HmcArgs(ctypes.Structure):
    _fields_ = [("d_z", ctypes.c_void_p), ("d_theta", ctypes.c_void_p), ("d_mass", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("L", ctypes.c_int), ("sigma_z", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("counter", ctypes.c_uint64), ("refresh_static", ctypes.c_int),
                ("d_out", ctypes.c_void_p), ("beta", ctypes.c_double), ("prior", ctypes.c_int),
                ("d_z_proposal", ctypes.c_void_p)]


class Hyper(ctypes.Structure):
    _fields_ = [("mu0", ctypes.c_double), ("tau_x", ctypes.c_double), ("tau_t", ctypes.c_double),
                ("theta0", ctypes.c_double), ("omega", ctypes.c_double), ("h", ctypes.c_double)]

    @classmethod
    def of(cls, hy):
        if isinstance(hy, Hyper):
            return hy
        return cls(*[float(v) for v in hy])


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_HyP = ctypes.POINTER(Hyper)

# name -> (restype, argtypes); mirrors include/hawkes.h
SIGNATURES = {
    "hawkes_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), _i64, _vp, _vp, ctypes.c_double, _vp]),
    "hawkes_plan_destroy": (ctypes.c_int, [_vp]),
    "hawkes_plan_size": (_i64, [_vp]),
    "hawkes_eval": (ctypes.c_int, [_vp, _HyP, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "hawkes_loglik": (ctypes.c_int, [_vp, _HyP, _vp, _vp, _vp]),
    "hawkes_grad": (ctypes.c_int, [_vp, _HyP, _vp, _vp, _vp, _vp, _vp]),
    "hawkes_hessdiag": (ctypes.c_int, [_vp, _HyP, _vp, _vp, _vp, _vp]),
    "hawkes_plan_status": (ctypes.c_int, [_vp]),
    "hawkes_copy_lambda": (ctypes.c_int, [_vp, _vp, _vp]),
    "hawkes_plan_epoch": (_i64, [_vp]),
    "hawkes_plan_set_cutoff": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hawkes_grad_theta_from_last": (ctypes.c_int, [_vp, _HyP, _i64, _vp, _vp, _vp]),
    "hawkes_plan_set_subset": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "hawkes_subset_grad": (ctypes.c_int, [_vp, _HyP, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "hmc_step": (ctypes.c_int, [_vp, _HyP, ctypes.POINTER(HmcArgs), _vp]),
    "hawkes_subset_trend_grad": (ctypes.c_int, [_vp, _HyP, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]),
    "hawkes_plan_set_tree": (ctypes.c_int, [_vp, _i64, _vp, _vp, ctypes.c_double]),
    "hawkes_tree_prior": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp]),
    "hawkes_mlp_num_params": (_i64, []),
    "hawkes_mlp_workspace_floats": (_i64, [_i64]),
    "hawkes_mlp_forward": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "hawkes_mlp_grad": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "hawkes_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _i64, _vp, _vp,
                                             _i64, _vp, _vp, _vp, _vp, _vp]),
    "hawkes_mlp_noalloc_max_batch": (_i64, []),
    "hawkes_mlp_train_step_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _i64, _vp,
                                                     _vp, _i64, _vp, _vp, _vp]),
    "hawkes_features": (ctypes.c_int, [_vp, _HyP, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "hawkes_mass_update": (ctypes.c_int, [_vp, _HyP, _vp, _vp, ctypes.c_double, ctypes.c_int, _i64, _vp, _vp]),
    "hawkes_subset_z": (ctypes.c_int, [_vp, _vp, ctypes.c_double, _vp, _vp]),
    "hawkes_subset_curvature": (ctypes.c_int, [_vp, _HyP, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp, _vp]),
    "hawkes_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hawkes_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "hawkes_exp2_bias": (ctypes.c_int, [_i64, ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "hawkes_exp2_bias_constant": (ctypes.c_double, []),
    "hawkes_exp2_rate": (ctypes.c_int, [_i64, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double), _vp]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def lib():
    return _lib


def check(code, where):
    if code != OK:
        raise HawkesError(code, where)


def ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)
