"""Python face of the library: a plan over one event set and its evaluations.

Only argument marshalling happens here; the work runs in libhawkes.so.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import Hyper, check, ptr, stream_handle


class Plan:
    """Sorted, device-resident event set (Sec. 2.1's data (x_n, t_n)).

    t  : [n] float64 CUDA tensor of event times
    xy : [n, 2] float64 CUDA tensor of locations
    t_start : window start T0 (<= min t)
    """

    def __init__(self, t: torch.Tensor, xy: torch.Tensor, t_start: float = 0.0):
        if t.dtype != torch.float64 or xy.dtype != torch.float64:
            raise TypeError("t and xy must be float64")
        if xy.dim() != 2 or xy.shape[1] != 2 or xy.shape[0] != t.shape[0]:
            raise ValueError("xy must be [n, 2] with n = len(t)")
        self.device = t.device
        self._t = t.contiguous()
        self._xy = xy.contiguous()
        self.n = int(t.shape[0])
        self.t_start = float(t_start)
        h = ctypes.c_void_p()
        check(_lib.lib().hawkes_plan_create(ctypes.byref(h), self.n, ptr(self._t), ptr(self._xy),
                                            self.t_start, stream_handle()), "hawkes_plan_create")
        self._h = h

    @classmethod
    def from_numpy(cls, t, x, y, t_start=0.0, device="cuda:0"):
        import numpy as np
        tt = torch.as_tensor(np.ascontiguousarray(t, dtype=np.float64), device=device)
        xy = torch.as_tensor(np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64)], 1), device=device)
        return cls(tt, xy.contiguous(), t_start)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().hawkes_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, k):
        return torch.empty(k, dtype=torch.float64, device=self.device)

    def eval(self, theta: torch.Tensor, hyper, loglik=True, grad_theta=False, grad_hyper=False,
             negH_theta=False, negH_hyper=False, out=None):
        """hawkes_eval.  Returns a dict of the requested CUDA tensors (caller order)."""
        if theta.dtype != torch.float64 or theta.shape != (self.n,):
            raise ValueError("theta must be float64 [n]")
        o = {} if out is None else out
        if loglik and "loglik" not in o:
            o["loglik"] = self._vec(1)
        if grad_theta and "grad_theta" not in o:
            o["grad_theta"] = self._vec(self.n)
        if grad_hyper and "grad_hyper" not in o:
            o["grad_hyper"] = self._vec(6)
        if negH_theta and "negH_theta" not in o:
            o["negH_theta"] = self._vec(self.n)
        if negH_hyper and "negH_hyper" not in o:
            o["negH_hyper"] = self._vec(6)
        hy = Hyper.of(hyper)
        th = theta.contiguous()  # referenced until the call returns and stream-ordered after it
        check(_lib.lib().hawkes_eval(self._h, ctypes.byref(hy), ptr(th),
                                     ptr(o.get("loglik") if loglik else None),
                                     ptr(o.get("grad_theta") if grad_theta else None),
                                     ptr(o.get("grad_hyper") if grad_hyper else None),
                                     ptr(o.get("negH_theta") if negH_theta else None),
                                     ptr(o.get("negH_hyper") if negH_hyper else None),
                                     stream_handle()), "hawkes_eval")
        return o

    def set_cutoff(self, enabled: bool):
        """hawkes_plan_set_cutoff: skip pair blocks whose terms all underflow."""
        check(_lib.lib().hawkes_plan_set_cutoff(self._h, int(bool(enabled))), "hawkes_plan_set_cutoff")

    def epoch(self) -> int:
        """hawkes_plan_epoch: evaluations run so far (pairs a backward with its forward)."""
        return int(_lib.lib().hawkes_plan_epoch(self._h))

    def grad_theta_from_last(self, hyper, epoch: int, negH: bool = False):
        """hawkes_grad_theta_from_last: the column pass alone on the intensities of
        the evaluation numbered `epoch`.  Returns (grad_theta, negH_theta or None),
        or None if the plan has evaluated something else since (HAWKES_E_STALE)."""
        g = self._vec(self.n)
        h = self._vec(self.n) if negH else None
        hy = Hyper.of(hyper)
        code = _lib.lib().hawkes_grad_theta_from_last(self._h, ctypes.byref(hy), int(epoch), ptr(g), ptr(h),
                                                      stream_handle())
        if code == _lib.E_STALE:
            return None
        check(code, "hawkes_grad_theta_from_last")
        return g, h

    def lam(self) -> torch.Tensor:
        """lambda_i of the last evaluation, caller order."""
        out = self._vec(self.n)
        check(_lib.lib().hawkes_copy_lambda(self._h, ptr(out), stream_handle()), "hawkes_copy_lambda")
        return out

    def status(self) -> int:
        """Synchronise and return (and clear) the sticky device status code."""
        return int(_lib.lib().hawkes_plan_status(self._h))
