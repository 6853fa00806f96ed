"""Learned diagonal preconditioner for the HMC step.

A 12 -> 64 -> 64 -> 1 tanh network predicts, for free event k, log H_k: the
log of Eq. 5's Hessian diagonal, which the paper uses as the HMC mass, from
cheap per-event features (grid-cell counts, recent-window counts, log theta,
time rank, time to the window end).  It is trained on the GPU by the library's
own forward, back-propagation and Adam kernels on exact Eq. 5 diagonals that
the library computes at saved HMC states.  The sampler folds the learned
estimate theta_k^2 exp(prediction) + P_kk (the prior's precision P added when
the mass is formed) into its running-average mass and still folds in the exact
estimate at a coarser interval; because any positive mass leaves the target
invariant, the sampler stays exact whatever the network predicts.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .sampler import HmcSampler

N_FEATURES = 12


def glorot_init(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in, bias in ((64, 12, 64), (64, 64, 64), (1, 64, 1)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(bias))
    flat = np.concatenate(parts)
    assert flat.shape[0] == int(_lib.lib().hawkes_mlp_num_params())
    return flat.astype(np.float32)


class LearnedPreconditioner:
    def __init__(self, sampler: HmcSampler, t: torch.Tensor, xy: torch.Tensor, seed: int = 0):
        self.s = sampler
        self.dev = sampler.dev
        self.t = t.contiguous()
        self.xy = xy.contiguous()
        self.gx0 = float(self.xy[:, 0].min().item()) - 1e-9
        self.gy0 = float(self.xy[:, 1].min().item()) - 1e-9
        self.np = int(_lib.lib().hawkes_mlp_num_params())
        self.params = torch.as_tensor(glorot_init(seed), device=self.dev)
        self.adam_m = torch.zeros(self.np, dtype=torch.float32, device=self.dev)
        self.adam_v = torch.zeros(self.np, dtype=torch.float32, device=self.dev)
        self.step_no = 0
        self.feat = torch.empty((sampler.m, N_FEATURES), dtype=torch.float32, device=self.dev)
        self.pred = torch.empty(sampler.m, dtype=torch.float32, device=self.dev)

    # ---- inputs and targets --------------------------------------------------------------
    def features(self) -> torch.Tensor:
        s = self.s
        _lib.check(_lib.lib().hawkes_features(s.plan.handle, ctypes.byref(s.hyper), _lib.ptr(self.t),
                                              _lib.ptr(self.xy), _lib.ptr(s.z), self.gx0, self.gy0,
                                              _lib.ptr(self.feat), _lib.stream_handle()), "hawkes_features")
        return self.feat

    def collect(self, n_states: int, eps: float, thin: int = 1):
        """Advance the sampler (current mass) and record the features and the
        training target log max(H_k, 1e-6) (Eq. 5 on the subset, computed by the
        library) at n_states states.  Returns (X [n_states*m, 12], T [n_states*m])."""
        m = self.s.m
        X = torch.empty((n_states * m, N_FEATURES), dtype=torch.float32, device=self.dev)
        T = torch.empty(n_states * m, dtype=torch.float32, device=self.dev)
        for k in range(n_states):
            for _ in range(thin):
                self.s.step(eps)
            X[k * m:(k + 1) * m].copy_(self.features())
            self.s.curvature(log_h=T[k * m:(k + 1) * m])
        return X, T

    # ---- training ------------------------------------------------------------------------------
    def train(self, X: torch.Tensor, T: torch.Tensor, steps: int = 2000, batch: int = 4096, lr: float = 2e-3,
              seed: int = 0, log_every: int = 0):
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        B = min(batch, n)
        work = torch.empty(int(_lib.lib().hawkes_mlp_workspace_floats(B)), dtype=torch.float32, device=self.dev)
        grad = torch.empty(self.np, dtype=torch.float64, device=self.dev)
        loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        err = torch.zeros(1, dtype=torch.int32, device=self.dev)
        X = X.contiguous()
        T = T.contiguous()
        hist = []
        # every step's batch rows drawn up front and copied once
        all_rows = torch.as_tensor(rng.integers(0, n, size=(steps, B)).astype(np.int32), device=self.dev)
        for it in range(steps):
            rows = all_rows[it]
            self.step_no += 1
            _lib.check(_lib.lib().hawkes_mlp_train_step(_lib.ptr(self.params), _lib.ptr(self.adam_m),
                                                        _lib.ptr(self.adam_v), self.step_no, ctypes.c_float(lr),
                                                        _lib.ptr(X), n, _lib.ptr(rows), _lib.ptr(T), B,
                                                        _lib.ptr(work), _lib.ptr(grad), _lib.ptr(loss),
                                                        _lib.ptr(err), _lib.stream_handle()),
                       "hawkes_mlp_train_step")
            if log_every and (it % log_every == 0 or it == steps - 1):
                hist.append((it, float(loss.item())))
        torch.cuda.synchronize()
        if int(err.item()) != 0:
            raise RuntimeError("a batch row index was out of range")
        return hist

    def evaluate(self, X: torch.Tensor, T: torch.Tensor) -> float:
        """Mean squared error of the prediction on (X, T), by the library's loss
        (hawkes_mlp_grad over all rows; its gradient is discarded)."""
        n = X.shape[0]
        work = torch.empty(int(_lib.lib().hawkes_mlp_workspace_floats(n)), dtype=torch.float32, device=self.dev)
        grad = torch.empty(self.np, dtype=torch.float64, device=self.dev)
        loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        _lib.check(_lib.lib().hawkes_mlp_grad(_lib.ptr(self.params), _lib.ptr(X.contiguous()), n, None,
                                              _lib.ptr(T.contiguous()), n, _lib.ptr(work), _lib.ptr(grad),
                                              _lib.ptr(loss), None, _lib.stream_handle()), "hawkes_mlp_grad")
        return float(loss.item())

    # ---- use in the sampler --------------------------------------------------------------------
    def predict(self) -> torch.Tensor:
        feat = self.features()
        _lib.check(_lib.lib().hawkes_mlp_forward(_lib.ptr(self.params), _lib.ptr(feat), self.s.m,
                                                 _lib.ptr(self.pred), _lib.stream_handle()), "hawkes_mlp_forward")
        return self.pred

    def fold_into_mass(self, sampler: HmcSampler):
        """One learned estimate folded into the sampler's running-average mass."""
        pred = self.predict()
        _lib.check(_lib.lib().hawkes_mass_update(sampler.plan.handle, ctypes.byref(sampler.hyper),
                                                 _lib.ptr(sampler.theta), _lib.ptr(pred), sampler.sigma_z,
                                                 sampler.prior, sampler.mass_count, _lib.ptr(sampler.mass),
                                                 _lib.stream_handle()), "hawkes_mass_update")
        sampler.mass_count += 1
