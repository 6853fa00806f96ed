"""Per-event inputs of the learned preconditioner, by their plain definition
(brute-force counting over all events).  Test infrastructure only.

For a free event m at (x_m, t_m), with r2_e = (x_e - x_m)^2 + (y_e - y_m)^2 and
dt_e = t_e - t_m:
  f0, f1  log1p(#{e != m : r2_e < r^2}) for r = h, 3h
  f2      log1p(#{e : r2_e < (3h)^2, 0 < dt_e <= 6/omega})  (the terms of f8)
  f3..f5  r = h:  log1p(#{e : r2_e < r^2, -1/omega <= dt_e < 0}),
                  log1p(#{e : r2_e < r^2, 0 < dt_e <= 1/omega}),
                  log1p(#{e : r2_e < r^2, 0 < dt_e <= 3/omega})
  f6, f7  the first two with r = 3h
  f8      max(log2 S_m, -32) / 8 with S_m the forward sum of the squared
          excitation kernel, sum over e with r2_e < (3h)^2, 0 < dt_e <= 6/omega
          of exp(-2 omega dt_e - r2_e / h^2) (Eq. 5's H_m without its weights)
  f9      z_m = log theta_m
  f10     #{e : t_e < t_m} / N     (time rank)
  f11     (T1 - t_m) / (T1 - T0)   (time to the window end)
r^2 is r * r and r2_e is formed as dx * dx + dy * dy, each rounded once in
FP64; 1/omega, 3/omega and 6/omega are 1.0 / omega, 3.0 / omega and
6.0 / omega in FP64.  The grid
origin (gx0, gy0) is accepted for the library's signature and does not change
any count.
"""
from __future__ import annotations

import numpy as np


def features(t, x, y, idx, z, hyper, t0, gx0, gy0):
    t = np.asarray(t, np.float64)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    idx = np.asarray(idx, np.int64)
    _, _, _, _, omega, h = [float(v) for v in hyper]
    n = t.shape[0]
    T1 = float(t.max())
    span = T1 - t0
    w1 = 1.0 / omega
    w3 = 3.0 / omega
    w6 = 6.0 / omega
    F = np.zeros((idx.shape[0], 12))
    for r, m in enumerate(idx):
        dx = x - x[m]
        dy = y - y[m]
        r2 = dx * dx + dy * dy
        dt = t - t[m]
        for c, rad in enumerate((h, 3.0 * h)):
            F[r, c] = np.log1p(np.sum(r2 < rad * rad) - 1)
        for base, rad in ((3, h), (6, 3.0 * h)):
            near = r2 < rad * rad
            F[r, base + 0] = np.log1p(np.sum(near & (dt >= -w1) & (dt < 0.0)))
            F[r, base + 1] = np.log1p(np.sum(near & (dt > 0.0) & (dt <= w1)))
            if base == 3:
                F[r, base + 2] = np.log1p(np.sum(near & (dt > 0.0) & (dt <= w3)))
        sel = (r2 < (3.0 * h) * (3.0 * h)) & (dt > 0.0) & (dt <= w6)
        F[r, 2] = np.log1p(np.sum(sel))
        s_m = np.sum(np.exp(-2.0 * omega * dt[sel] - r2[sel] / (h * h)))
        F[r, 8] = max(np.log2(s_m) if s_m > 0.0 else -np.inf, -32.0) / 8.0
        F[r, 9] = z[r]
        F[r, 10] = np.sum(t < t[m]) / n
        F[r, 11] = (T1 - t[m]) / span if span > 0 else 0.0
    return F
