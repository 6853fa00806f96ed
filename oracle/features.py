"""Per-event inputs of the learned preconditioner, by their plain definition
(brute-force counting).  Test infrastructure only.

For a free event m at (x_m, t_m), with cell(e; s) = (floor((x_e - gx0)/s),
floor((y_e - gy0)/s)) and bin(e) = floor((t_e - T0) * omega):
  f0..f2  log1p(#other events in m's cell), cell sizes s = h, 3h, tau_x
  f3..f5  cell size h:  log1p(#events with bin = bin_m - 1),
                        log1p(#events with bin = bin_m + 1),
                        log1p(#events with bin_m + 1 <= bin <= bin_m + 3)
  f6..f8  the same three with cell size 3h
  f9      z_m = log theta_m
  f10     #{e : t_e < t_m} / N     (time rank)
  f11     (T1 - t_m) / (T1 - T0)   (time to the window end)
The grid origin (gx0, gy0) is part of the input.
"""
from __future__ import annotations

import numpy as np


def features(t, x, y, idx, z, hyper, t0, gx0, gy0):
    t = np.asarray(t, np.float64)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    idx = np.asarray(idx, np.int64)
    _, tau_x, _, _, omega, h = [float(v) for v in hyper]
    n = t.shape[0]
    T1 = float(t.max())
    span = T1 - t0
    bins = np.floor((t - t0) * omega)
    F = np.zeros((idx.shape[0], 12))

    def cell(s):
        return np.floor((x - gx0) / s), np.floor((y - gy0) / s)

    cells = {s: cell(s) for s in (h, 3.0 * h, tau_x)}
    for r, m in enumerate(idx):
        for c, s in enumerate((h, 3.0 * h, tau_x)):
            cx, cy = cells[s]
            same = (cx == cx[m]) & (cy == cy[m])
            F[r, c] = np.log1p(same.sum() - 1)
        for base, s in ((3, h), (6, 3.0 * h)):
            cx, cy = cells[s]
            same = (cx == cx[m]) & (cy == cy[m])
            b = bins[m]
            F[r, base + 0] = np.log1p(np.sum(same & (bins == b - 1)))
            F[r, base + 1] = np.log1p(np.sum(same & (bins == b + 1)))
            F[r, base + 2] = np.log1p(np.sum(same & (bins >= b + 1) & (bins <= b + 3)))
        F[r, 9] = z[r]
        F[r, 10] = np.sum(t < t[m]) / n
        F[r, 11] = (T1 - t[m]) / span if span > 0 else 0.0
    return F
