"""Phylogenetic Brownian prior of Sec. 2.2 (Eq. 2) by its plain definition:
the dense covariance V of the tips and a Cholesky factorisation.  Test
infrastructure only.

For a bifurcating tree with branch lengths w and root variance factor tau0,
V_nm = tau0 + depth(MRCA(n, m)), where depth is the summed branch length from
the root; V_nn is tau0 plus the depth of tip n.  Then
  log p(z) = -(M log(2 pi sigma^2) + log|V| + z^T V^{-1} z / sigma^2) / 2,
  grad     = -V^{-1} z / sigma^2.
"""
from __future__ import annotations

import numpy as np


def covariance(parent, length, tau0):
    """Dense V [M, M] for a tree given as parent[] (-1 at the root) over
    2M - 1 nodes whose first M are the tips."""
    parent = np.asarray(parent, dtype=np.int64)
    length = np.asarray(length, dtype=np.float64)
    n = parent.shape[0]
    m = (n + 1) // 2
    depth = np.zeros(n)
    order = []
    # depths by walking up from every node (memoised)
    done = np.zeros(n, dtype=bool)
    root = int(np.where(parent < 0)[0][0])
    done[root] = True

    def dep(v):
        path = []
        while not done[v]:
            path.append(v)
            v = parent[v]
        for u in reversed(path):
            depth[u] = depth[parent[u]] + length[u]
            done[u] = True

    for v in range(n):
        dep(v)
    # ancestor sets of the tips
    anc = []
    for k in range(m):
        a, v = [], k
        while v >= 0:
            a.append(v)
            v = parent[v]
        anc.append(a)
    V = np.empty((m, m))
    for i in range(m):
        si = set(anc[i])
        for j in range(i, m):
            # first ancestor of j (walking up) that is also an ancestor of i
            mrca = next(v for v in anc[j] if v in si)
            V[i, j] = V[j, i] = tau0 + depth[mrca]
    return V


def logpdf_and_grad(z, V, sigma):
    z = np.asarray(z, dtype=np.float64)
    m = z.shape[0]
    L = np.linalg.cholesky(V)
    y = np.linalg.solve(L, z)
    quad = float(y @ y)
    vz = np.linalg.solve(L.T, y)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    logp = -0.5 * (m * np.log(2 * np.pi * sigma ** 2) + logdet + quad / sigma ** 2)
    return logp, -vz / sigma ** 2, quad
