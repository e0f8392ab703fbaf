"""Fiber-orientation outputs of an RVE (test infrastructure; only tests,
smoke() and bench.py's CPU baseline use the oracle).

The paper tracks the reorientation of the fibers during loading and sends an
orientation measure of each RVE to the macroscale (Section 4, coupling: the
orientation tensor written with each converged step; Section 6: the degree
of alignment as the second Legendre polynomial of the angle between a
fiber's direction and a reference direction, averaged over the fibers).

Readings (the paper gives no formula for the tensor): the orientation tensor
is Omega = <n n^T>, the plain average over the fibers of the RVE of the dyad
of the unit direction n = (x_j - x_i) / |x_j - x_i| in the current
configuration, unweighted like P2; P2 = <(3 (n . e)^2 - 1) / 2> with e the
reference direction normalised.  Then P2 = (3 e.Omega.e - 1) / 2 and
trace Omega = 1.

Plain loops, FP64; written from the definitions, sharing nothing with the
HIP path.
"""
from __future__ import annotations

import math

import numpy as np


def orientation(x, fib, e):
    """(Omega [3,3], P2) of one network at positions x [N,3] (fibers fib [M,2])."""
    x = np.asarray(x, dtype=np.float64)
    fib = np.asarray(fib)
    ex, ey, ez = (float(v) for v in e)
    en = math.sqrt(ex * ex + ey * ey + ez * ez)
    ex, ey, ez = ex / en, ey / en, ez / en
    om = [[0.0] * 3 for _ in range(3)]
    p2 = 0.0
    m = len(fib)
    for k in range(m):
        i, j = int(fib[k, 0]), int(fib[k, 1])
        d = [x[j, 0] - x[i, 0], x[j, 1] - x[i, 1], x[j, 2] - x[i, 2]]
        ln = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        n = [d[0] / ln, d[1] / ln, d[2] / ln]
        for a in range(3):
            for b in range(3):
                om[a][b] += n[a] * n[b]
        c = n[0] * ex + n[1] * ey + n[2] * ez
        p2 += 0.5 * (3.0 * c * c - 1.0)
    return np.array(om) / m, p2 / m


def orientation_batch(batch, x, e):
    """Per RVE of a packed batch: Omega [R,3,3] and P2 [R] at positions x [NN,3]."""
    R = batch.n_rve
    om = np.empty((R, 3, 3))
    p2 = np.empty(R)
    for r in range(R):
        n0, n1 = batch.node_off[r], batch.node_off[r + 1]
        f0, f1 = batch.fib_off[r], batch.fib_off[r + 1]
        om[r], p2[r] = orientation(x[n0:n1], batch.fib[f0:f1], e)
    return om, p2
