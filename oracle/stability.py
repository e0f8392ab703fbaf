"""Validity and stability of a given network state (test infrastructure).

A sub-isostatic fiber network can have several stable equilibria under one
F (the paper notes the networks bifurcate), so two correct relaxations may
end in different states.  Where a GPU result differs from the oracle's, the
tests check the GPU state itself with the oracle's own arithmetic:

* ``equilibrium``: the free-node residual |f_free| and the reaction norm
  |f_bnd| of the internal forces at the state (O5), and the boundary-
  reaction stress of the state (O9);
* ``is_stable``: whether the free-free stiffness K_ff at the state is
  positive definite up to a relative shift, lambda_min >= -rel lambda_max
  (a stable equilibrium: a local minimum of the stored energy), tested by a
  Cholesky factorisation of K_ff + rel lambda_max I with lambda_max from a
  power iteration (which never overestimates it, so the test is not looser
  than the stated bound).

Both use only ``forces``, ``stress`` and ``stiffness_dense`` of the C
oracle, which are pinned against finite differences and closed forms.
"""
from __future__ import annotations

import numpy as np

from . import forces, rest_lengths, stiffness_dense, stress


def equilibrium(net, F, x, opts, V0=1.0, L0=None):
    """(|f_free|_2, |f_bnd|_2, sigma[3,3]) of the internal forces at positions x."""
    fib = np.asarray(net.fib, np.int32)
    L0 = rest_lengths(net.X, fib) if L0 is None else np.asarray(L0, np.float64)
    f, _, _ = forces(x, fib, L0, opts)
    ib = np.asarray(net.is_bnd, bool)
    return (float(np.linalg.norm(f[~ib])), float(np.linalg.norm(f[ib])),
            stress(x, f, net.is_bnd, F, V0))


def is_stable(net, x, opts, rel=1e-8, max_dof=6000, L0=None):
    """True if K_ff at x has lambda_min >= -rel lambda_max (None above max_dof free DOFs)."""
    fib = np.asarray(net.fib, np.int32)
    L0 = rest_lengths(net.X, fib) if L0 is None else np.asarray(L0, np.float64)
    free = np.repeat(~np.asarray(net.is_bnd, bool), 3)
    if free.sum() > max_dof:
        return None
    if free.sum() == 0:
        return True
    K = stiffness_dense(x, fib, L0, opts)[np.ix_(free, free)]
    v = np.random.default_rng(0).standard_normal(K.shape[0])
    lam = 0.0
    for _ in range(50):
        w = K @ v
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            break
        v = w / lam
    lam_max = abs(float(v @ (K @ v))) if lam > 0 else 0.0
    try:
        np.linalg.cholesky(K + (rel * lam_max + 1e-300) * np.eye(K.shape[0]))
        return True
    except np.linalg.LinAlgError:
        return False
