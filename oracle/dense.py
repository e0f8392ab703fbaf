"""Dense-matrix oracle checks for small networks (test infrastructure).

* ``newton``: brute-force Newton on the stored energy for tiny networks
  (an independent route to the same static equilibrium the relaxation
  reaches; the paper's implicit micro solver, Section 3.2, is a Newton
  method on the same truss).
* ``tangent_forward``: the exact linearisation dsigma/dF of the boundary-
  reaction stress at a converged state.  For each direction E = e_k e_l the
  boundary moves by dx_b = E Xm_b, the free nodes follow from
  K_ff dx_f = -K_fb dx_b, the reactions change by df_b = K_bf dx_f + K_bb dx_b,
  and dsigma = (sum_b df_b x_b^T + f_b (E Xm_b)^T)/(J V0) - sigma (F^-1)_lk
  (derivative of J = det F is J F^-T).  Singular K_ff (mechanisms) is
  handled with the minimum-norm solution.
* ``tangent_fd``: central finite differences of relaxed stresses in F.

The stiffness comes from ``or_stiffness_dense`` in the C oracle; its
agreement with finite differences of the forces is itself a pinned test.
"""
from __future__ import annotations

import numpy as np

from . import (INIT_GIVEN, forces, make_opts, rest_lengths, solve, stiffness_dense, stress)


def _centred(X):
    return np.asarray(X, dtype=np.float64) - 0.5


def energy_and_grad(x, fib, L0, opts):
    f, _, W = forces(x, fib, L0, opts)
    return W, f


def newton(net, F, opts, x0=None, tol=1e-14, max_iter=200):
    """Minimise the stored energy over free positions (boundary fixed at F Xm).

    Returns (x, sigma, |r|, stable) where stable means the final K_ff is
    positive definite (Cholesky succeeds)."""
    Xm = _centred(net.X)
    fib = np.asarray(net.fib, np.int32)
    L0 = rest_lengths(net.X, fib)
    ib = np.asarray(net.is_bnd, bool)
    x = Xm @ F.T if x0 is None else np.array(x0, dtype=np.float64)
    x[ib] = Xm[ib] @ F.T
    free = np.repeat(~ib, 3)
    rnorm = np.inf
    for _ in range(max_iter):
        W, f = energy_and_grad(x, fib, L0, opts)
        g = f.ravel()[free]
        rnorm = np.linalg.norm(g)
        if rnorm <= tol:
            break
        K = stiffness_dense(x, fib, L0, opts)[np.ix_(free, free)]
        try:
            step = -np.linalg.solve(K, g)
        except np.linalg.LinAlgError:
            step = -np.linalg.lstsq(K, g, rcond=None)[0]
        if g @ step >= 0:            # not a descent direction: fall back to steepest descent
            step = -g / max(1.0, np.abs(np.diag(K)).max())
        t = 1.0
        xs = x.copy()
        while t > 1e-12:
            xt = xs.copy()
            xt.ravel()[free] += t * step
            Wt, _ = energy_and_grad(xt, fib, L0, opts)
            if Wt <= W + 1e-4 * t * (g @ step) or abs(Wt - W) <= 1e-15 * max(1.0, abs(W)):
                x = xt
                break
            t *= 0.5
        else:
            break
    W, f = energy_and_grad(x, fib, L0, opts)
    K = stiffness_dense(x, fib, L0, opts)[np.ix_(free, free)]
    try:
        np.linalg.cholesky(K)
        stable = True
    except np.linalg.LinAlgError:
        stable = False
    sig = stress(x, f, net.is_bnd, F)
    return x, sig, float(np.linalg.norm(f.ravel()[free])), stable


def tangent_forward(net, F, x, opts, V0=1.0):
    """Exact dsigma/dF (9x9, row 3i+j = sigma_ij, column 3k+l = F_kl) at the
    equilibrium x (boundary nodes at F Xm)."""
    Xm = _centred(net.X)
    fib = np.asarray(net.fib, np.int32)
    L0 = rest_lengths(net.X, fib)
    ib = np.asarray(net.is_bnd, bool)
    n = len(Xm)
    K = stiffness_dense(x, fib, L0, opts)
    free = np.repeat(~ib, 3)
    bnd = ~free
    Kff = K[np.ix_(free, free)]
    f, _, _ = forces(x, fib, L0, opts)
    J = np.linalg.det(F)
    sig = stress(x, f, net.is_bnd, F, V0)
    Finv = np.linalg.inv(F)
    out = np.zeros((9, 9))
    Kff_pinv = None
    for k in range(3):
        for l in range(3):
            E = np.zeros((3, 3)); E[k, l] = 1.0
            dx = np.zeros((n, 3))
            dx[ib] = Xm[ib] @ E.T
            rhs = -(K[:, bnd] @ dx.ravel()[bnd])[free]
            try:
                dxf = np.linalg.solve(Kff, rhs)
                if not np.all(np.isfinite(dxf)):
                    raise np.linalg.LinAlgError
            except np.linalg.LinAlgError:
                if Kff_pinv is None:
                    Kff_pinv = np.linalg.pinv(Kff, rcond=1e-12, hermitian=True)
                dxf = Kff_pinv @ rhs
            full = dx.ravel().copy()
            full[free] = dxf
            df = (K @ full).reshape(n, 3)
            dtau = df[ib].T @ x[ib] + f[ib].T @ dx[ib]
            dsig = dtau / (J * V0) - sig * Finv[l, k]
            out[:, 3 * k + l] = dsig.ravel()
    return out


def tangent_fd(net, F, x_base, c, opts, h=1e-6, V0=1.0):
    """Central finite differences of the relaxed stress in each F_kl.

    Each +/- solve starts from the converged base state shifted by the
    affine part of the perturbation (warm start)."""
    Xm = _centred(net.X)
    out = np.zeros((9, 9))
    o = make_opts(law=opts.law, EA=opts.EA, B=opts.B, rhoA=opts.rhoA, alpha=opts.alpha,
                  tol_abs=opts.tol_abs, tol_rel=opts.tol_rel, n_max=opts.n_max, init=INIT_GIVEN,
                  mass=opts.mass)
    for k in range(3):
        for l in range(3):
            E = np.zeros((3, 3)); E[k, l] = 1.0
            s = []
            for sgn in (1.0, -1.0):
                Fp = F + sgn * h * E
                x0 = x_base + sgn * h * (Xm @ E.T)
                r = solve(net, Fp, c, o, x0=x0, V0=V0)
                s.append(r["sigma"])
            out[:, 3 * k + l] = ((s[0] - s[1]) / (2 * h)).ravel()
    return out
