"""The paper's material tangent by finite differences (test infrastructure;
only tests, smoke() and bench.py's CPU baseline use the oracle).

Section 3.2 (material stiffness): the updated-Lagrangian spatial tangent C
is the push-forward C_mnpq = F_mi F_nj A_ijrs F_pr F_qs / J of
A = dPi/dE (Pi the second Piola-Kirchhoff stress, E the Green-Lagrange
strain).  Because Pi does not change under a rotation of the deformed
state, A follows from derivatives in the right stretch U (F = R U):
dPi/dE = dPi/dU (dE/dU)^-1.  With Mandel 6x6 matrices [M] = [dE/dU],
[T] the six probing directions (columns, symmetric positive semi-definite
stretch increments) and [P] the forward differences
(Pi(U + h T_c) - Pi(U)) / h (columns c), [P] = [A][M][T], so
[A] = [P] ([M][T])^-1.

Readings:
* Mandel order (11, 22, 33, 23, 13, 12) with sqrt(2) on the shear entries
  of vectors and of 6x6 representations of minor-symmetric 4th-order
  tensors (the order the paper's printed [M] uses: rows 4..6 carry
  U22 + U33, U11 + U33, U11 + U22).
* Pi(U) is taken from the base solve under F (objectivity); the six probe
  solves run under F = U + h T_c (no rotation), each warm-started from the
  base state rotated back, x0 = (U + h T_c) Xm + R^T (x - F Xm).
* Pi = J F^-1 sigma F^-T from the Cauchy stress of the solve.

Library routines used as steps: numpy eigh (the polar decomposition through
U = sqrt(F^T F)), numpy solve/inv for the 6x6 and 3x3 algebra.
"""
from __future__ import annotations

import math

import numpy as np

from . import INIT_GIVEN, make_opts, solve

S2 = math.sqrt(2.0)
MANDEL = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
WEIGHT = [1.0, 1.0, 1.0, S2, S2, S2]


def to_mandel_vec(S):
    S = np.asarray(S, dtype=np.float64)
    return np.array([WEIGHT[I] * S[i, j] for I, (i, j) in enumerate(MANDEL)])


def from_mandel_vec(v):
    S = np.zeros((3, 3))
    for I, (i, j) in enumerate(MANDEL):
        S[i, j] = S[j, i] = v[I] / WEIGHT[I]
    return S


def to_mandel_mat(A4):
    """6x6 Mandel matrix of a 4th-order tensor with both minor symmetries."""
    out = np.zeros((6, 6))
    for I, (i, j) in enumerate(MANDEL):
        for J, (k, l) in enumerate(MANDEL):
            out[I, J] = WEIGHT[I] * WEIGHT[J] * A4[i, j, k, l]
    return out


def from_mandel_mat(A6):
    A4 = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(MANDEL):
        for J, (k, l) in enumerate(MANDEL):
            v = A6[I, J] / (WEIGHT[I] * WEIGHT[J])
            for a, b in ((i, j), (j, i)):
                for c, d in ((k, l), (l, k)):
                    A4[a, b, c, d] = v
    return A4


def dE_dU(U):
    """4th-order dE_kl/dU_pq on symmetric increments: the symmetrised
    (delta_kq U_pl + delta_lq U_pk + delta_kp U_ql + delta_lp U_qk) / 4."""
    d = np.eye(3)
    M = np.zeros((3, 3, 3, 3))
    for k in range(3):
        for l in range(3):
            for p in range(3):
                for q in range(3):
                    M[k, l, p, q] = 0.25 * (d[k, q] * U[p, l] + d[l, q] * U[p, k] + d[k, p] * U[q, l]
                                            + d[l, p] * U[q, k])
    return M


def probe_directions():
    """The six probing directions of the paper: Mandel columns of [T]."""
    return 0.5 * np.array([[1, 0, 0, 0, S2, S2],
                           [0, 1, 0, S2, 0, S2],
                           [0, 0, 1, S2, S2, 0],
                           [0, 0, 0, 2, 0, 0],
                           [0, 0, 0, 0, 2, 0],
                           [0, 0, 0, 0, 0, 2]], dtype=np.float64)


def polar(F):
    """F = R U with U symmetric positive definite."""
    w, V = np.linalg.eigh(F.T @ F)
    U = (V * np.sqrt(w)) @ V.T
    R = F @ np.linalg.inv(U)
    return R, U


def pk2(F, sigma):
    Fi = np.linalg.inv(F)
    return np.linalg.det(F) * Fi @ sigma @ Fi.T


def push_forward(F, A4):
    J = np.linalg.det(F)
    return np.einsum("mi,nj,ijrs,pr,qs->mnpq", F, F, A4, F, F) / J


def fd_tangent(net, F, x_base, sigma_base, c, opts, h=1e-4, V0=1.0):
    """Mandel 6x6 spatial tangent C (and A, P, [M][T]) of one RVE at its
    converged base state (positions x_base, Cauchy stress sigma_base under
    F).  Returns dict(C, A, P, MT, status) with status the worst probe
    status."""
    Xm = np.asarray(net.X, dtype=np.float64) - 0.5
    R, U = polar(F)
    MT = to_mandel_mat(dE_dU(U)) @ probe_directions()
    Pi0 = pk2(F, sigma_base)
    o = make_opts(law=opts.law, EA=opts.EA, B=opts.B, rhoA=opts.rhoA, alpha=opts.alpha, tol_abs=opts.tol_abs,
                  tol_rel=opts.tol_rel, n_max=opts.n_max, init=INIT_GIVEN, mass=opts.mass)
    fluct = x_base - Xm @ F.T            # zero on boundary nodes
    T = probe_directions()
    P = np.zeros((6, 6))
    worst = 0
    for col in range(6):
        Fp = U + h * from_mandel_vec(T[:, col])
        x0 = Xm @ Fp.T + fluct @ R
        r = solve(net, Fp, c, o, x0=x0, V0=V0)
        worst = max(worst, int(r["status"]))
        P[:, col] = (to_mandel_vec(pk2(Fp, r["sigma"])) - to_mandel_vec(Pi0)) / h
    A6 = P @ np.linalg.inv(MT)
    C6 = to_mandel_mat(push_forward(F, from_mandel_mat(A6)))
    return dict(C=C6, A=A6, P=P, MT=MT, status=worst)


def A_from_dsigma_dF(F, sigma, dsdF):
    """Exact A = dPi/dE (Mandel 6x6) from the exact dsigma/dF (9x9, row
    3i+j, column 3k+l): dPi for a stretch increment dU at F = R U is the
    derivative along dF = R dU, and dE = [dE/dU] dU."""
    R, U = polar(F)
    Fi = np.linalg.inv(F)
    J = np.linalg.det(F)
    Minv = np.linalg.inv(to_mandel_mat(dE_dU(U)))
    cols = []
    for J6 in range(6):
        e = np.zeros(6); e[J6] = 1.0
        dU = from_mandel_vec(e)
        dF = R @ dU
        dsig = (dsdF @ dF.ravel()).reshape(3, 3)
        dJ = J * np.trace(Fi @ dF)
        dFi = -Fi @ dF @ Fi
        dPi = dJ * Fi @ sigma @ Fi.T + J * (dFi @ sigma @ Fi.T + Fi @ dsig @ Fi.T + Fi @ sigma @ dFi.T)
        cols.append(to_mandel_vec(dPi))
    dPi_dU = np.array(cols).T            # Mandel columns per unit Mandel stretch direction
    return dPi_dU @ Minv
