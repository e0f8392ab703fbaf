"""Pins of the oracle's finite-difference material tangent (Section 3.2),
CPU only.

* The Mandel matrix [dE/dU] built from the 4th-order definition equals the
  6x6 matrix the paper prints (as a function of U), for random SPD U.
* Mandel conventions: round trips and inner-product preservation.
* The probe directions the paper prints are positive semi-definite stretch
  increments spanning all six symmetric directions.
* Polar decomposition: R orthogonal, U symmetric positive definite, R U = F.
* On the relaxed lattice (affine, closed-form stress) the forward-difference
  A = dPi/dE agrees to O(h) with A from central differences of the closed
  form, and with A from the exact linearisation dsigma/dF.
* On a small Voronoi network in tension the same O(h) agreement with the
  exact linearisation, and A has the major symmetry of a hyperelastic
  material (exactly for the linearisation, to O(h) for the differences).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense
from oracle import fd_tangent as fdt
from paper_2306_09427_amd import synth
from tests.test_oracle_pins import lattice_stress

S2 = math.sqrt(2.0)


def printed_M(U):
    """The 6x6 Mandel form of dE/dU as printed in Section 3.2."""
    return 0.5 * np.array([
        [2 * U[0, 0], 0, 0, 0, S2 * U[0, 2], S2 * U[0, 1]],
        [0, 2 * U[1, 1], 0, S2 * U[1, 2], 0, S2 * U[0, 1]],
        [0, 0, 2 * U[2, 2], S2 * U[1, 2], S2 * U[0, 2], 0],
        [0, S2 * U[1, 2], S2 * U[1, 2], U[1, 1] + U[2, 2], U[0, 1], U[0, 2]],
        [S2 * U[0, 2], 0, S2 * U[0, 2], U[0, 1], U[0, 0] + U[2, 2], U[1, 2]],
        [S2 * U[0, 1], S2 * U[0, 1], 0, U[0, 2], U[1, 2], U[0, 0] + U[1, 1]]])


def rand_spd(rng):
    A = rng.standard_normal((3, 3))
    return np.eye(3) + 0.2 * (A + A.T)


def test_mandel_dE_dU_matches_printed_matrix():
    rng = np.random.default_rng(0)
    for _ in range(5):
        U = rand_spd(rng)
        np.testing.assert_allclose(fdt.to_mandel_mat(fdt.dE_dU(U)), printed_M(U), atol=1e-15)
        # and it is the derivative of E = (U U - I)/2 along symmetric increments
        dU = fdt.from_mandel_vec(rng.standard_normal(6))
        h = 1e-6
        E = lambda V: 0.5 * (V @ V - np.eye(3))
        dE = (E(U + h * dU) - E(U - h * dU)) / (2 * h)
        np.testing.assert_allclose(fdt.to_mandel_vec(dE), printed_M(U) @ fdt.to_mandel_vec(dU), atol=1e-9)


def test_mandel_conventions():
    rng = np.random.default_rng(1)
    S = fdt.from_mandel_vec(rng.standard_normal(6))
    W = fdt.from_mandel_vec(rng.standard_normal(6))
    np.testing.assert_allclose(fdt.from_mandel_vec(fdt.to_mandel_vec(S)), S, atol=1e-15)
    assert abs(np.sum(S * W) - fdt.to_mandel_vec(S) @ fdt.to_mandel_vec(W)) <= 1e-14
    A6 = rng.standard_normal((6, 6))
    np.testing.assert_allclose(fdt.to_mandel_mat(fdt.from_mandel_mat(A6)), A6, atol=1e-14)
    # 6x6 product = double contraction
    A4 = fdt.from_mandel_mat(A6)
    np.testing.assert_allclose(fdt.to_mandel_vec(np.einsum("ijkl,kl->ij", A4, S)), A6 @ fdt.to_mandel_vec(S),
                               atol=1e-13)


def test_probe_directions_are_psd_and_span():
    T = fdt.probe_directions()
    assert np.linalg.matrix_rank(T) == 6
    for c in range(6):
        w = np.linalg.eigvalsh(fdt.from_mandel_vec(T[:, c]))
        assert w.min() >= -1e-15 and w.max() > 0


def test_polar():
    rng = np.random.default_rng(2)
    F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
    R, U = fdt.polar(F)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(R) - 1) <= 1e-14
    np.testing.assert_allclose(U, U.T, atol=1e-15)
    assert np.linalg.eigvalsh(U).min() > 0
    np.testing.assert_allclose(R @ U, F, atol=1e-14)


def _A_closed_lattice(n, F, law):
    """A = dPi/dE of the lattice closed form, by central differences in U."""
    R, U = fdt.polar(F)
    Minv = np.linalg.inv(fdt.to_mandel_mat(fdt.dE_dU(U)))
    h = 1e-6
    cols = []
    for J in range(6):
        e = np.zeros(6); e[J] = 1.0
        dU = fdt.from_mandel_vec(e)
        Pp = fdt.pk2(U + h * dU, lattice_stress(n, U + h * dU, law))
        Pm = fdt.pk2(U - h * dU, lattice_stress(n, U - h * dU, law))
        cols.append(fdt.to_mandel_vec((Pp - Pm) / (2 * h)))
    return np.array(cols).T @ Minv


@pytest.mark.parametrize("law", [oracle.LINEAR, oracle.EXP])
def test_lattice_fd_tangent_matches_closed_form(law):
    n = 3
    net = synth.lattice_network(n)
    F = np.array([[1.12, 0.04, 0.0], [0.0, 1.08, 0.03], [0.02, 0.0, 1.1]])
    o = oracle.make_opts(law=law, alpha=0.5, tol_abs=1e-13, tol_rel=0.0, n_max=400000)
    base = oracle.solve(net, F, 2.0, o)
    assert base["status"] == 0
    h = 1e-5
    out = fdt.fd_tangent(net, F, base["x"], base["sigma"], 2.0, o, h=h)
    assert out["status"] == 0
    A_ref = _A_closed_lattice(n, F, law)
    err = np.abs(out["A"] - A_ref).max() / np.abs(A_ref).max()
    assert err <= 50 * h
    # exact linearisation route
    A_lin = fdt.A_from_dsigma_dF(F, base["sigma"], dense.tangent_forward(net, F, base["x"], o))
    assert np.abs(A_lin - A_ref).max() / np.abs(A_ref).max() <= 1e-7
    # objectivity: the same A for F and Q F
    Q = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))[0]
    Q = Q if np.linalg.det(Q) > 0 else -Q
    A_rot = fdt.A_from_dsigma_dF(Q @ F, base["sigma"] * 0 + Q @ base["sigma"] @ Q.T,
                                 dense.tangent_forward(net, Q @ F, (net.X - 0.5) @ (Q @ F).T, o))
    assert np.abs(A_rot - A_ref).max() / np.abs(A_ref).max() <= 1e-7


def test_network_fd_tangent_matches_linearisation():
    net = synth.voronoi_network(20, [21, 3, 0])
    F = np.array([[1.1, 0.02, 0.0], [0.0, 1.06, 0.01], [0.01, 0.0, 1.05]])
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-12, n_max=400000)
    base = oracle.solve(net, F, 2.0, o)
    assert base["status"] == 0
    h = 1e-5
    out = fdt.fd_tangent(net, F, base["x"], base["sigma"], 2.0, o, h=h)
    assert out["status"] == 0
    A_lin = fdt.A_from_dsigma_dF(F, base["sigma"], dense.tangent_forward(net, F, base["x"], o))
    err = np.abs(out["A"] - A_lin).max() / np.abs(A_lin).max()
    assert err <= 1e-3
    # a truss network is hyperelastic (Pi = dW/dE): A has the major symmetry,
    # exactly for the linearisation and to O(h) for the differences
    scale = np.abs(A_lin).max()
    assert np.abs(A_lin - A_lin.T).max() <= 1e-9 * scale
    assert np.abs(out["A"] - out["A"].T).max() <= 1e-3 * scale
