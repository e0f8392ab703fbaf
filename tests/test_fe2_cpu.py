"""Pins of the FE^2 driver's macroscale (CPU; Algorithm 1's macro loop).

* Gauss-point deformation gradients equal those of the hex-mesh workload
  generator for the same nodal displacements (an independent per-point
  loop), and are exact for an affine field.
* Patch test: a constant stress P gives zero internal force at interior
  nodes and the face resultants P n A on the x faces.
* dP/dF from (sigma, d sigma/dF) equals the central difference of
  P = J sigma F^-T for a closed-form material (compressible neo-Hookean).
* The assembled stiffness equals the central difference of the internal
  force.
* With that material at every Gauss point the driver converges
  quadratically to the homogeneous uniaxial solution, whose lateral stretch
  solves sigma_yy = 0 (scalar root).
* With gripped x faces the solution is not homogeneous; the driver still
  converges quadratically, the fixed DOFs are the two x faces, and the
  reactions on the two faces balance.
* With every boundary node on an affine map the homogeneous material's
  solution is that affine map: the predictor already satisfies equilibrium.
* A failing step is retried with half the increment after the micro state
  is restored from the last checkpoint.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2306_09427_amd import fe2, synth

MU, LAM = 1.0, 2.0


def nh_sigma(F):
    """Compressible neo-Hookean Cauchy stress, (n,3,3)."""
    J = np.linalg.det(F)
    b = F @ np.transpose(F, (0, 2, 1))
    return (MU * (b - np.eye(3)) + LAM * np.log(J)[:, None, None] * np.eye(3)) / J[:, None, None]


def fd_dsdF(F, fun=nh_sigma, h=1e-6):
    n = len(F)
    out = np.zeros((n, 9, 9))
    for c in range(9):
        E = np.zeros(9); E[c] = h
        E = E.reshape(3, 3)
        out[:, :, c] = ((fun(F + E) - fun(F - E)) / (2 * h)).reshape(n, 9)
    return out


class NeoHookeMicro:
    """A closed-form stand-in for the RVE batch (same interface)."""

    def __init__(self, fail_above=None):
        self.F = None
        self.fail_above = fail_above
        self.restored = 0
        self.solves = 0

    def solve(self, F):
        prev = self.F if self.F is not None else np.eye(3)    # the undeformed start
        self.F = F.copy()
        self.solves += 1
        st = np.zeros(len(F), np.int32)
        if self.fail_above is not None and np.abs(F - prev).max() > self.fail_above:
            st[:] = 2
        return nh_sigma(F), st, np.zeros(len(F), np.int64)

    def tangent(self):
        return fd_dsdF(self.F), np.zeros(len(self.F), np.int32)

    def checkpoint(self):
        return None if self.F is None else self.F.copy()

    def restore(self, state):
        self.restored += 1
        self.F = state


def test_gradients_match_workload_generator():
    mesh = fe2.HexMesh(3, 2, 2)
    u = synth.hex_mesh_u(mesh.X)
    np.testing.assert_allclose(mesh.deformation_gradients(u), synth.hex_mesh_F(3, 2, 2), rtol=0, atol=1e-14)
    G = np.array([[0.1, 0.02, -0.03], [0.0, -0.04, 0.05], [0.01, 0.02, 0.03]])
    Fg = mesh.deformation_gradients(mesh.X @ G.T)
    np.testing.assert_allclose(Fg, np.broadcast_to(np.eye(3) + G, Fg.shape), atol=1e-14)


def test_patch_test_constant_stress():
    mesh = fe2.HexMesh(3, 2, 2)
    P = np.array([[1.0, 0.2, -0.3], [0.4, 2.0, 0.1], [-0.2, 0.3, 0.5]])
    f = mesh.internal_force(np.broadcast_to(P, (mesh.n_gp, 3, 3)).copy())
    X = mesh.X
    interior = (X[:, 0] > 0) & (X[:, 0] < 3) & (X[:, 1] > 0) & (X[:, 1] < 2) & (X[:, 2] > 0) & (X[:, 2] < 2)
    assert interior.sum() > 0
    assert np.abs(f[interior]).max() <= 1e-14
    area = 2 * 2
    np.testing.assert_allclose(f[X[:, 0] == 3].sum(0), P[:, 0] * area, atol=1e-13)
    np.testing.assert_allclose(f[X[:, 0] == 0].sum(0), -P[:, 0] * area, atol=1e-13)
    np.testing.assert_allclose(f.sum(0), 0.0, atol=1e-12)


def test_first_pk_derivative():
    rng = np.random.default_rng(0)
    F = np.eye(3) + 0.15 * rng.standard_normal((4, 3, 3))
    sig = nh_sigma(F)
    _, A = fe2.first_pk(F, sig, fd_dsdF(F))
    P_of = lambda G: fe2.first_pk(G, nh_sigma(G))[0]
    A_fd = fd_dsdF(F, P_of)
    assert np.abs(A - A_fd).max() <= 1e-7 * np.abs(A_fd).max()


def test_stiffness_is_derivative_of_internal_force():
    mesh = fe2.HexMesh(2, 1, 1)
    rng = np.random.default_rng(1)
    u = 0.05 * rng.standard_normal((mesh.n_nodes, 3))
    F = mesh.deformation_gradients(u)
    _, A = fe2.first_pk(F, nh_sigma(F), fd_dsdF(F))
    K = mesh.stiffness(A).toarray()
    du = rng.standard_normal((mesh.n_nodes, 3))
    h = 1e-6
    fp = mesh.internal_force(fe2.first_pk(mesh.deformation_gradients(u + h * du), nh_sigma(mesh.deformation_gradients(u + h * du)))[0])
    fm = mesh.internal_force(fe2.first_pk(mesh.deformation_gradients(u - h * du), nh_sigma(mesh.deformation_gradients(u - h * du)))[0])
    d = ((fp - fm) / (2 * h)).ravel()
    assert np.abs(K @ du.ravel() - d).max() <= 1e-6 * np.abs(d).max()
    np.testing.assert_allclose(K, K.T, atol=1e-8 * np.abs(K).max())   # hyperelastic: symmetric


def test_driver_homogeneous_uniaxial_solution():
    mesh = fe2.HexMesh(3, 2, 2)
    micro = NeoHookeMicro()
    drv = fe2.FE2(mesh, micro, tol=1e-12, max_newton=12)
    lam = 1.2
    hist = drv.run(lam, 2)
    assert all(h.converged for h in hist) and len(hist) == 2
    mu = brentq(lambda m: nh_sigma(np.diag([lam, m, m])[None])[0, 1, 1], 0.5, 1.0)
    np.testing.assert_allclose(drv.F, np.broadcast_to(np.diag([lam, mu, mu]), drv.F.shape), atol=1e-9)
    # quadratic convergence: each residual at most ~ the square of the previous (times a constant)
    r = hist[-1].residual
    assert len(r) <= 7
    for a, b in zip(r[1:-1], r[2:]):
        assert b <= 10 * a * a + 1e-13


def test_failed_step_is_cut_back_and_restored():
    mesh = fe2.HexMesh(2, 1, 1)
    micro = NeoHookeMicro(fail_above=0.08)        # increments of F above 0.08 "fail"
    drv = fe2.FE2(mesh, micro, tol=1e-10)
    hist = drv.run(1.2, 1)                        # one step of 0.2 must be cut to 0.05
    assert micro.restored >= 2
    assert not hist[0].converged and hist[-1].converged
    assert abs(drv.lam - 1.2) <= 1e-14
    with pytest.raises(RuntimeError):
        fe2.FE2(mesh, NeoHookeMicro(fail_above=1e-9), tol=1e-10).run(1.2, 1, max_cutbacks=2)


def test_driver_clamped_converges():
    mesh = fe2.HexMesh(3, 2, 2)
    dofs, vals = mesh.boundary_dofs(1.1, "clamped")
    x_faces = (mesh.X[:, 0] == 0) | (mesh.X[:, 0] == 3)
    assert len(dofs) == 3 * x_faces.sum()
    drv = fe2.FE2(mesh, NeoHookeMicro(), tol=1e-12, max_newton=12, bc="clamped")
    hist = drv.run(1.1, 2)
    assert hist[-1].converged
    r = hist[-1].residual
    for a, b in zip(r[1:-1], r[2:]):
        assert b <= 10 * a * a + 1e-13
    assert np.ptp(drv.F[:, 1, 1]) > 1e-3                 # lateral contraction varies along x
    P, _ = fe2.first_pk(drv.F, drv.sigma)
    f = mesh.internal_force(P)
    np.testing.assert_allclose(f[mesh.X[:, 0] == 0].sum(0), -f[mesh.X[:, 0] == 3].sum(0), atol=1e-10)
    with pytest.raises(ValueError):
        mesh.boundary_dofs(1.1, "periodic")


def test_driver_affine_boundary_homogeneous():
    mesh = fe2.HexMesh(3, 3, 3)
    dofs, vals = mesh.boundary_dofs(1.1, "affine")
    on = np.zeros(mesh.n_nodes, bool)
    for k in range(3):
        on |= (mesh.X[:, k] == 0) | (mesh.X[:, k] == 3)
    assert len(dofs) == 3 * on.sum()
    drv = fe2.FE2(mesh, NeoHookeMicro(), tol=1e-12, bc="affine")
    hist = drv.run(1.1, 2)
    assert all(h.converged for h in hist)
    np.testing.assert_allclose(drv.F, np.broadcast_to(np.diag([1.1, 1.05, 1.05]), drv.F.shape), atol=1e-12)
    assert all(len(h.residual) <= 2 for h in hist)
