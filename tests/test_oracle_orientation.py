"""Pins of the oracle's fiber-orientation outputs (CPU).

The orientation tensor Omega = <n n^T> and the degree of alignment
P2 = <(3 cos^2 theta - 1)/2> (Section 6: second Legendre polynomial of the
angle between the fiber direction and a reference direction, averaged over
the fibers) are pinned to what geometry fixes: the six axis directions
(isotropic: Omega = I/3, P2 = 0 for every e), fully aligned and fully
perpendicular sets (P2 = 1 and -1/2, the range the paper states), the
relaxed lattice under any F (affine: fibers along F e_k, equal counts per
axis), rotation covariance, and the identities trace Omega = 1 and
P2 = (3 e.Omega.e - 1)/2.
"""
import numpy as np
import pytest

import oracle
from oracle import orientation as orient
from paper_2306_09427_amd import synth


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_axis_star_is_isotropic():
    # six fibers from the origin along +-e_k
    x = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 2, 0], [0, -1, 0], [0, 0, 3], [0, 0, -0.5]], float)
    fib = np.array([[0, k] for k in range(1, 7)])
    for e in ([1, 0, 0], [0.3, -0.2, 0.9], [1, 1, 1]):
        om, p2 = orient.orientation(x, fib, e)
        np.testing.assert_allclose(om, np.eye(3) / 3, atol=1e-15)
        assert abs(p2) <= 1e-15


def test_aligned_and_perpendicular_limits():
    rng = np.random.default_rng(1)
    e = np.array([0.2, 0.5, -0.3])
    eu = e / np.linalg.norm(e)
    # all fibers parallel (either sense) to e
    pts = [np.zeros(3)]
    for s in rng.uniform(-2, 2, 7):
        pts.append(s * e if abs(s) > 0.1 else 0.5 * e)
    x = np.array(pts)
    fib = np.array([[0, k] for k in range(1, len(pts))])
    om, p2 = orient.orientation(x, fib, e)
    assert abs(p2 - 1.0) <= 1e-14
    np.testing.assert_allclose(om, np.outer(eu, eu), atol=1e-14)
    # all fibers perpendicular to e
    u = np.cross(eu, [1.0, 0, 0]); u /= np.linalg.norm(u)
    w = np.cross(eu, u)
    x = np.array([np.zeros(3)] + [np.cos(t) * u + np.sin(t) * w for t in rng.uniform(0, 6.3, 9)])
    fib = np.array([[0, k] for k in range(1, 10)])
    om, p2 = orient.orientation(x, fib, e)
    assert abs(p2 + 0.5) <= 1e-14
    assert abs(eu @ om @ eu) <= 1e-14


@pytest.mark.parametrize("law", [oracle.LINEAR, oracle.EXP])
def test_relaxed_lattice_matches_affine_directions(law):
    net = synth.lattice_network(3)
    F = np.array([[1.1, 0.05, 0.0], [0.02, 1.04, 0.03], [0.0, -0.01, 1.06]])
    o = oracle.make_opts(law=law, alpha=0.5, tol_abs=1e-13, tol_rel=0.0, n_max=200000)
    out = oracle.solve(net, F, 2.0, o)
    assert out["status"] == 0
    e = np.array([1.0, 0.2, -0.1])
    om, p2 = orient.orientation(out["x"], net.fib, e)
    # equal numbers of fibers along each axis, each mapped to F e_k
    expect = np.zeros((3, 3))
    for k in range(3):
        n = F[:, k] / np.linalg.norm(F[:, k])
        expect += np.outer(n, n) / 3
    np.testing.assert_allclose(om, expect, atol=1e-12)
    eu = e / np.linalg.norm(e)
    assert abs(p2 - 0.5 * (3 * eu @ expect @ eu - 1)) <= 1e-12


def test_rotation_covariance_and_identities():
    net = synth.voronoi_network(40, [9, 1, 0])
    x = net.X - 0.5 + 0.01 * np.random.default_rng(2).standard_normal(net.X.shape)
    e = np.array([0.3, -1.0, 0.4])
    om, p2 = orient.orientation(x, net.fib, e)
    assert abs(np.trace(om) - 1) <= 1e-14
    np.testing.assert_allclose(om, om.T, atol=0)
    eu = e / np.linalg.norm(e)
    assert abs(p2 - 0.5 * (3 * eu @ om @ eu - 1)) <= 1e-14
    assert -0.5 - 1e-15 <= p2 <= 1 + 1e-15
    Q = _rot(5)
    om_q, p2_q = orient.orientation(x @ Q.T, net.fib, Q @ e)
    np.testing.assert_allclose(om_q, Q @ om @ Q.T, atol=1e-14)
    assert abs(p2_q - p2) <= 1e-14
