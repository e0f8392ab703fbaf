"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, brute force, or a finite difference.  Together they are
chosen so that a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_09427_amd import synth

LIN, EXP = oracle.LINEAR, oracle.EXP


def rand_rotation(rng):
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def law_T(law, eps, EA=1.0, B=10.0):
    """Fiber axial force written out independently of the oracle."""
    if law == EXP and eps >= 0:
        return EA * np.expm1(B * eps) / B
    return EA * eps


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("law", [LIN, EXP])
def test_identity_F_is_stress_free(law):
    """F = I: every fiber keeps its rest length, so R0 = 0, sigma = 0, 0 iterations."""
    net = synth.voronoi_network(60, [11, 0, 0])
    r = oracle.solve(net, np.eye(3), 1.0, oracle.make_opts(law=law, tol_abs=1e-12))
    assert r["status"] == oracle.CONVERGED
    assert r["iters"] == 0
    assert np.max(np.abs(r["sigma"])) < 1e-13


# ------------------------------------------------------------------ P2
@pytest.mark.parametrize("law", [LIN, EXP])
def test_single_fiber_closed_form(law):
    """Both ends on the boundary: sigma = T(eps) l n n^T / (J V0)."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        Xa, Xb = rng.random(3), rng.random(3)
        net = synth.single_fiber_network(Xa, Xb)
        F = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        if np.linalg.det(F) <= 0:
            continue
        V0 = 0.7
        r = oracle.solve(net, F, 1.0, oracle.make_opts(law=law), V0=V0)
        d = F @ (Xb - Xa)
        l = np.linalg.norm(d)
        eps = l / np.linalg.norm(Xb - Xa) - 1.0
        expect = law_T(law, eps) * np.outer(d, d) / l / (np.linalg.det(F) * V0)
        assert r["iters"] == 0
        np.testing.assert_allclose(r["sigma"], expect, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------ P3
@pytest.mark.parametrize("law", [LIN, EXP])
def test_chain_equal_strain(law):
    """A zig-zag chain between two boundary nodes straightens under tension;
    every segment then has the same strain eps = l_total/sum(L0) - 1."""
    rng = np.random.default_rng(5)
    k = 5
    t = np.linspace(0.0, 1.0, k + 1)
    pts = np.stack([0.2 + 0.6 * t, 0.5 + 0.03 * rng.standard_normal(k + 1),
                    0.5 + 0.03 * rng.standard_normal(k + 1)], 1)
    pts[0, 1:] = pts[-1, 1:] = 0.5
    net = synth.chain_network(pts)
    L0 = np.linalg.norm(np.diff(pts, axis=0), axis=1)
    F = np.array([[1.3, 0.05, 0.0], [0.02, 0.95, 0.0], [0.0, 0.0, 1.0]])
    # the reference start puts the end segments at large strain, which the
    # exponential law turns into an explosive force, so that law starts affine
    init = oracle.INIT_REFERENCE if law == LIN else oracle.INIT_AFFINE
    r = oracle.solve(net, F, 2.0, oracle.make_opts(law=law, tol_abs=1e-12, n_max=2_000_000,
                                                   init=init, alpha=0.5))
    assert r["status"] == oracle.CONVERGED and r["iters"] > 10
    d = F @ (pts[-1] - pts[0])
    ltot = np.linalg.norm(d)
    eps = ltot / L0.sum() - 1.0
    assert eps > 0
    expect = law_T(law, eps) * np.outer(d, d) / ltot / np.linalg.det(F)
    np.testing.assert_allclose(r["sigma"], expect, rtol=1e-9, atol=1e-12)
    # every segment at the common strain
    seg = np.linalg.norm(np.diff(r["x"], axis=0), axis=1)
    np.testing.assert_allclose(seg / L0 - 1.0, eps, atol=1e-9)


# ------------------------------------------------------------------ P4
def lattice_stress(n, F, law):
    """Closed-form stress of the n^3 lattice at its affine state (virial):
    sigma = 1/J sum_k (n+1)^2 T(|F e_k| - 1) (F e_k)(F e_k)^T / |F e_k|."""
    s = np.zeros((3, 3))
    for k in range(3):
        a = F[:, k]
        la = np.linalg.norm(a)
        s += (n + 1) ** 2 * law_T(law, la - 1.0) * np.outer(a, a) / la
    return s / np.linalg.det(F)


@pytest.mark.parametrize("law", [LIN, EXP])
@pytest.mark.parametrize("n", [2, 3, 5])
def test_cubic_lattice_affine_stress(law, n):
    rng = np.random.default_rng(100 + n)
    net = synth.lattice_network(n)
    while True:
        F = np.eye(3) * 1.1 + 0.05 * rng.standard_normal((3, 3))
        if min(np.linalg.norm(F, axis=0)) >= 1.02:
            break
    Xm = net.X - 0.5
    x0 = Xm @ F.T + 0.01 * rng.standard_normal(Xm.shape)      # random start
    o = oracle.make_opts(law=law, tol_abs=1e-12, init=oracle.INIT_GIVEN, n_max=2_000_000)
    r = oracle.solve(net, F, 2.0, o, x0=x0)
    assert r["status"] == oracle.CONVERGED and r["iters"] > 10
    np.testing.assert_allclose(r["sigma"], lattice_stress(n, F, law), rtol=1e-10, atol=1e-12)
    # the relaxed state is the affine one
    np.testing.assert_allclose(r["x"], Xm @ F.T, atol=1e-9)


# ------------------------------------------------------------------ P5/P6/P7
def test_balance_and_virial_invariants():
    """At the relaxed state: reactions sum to ~0 (momentum), tau is ~symmetric
    (moment), and tau equals the fiber virial sum T l n n^T."""
    net = synth.voronoi_network(80, [12, 0, 0])
    F = np.diag([1.15, 1.05, 1.0])
    o = oracle.make_opts(law=EXP, tol_abs=1e-11, n_max=2_000_000, alpha=0.5)
    r = oracle.solve(net, F, 2.0, o)
    assert r["status"] == oracle.CONVERGED
    fib = net.fib
    L0 = oracle.rest_lengths(net.X, fib)
    f, _, _ = oracle.forces(r["x"], fib, L0, o)
    ib = net.is_bnd.astype(bool)
    Rf = np.linalg.norm(f[~ib])
    assert Rf <= 1e-11 * 1.0001
    nfree = int((~ib).sum())
    # P5 momentum: sum over all nodes is exactly zero, so the boundary sum is
    # bounded by the free residual
    assert np.linalg.norm(f[ib].sum(0)) <= np.sqrt(nfree) * Rf + 1e-13
    # P7 virial: sum_all f_a x_a^T == sum_f T l n n^T
    x = r["x"]
    d = x[fib[:, 1]] - x[fib[:, 0]]
    l = np.linalg.norm(d, axis=1)
    T = np.array([law_T(EXP, e) for e in l / L0 - 1.0])
    vir = np.einsum("f,fi,fj->ij", T / l, d, d)
    tau_b = f[ib].T @ x[ib]
    xf2 = np.sqrt((x[~ib] ** 2).sum())
    assert np.abs(tau_b - vir).max() <= Rf * xf2 + 1e-12
    # P6 moment balance
    assert np.abs(tau_b - tau_b.T).max() <= 2 * Rf * xf2 + 1e-12
    J = np.linalg.det(F)
    np.testing.assert_allclose(r["sigma"], tau_b / J, rtol=1e-12)


# ------------------------------------------------------------------ P8
def test_objectivity():
    """sigma(QF) = Q sigma(F) Q^T (the time-step rule is rotation invariant)."""
    rng = np.random.default_rng(8)
    net = synth.voronoi_network(60, [13, 0, 0])
    F = np.diag([1.2, 1.1, 1.05])
    Q = rand_rotation(rng)
    o = oracle.make_opts(law=EXP, tol_abs=1e-11, n_max=2_000_000, alpha=0.5)
    a = oracle.solve(net, F, 2.0, o)
    b = oracle.solve(net, Q @ F, 2.0, o)
    assert a["status"] == b["status"] == oracle.CONVERGED
    np.testing.assert_allclose(b["sigma"], Q @ a["sigma"] @ Q.T, rtol=1e-8, atol=1e-10)


# ------------------------------------------------------------------ P9
def test_EA_linearity():
    """sigma(s EA) = s sigma(EA) with c scaled by sqrt(s) and the tolerance by s:
    the scaled relaxation is the same trajectory in rescaled time."""
    net = synth.voronoi_network(60, [14, 0, 0])
    F = np.diag([1.2, 1.1, 1.05])
    s = 7.0
    a = oracle.solve(net, F, 2.0, oracle.make_opts(law=EXP, EA=1.0, tol_abs=1e-11, alpha=0.5))
    b = oracle.solve(net, F, 2.0 * np.sqrt(s), oracle.make_opts(law=EXP, EA=s, tol_abs=s * 1e-11, alpha=0.5))
    assert a["status"] == b["status"] == oracle.CONVERGED
    assert abs(a["iters"] - b["iters"]) <= 2
    np.testing.assert_allclose(b["sigma"], s * a["sigma"], rtol=1e-8, atol=1e-10)


# ------------------------------------------------------------------ P10
def test_fictitious_parameter_independence():
    """On a network with a unique equilibrium (lattice), sigma does not depend
    on the damping, the time-step safety factor, rhoA or the mass choice."""
    net = synth.lattice_network(3)
    F = np.array([[1.2, 0.05, 0.0], [0.0, 1.1, 0.02], [0.03, 0.0, 1.08]])
    ref = lattice_stress(3, F, EXP)
    rng = np.random.default_rng(1)
    x0 = (net.X - 0.5) @ F.T + 0.01 * rng.standard_normal(net.X.shape)
    for c, alpha, rhoA, mass in [(1.0, 0.9, 1.0, 0), (4.0, 0.5, 3.0, 0), (0.3, 0.7, 1.0, 1)]:
        o = oracle.make_opts(law=EXP, tol_abs=1e-12, alpha=alpha, rhoA=rhoA, mass=mass,
                             init=oracle.INIT_GIVEN, n_max=2_000_000)
        r = oracle.solve(net, F, c, o, x0=x0)
        assert r["status"] == oracle.CONVERGED
        np.testing.assert_allclose(r["sigma"], ref, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------------ P11
@pytest.mark.parametrize("law", [LIN, EXP])
def test_relaxation_matches_brute_force_newton(law):
    F = np.array([[1.2, 0.04, 0.0], [0.0, 1.12, 0.03], [0.02, 0.0, 1.1]])
    checked = 0
    for seed in range(6):
        net = synth.voronoi_network(15, [15, seed, 0])
        if net.n_free == 0 or net.n_free > 50:
            continue
        xN, sN, rN, stable = dense.newton(net, F, oracle.make_opts(law=law))
        if not stable or rN > 1e-12:
            continue
        o = oracle.make_opts(law=law, tol_abs=1e-12, n_max=5_000_000, alpha=0.5)
        r = oracle.solve(net, F, 2.0, o)
        assert r["status"] == oracle.CONVERGED
        scale = np.abs(sN).max()
        assert np.abs(r["sigma"] - sN).max() <= 1e-9 * scale
        checked += 1
    assert checked >= 2


# ------------------------------------------------------------------ P12
@pytest.mark.parametrize("law", [LIN, EXP])
def test_forces_and_stiffness_are_derivatives(law):
    """f = dW/dx and K = df/dx by central differences (h = 1e-6)."""
    rng = np.random.default_rng(12)
    net = synth.voronoi_network(10, [16, 0, 0])
    o = oracle.make_opts(law=law)
    L0 = oracle.rest_lengths(net.X, net.fib)
    x = (net.X - 0.5) @ (np.eye(3) * 1.1).T + 0.01 * rng.standard_normal(net.X.shape)
    f, G, W = oracle.forces(x, net.fib, L0, o)
    K = oracle.stiffness_dense(x, net.fib, L0, o)
    h = 1e-6
    n = len(x)
    fd_f = np.zeros(3 * n)
    fd_K = np.zeros((3 * n, 3 * n))
    for k in range(3 * n):
        xp = x.copy(); xp.ravel()[k] += h
        xm = x.copy(); xm.ravel()[k] -= h
        fp, _, Wp = oracle.forces(xp, net.fib, L0, o)
        fm, _, Wm = oracle.forces(xm, net.fib, L0, o)
        fd_f[k] = (Wp - Wm) / (2 * h)
        fd_K[:, k] = (fp - fm).ravel() / (2 * h)
    np.testing.assert_allclose(f.ravel(), fd_f, atol=1e-7 * max(1, np.abs(f).max()))
    np.testing.assert_allclose(K, fd_K, atol=1e-6 * max(1, np.abs(K).max()))
    # Gershgorin sums bound the spectrum of the stiffness
    lam = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert lam.max() <= np.repeat(G, 3).max() * (1 + 1e-12)


def test_timestep_bound_is_stable_on_linear_problem():
    """For the linear law the Gershgorin bound dominates the true lambda_max(M^-1 K)."""
    net = synth.voronoi_network(40, [17, 0, 0])
    o = oracle.make_opts(law=LIN)
    L0 = oracle.rest_lengths(net.X, net.fib)
    x = (net.X - 0.5) @ np.diag([1.1, 1.0, 0.95]).T
    _, G, _ = oracle.forces(x, net.fib, L0, o)
    K = oracle.stiffness_dense(x, net.fib, L0, o)
    M = np.zeros(net.n_nodes)
    np.add.at(M, net.fib[:, 0], 0.5 * L0); np.add.at(M, net.fib[:, 1], 0.5 * L0)
    fr = ~net.is_bnd.astype(bool)
    idx = np.repeat(fr, 3)
    Mi = np.repeat(1.0 / np.sqrt(M), 3)[idx]
    A = Mi[:, None] * K[np.ix_(idx, idx)] * Mi[None, :]
    lam = np.linalg.eigvalsh(0.5 * (A + A.T)).max()
    assert lam <= (G[fr] / M[fr]).max() * (1 + 1e-12)


# ------------------------------------------------------------------ P13/P15
def test_tangent_forward_matches_fd_and_is_objective():
    F = np.array([[1.2, 0.04, 0.0], [0.0, 1.12, 0.03], [0.02, 0.0, 1.1]])
    o = oracle.make_opts(law=EXP, tol_abs=1e-13, n_max=5_000_000, alpha=0.5)
    done = 0
    for seed in range(6):
        net = synth.voronoi_network(15, [15, seed, 0])
        if net.n_free == 0:
            continue
        r = oracle.solve(net, F, 2.0, o)
        if r["status"] != oracle.CONVERGED:
            continue
        xN, sN, rN, stable = dense.newton(net, F, o, x0=r["x"])
        if not stable:
            continue
        Cf = dense.tangent_forward(net, F, xN, o)
        Cd = dense.tangent_fd(net, F, xN, 2.0, o, h=1e-5)
        scale = np.abs(Cf).max()
        assert np.abs(Cf - Cd).max() <= 1e-5 * scale
        # P15: d sigma along an infinitesimal rotation W F equals W sigma - sigma W
        Wsk = np.array([[0.0, 0.3, -0.2], [-0.3, 0.0, 0.5], [0.2, -0.5, 0.0]])
        dF = (Wsk @ F).ravel()
        dsig = (Cf @ dF).reshape(3, 3)
        np.testing.assert_allclose(dsig, Wsk @ sN - sN @ Wsk, atol=1e-8 * scale)
        done += 1
    assert done >= 2


# ------------------------------------------------------------------ P14
def test_lattice_tangent_matches_closed_form_derivative():
    net = synth.lattice_network(3)
    F = np.array([[1.2, 0.05, 0.0], [0.0, 1.1, 0.02], [0.03, 0.0, 1.08]])
    o = oracle.make_opts(law=EXP)
    x = (net.X - 0.5) @ F.T
    C = dense.tangent_forward(net, F, x, o)
    h = 1e-6
    Cd = np.zeros((9, 9))
    for k in range(9):
        E = np.zeros(9); E[k] = h
        Cd[:, k] = ((lattice_stress(3, F + E.reshape(3, 3), EXP)
                     - lattice_stress(3, F - E.reshape(3, 3), EXP)) / (2 * h)).ravel()
    np.testing.assert_allclose(C, Cd, atol=1e-6 * np.abs(Cd).max())


def test_bad_F_and_nonfinite_status():
    net = synth.voronoi_network(20, [18, 0, 0])
    o = oracle.make_opts(law=EXP)
    r = oracle.solve(net, np.diag([1.0, 1.0, -1.0]), 1.0, o)
    assert r["status"] == oracle.BAD_F and np.all(np.isnan(r["sigma"]))
    F = np.eye(3); F[0, 1] = np.nan
    assert oracle.solve(net, F, 1.0, o)["status"] == oracle.BAD_F
    r = oracle.solve(net, np.diag([1.1, 1, 1]), 1.0, oracle.make_opts(law=EXP, n_max=3, tol_abs=0))
    assert r["status"] == oracle.MAXITER and r["iters"] == 3 and np.all(np.isfinite(r["sigma"]))


def test_batch_driver_matches_single_solves():
    batch, F = synth.make_config_batch(2, idx=[0, 5, 9], workers=1)
    o = oracle.make_opts(law=EXP, tol_rel=1e-8, tol_abs=0, n_max=2000, alpha=0.5)
    rb = oracle.solve_batch(batch, F, 1.0, o, threads=3)
    for k in range(3):
        rs = oracle.solve(batch.network(k), F[k], 1.0, o)
        assert rs["iters"] == rb["iters"][k] and rs["status"] == rb["status"][k]
        np.testing.assert_array_equal(rs["sigma"], rb["sigma"][k])


# ------------------------------------------------------------------ O6 pin
def test_gershgorin_sums_equal_block_row_norms():
    """G_a = 2 sum_{fibers at a} |B_f|_2, and each off-diagonal 3x3 block of
    the (finite-difference-pinned) stiffness is -B_f, so G_a must equal twice
    the sum of the spectral norms of node a's off-diagonal blocks."""
    rng = np.random.default_rng(21)
    net = synth.voronoi_network(12, [19, 0, 0])
    for law in (LIN, EXP):
        o = oracle.make_opts(law=law)
        L0 = oracle.rest_lengths(net.X, net.fib)
        x = (net.X - 0.5) @ np.diag([1.15, 0.9, 1.05]).T + 0.01 * rng.standard_normal(net.X.shape)
        _, G, _ = oracle.forces(x, net.fib, L0, o)
        K = oracle.stiffness_dense(x, net.fib, L0, o)
        n = net.n_nodes
        pairs = {tuple(sorted(p)) for p in net.fib.tolist()}
        assert len(pairs) == len(net.fib)          # no parallel fibers
        for a in range(n):
            s = 0.0
            for b in range(n):
                if b != a:
                    s += np.linalg.norm(K[3 * a:3 * a + 3, 3 * b:3 * b + 3], 2)
            assert G[a] == pytest.approx(2.0 * s, rel=1e-12)


# ------------------------------------------------------------------ O8 pin
def _one_dof_chain(L=0.2):
    """Boundary - free - boundary on the x axis, equal rest lengths L.  An
    axial displacement u of the middle node is exactly linear: stiffness
    k = 2 EA/L, lumped mass M = rhoA L, so omega^2 = 2 EA / (rhoA L^2), and
    the Gershgorin ratio is G/M = 4 EA/(rhoA L^2) = 2 omega^2 for all
    |u| < L, so dt = alpha sqrt(2)/omega is constant."""
    pts = np.array([[0.5 - L, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5 + L, 0.5, 0.5]])
    return synth.chain_network(pts), pts


@pytest.mark.parametrize("c", [0.0, 0.7])
def test_central_difference_trajectory_closed_form(c):
    """Two-step central difference with mass-proportional damping on one DOF:
    u_{n+2} = (2 - c dt - w^2 dt^2) u_{n+1} - (1 - c dt) u_n with
    u_1 = (1 - w^2 dt^2 / 2) u_0 (start at rest).  Its closed form is
    A z1^n + B z2^n with z1, z2 the roots of the characteristic polynomial
    (for c = 0 this is u_0 cos(n theta), cos theta = 1 - w^2 dt^2 / 2)."""
    L, EA, alpha, u0 = 0.2, 1.3, 0.8, 0.01
    net, pts = _one_dof_chain(L)
    w = np.sqrt(2 * EA / L ** 2)
    dt = alpha * np.sqrt(2) / w
    p = w * w * dt * dt
    z = np.roots([1.0, -(2 - c * dt - p), 1 - c * dt]).astype(complex)
    A = np.linalg.solve(np.array([[1, 1], z]), np.array([u0, u0 * (1 - p / 2)], dtype=complex))
    for N in (1, 2, 7, 40):
        x0 = pts - 0.5
        x0[1, 0] += u0
        o = oracle.make_opts(law=LIN, EA=EA, alpha=alpha, tol_abs=0.0, n_max=N, init=oracle.INIT_GIVEN)
        r = oracle.solve(net, np.eye(3), c, o, x0=x0)
        assert r["iters"] == N
        uN = (A * z ** N).sum().real
        assert r["x"][1, 0] == pytest.approx(uN, abs=1e-14)
        assert np.abs(r["x"][1, 1:]).max() < 1e-15
    if c == 0.0:
        theta = np.arccos(1 - p / 2)
        assert (A * z ** 40).sum().real == pytest.approx(u0 * np.cos(40 * theta), abs=1e-14)


# ---------------------------------------------------------------- state validity and stability
def test_stability_of_a_chain_in_tension_and_compression():
    """Two boundary nodes and one free node on a line: in tension K_ff is
    k_t/L0 (2x) along the line and 2 T/l across it, positive definite; in
    compression the transverse stiffness 2 T/l < 0 makes it indefinite."""
    from oracle.stability import equilibrium, is_stable
    net = synth.chain_network([[0.0, 0.5, 0.5], [0.5, 0.5, 0.5], [1.0, 0.5, 0.5]])
    o = oracle.make_opts(law=oracle.LINEAR)
    Xm = net.X - 0.5
    for lam, stable in ((1.1, True), (0.9, False)):
        F = np.diag([lam, 1.0, 1.0])
        x = Xm @ F.T
        R, Fb, sig = equilibrium(net, F, x, o)
        assert R < 1e-14                       # the affine state of a symmetric chain is an equilibrium
        T = lam - 1.0                          # linear law, EA = 1, eps = lam - 1
        assert abs(Fb - np.sqrt(2) * abs(T)) < 1e-14
        assert abs(sig[0, 0] - T * lam / lam) < 1e-14   # sigma_11 = T l / (J V0) with l = lam/2 per fiber, 2 fibers
        assert is_stable(net, x, o) is stable


def test_stability_of_relaxed_lattice_and_floppy_mode():
    """A relaxed n^3 lattice in tension is stable.  A free node hanging on a
    single fiber has K_ff = (k_t/L0) n n^T + (T/l)(I - n n^T): at the rest
    length (T = 0) it is semidefinite with two zero eigenvalues (a floppy
    mode), which the relative shift accepts as stable; shortened (T < 0) the
    two transverse eigenvalues T/l are negative: unstable."""
    from oracle.stability import is_stable
    o = oracle.make_opts(law=oracle.EXP)
    net = synth.lattice_network(3)
    Xm = net.X - 0.5
    assert is_stable(net, Xm @ np.diag([1.1, 1.05, 1.08]).T, o) is True
    hang = synth.Network(np.array([[0.0, 0.5, 0.5], [0.4, 0.5, 0.5]]), np.array([1, 0], np.uint8),
                         np.array([[0, 1]], np.int32))
    x = hang.X - 0.5
    assert is_stable(hang, x, o) is True
    x2 = x.copy()
    x2[1, 0] -= 0.1
    assert is_stable(hang, x2, o) is False
