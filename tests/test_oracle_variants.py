"""Pins of the oracle's dynamic-relaxation alternatives (Section 3.2: kinetic
damping, an automatically updated damping coefficient, the energy-balance
check), CPU only.

* Viscous mode of the variant routine is the ordinary relaxation: same
  iterations, same stress.
* Every mode reaches the closed-form stress of the relaxed lattice from a
  random start, and the brute-force Newton equilibrium of tiny networks.
* Kinetic damping relaxes a single mode within a few of its periods (the
  first reset falls near the equilibrium), far faster than a light viscous
  damping.
* Adaptive damping on a one-DOF linear system: the Rayleigh quotient of the
  displacement is k/m, so the coefficient is critical damping 2 sqrt(k/m),
  which relaxes the mode in far fewer steps than a small constant c; for the
  transverse mode of the same pre-tensioned chain the stiffness is the
  geometric one, 2 T / l.
* On config-2 networks (many modes) kinetic damping converges within twice
  the iterations of the tuned viscous damping (a wrong reset test turns it
  into a slow gradient descent).
* Energy bookkeeping: on a damped linear chain the balance
  W + KE + Wd - W_start shrinks like dt^2 (halving alpha divides it by about
  four), so no term is missing; an unstable run (exponential fibers at
  alpha 0.9) is stopped by the check before it turns non-finite, while
  stable runs never trip it.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_09427_amd import synth
from tests.test_oracle_pins import lattice_stress

MODES = [oracle.DAMP_VISCOUS, oracle.DAMP_KINETIC, oracle.DAMP_ADAPTIVE]


def test_viscous_variant_is_the_ordinary_relaxation():
    batch, F = synth.make_config_batch(2, idx=np.arange(3))
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-8, n_max=30000,
                         mass=oracle.MASS_SCALED)
    for r in range(3):
        net = batch.network(r)
        a = oracle.solve(net, F[r], 0.1, o)
        b = oracle.solve_variant(net, F[r], 0.1, o, damping=oracle.DAMP_VISCOUS)
        assert a["status"] == b["status"] and a["iters"] == b["iters"]
        np.testing.assert_array_equal(a["sigma"], b["sigma"])
        assert b["c"] == 0.1


@pytest.mark.parametrize("law", [oracle.LINEAR, oracle.EXP])
@pytest.mark.parametrize("damping", MODES)
def test_lattice_closed_form_every_mode(law, damping):
    n = 3
    net = synth.lattice_network(n)
    F = np.array([[1.12, 0.04, 0.0], [0.0, 1.08, 0.03], [0.02, 0.0, 1.1]])
    o = oracle.make_opts(law=law, alpha=0.5, tol_abs=1e-12, tol_rel=0.0, n_max=400000, init=oracle.INIT_GIVEN)
    x0 = (net.X - 0.5) @ F.T + 0.02 * np.random.default_rng(4).standard_normal(net.X.shape)
    r = oracle.solve_variant(net, F, 2.0, o, damping=damping, energy_check=True, x0=x0)
    assert r["status"] == oracle.CONVERGED
    ref = lattice_stress(n, F, law)
    assert np.abs(r["sigma"] - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("damping", [oracle.DAMP_KINETIC, oracle.DAMP_ADAPTIVE])
def test_matches_brute_force_newton(damping):
    F = np.array([[1.2, 0.04, 0.0], [0.0, 1.12, 0.03], [0.02, 0.0, 1.1]])
    checked = 0
    for seed in range(6):
        net = synth.voronoi_network(15, [15, seed, 0])
        if net.n_free == 0 or net.n_free > 50:
            continue
        xN, sN, rN, stable = dense.newton(net, F, oracle.make_opts(law=oracle.EXP))
        if not stable or rN > 1e-12:
            continue
        o = oracle.make_opts(law=oracle.EXP, tol_abs=1e-12, n_max=5_000_000, alpha=0.5)
        r = oracle.solve_variant(net, F, 2.0, o, damping=damping)
        assert r["status"] == oracle.CONVERGED
        assert np.abs(r["sigma"] - sN).max() <= 1e-9 * np.abs(sN).max()
        checked += 1
    assert checked >= 2


def _axial_one_dof():
    """One free node between two boundary nodes on the x axis (two fibers of
    rest length 0.3), displaced along x only: a linear one-DOF system with
    stiffness k = 2 EA / L0 and lumped mass m = rhoA L0."""
    net = synth.chain_network([[0.2, 0.5, 0.5], [0.5, 0.5, 0.5], [0.8, 0.5, 0.5]])
    F = np.diag([1.1, 1.0, 1.0])
    x0 = (net.X - 0.5) @ F.T
    x0[1, 0] += 0.01
    return net, F, x0


def test_adaptive_coefficient_is_critical_damping():
    net, F, x0 = _axial_one_dof()
    o = oracle.make_opts(law=oracle.LINEAR, EA=1.0, alpha=0.5, tol_abs=1e-13, tol_rel=0.0, n_max=100000,
                         init=oracle.INIT_GIVEN)
    r = oracle.solve_variant(net, F, 0.0, o, damping=oracle.DAMP_ADAPTIVE, x0=x0)
    assert r["status"] == oracle.CONVERGED
    L0, EA = 0.3, 1.0
    assert abs(r["c"] - 2.0 * np.sqrt((2 * EA / L0) / L0)) <= 1e-12 * r["c"]
    assert abs(r["x"][1, 0]) <= 1e-12            # back at the centre (F Xm = 0 there)
    # critical damping brings the single mode in far fewer steps than c = 0.1
    slow = oracle.solve_variant(net, F, 0.1, o, damping=oracle.DAMP_VISCOUS, x0=x0)
    assert r["iters"] * 3 < slow["iters"]


def test_energy_balance_is_second_order_in_dt():
    net, F, x0 = _axial_one_dof()
    x0[1, 1] += 0.02                              # add a transverse (softer) component
    errs = []
    for alpha in (0.4, 0.2, 0.1):
        o = oracle.make_opts(law=oracle.LINEAR, alpha=alpha, tol_abs=1e-30, tol_rel=0.0, n_max=int(60 / alpha),
                             init=oracle.INIT_GIVEN)
        r = oracle.solve_variant(net, F, 0.5, o, damping=oracle.DAMP_VISCOUS, x0=x0)
        errs.append(r["energy"])
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_energy_check_stops_unstable_runs_only():
    batch, F = synth.make_config_batch(2, idx=np.arange(3))
    for alpha, unstable in ((0.9, True), (0.5, False)):
        o = oracle.make_opts(law=oracle.EXP, alpha=alpha, tol_abs=0.0, tol_rel=1e-8, n_max=20000,
                             mass=oracle.MASS_SCALED)
        for r in range(3):
            net = batch.network(r)
            chk = oracle.solve_variant(net, F[r], 0.1, o, energy_check=True, energy_tol=0.05)
            free = oracle.solve_variant(net, F[r], 0.1, o, energy_check=False)
            if unstable:
                assert free["status"] == oracle.NONFINITE
                assert chk["status"] == oracle.ENERGY and chk["iters"] < free["iters"]
            else:
                assert chk["status"] == free["status"] != oracle.ENERGY
                assert chk["iters"] == free["iters"] and chk["energy"] <= 0.05


def test_kinetic_damping_relaxes_a_single_mode_quickly():
    net, F, x0 = _axial_one_dof()
    o = oracle.make_opts(law=oracle.LINEAR, EA=1.0, alpha=0.5, tol_abs=1e-13, tol_rel=0.0, n_max=100000,
                         init=oracle.INIT_GIVEN)
    kin = oracle.solve_variant(net, F, 0.1, o, damping=oracle.DAMP_KINETIC, x0=x0)
    visc = oracle.solve_variant(net, F, 0.1, o, damping=oracle.DAMP_VISCOUS, x0=x0)
    assert kin["status"] == oracle.CONVERGED and visc["status"] == oracle.CONVERGED
    assert kin["iters"] < 300 and kin["iters"] * 10 < visc["iters"]
    assert abs(kin["x"][1, 0]) <= 1e-12
    assert kin["c"] == 0.0


def test_adaptive_coefficient_sees_the_geometric_stiffness():
    net, F, x0 = _axial_one_dof()
    x0[1, 0] -= 0.01
    x0[1, 1] += 0.01                     # transverse displacement only
    o = oracle.make_opts(law=oracle.LINEAR, EA=1.0, alpha=0.5, tol_abs=1e-13, tol_rel=0.0, n_max=100000,
                         init=oracle.INIT_GIVEN)
    r = oracle.solve_variant(net, F, 0.0, o, damping=oracle.DAMP_ADAPTIVE, x0=x0)
    assert r["status"] == oracle.CONVERGED
    L0, l, m = 0.3, 0.33, 0.3
    T = 1.0 * (l / L0 - 1.0)
    assert abs(r["c"] - 2.0 * np.sqrt(2.0 * T / l / m)) <= 1e-9 * r["c"]


def test_kinetic_damping_on_networks_keeps_pace_with_viscous():
    batch, F = synth.make_config_batch(2, idx=[1, 3])
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-8, n_max=60000, mass=oracle.MASS_SCALED)
    for r in range(2):
        net = batch.network(r)
        kin = oracle.solve_variant(net, F[r], 0.1, o, damping=oracle.DAMP_KINETIC)
        visc = oracle.solve_variant(net, F[r], 0.1, o, damping=oracle.DAMP_VISCOUS)
        assert kin["status"] == oracle.CONVERGED and visc["status"] == oracle.CONVERGED
        assert kin["iters"] <= 2 * visc["iters"]
