"""Pins of the oracle's stagnation stop (the optional end of the convergence
loop, Section 3.2, for tolerances below what the arithmetic can reach),
CPU only.

The rule: after stall_checks consecutive convergence tests in which the
residual R did not fall below half of its reference value (R of the start,
replaced by R each time R falls below half of it), with R and the
damping-force norm both within floor_tol_rel |f_bnd|, the run stops as
stagnated; its stress is evaluated as for a converged run.

* Relaxed lattice from a perturbed start with an unreachable tolerance:
  the run stops as stagnated once the FP64 residual has levelled off,
  R <= floor_tol_rel |f_bnd| there and the stress is the closed form; with
  the stop off (or a floor below the FP64 residual) the same run goes on
  to n_max and ends on the same stress.
* Both norms are tested: an undamped run (c = 0, so the damping-force
  norm is zero throughout) whose residual oscillates far above the floor
  is never stopped.
* The window counts tests: with an unbounded floor and a window of one
  test the run stops at the first iteration (one step does not halve R);
  a window of 50 outlasts every geometric halving of the lattice's
  residual and ends where the window of 20 ends (the floor), not at
  iteration 50 (a missing reset would stop there).
* A floor that no residual reaches (1e-300, window of one test) leaves
  the relaxation bit for bit unchanged: the rule only ever stops a run.
"""
import numpy as np

import oracle
from paper_2306_09427_amd import synth
from tests.test_oracle_pins import lattice_stress

F_LAT = np.array([[1.12, 0.04, 0.0], [0.0, 1.08, 0.03], [0.02, 0.0, 1.1]])


def _lattice():
    net = synth.lattice_network(3)
    x0 = (net.X - 0.5) @ F_LAT.T + 0.02 * np.random.default_rng(4).standard_normal(net.X.shape)
    return net, x0


def _opts(**kw):
    base = dict(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-30, n_max=400000, init=oracle.INIT_GIVEN)
    base.update(kw)
    return oracle.make_opts(**base)


def _bnd_norm(net, x):
    fib = np.asarray(net.fib, np.int32)
    f, _, _ = oracle.forces(x, fib, oracle.rest_lengths(net.X, fib), _opts())
    return np.linalg.norm(f[np.asarray(net.is_bnd, bool)])


def test_stagnation_stops_on_the_closed_form():
    net, x0 = _lattice()
    ref = lattice_stress(3, F_LAT, oracle.EXP)
    r = oracle.solve(net, F_LAT, 2.0, _opts(floor_tol_rel=1e-12, stall_checks=50), x0=x0)
    assert r["status"] == oracle.STAGNATED and 50 < r["iters"] < 2000
    B = _bnd_norm(net, r["x"])
    assert r["R"] <= 1e-12 * B and r["D"] <= 1e-12 * B
    assert np.abs(r["sigma"] - ref).max() <= 1e-9 * np.abs(ref).max()
    n_stop = r["iters"]
    for kw in (dict(floor_tol_rel=0.0), dict(floor_tol_rel=1e-20, stall_checks=50)):
        q = oracle.solve(net, F_LAT, 2.0, _opts(n_max=n_stop + 500, **kw), x0=x0)
        assert q["status"] == oracle.MAXITER and q["iters"] == n_stop + 500
        assert np.abs(q["sigma"] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_undamped_run_above_the_floor_is_not_stopped():
    net, x0 = _lattice()
    r = oracle.solve(net, F_LAT, 0.0, _opts(floor_tol_rel=1e-6, stall_checks=10, n_max=3000), x0=x0)
    assert r["status"] == oracle.MAXITER and r["D"] == 0.0
    assert r["R"] > 1e-6 * _bnd_norm(net, r["x"])


def test_window_counts_tests_without_halving():
    net, x0 = _lattice()
    stops = {}
    for W in (1, 20, 50):
        r = oracle.solve(net, F_LAT, 2.0, _opts(floor_tol_rel=1e300, stall_checks=W, n_max=5000), x0=x0)
        assert r["status"] == oracle.STAGNATED
        stops[W] = r
    assert stops[1]["iters"] == 1
    # the geometric phase halves R well within 20 tests, so both windows
    # run into the FP64 level: there the 50-test window ends 30 tests later
    assert stops[50]["iters"] > 200
    assert stops[50]["iters"] >= stops[20]["iters"] + 30
    ref = lattice_stress(3, F_LAT, oracle.EXP)
    for W in (20, 50):
        assert np.abs(stops[W]["sigma"] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_floor_off_is_the_ordinary_relaxation():
    batch, F = synth.make_config_batch(2, idx=np.arange(2))
    for r in range(2):
        net = batch.network(r)
        o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-6, n_max=30000,
                             mass=oracle.MASS_SCALED)
        o2 = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-6, n_max=30000,
                              mass=oracle.MASS_SCALED, floor_tol_rel=1e-300, stall_checks=1)
        a, b = oracle.solve(net, F[r], 0.1, o), oracle.solve(net, F[r], 0.1, o2)
        assert a["status"] == b["status"] and a["iters"] == b["iters"]
        np.testing.assert_array_equal(a["sigma"], b["sigma"])
