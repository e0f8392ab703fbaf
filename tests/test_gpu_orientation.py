"""GPU fiber-orientation outputs (orientation tensor, degree of alignment P2)
against the oracle (oracle/orientation.py, pinned in
tests/test_oracle_orientation.py) at the oracle's own converged state, and
against the affine closed form on a relaxed lattice.

Tolerances: FP64 states converged to tol_rel 1e-8 on both sides agree in the
orientation outputs to 1e-6 (absolute; the outputs are O(1)); the mixed
state to 1e-4.  The closed form holds to 1e-10 (lattice relaxed to
tol_abs 1e-13).
"""
import numpy as np
import pytest

import oracle
from oracle import orientation as orient
from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu
E = np.array([1.0, 0.3, -0.2])


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def test_orientation_config2_matches_oracle(rb):
    log("orientation config2 subset")
    idx = np.array([0, 1, 2, 5, 9, 11])
    batch, F = synth.make_config_batch(2, idx=idx)
    common = dict(law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, n_max=100000)
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-8, n_max=100000, mass=oracle.MASS_SCALED)
    ref = oracle.solve_batch(batch, F, 0.1, o)
    om_ref, p2_ref = orient.orientation_batch(batch, ref["x"], E)
    for prec, tol_rel, bar in ((rb.FP64, 1e-8, 1e-6), (rb.MIXED, 1e-5, 1e-4)):
        b = rb.Batch(batch, precision=prec, tol_rel=tol_rel, **common)
        with pytest.raises(rb.RVEError):
            b.orientation(E)          # no state before the first solve
        sig, st = b.solve(F)
        om, p2 = b.orientation(E)
        with pytest.raises(rb.RVEError):
            b.orientation((0.0, 0.0, 0.0))
        both = (st == 0) & (ref["status"] == 0)
        assert both.sum() >= 3
        d_om = np.abs(om - om_ref).reshape(len(idx), -1).max(1)
        d_p2 = np.abs(p2 - p2_ref)
        log(f"  precision {prec}: {both.sum()} jointly converged, max |dOmega| {d_om[both].max():.2e}, "
            f"max |dP2| {d_p2[both].max():.2e}")
        assert d_om[both].max() <= bar and d_p2[both].max() <= bar
        np.testing.assert_allclose(np.trace(om, axis1=1, axis2=2), 1.0, atol=1e-12)
        b.close()


def test_orientation_lattice_closed_form(rb):
    log("orientation lattice closed form")
    nets = [synth.lattice_network(3), synth.lattice_network(4)]
    batch = synth.pack(nets)
    F = np.array([[[1.1, 0.05, 0.0], [0.02, 1.04, 0.03], [0.0, -0.01, 1.06]],
                  [[1.05, 0.0, 0.02], [0.0, 1.1, 0.0], [0.01, 0.03, 1.08]]])
    b = rb.Batch(batch, precision=rb.FP64, law=rb.LAW_LINEAR, alpha=0.5, c=2.0, tol_abs=1e-13, n_max=200000)
    sig, st = b.solve(F)
    assert (st == 0).all()
    om, p2 = b.orientation(E)
    eu = E / np.linalg.norm(E)
    for r in range(2):
        expect = sum(np.outer(F[r][:, k], F[r][:, k]) / (F[r][:, k] @ F[r][:, k]) for k in range(3)) / 3
        assert np.abs(om[r] - expect).max() <= 1e-10
        assert abs(p2[r] - 0.5 * (3 * eu @ expect @ eu - 1)) <= 1e-10
    b.close()
