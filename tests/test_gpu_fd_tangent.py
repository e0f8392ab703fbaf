"""GPU finite-difference material tangent (the paper's method, Section 3.2)
against the oracle (oracle/fd_tangent.py, pinned in
tests/test_oracle_fd_tangent.py).

* Small networks in tension: the GPU's C and A against the oracle's
  finite-difference tangent at the oracle's own converged state, same h.
  Both base states and all probes are converged to tol_rel 1e-11, so the
  difference quotients agree to ~tol / h; bar 1e-5 (relative to max |A|).
* A 300-seed RVE: the GPU's A against the oracle's exact linearisation
  (dense dsigma/dF turned into dPi/dE), bar 50 h (the forward difference is
  first order).
* Status: RVEs whose base solve did not converge report "no state" and NaN.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from oracle import fd_tangent as fdt
from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu
FT = np.array([[1.1, 0.02, 0.0], [0.0, 1.06, 0.01], [0.01, 0.0, 1.05]])


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def _opts(rb, **kw):
    d = dict(precision=rb.FP64, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-11,
             n_max=400000)
    d.update(kw)
    return d


def test_fd_tangent_matches_oracle_fd(rb):
    log("fd tangent small networks")
    nets = [synth.voronoi_network(40, [71, s, 0]) for s in range(3)]
    batch = synth.pack(nets)
    F = np.tile(FT, (len(nets), 1, 1))
    h = 1e-4
    b = rb.Batch(batch, **_opts(rb))
    sig, st = b.solve(F)
    assert (st == 0).all()
    C, A, fst = b.fd_tangent(h)
    b.close()
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-11, n_max=400000,
                         mass=oracle.MASS_SCALED)
    for k, net in enumerate(nets):
        base = oracle.solve(net, F[k], 0.1, o)
        assert base["status"] == 0 and fst[k] == 0
        ref = fdt.fd_tangent(net, F[k], base["x"], base["sigma"], 0.1, o, h=h)
        assert ref["status"] == 0
        ea = np.abs(A[k] - ref["A"]).max() / np.abs(ref["A"]).max()
        ec = np.abs(C[k] - ref["C"]).max() / np.abs(ref["C"]).max()
        log(f"  rve {k}: A rel diff {ea:.2e}, C rel diff {ec:.2e}")
        assert ea <= 1e-5 and ec <= 1e-5


def test_fd_tangent_matches_linearisation_and_status(rb):
    log("fd tangent vs exact linearisation")
    batch, _ = synth.make_config_batch(4, idx=[0, 3])
    F = np.stack([FT, np.eye(3) + np.diag([0.2, -0.15, -0.15])])   # the second: compressed, may not converge
    h = 1e-5
    b = rb.Batch(batch, **_opts(rb, n_max=20000))
    sig, st = b.solve(F)
    C, A, fst = b.fd_tangent(h)
    b.close()
    assert st[0] == 0 and fst[0] == 0
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-11, n_max=400000,
                         mass=oracle.MASS_SCALED)
    net = batch.network(0)
    base = oracle.solve(net, F[0], 0.1, o)
    assert base["status"] == 0
    A_lin = fdt.A_from_dsigma_dF(F[0], base["sigma"], dense.tangent_forward(net, F[0], base["x"], o))
    err = np.abs(A[0] - A_lin).max() / np.abs(A_lin).max()
    log(f"  300-seed RVE: FD A vs exact linearisation {err:.2e}")
    assert err <= 50 * h
    if st[1] != 0:
        assert fst[1] == rb.ST_NO_STATE and np.isnan(C[1]).all()
    with pytest.raises(rb.RVEError):
        b2 = rb.Batch(batch, **_opts(rb))
        try:
            b2.fd_tangent(h)        # no solve yet
        finally:
            b2.close()
