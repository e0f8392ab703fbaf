"""GPU state export / import (checkpoint, restart, warm starts across batches).

* The exported fluctuation is the converged state: x = F Xm + h matches the
  oracle's converged positions (FP64, tol_rel 1e-8 on both sides: 1e-6
  absolute on O(1) coordinates), boundary rows are exactly 0, and
  F Xm + h equals rve_batch_positions.
* A second batch built from the same networks that imports the state gives
  the same stress (the same FP64 stress kernel on the same state: bitwise),
  the same tangent and orientation (bitwise: same kernels, same inputs), and
  a warm-started solve under a new F identical to the warm-started solve of
  the original batch (statuses, iterations and stress bitwise).
* Device-pointer export/import equals the host path bitwise; a mixed
  precision state round-trips the same way.
* Imported statuses are checked: out-of-range codes become NONFINITE, a
  non-positive det F becomes BAD_F, and both give NaN stress.
"""
import numpy as np
import pytest

import oracle
from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu
IDX = np.array([0, 1, 2, 5, 9, 11])


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def _common(rb, **kw):
    d = dict(law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, n_max=100000)
    d.update(kw)
    return d


def test_export_matches_oracle_and_positions(rb):
    log("state export vs oracle, FP64")
    batch, F = synth.make_config_batch(2, idx=IDX)
    b = rb.Batch(batch, precision=rb.FP64, tol_rel=1e-8, **_common(rb))
    with pytest.raises(rb.RVEError):
        b.export_state()              # no state before the first solve
    sig, st = b.solve(F)
    Fe, h, ste = b.export_state()
    np.testing.assert_array_equal(Fe, F)
    np.testing.assert_array_equal(ste, st)
    isb = np.asarray(batch.is_bnd).astype(bool)
    assert (h[isb] == 0).all()
    Xm = np.asarray(batch.X) - 0.5
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-8, n_max=100000, mass=oracle.MASS_SCALED)
    ref = oracle.solve_batch(batch, F, 0.1, o)
    worst = 0.0
    for r in range(len(IDX)):
        n0, n1 = batch.node_off[r], batch.node_off[r + 1]
        x = Xm[n0:n1] @ F[r].T + h[n0:n1]
        np.testing.assert_allclose(b.positions(r), x, rtol=0, atol=1e-14)
        if st[r] == 0 and ref["status"][r] == 0:
            worst = max(worst, np.abs(x - ref["x"][n0:n1]).max())
    log(f"  max |x_gpu - x_oracle| over jointly converged RVEs: {worst:.2e}")
    assert worst <= 1e-6
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_import_reproduces_state_tangent_and_warm_solve(rb, prec):
    log(f"state import round trip, {prec}")
    p, tol = (rb.FP64, 1e-8) if prec == "fp64" else (rb.MIXED, 1e-5)
    batch, F = synth.make_config_batch(2, idx=IDX)
    opts = _common(rb, precision=p, tol_rel=tol, cg_tol=1e-8)
    b1 = rb.Batch(batch, **opts)
    sig1, st1 = b1.solve(F)
    Fe, h, ste = b1.export_state()
    b2 = rb.Batch(batch, **opts)
    sig2 = b2.import_state(Fe, h, ste)
    np.testing.assert_array_equal(sig2[st1 < 2], sig1[st1 < 2])
    # tangent and orientation at the imported state
    t1, ts1 = b1.tangent()
    t2, ts2 = b2.tangent()
    np.testing.assert_array_equal(ts2, ts1)
    ok = ts1 == 0
    assert ok.sum() >= 3
    np.testing.assert_array_equal(t2[ok], t1[ok])
    o1, _ = b1.orientation()
    o2, _ = b2.orientation()
    np.testing.assert_array_equal(o2, o1)
    # a warm-started increment continues identically from either batch
    F2 = F @ (np.eye(3) + np.diag([0.01, -0.005, -0.005]))
    for bb in (b1, b2):
        bb.set_opts(init=rb.INIT_WARM, **opts)
    s1, w1, d1 = b1.solve(F2, stats=True)
    s2, w2, d2 = b2.solve(F2, stats=True)
    np.testing.assert_array_equal(w2, w1)
    np.testing.assert_array_equal(d2["iters"], d1["iters"])
    np.testing.assert_array_equal(s2[w1 < 2], s1[w1 < 2])
    log(f"  warm increment: statuses {np.bincount(w1, minlength=4)}, iterations {d1['iters'].tolist()}")
    b1.close()
    b2.close()


def test_device_pointers_and_status_checks(rb):
    import torch
    log("state export/import through device pointers")
    dev = torch.device("cuda:0")
    batch, F = synth.make_config_batch(2, idx=IDX)
    opts = _common(rb, precision=rb.MIXED, tol_rel=1e-5)
    b1 = rb.Batch(batch, **opts)
    sig1, st1 = b1.solve(F)
    Fh, hh, sth = b1.export_state()
    like = torch.empty(1, device=dev)
    Fd, hd, std = b1.export_state(like=like)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Fd.cpu().numpy(), Fh)
    np.testing.assert_array_equal(hd.cpu().numpy(), hh)
    np.testing.assert_array_equal(std.cpu().numpy(), sth)
    b2 = rb.Batch(batch, **opts)
    sigd = b2.import_state(Fd, hd, std)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sigd.cpu().numpy()[st1 < 2], sig1[st1 < 2])
    # status checks: an out-of-range code and a reflected F
    st_bad = sth.copy()
    st_bad[0] = 9
    F_bad = Fh.copy()
    F_bad[1] = F_bad[1] @ np.diag([1.0, 1.0, -1.0])
    sig3 = b2.import_state(F_bad, hh, st_bad)
    _, _, st3 = b2.export_state()
    assert st3[0] == rb.ST_NONFINITE and st3[1] == rb.ST_BAD_F
    assert np.isnan(sig3[0]).all() and np.isnan(sig3[1]).all()
    np.testing.assert_array_equal(st3[2:], sth[2:])
    with pytest.raises(ValueError):
        b2.import_state(Fd, hd.float(), std)
    b1.close()
    b2.close()
