"""GPU stagnation stop (status RVE_ST_STAGNATED) against the oracle's rule
(pinned in tests/test_oracle_floor.py).

* FP64, config-2 RVEs, an unreachable tol_rel (1e-30) with floor_tol_rel
  1e-11 and a window of 64 tests, on the resident and the streamed
  engine: the GPU and the oracle run the same iteration in a different
  summation order, so on at least 80% of the RVEs they end with the same
  status after the same number of iterations, and there the stresses agree
  to 1e-6; RVEs that stop as stagnated have R and the damping-force norm
  within 1e-11 |f_bnd|.
* Mixed precision asked for tol_rel 1e-8, below the float floor: without
  the stop (at least 90% of) the RVEs run to n_max; with floor_tol_rel 3e-5 and a window of
  32 tests (every 8 iterations) at least half of them stop as stagnated,
  in fewer iterations, with R within the floor, and at least 80% of those
  the FP64 oracle converges (tol_rel 1e-8) are within the mixed-precision
  stress tolerance 1e-4 of it.  A stagnated RVE gets no tangent
  (RVE_ST_NO_STATE) and keeps its status through export and import.
"""
import numpy as np
import pytest

import oracle
from paper_2306_09427_amd import synth
from tests.gpu_common import log, rel_err, require_gpu

pytestmark = pytest.mark.gpu
IDX = np.array([0, 1, 2, 3, 5, 9])


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


@pytest.mark.parametrize("engine", ["auto", "streamed"])
def test_fp64_matches_oracle(rb, engine):
    log(f"stagnation stop, FP64, {engine} engine, config2 subset vs oracle")
    batch, F = synth.make_config_batch(2, idx=IDX)
    eng = rb.ENGINE_AUTO if engine == "auto" else rb.ENGINE_STREAMED
    b = rb.Batch(batch, precision=rb.FP64, law=rb.LAW_EXP, mass=rb.MASS_SCALED, alpha=0.5, c=0.1, tol_abs=0.0,
                 tol_rel=1e-30, n_max=60000, check_every=1, engine=eng, floor_tol_rel=1e-11, stall_checks=64)
    sig, st, stats = b.solve(F, stats=True)
    b.close()
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-30, n_max=60000,
                         mass=oracle.MASS_SCALED, floor_tol_rel=1e-11, stall_checks=64)
    ref = oracle.solve_batch(batch, F, 0.1, o)
    log(f"  statuses GPU {st.tolist()} oracle {ref['status'].tolist()}")
    log(f"  iterations GPU {stats['iters'].tolist()} oracle {ref['iters'].tolist()}")
    same = (st == ref["status"]) & (stats["iters"] == ref["iters"])
    err = rel_err(sig, ref["sigma"])
    log(f"  sigma rel err (same status and iterations): {err[same].tolist()}")
    assert same.mean() >= 0.8 and err[same].max() <= 1e-6
    stag = st == rb.ST_STAGNATED
    assert stag.sum() >= 2
    assert (stats["R"][stag] <= 1e-11 * stats["Fb"][stag]).all()
    assert (stats["D"][stag] <= 1e-11 * stats["Fb"][stag]).all()


def test_mixed_stops_at_the_float_floor(rb):
    idx = np.arange(0, 64, 4)
    log(f"stagnation stop, mixed precision, {len(idx)} config2 RVEs")
    batch, F = synth.make_config_batch(2, idx=idx)
    common = dict(precision=rb.MIXED, law=rb.LAW_EXP, mass=rb.MASS_SCALED, alpha=0.5, c=0.1, tol_abs=0.0,
                  tol_rel=1e-8, n_max=60000, check_every=8)
    b = rb.Batch(batch, **common)
    _, st_off, s_off = b.solve(F, stats=True)
    b.close()
    b = rb.Batch(batch, floor_tol_rel=3e-5, stall_checks=32, **common)
    sig, st, stats = b.solve(F, stats=True)
    log(f"  without the stop: {st_off.tolist()}")
    log(f"  with the stop:    {st.tolist()}, iterations {stats['iters'].tolist()}")
    capped = st_off == rb.ST_MAXITER
    assert capped.mean() >= 0.9
    stag = st == rb.ST_STAGNATED
    assert stag.sum() >= len(idx) // 2
    assert np.isin(st[capped], (rb.ST_MAXITER, rb.ST_STAGNATED)).all()
    assert (stats["iters"][stag] < s_off["iters"][stag]).all()
    assert (stats["R"][stag] <= 3e-5 * stats["Fb"][stag]).all()
    assert (stats["D"][stag] <= 3e-5 * stats["Fb"][stag]).all()
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-8, n_max=60000,
                         mass=oracle.MASS_SCALED)
    ref = oracle.solve_batch(batch, F, 0.1, o)
    both = stag & (ref["status"] == oracle.CONVERGED)
    err = rel_err(sig, ref["sigma"])
    log(f"  sigma rel err vs the FP64 oracle (tol_rel 1e-8) on {both.sum()} stagnated: {err[both].tolist()}")
    assert both.sum() >= 4 and np.mean(err[both] <= 1e-4) >= 0.8
    ds, tst = b.tangent()
    assert (tst[stag] == rb.ST_NO_STATE).all()
    Fe, h, se = b.export_state()
    sig2 = b.import_state(Fe, h, se)
    _, _, se2 = b.export_state()
    b.close()
    np.testing.assert_array_equal(se2, st)
    assert rel_err(sig2[stag], sig[stag]).max() <= 1e-6
