"""Incidence engine (node state in registers, one fiber record per
node-fiber incidence read from global memory each iteration), GPU.

RVE_ENGINE_INCIDENCE puts every RVE within the engine's limits (free nodes
of degree <= 16; positions in LDS up to 12288 free nodes, the global mode
above) on it, so small networks exercise it quickly; AUTO gives it the RVEs
beyond the register-resident capacity.

* config 2 RVEs: statuses as on the resident engine (except within 2% of
  the cap) and every jointly converged RVE within 1e-4 of the resident
  engine's stress, or a different equilibrium verified with the oracle's
  arithmetic at the incidence engine's state (gpu_common.grade_parity);
* bitwise repeatable, and independent of the work order;
* a warm start from its own state converges at the first test (the state is
  written in the packed order and read back through the rank permutation);
* kinetic damping: the kinetic build converges like the resident one;
* 2000-seed RVEs: AUTO takes them on the incidence kernel, statuses and
  stresses as on the streamed kernel (same grading); the largest RVEs of
  the FE^2 workload (above 12288 free nodes) on its global mode likewise;
* RVE_ENGINE_INCIDENCE with RVE_FP64 is rejected.
Parity with the FP64 oracle's stored results at the full workload shapes is
in test_gpu_fullshape.py (engine 4).
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
import oracle
from tests.gpu_common import grade_parity, log, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _kw(rb, engine, **extra):
    kw = dict(precision=rb.MIXED, law=rb.LAW_EXP, mass=rb.MASS_SCALED, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5,
              n_max=40000, check_every=8, engine=engine)
    kw.update(extra)
    return kw


def _oracle_opts(kw):
    return oracle.make_opts(law=oracle.EXP, mass=kw["mass"], alpha=kw["alpha"], tol_abs=0.0, tol_rel=1e-5,
                            n_max=kw["n_max"])


def _compare(b, batch, F, sig, st, it, ref_sig, ref_st, ref_it, kw, label):
    near_cap = (it >= 0.98 * kw["n_max"]) | (ref_it >= 0.98 * kw["n_max"])
    miss = (st != ref_st) & ~near_cap
    log(f"  [{label}] statuses {np.bincount(st, minlength=4).tolist()} vs {np.bincount(ref_st, minlength=4).tolist()}, "
        f"mismatches away from the cap {int(miss.sum())}")
    assert not miss.any(), np.where(miss)[0]
    grade = grade_parity(b, batch, F, sig, st, ref_sig, ref_st, 1e-4, _oracle_opts(kw), label, residual_rel=1e-4)
    assert grade["both"] >= 1
    both = (st == 0) & (ref_st == 0)
    ratio = np.median(it[both] / np.maximum(ref_it[both], 1))
    log(f"  [{label}] median iteration ratio {ratio:.3f}")
    assert 0.8 <= ratio <= 1.25


@pytest.fixture(scope="module")
def cfg2():
    return synth.make_config_batch(2, idx=np.arange(96))


def test_incidence_matches_resident_engine(cfg2):
    rb = require_gpu()
    batch, F = cfg2
    kw = _kw(rb, rb.ENGINE_INCIDENCE)
    b = rb.Batch(batch, **kw)
    log(f"groups {b.describe()}")
    assert b.describe().startswith("incidence(")
    sig, st, x = b.solve(F, stats=True)
    ref = rb.Batch(batch, **_kw(rb, rb.ENGINE_AUTO))
    log(f"reference groups {ref.describe()}")
    rsig, rst, rx = ref.solve(F, stats=True)
    _compare(b, batch, F, sig, st, x["iters"], rsig, rst, rx["iters"], kw, "incidence vs resident")
    b.close()
    ref.close()


def test_incidence_is_repeatable_and_order_independent(cfg2):
    rb = require_gpu()
    batch, F = cfg2
    b = rb.Batch(batch, **_kw(rb, rb.ENGINE_INCIDENCE, work_order=rb.ORDER_COST))
    s1, t1, x1 = b.solve(F, stats=True)   # host order
    s2, t2, x2 = b.solve(F, stats=True)   # cost order of the first solve
    assert np.array_equal(s1, s2, equal_nan=True) and np.array_equal(t1, t2)
    assert np.array_equal(x1["iters"], x2["iters"])
    b.close()


def test_incidence_warm_start_converges_at_once(cfg2):
    rb = require_gpu()
    batch, F = cfg2
    kw = _kw(rb, rb.ENGINE_INCIDENCE)
    b = rb.Batch(batch, **kw)
    s1, t1, x1 = b.solve(F, stats=True)
    b.set_opts(**dict(kw, init=rb.INIT_WARM))
    s2, t2, x2 = b.solve(F, stats=True)
    ok = t1 == 0
    log(f"warm start: iterations of the converged RVEs {np.unique(x2['iters'][ok]).tolist()}")
    assert np.all(t2[ok] == 0)
    assert np.all(x2["iters"][ok] <= kw["check_every"])
    assert np.max(rel_err(s2[ok], s1[ok])) <= 1e-4
    b.close()


def test_incidence_kinetic_damping(cfg2):
    rb = require_gpu()
    batch, F = cfg2
    kw = _kw(rb, rb.ENGINE_INCIDENCE, damping=rb.DAMP_KINETIC)
    b = rb.Batch(batch, **kw)
    sig, st, x = b.solve(F, stats=True)
    ref = rb.Batch(batch, **_kw(rb, rb.ENGINE_AUTO, damping=rb.DAMP_KINETIC))
    rsig, rst, rx = ref.solve(F, stats=True)
    _compare(b, batch, F, sig, st, x["iters"], rsig, rst, rx["iters"], kw, "kinetic incidence vs resident")
    b.close()
    ref.close()


def test_large_rves_take_the_incidence_kernel():
    rb = require_gpu()
    batch, F = synth.make_config_batch(3, idx=np.arange(4))
    kw = _kw(rb, rb.ENGINE_AUTO, n_max=100000)
    b = rb.Batch(batch, **kw)
    log(f"groups {b.describe()}")
    assert b.describe().startswith("incidence(") and ";" == b.describe()[-1] and b.describe().count(";") == 1
    sig, st, x = b.solve(F, stats=True)
    ref = rb.Batch(batch, **_kw(rb, rb.ENGINE_STREAMED, n_max=100000))
    rsig, rst, rx = ref.solve(F, stats=True)
    _compare(b, batch, F, sig, st, x["iters"], rsig, rst, rx["iters"], kw, "large RVEs incidence vs streamed")
    b.close()
    ref.close()


def test_global_mode_on_the_largest_rves():
    """RVEs above 12288 free nodes (the largest of the FE^2 workload) run the
    incidence engine's global mode (node state in global arrays); statuses
    and stresses as on the streamed kernel (same grading), in both
    dampings."""
    rb = require_gpu()
    seeds = np.array([synth.seed_count(5, r) for r in range(8192)])
    idx = np.sort(np.argsort(seeds)[-6:])
    batch, F = synth.make_config_batch(5, idx=idx)
    nfree = [int((batch.is_bnd[batch.node_off[r]:batch.node_off[r + 1]] == 0).sum()) for r in range(batch.n_rve)]
    log(f"free nodes {nfree}")
    for damping in (rb.DAMP_VISCOUS, rb.DAMP_KINETIC):
        kw = _kw(rb, rb.ENGINE_AUTO, n_max=100000, damping=damping)
        b = rb.Batch(batch, **kw)
        d = b.describe()
        log(f"groups {d}")
        assert "incidence(global," in d and "streamed" not in d
        sig, st, x = b.solve(F, stats=True)
        ref = rb.Batch(batch, **_kw(rb, rb.ENGINE_STREAMED, n_max=100000, damping=damping))
        rsig, rst, rx = ref.solve(F, stats=True)
        _compare(b, batch, F, sig, st, x["iters"], rsig, rst, rx["iters"], kw, f"global mode vs streamed, damping {damping}")
        b2 = rb.Batch(batch, **kw)
        s2, t2 = b2.solve(F)
        assert np.array_equal(sig, s2, equal_nan=True) and np.array_equal(st, t2)   # repeatable
        for h in (b, ref, b2):
            h.close()


def test_incidence_engine_rejects_fp64():
    rb = require_gpu()
    batch, _ = synth.make_config_batch(2, idx=np.arange(2))
    with pytest.raises(rb.RVEError):
        rb.Batch(batch, precision=rb.FP64, engine=rb.ENGINE_INCIDENCE)
