"""Team engine: RVEs too large for one CU relaxed by k workgroups that
exchange partition-boundary state through global memory once per iteration.

Against the streamed engine (one workgroup per RVE, same arithmetic in a
different order of the reductions): FP64 statuses equal and stresses within
1e-9; mixed stresses within 1e-4 on RVEs converged in both runs.  Against
the oracle: tests/test_gpu_fullshape.py (the 2000-seed RVEs and the large
RVEs of the FE2 workload run on this engine).  The give-up path of the team
barrier is forced from the host with a one-poll limit.
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


@pytest.fixture(scope="module")
def large():
    # FE2-workload RVEs above the resident capacity (up to 3000 seeds) and two 2000-seed RVEs
    seeds = np.array([synth.seed_count(5, r) for r in range(8192)])
    idx = np.argsort(seeds)[-6:]
    b5, F5 = synth.make_config_batch(5, idx=np.sort(idx))
    b3, F3 = synth.make_config_batch(3, idx=[0, 1])
    nets = [b5.network(r) for r in range(b5.n_rve)] + [b3.network(r) for r in range(b3.n_rve)]
    return synth.pack(nets), np.concatenate([F5, F3])


KW = dict(law=1, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, check_every=8)


@pytest.mark.parametrize("prec,tol_rel,n_max,sig_tol", [(0, 1e-8, 30000, 1e-9), (1, 1e-5, 30000, 1e-4)])
@pytest.mark.parametrize("damping", [0, 1])
def test_team_matches_streamed(rb, large, prec, tol_rel, n_max, sig_tol, damping):
    batch, F = large
    runs = {}
    for name, eng in (("team", rb.ENGINE_TEAM), ("streamed", rb.ENGINE_STREAMED)):
        b = rb.Batch(batch, precision=prec, engine=eng, tol_rel=tol_rel, n_max=n_max, damping=damping, **KW)
        d = b.describe()
        sig, st, stats = b.solve(F, stats=True)
        runs[name] = (sig, st, stats["iters"])
        log(f"  precision {prec} damping {damping} {name}: {d} status {np.bincount(st, minlength=4).tolist()} "
            f"iters {stats['iters'].tolist()}")
        if name == "team":
            assert "team(" in d
        b.close()
    (s1, t1, i1), (s0, t0, i0) = runs["team"], runs["streamed"]
    near = (i1 >= 0.98 * n_max) | (i0 >= 0.98 * n_max)
    assert np.all((t1 == t0) | near), (t1, t0)
    both = (t1 == 0) & (t0 == 0)
    err = rel_err(s1[both], s0[both])
    log(f"  team vs streamed: {int(both.sum())} both converged, sigma max rel diff {err.max() if both.any() else 0:.2e}")
    assert both.sum() >= 2
    assert np.all(err <= sig_tol), err
    if prec == 0:
        it_d = np.abs(i1[both] - i0[both]) / np.maximum(i0[both], 1)
        assert np.median(it_d) <= 0.01


def test_team_warm_start_and_repeatable(rb, large):
    batch, F = large
    b = rb.Batch(batch, precision=1, engine=rb.ENGINE_TEAM, tol_rel=1e-5, n_max=30000, **KW)
    assert "team(" in b.describe()
    s1, t1 = b.solve(F)
    s2, t2 = b.solve(F)
    assert np.array_equal(s1, s2, equal_nan=True) and np.array_equal(t1, t2)
    b.set_opts(precision=1, engine=rb.ENGINE_TEAM, init=rb.INIT_WARM, tol_rel=1e-5, n_max=30000, **KW)
    s3, t3, st3 = b.solve(F * (1 + 1e-4), stats=True)
    log(f"  warm increment: iterations {st3['iters'].tolist()}, status {t3.tolist()}")
    assert np.all(t3[t1 == 0] == 0)
    b.close()


def test_team_gives_up_cleanly_at_a_one_poll_limit(rb, large):
    """Forced from the host: every team barrier may poll once, so teams give
    up (the kernel exits normally); the call reports RVE_EDEVICE and the
    team RVEs it did not finish are non-finite with NaN stress; with the
    default limit the same batch solves again."""
    batch, F = large
    b = rb.Batch(batch, precision=1, engine=rb.ENGINE_TEAM, tol_rel=1e-5, n_max=30000, **KW)
    b.team_spin_limit(1)
    with pytest.raises(rb.RVEError) as e:
        b.solve(F)
    assert e.value.code == rb.EDEVICE and "team" in str(e.value)
    b.team_spin_limit(1 << 24)
    sig, st = b.solve(F)
    assert np.all(np.isin(st, (0, 1)))
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_chooses_team_or_streamed_by_measurement(rb, large, precision):
    """The autotuner times the team engine against the streamed kernel on
    the RVEs no resident build holds and the incidence kernel does not take
    (all eight in FP64, the six largest in mixed precision), and keeps the
    team where it takes less CU-time (validated: same iterations and final
    states within 5% of the streamed run); the RVEs the incidence kernel
    takes stay on it."""
    batch, F = large
    b = rb.Batch(batch, precision=precision, tol_rel=1e-5 if precision else 1e-8, n_max=30000, **KW)
    before = b.describe()
    b.autotune(F, 200)
    after = b.describe()
    log(f"  before autotune: {before}; after: {after}")
    assert "team(" not in before
    if precision == 1:
        # the two 2000-seed RVEs stay on the incidence kernel; the six
        # largest (beyond its limits) may move from the streamed kernel to a team
        inc = [g for g in before.split(";") if g.startswith("incidence(")]
        assert inc == [g for g in after.split(";") if g.startswith("incidence(")] and inc[0].endswith(":2")
    sig, st = b.solve(F)
    assert np.all(np.isin(st, (0, 1)))
    b.close()
