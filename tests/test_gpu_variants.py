"""Every relaxation kernel variant gives the same answer.

The batch of 64 config-2 RVEs is solved with the automatic choice, with the
workgroup size forced to 256, 512 and 1024 threads (each picks other
register-resident variants, or the streamed kernel where none of that size
holds an RVE without spilling), and on the streamed engine alone.  FP64:
statuses, iteration counts and stresses agree (the same arithmetic in a
different work distribution; stresses to 1e-10).  Mixed: stresses of RVEs
converged in both runs agree to 1e-4 (the FP32 trajectories differ in
rounding order only where the work distribution differs).
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


@pytest.mark.parametrize("prec", [0, pytest.param(1, marks=pytest.mark.skip(
    reason="a run of this mixed-precision case faulted the GPU (illegal memory access) and the cause is not "
           "known; the (512,8,4) and (256,16,8) builds it used are switched off and the case stays off the GPU"))])
def test_variants_agree(rb, prec):
    batch, F = synth.make_config_batch(2, idx=np.arange(64))
    common = dict(law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-8 if prec == 0 else 1e-5,
                  n_max=100000, check_every=8)
    runs = {}
    for name, kw in (("streamed", dict(engine=rb.ENGINE_STREAMED)), ("auto", {}), ("t256", dict(threads_per_rve=256)),
                     ("t512", dict(threads_per_rve=512)), ("t1024", dict(threads_per_rve=1024))):
        b = rb.Batch(batch, precision=prec, **common, **kw)
        sig, st, stats = b.solve(F, stats=True)
        runs[name] = (sig, st, stats["iters"])
        log(f"  precision {prec} {name}: {b.describe()} status {np.bincount(st, minlength=4).tolist()}")
        b.close()
    s0, st0, it0 = runs["streamed"]
    assert (st0 == 0).sum() >= 32
    for name in ("auto", "t256", "t512", "t1024"):
        s, st, it = runs[name]
        both = (st == 0) & (st0 == 0)
        err = rel_err(s[both], s0[both])
        log(f"  precision {prec} {name} vs streamed: sigma max rel diff {err.max():.2e}")
        if prec == 0:
            assert (st == st0).all() and (it == it0).all()
            assert err.max() <= 1e-10
        else:
            assert both.sum() >= 0.9 * (st0 == 0).sum()
            assert err.max() <= 1e-4
