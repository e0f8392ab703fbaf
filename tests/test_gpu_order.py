"""Work-list order by the previous solve's cost, GPU.

After a first solve, a resident or incidence launch group (and a streamed
one under work_order RVE_ORDER_COST) takes its RVEs in longest-processing-time order
of the previous solve (iterations x fibers, a bitonic sort on the device).  The order only decides which
persistent workgroup takes which RVE when, so every result must be bitwise
the one of a batch that solves in the host's order; a wrong permutation
(an RVE taken twice, another never) would leave that RVE's outputs from the
previous call, which the second F exposes.
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


def _kw(rb, precision, engine, order):
    return dict(precision=precision, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0,
                tol_rel=1e-5 if precision == 1 else 1e-8, n_max=20000, check_every=8, engine=engine,
                work_order=order)


@pytest.mark.parametrize("precision,engine,order", [(1, 0, 0), (0, 0, 0), (1, 1, 2), (1, 0, 1)])
def test_cost_order_gives_the_same_results(precision, engine, order):
    rb = require_gpu()
    idx = np.arange(96)
    batch, F1 = synth.make_config_batch(2, idx=idx)
    F2 = np.eye(3)[None] + 0.8 * (F1 - np.eye(3)[None])
    kw = _kw(rb, precision, engine, order)
    b = rb.Batch(batch, **kw)
    s1, t1, x1 = b.solve(F1, stats=True)       # host order (most fibers first)
    s1b, t1b, x1b = b.solve(F1, stats=True)    # order by the first solve's cost
    s2, t2, x2 = b.solve(F2, stats=True)       # order by F1's cost, new F
    log(f"groups {b.describe()}; statuses {np.bincount(t2, minlength=4).tolist()}")
    fresh = rb.Batch(batch, **kw)
    r2, u2, y2 = fresh.solve(F2, stats=True)
    assert np.array_equal(s1, s1b, equal_nan=True) and np.array_equal(t1, t1b)
    assert np.array_equal(x1["iters"], x1b["iters"])
    assert np.array_equal(s2, r2, equal_nan=True) and np.array_equal(t2, u2)
    assert np.array_equal(x2["iters"], y2["iters"])
    assert not np.array_equal(s2, s1, equal_nan=True)
    b.close()
    fresh.close()


def test_switching_work_order_restores_host_order():
    """Cost order, then host order through set_opts, on a resident batch."""
    rb = require_gpu()
    batch, F1 = synth.make_config_batch(2, idx=np.arange(64))
    F2 = np.eye(3)[None] + 0.8 * (F1 - np.eye(3)[None])
    b = rb.Batch(batch, **_kw(rb, 1, 0, rb.ORDER_COST))
    b.solve(F1)
    b.solve(F1)
    b.set_opts(**_kw(rb, 1, 0, rb.ORDER_HOST))
    s2, t2, x2 = b.solve(F2, stats=True)
    fresh = rb.Batch(batch, **_kw(rb, 1, 0, rb.ORDER_AUTO))
    r2, u2, y2 = fresh.solve(F2, stats=True)
    assert np.array_equal(s2, r2, equal_nan=True) and np.array_equal(t2, u2)
    assert np.array_equal(x2["iters"], y2["iters"])
    b.close()
    fresh.close()


def test_work_order_is_validated():
    rb = require_gpu()
    batch, _ = synth.make_config_batch(2, idx=np.arange(4))
    with pytest.raises(rb.RVEError):
        rb.Batch(batch, precision=1, work_order=3)
