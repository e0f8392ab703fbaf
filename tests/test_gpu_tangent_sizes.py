"""GPU tangent across RVE sizes: every task kernel of the tangent.

RVEs of 100 to 2200 seeds land in each launch group of rve_batch_tangent:
resident workgroups of 256, 512 and 1024 threads with registers and LDS (up
to 2048 free nodes), the lean resident variants (search direction in LDS, up
to 4096 and 8192 free nodes) and the 1024-thread streamed kernel above that.

* Every size: the default engine against the 64-thread streamed reference
  path (engine STREAMED; the same equations, one wavefront per right-hand
  side, vectors in global memory) at the same converged FP64 state:
  relative difference <= 1e-7 (both solve to cg_tol = 1e-10).
* The three smaller RVEs: both paths against the oracle's exact dense
  linearisation at the oracle's own converged state (<= 1e-5, the bar of
  test_gpu_tangent.py).

F stretches every RVE (all principal stretches > 1), so the networks are in
tension and K_ff is positive definite.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu

SEEDS = [100, 200, 400, 700, 1400, 2200]
F0 = np.array([[1.08, 0.02, 0.0], [0.0, 1.05, 0.01], [0.01, 0.0, 1.04]])
OPTS = dict(law=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-9, n_max=200000)


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def test_tangent_every_kernel_size(rb):
    nets = [synth.voronoi_network(n, [4242, i, 0]) for i, n in enumerate(SEEDS)]
    batch = synth.pack(nets)
    R = len(nets)
    nf = np.array([n.n_free for n in nets])
    log(f"tangent sizes: free nodes {nf.tolist()}")
    # one RVE per launch group (free-node capacities 512, 1024, 2048, 4096, 8192, above)
    caps = [512, 1024, 2048, 4096, 8192]
    groups = [int(np.searchsorted(caps, v)) for v in nf]
    assert sorted(groups) == list(range(6)), groups
    F = np.tile(F0, (R, 1, 1))
    b = rb.Batch(batch, precision=rb.FP64, mass=1, cg_tol=1e-10, **{**OPTS, "law": rb.LAW_EXP})
    sig, st = b.solve(F)
    log(f"  solve status {st.tolist()}")
    assert (st == 0).all()
    C_auto, s_auto = b.tangent()
    o = b.opts
    o.engine = rb.ENGINE_STREAMED
    b.set_opts(o)
    C_ref, s_ref = b.tangent()
    b.close()
    for k in range(R):
        d = np.abs(C_auto[k] - C_ref[k]).max() / np.abs(C_ref[k]).max()
        log(f"  rve {k} (nf {nf[k]}): status {s_auto[k]}/{s_ref[k]}, resident vs reference {d:.2e}")
        assert s_auto[k] == 0 and s_ref[k] == 0
        assert d <= 1e-7

    # the smaller three against the oracle's dense linearisation at its own state
    small = np.arange(3)
    sub = batch.subset(small)
    oo = oracle.make_opts(law=oracle.EXP, alpha=OPTS["alpha"], tol_abs=0.0, tol_rel=OPTS["tol_rel"],
                          n_max=OPTS["n_max"], mass=oracle.MASS_SCALED)
    ref = oracle.solve_batch(sub, F[small], OPTS["c"], oo)
    for k in small:
        assert ref["status"][k] == 0
        net = sub.network(k)
        x = ref["x"][sub.node_off[k]:sub.node_off[k + 1]]
        Cr = dense.tangent_forward(net, F[k], x, oo)
        for name, C in (("resident", C_auto), ("reference", C_ref)):
            err = np.abs(C[k] - Cr).max() / np.abs(Cr).max()
            log(f"  rve {k}: {name} vs dense oracle {err:.2e}")
            assert err <= 1e-5
