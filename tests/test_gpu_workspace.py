"""GPU caller-owned workspace (rve_batch_workspace_size / bind_workspace).

* A batch working in a bound torch tensor gives bitwise the same stresses,
  statuses, tangents, VJPs, orientation outputs and exported state as a
  batch that allocates its own work areas (same kernels, same inputs; the
  streamed engine so that the streamed workspace is used too).
* With the workspace bound, solve, tangent, VJP, orientation and export
  allocate no device memory: the device's free memory does not change
  across them (1 MiB slack for runtime bookkeeping) while the unbound batch
  needs at least the tangent slots.
* Binding rejects memory that is too small, misaligned or on the host;
  rebinding (None, then a new tensor) rebuilds the tangent tables and keeps
  the results.
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu
IDX = np.arange(0, 64, 4)


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def _all(b, F, g):
    sig, st = b.solve(F)
    ds, tst = b.tangent()
    it = b.tangent_iters()
    gF, vst = b.vjp(g)
    om, p2 = b.orientation((1.0, 0.0, 0.0))
    Fe, h, se = b.export_state()
    return [sig, st, ds, tst, it, gF, vst, om, p2, Fe, h, se]


def test_bound_workspace_matches_and_allocates_nothing(rb):
    import torch
    dev = torch.device("cuda:0")
    batch, F = synth.make_config_batch(2, idx=IDX)
    g = np.random.default_rng(3).standard_normal((len(IDX), 3, 3))
    opts = dict(precision=rb.MIXED, law=rb.LAW_EXP, mass=rb.MASS_SCALED, alpha=0.5, c=0.1, tol_abs=0.0,
                tol_rel=1e-5, n_max=100000, check_every=8, engine=rb.ENGINE_STREAMED)
    log("workspace: library-owned reference")
    b0 = rb.Batch(batch, **opts)
    ref = _all(b0, F, g)
    b0.close()
    b1 = rb.Batch(batch, **opts)
    need = b1.workspace_size()
    log(f"  workspace size {need / 2**20:.1f} MiB for {len(IDX)} RVEs")
    ws = torch.empty(need + 4096, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    buf = ws[off:off + need]
    with pytest.raises(rb.RVEError):
        b1.bind_workspace(ws[off:off + need - 256])                 # too small
    with pytest.raises(rb.RVEError):
        b1.bind_workspace(ws[off + 1:off + 1 + need])              # misaligned
    with pytest.raises(rb.RVEError):
        b1.bind_workspace(torch.empty(need, dtype=torch.uint8))     # host memory
    b1.bind_workspace(buf)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    out = _all(b1, F, g)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(dev)[0]
    log(f"  device free memory change across the calls: {(free0 - free1) / 2**20:.3f} MiB")
    assert abs(free0 - free1) <= 2**20
    for a, r in zip(out, ref):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(r))
    # unbind, then bind a fresh tensor: tables are rebuilt, results unchanged
    b1.bind_workspace(None)
    with pytest.raises(rb.RVEError):
        b1.tangent_iters()
    ws2 = torch.zeros(need + 512, dtype=torch.uint8, device=dev)
    off2 = (-ws2.data_ptr()) % 256
    b1.bind_workspace(ws2[off2:off2 + need])
    out2 = _all(b1, F, g)
    for a, r in zip(out2, ref):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(r))
    b1.close()
