"""Solve + tangent captured in one HIP graph (FE^2-shaped step) and replayed.

Each replay is compared bitwise with the eager result, with eager library
work and synchronisations between replays.  The library resets its work
counters with a kernel, not a memset node, so the graph replays cleanly.
"""
import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("engine", [0, 4])
def test_graph_replay_matches_eager(engine):
    """engine 0: resident kernels; 4: the incidence kernel (its per-solve
    records are written by the kernel itself, no memset node)."""
    rb = require_gpu()
    import torch
    log(f"graph capture of solve + tangent, engine {engine}")
    batch, F = synth.make_config_batch(4, idx=np.arange(6))
    b = rb.Batch(batch, precision=rb.MIXED, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5,
                 n_max=20000, check_every=8, cg_tol=1e-6, engine=engine)
    log(f"  groups {b.describe()}")
    s = torch.cuda.Stream()
    Fd = torch.tensor(F, device="cuda")
    with torch.cuda.stream(s):
        sig_e, st_e = b.solve(Fd)            # eager reference (also allocates every workspace)
        C_e, ct_e = b.tangent(like=Fd)
    s.synchronize()
    sig_e, st_e, C_e, ct_e = (t.clone() for t in (sig_e, st_e, C_e, ct_e))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        sig_g, st_g = b.solve(Fd)
        C_g, ct_g = b.tangent(like=Fd)
    for rep in range(3):
        with torch.cuda.stream(s):
            b.solve(Fd * 1.01)                   # eager work between replays
        s.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(st_g, st_e) and torch.equal(ct_g, ct_e), rep
        assert torch.equal(torch.nan_to_num(sig_g), torch.nan_to_num(sig_e)), rep
        assert torch.equal(torch.nan_to_num(C_g), torch.nan_to_num(C_e)), rep
    b.close()
