"""The allocation-free solve (rve_batch_solve_static) against rve_batch_solve.

Its kernels are the solve's own; only the work areas (launch counters, the
team engine's work area and the streamed engine's workspace) come from the
library's fixed device scratch array instead of allocations.  Two calls in a row on batches of
decreasing size (the second reuses the array the first left behind) must
reproduce rve_batch_solve bitwise (same kernels, same arithmetic), on the
streamed, team and incidence engines and on the automatic engine choice, and
no device memory may be allocated by the call.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


def test_static_solve_matches_solve_twice_shrinking():
    import torch
    rb = require_gpu()
    big, Fb = synth.make_config_batch(2, idx=np.arange(24))
    small, Fs = synth.make_config_batch(5, idx=[3, 8, 13, 21, 89, 144])   # includes RVEs above every resident tier
    kw = dict(law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5, n_max=20000, check_every=8)
    for prec in (rb.MIXED, rb.FP64):
        engines = (rb.ENGINE_STREAMED, rb.ENGINE_AUTO, rb.ENGINE_TEAM) + ((rb.ENGINE_INCIDENCE,) if prec == rb.MIXED else ())
        for engine in engines:
            for name, batch, F in (("24 config-2 RVEs", big, Fb), ("6 config-5 RVEs", small, Fs)):
                b = rb.Batch(batch, precision=prec, engine=engine, **kw)
                s_ref, st_ref = b.solve(F)
                Fd = torch.tensor(F, device="cuda")
                sig_d = torch.empty((len(F), 3, 3), dtype=torch.float64, device="cuda")
                st_d = torch.empty(len(F), dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                b.set_stream(C.c_void_p(torch.cuda.current_stream().cuda_stream))
                rc = rb.lib().rve_batch_solve_static(b._h, Fd.data_ptr(), sig_d.data_ptr(), st_d.data_ptr(),
                                                     rb.PTR_DEVICE)
                torch.cuda.synchronize()
                free1 = torch.cuda.mem_get_info()[0]
                assert rc == rb.OK, rb.last_error()
                s_st, st_st = sig_d.cpu().numpy(), st_d.cpu().numpy()
                log(f"  precision {prec} engine {engine} {name}: {b.describe()} statuses "
                    f"{np.bincount(st_st, minlength=4).tolist()}, free memory change {free0 - free1} B")
                assert np.array_equal(st_st, st_ref)
                assert np.array_equal(s_st, s_ref, equal_nan=True)
                assert free1 == free0
                b.close()
