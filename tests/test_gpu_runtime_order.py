"""The library links the system HIP runtime and torch carries its own: a
program that solves with host arrays first and uses torch tensors afterwards
must still see the GPU from torch (the binding lets torch open the device
before the library does).  Run in a fresh process, so that nothing before it
has touched the GPU."""
import os
import subprocess
import sys

import pytest

from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r"""
import numpy as np
from paper_2306_09427_amd import binding as rb, synth
batch, F = synth.make_config_batch(2, idx=[0, 1], workers=1)
b = rb.Batch(batch, precision=rb.MIXED, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5,
             n_max=20000)
sig, st = b.solve(F)
import torch
Fd = torch.tensor(F, device="cuda:0")
sig_d, st_d = b.solve(Fd)
torch.cuda.synchronize()
assert np.array_equal(sig_d.cpu().numpy(), sig), "device and host paths differ"
b.close()
print("ok", flush=True)
"""


def test_numpy_first_then_torch():
    require_gpu()
    r = subprocess.run([sys.executable, "-c", PROG], cwd=ROOT, capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "ok" in r.stdout
