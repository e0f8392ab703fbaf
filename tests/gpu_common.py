"""Shared helpers of the GPU tests (not collected by pytest)."""
import os

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_09427_amd import binding as rb
    if not os.path.exists(rb.LIB_PATH):
        pytest.fail("librvebatch.so is not built (run __graft_entry__.build())")
    return rb


def rel_err(a, b):
    """max |a - b| / max |b| per RVE (stress tensors [R,3,3])."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)


def log(msg):
    print(msg, flush=True)
