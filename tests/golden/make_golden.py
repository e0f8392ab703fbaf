"""Write oracle reference results for the full-shape GPU parity tests.

Calls only the seeded input generator and the FP64 CPU oracle; the outputs
(tests/golden/*.npz) hold per-RVE stress, status and iteration counts of the
oracle with the options recorded next to them.  Regenerate with
    python tests/golden/make_golden.py [case ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2306_09427_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

RELAX = dict(law=oracle.EXP, mass=oracle.MASS_SCALED, alpha=0.5, tol_abs=0.0, tol_rel=1e-8)


def cfg5_sample(k=16):
    """k RVEs of the 8192-RVE FE^2 workload spread over its size range."""
    seeds = np.array([synth.seed_count(5, r) for r in range(8192)])
    order = np.argsort(seeds, kind="stable")
    return np.sort(order[np.linspace(0, 8191, k).round().astype(int)])


CASES = {
    "cfg2_64": dict(config=2, idx=list(range(64)), c=0.1, n_max=100000),
    "cfg3_4": dict(config=3, idx=list(range(4)), c=0.1, n_max=200000),
    "cfg5_16": dict(config=5, idx=None, c=0.1, n_max=100000),
}


def make(name):
    case = CASES[name]
    idx = case["idx"] if case["idx"] is not None else cfg5_sample().tolist()
    batch, F = synth.make_config_batch(case["config"], idx=idx)
    o = oracle.make_opts(n_max=case["n_max"], **RELAX)
    t = time.time()
    r = oracle.solve_batch(batch, F, case["c"], o, threads=os.cpu_count())
    opts = dict(RELAX, c=case["c"], n_max=case["n_max"], config=case["config"])
    np.savez(os.path.join(HERE, f"{name}.npz"), idx=np.array(idx), sigma=r["sigma"], status=r["status"],
             iters=r["iters"], R=r["R"], opts=json.dumps(opts))
    print(f"{name}: {time.time() - t:.0f}s status {np.bincount(r['status'], minlength=4).tolist()}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
