"""Relax one of the five synthetic workloads on cuda:0 and print one JSON line.

    python -m paper_2306_09427_amd.run_config --config 3 [--precision mixed|fp64]

The workloads are those of synth.make_config_batch (config 1: one 100-seed
RVE, linear fibers; 2-5: exponential fibers).  The line gives the kernel
groups the batch chose (rve_batch_describe and per group), the wall time and the HIP-event time of every
launch group of one solve (after one untimed warm-up solve), the statuses,
and the algorithmic HBM bytes of every group (per iteration and RVE
20 B per fiber + 52 B per free node in mixed precision, 32 B + 104 B in
FP64: read the network, read and write the state) with the rate they
imply.  Used to profile a workload other than the benchmark's under
rocprofv3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--n-rve", type=int, default=None, help="first n RVEs of the workload (default: all)")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--c", type=float, default=0.1)
    ap.add_argument("--tol-rel", type=float, default=1e-5)
    ap.add_argument("--n-max", type=int, default=100000)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--cache", default=None, help="npz file holding the generated networks (written if absent)")
    ap.add_argument("--threads-per-rve", type=int, default=0, help="force resident builds of this workgroup size")
    ap.add_argument("--engine", choices=["auto", "streamed", "team", "incidence"], default="auto")
    ap.add_argument("--tangent", action="store_true", help="also one tangent dsigma/dF call after the timed solve")
    ap.add_argument("--tangent-rhs", type=int, default=0, choices=[0, 1, 3],
                    help="right-hand sides per tangent task (0: library choice, 3: blocked)")
    ap.add_argument("--damping", choices=["viscous", "kinetic"], default="viscous")
    ap.add_argument("--solves", type=int, default=1, help="timed solves (after one untimed warm-up solve)")
    ap.add_argument("--autotune", type=int, default=0, metavar="N_ITER",
                    help="run rve_batch_autotune with this many iterations under F before the solves (0: no)")
    ap.add_argument("--work-order", choices=["auto", "host", "cost"], default="auto",
                    help="order of the RVEs in a launch (the warm-up solve is always in host order)")
    args = ap.parse_args(argv)

    import torch

    from . import binding as rb
    from . import synth

    if not torch.cuda.is_available():
        print("run_config needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    t0 = time.time()
    batch = None
    if args.cache and os.path.exists(args.cache):
        z = np.load(args.cache)
        batch = synth.Batch(z["node_off"], z["fib_off"], z["X"], z["is_bnd"], z["fib"])
        F = z["F"]
    if batch is None:
        batch, F = synth.make_config_batch(args.config, n_rve=args.n_rve)
        if args.cache:
            np.savez(args.cache, node_off=batch.node_off, fib_off=batch.fib_off, X=batch.X, is_bnd=batch.is_bnd,
                     fib=batch.fib, F=F)
    t_gen = time.time() - t0
    nfib = np.diff(batch.fib_off)
    nfree = np.array([int((batch.is_bnd[batch.node_off[r]:batch.node_off[r + 1]] == 0).sum())
                      for r in range(batch.n_rve)])
    fp64 = args.precision == "fp64"
    law = rb.LAW_LINEAR if args.config == 1 else rb.LAW_EXP
    b = rb.Batch(batch, precision=rb.FP64 if fp64 else rb.MIXED, law=law, mass=rb.MASS_SCALED, alpha=args.alpha,
                 c=args.c, tol_abs=0.0, tol_rel=args.tol_rel, n_max=args.n_max, check_every=args.check_every,
                 threads_per_rve=args.threads_per_rve,
                 engine={"auto": rb.ENGINE_AUTO, "streamed": rb.ENGINE_STREAMED, "team": rb.ENGINE_TEAM,
                         "incidence": rb.ENGINE_INCIDENCE}[args.engine],
                 damping=rb.DAMP_KINETIC if args.damping == "kinetic" else rb.DAMP_VISCOUS,
                 tangent_rhs=args.tangent_rhs,
                 work_order={"auto": rb.ORDER_AUTO, "host": rb.ORDER_HOST, "cost": rb.ORDER_COST}[args.work_order])
    b.profile(True)
    Fd = torch.tensor(F, device=dev)
    tune_s = None
    if args.autotune > 0:
        t_tune = time.perf_counter()
        b.autotune(Fd, n_iter=args.autotune)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t_tune
    b.solve(Fd)
    torch.cuda.synchronize()
    warm_relax_ms, _ = b.kernel_ms()
    warm_group_ms = [float(x) for x in b.groups()[2]]
    t1 = time.perf_counter()
    for _ in range(max(1, args.solves)):
        sig, st, stats = b.solve(Fd, stats=True)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / max(1, args.solves)
    relax_ms, stress_ms = b.kernel_ms()
    g_of, g_var, g_ms = b.groups()
    b_desc = b.describe()
    tangent = None
    if args.tangent:
        C, ct = b.tangent(like=Fd)   # builds the tangent's records
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        C, ct = b.tangent(like=Fd)
        torch.cuda.synchronize()
        tangent = {"ms": 1e3 * (time.perf_counter() - t2), "status_counts": np.bincount(ct.cpu().numpy(), minlength=7).tolist(),
                   "inner_iters": int(b.tangent_iters().sum())}
    st = st.cpu().numpy()
    it = stats["iters"].cpu().numpy()
    bpf, bpn = (32, 104) if fp64 else (20, 52)
    groups = []
    for g in range(len(g_ms)):
        sel = g_of == g
        if not sel.any():
            continue
        alg = float((it[sel] * (bpf * nfib[sel] + bpn * nfree[sel])).sum())
        kern = ("resident(%s)" % rb_variant(int(g_var[g]))) if g_var[g] >= 0 else (
            "streamed" if g_var[g] == rb.GROUP_STREAMED else "incidence" if g_var[g] == rb.GROUP_INCIDENCE
            else "incidence(global)" if g_var[g] == rb.GROUP_INCIDENCE_GLOBAL else "team(%d)" % (-1 - int(g_var[g])))
        groups.append({"kernel": kern,
                       "rves": int(sel.sum()), "ms": float(g_ms[g]), "algorithmic_bytes": alg,
                       "algorithmic_GB_per_s": alg / (float(g_ms[g]) / 1e3) / 1e9 if g_ms[g] > 0 else None})
    b.close()
    print(json.dumps({"config": args.config, "precision": args.precision, "n_rve": int(batch.n_rve),
                      "fibers": int(nfib.sum()), "free_nodes": int(nfree.sum()), "generate_s": t_gen,
                      "work_order": args.work_order, "autotune_s": tune_s, "describe": b_desc, "solve_ms": ms, "relax_ms": relax_ms, "stress_ms": stress_ms,
                      "warmup_relax_ms": warm_relax_ms, "warmup_group_ms": warm_group_ms,
                      "status_counts": np.bincount(st, minlength=4).tolist(),
                      "iters_median": float(np.median(it)), "iters_total": int(it.sum()), "groups": groups,
                      "tangent": tangent}),
          flush=True)
    return 0


# resident kernel variants (threads, fiber slots, node slots per thread), in
# the library's order
VARIANTS = [(256, 4, 2), (512, 4, 2), (768, 4, 2), (512, 6, 3), (1024, 4, 2), (1024, 6, 3)]


def rb_variant(v: int) -> str:
    return "%d,%d,%d" % VARIANTS[v]


if __name__ == "__main__":
    sys.exit(main())
