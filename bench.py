#!/usr/bin/env python3
"""Benchmark of the batched RVE relaxation on one MI355X.

Workload: 4096 Voronoi fiber-network RVEs of uneven size (200-400 uniform
seeds each), exponential-stiffening fibers (EA = 1, B = 10, linear in
compression), per-RVE F = I + 0.1 G with G symmetric (upper entries N(0,1)
clipped to [-1, 1]), affine boundary condition, damped dynamic relaxation to
|f_free| <= tol_rel |f_bnd|, homogenized Cauchy stress from the boundary
reactions.  One step = one rve_batch_solve of the whole batch in mixed
precision from the affine start, inputs resident in HBM (device pointers).

`value` counts the RVEs of a step that converged AND whose stress is within
1e-4 (relative, max-norm) of an FP64 solve of the same RVE converged to
tol_rel 1e-8 (the batched FP64 GPU engine, itself parity-tested against the
FP64 CPU oracle); RVEs whose FP64 reference did not converge cannot be
verified and do not count.  That count divided by the step time is the
metric's "RVE solves/s (sigma rel-err <= 1e-4)".

Also measured: the same batch in FP64 at the same tolerance (the plain FP64
batched speed baseline), the plain FP64 one-RVE-at-a-time engine on a few
RVEs (extrapolated per fiber evaluation), kinetic damping and the
stagnation stop (side lines, same accuracy count), the tangent dsigma/dF,
a timed leg of 512 large RVEs (2000 seeds each) on the HBM-streamed
kernel with its fraction of the HBM peak, and the CPU oracle on a bounded
sample (cpu_baseline).  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12            # B/s, MI355X HBM3E
# FP32 vector peaks of MI355X: the published 157.3 TFLOP/s counts packed
# (two-wide) FP32 FMAs; 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz =
# 78.6 TFLOP/s without them, which is what code compiled without packed
# FP32 instructions (as this library is) can reach.
PEAK_FP32_PUBLISHED = 157.3e12
PEAK_FP32_NONPACKED = 78.6e12

VARIANTS = [(256, 4, 2), (512, 4, 2), (768, 4, 2), (512, 6, 3), (1024, 4, 2), (1024, 6, 3)]


def rb_variant_name(v):
    return "%d,%d,%d" % VARIANTS[v]


# Committed rocprofv3 summaries: key -> (summary file, kernel source)
TRAFFIC_PROFILES = {
    "relax_cfg2": ("dr_resident_kernel_4096rve_200-400seeds_mixed.md", "rve_kernels.hip"),
    "relax_cfg3": ("dr_incidence_kernel_512rve_2000seeds_mixed.md", "rve_kernels.hip"),
    "tangent": ("tangent_4096rve_200-400seeds_mixed.md", "rve_tangent.hip"),
}


def measured_traffic(key):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    committed rocprofv3 summary, or None when there is none or the kernel
    source changed since it was taken."""
    if key not in TRAFFIC_PROFILES:
        return None
    md, srcname = TRAFFIC_PROFILES[key]
    path = os.path.join(ROOT, "profiles", md)
    src = os.path.join(ROOT, "paper_2306_09427_amd", "csrc", srcname)
    if not os.path.exists(path):
        return None
    fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                  if ": " in line and " " not in line.split(": ", 1)[0])
    if fields.get("kernel_source_sha256", "").strip() != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_or_make(config, n_rve, cache):
    from paper_2306_09427_amd import synth
    if cache and os.path.exists(cache):
        z = np.load(cache)
        if int(z["node_off"].shape[0]) == n_rve + 1:
            return synth.Batch(z["node_off"], z["fib_off"], z["X"], z["is_bnd"], z["fib"]), z["F"]
    batch, F = synth.make_config_batch(config, n_rve=n_rve)
    if cache:
        np.savez(cache, node_off=batch.node_off, fib_off=batch.fib_off, X=batch.X, is_bnd=batch.is_bnd,
                 fib=batch.fib, F=F)
    return batch, F


def rel_err(a, b):
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)


def timed_solves(b, Fd, steps, warmup, first=None):
    import torch
    for w in range(warmup):
        t0 = time.perf_counter()
        b.solve(Fd)
        torch.cuda.synchronize()
        if w == 0 and first is not None:
            # the first solve of a batch takes its RVEs in the host's order
            # (most fibers first); later solves order them by the previous
            # solve's cost (iterations x fibers)
            first.append(1e3 * (time.perf_counter() - t0))
    gms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sig, st, stats = b.solve(Fd, stats=True)
        gms.append(b.groups()[2])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return ms, sig.cpu().numpy(), st.cpu().numpy(), stats["iters"].cpu().numpy(), np.mean(np.array(gms), axis=0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-rve", type=int, default=4096)
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--c", type=float, default=0.1)
    ap.add_argument("--mass", type=int, default=1)
    ap.add_argument("--tol-rel", type=float, default=1e-5)
    ap.add_argument("--ref-tol-rel", type=float, default=1e-8, help="tolerance of the FP64 accuracy reference")
    ap.add_argument("--n-max", type=int, default=100000)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--naive-sample", type=int, default=4)
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--cfg3-rves", type=int, default=512, help="RVEs of the large-RVE (2000 seeds) leg; 0 skips it")
    ap.add_argument("--cfg3-streamed", type=int, default=1, help="also time the large-RVE leg on the streamed kernel (0: skip)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tangent", action="store_true")
    ap.add_argument("--no-kinetic", action="store_true", help="skip the kinetic-damping line")
    ap.add_argument("--no-floor", action="store_true", help="skip the stagnation-stop line")
    ap.add_argument("--tangent-steps", type=int, default=2)
    ap.add_argument("--cap-lines", type=int, nargs="*", default=[40000, 20000],
                    help="extra timed solves at these iteration caps (yield against time)")
    ap.add_argument("--autotune", action="store_true", help="autotune the mixed-precision kernel variants")
    ap.add_argument("--cache", default="/tmp/rve_bench_cfg2.npz",
                    help="network cache: loaded when present (no worker processes), else written")
    ap.add_argument("--cache3", default="/tmp/rve_bench_cfg3.npz")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run a plain device copy of this many MiB 10 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: RVEs are independent, so a multi-GPU run is the same kernel on a "
              "shard per GPU; only --gpus 1 is supported here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_09427_amd import binding as rb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n, "launches": 10}))
        return

    t0 = time.time()
    batch, F = load_or_make(2, args.n_rve, args.cache)
    nfib = np.diff(batch.fib_off)
    nfree = np.array([int((batch.is_bnd[batch.node_off[r]:batch.node_off[r + 1]] == 0).sum())
                      for r in range(batch.n_rve)])
    log(f"{batch.n_rve} RVEs ready in {time.time() - t0:.1f}s: fibers {nfib.sum()} (mean {nfib.mean():.0f}), "
        f"free nodes {nfree.sum()}")
    common = dict(law=rb.LAW_EXP, mass=args.mass, alpha=args.alpha, c=args.c, tol_abs=0.0, tol_rel=args.tol_rel,
                  n_max=args.n_max, check_every=args.check_every)
    Fd = torch.tensor(F, device=dev)

    # ---------------- mixed precision, timed (the step)
    b = rb.Batch(batch, precision=rb.MIXED, **common)
    if args.autotune:
        b.autotune(Fd, 300)
    groups = b.describe()
    log(f"mixed kernel groups: {groups}")
    b.profile(True)
    first_ms = []
    ms_per_step, sig, st, iters, g_ms = timed_solves(b, Fd, args.steps, args.warmup, first_ms)
    g_of, g_var, _ = b.groups()
    relax_ms, stress_ms = b.kernel_ms()
    elem_updates = float((iters * nfib).sum())
    at_cap = st == 1
    log(f"mixed: {ms_per_step:.1f} ms/step, relax {relax_ms:.1f} ms, status {np.bincount(st, minlength=4).tolist()}, "
        f"iters median {np.median(iters):.0f}, share of iterations on RVEs at n_max "
        f"{iters[at_cap].sum() / max(iters.sum(), 1):.3f}")

    # ---------------- FP64 accuracy reference (GPU, tol_rel 1e-8), not timed for the value
    bref = rb.Batch(batch, precision=rb.FP64, **dict(common, tol_rel=args.ref_tol_rel))
    tr = time.perf_counter()
    ref_sig, ref_st = bref.solve(Fd)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - tr
    ref_sig, ref_st = ref_sig.cpu().numpy(), ref_st.cpu().numpy()
    ref_groups = bref.describe()
    bref.close()
    log(f"fp64 reference (tol_rel {args.ref_tol_rel:g}): {t_ref:.1f}s, status {np.bincount(ref_st, minlength=4).tolist()}")

    def accurate(s, stt, ok_status=(0,)):
        err = rel_err(s, ref_sig)
        ok = np.isin(stt, ok_status) & (ref_st == 0)
        return ok & (err <= 1e-4), ok, err

    acc, both, err = accurate(sig, st)
    value = int(acc.sum()) / (ms_per_step / 1e3)

    # dominant launch group and its roofline
    # the relaxation of one step: every launch group (concurrent streams),
    # from the first group's start to the join, HIP events on those streams
    def gname(g):
        return (f"dr_resident_kernel<float,{rb_variant_name(int(g_var[g]))}>" if g_var[g] >= 0
                else "dr_streamed_kernel<float,1024>" if g_var[g] == rb.GROUP_STREAMED
                else "dr_incidence_kernel" if g_var[g] == rb.GROUP_INCIDENCE
                else "dr_incidence_global_kernel" if g_var[g] == rb.GROUP_INCIDENCE_GLOBAL
                else f"dr_team_kernel<float> x{-1 - int(g_var[g])}")
    dom_ms = float(relax_ms)
    alg_bytes = float((iters * (20 * nfib + 52 * nfree)).sum())
    alg_flops = float((iters * (53 * nfib + 40 * nfree)).sum())
    flop_rate = alg_flops / (dom_ms / 1e3)
    dom_name = " + ".join(gname(g) for g in range(len(g_ms))) + " (one launch each, concurrent streams)"
    group_lines = []
    for g in range(len(g_ms)):
        m = g_of == g
        fl = float((iters[m] * (53 * nfib[m] + 40 * nfree[m])).sum())
        group_lines.append({"kernel": gname(g), "rves": int(m.sum()), "ms": float(g_ms[g]),
                            "iters": int(iters[m].sum()), "fibers": int(nfib[m].sum()),
                            "algorithmic_flops": fl, "tflops_over_own_span": fl / (float(g_ms[g]) / 1e3) / 1e12})

    out = {
        "metric": "RVE solves/sec (sigma rel-err <= 1e-4) mixed vs FP64 plain; fraction of HBM peak",
        "value": value,
        "unit": "RVE solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fibers/state, f64 reductions and stress",
        "data": "synthetic",
        "config": {"workload": "4096 Voronoi RVEs, 200-400 seeds, exp fibers B=10, F=I+0.1G, mixed precision",
                   "n_rve": int(batch.n_rve), "fibers": int(nfib.sum()), "free_nodes": int(nfree.sum()),
                   "alpha": args.alpha, "c": args.c, "mass": ["lumped", "scaled"][args.mass],
                   "tol_rel": args.tol_rel, "n_max": args.n_max, "check_every": args.check_every},
        "value_definition": ("RVEs of a step that converged and are within 1e-4 of the FP64 GPU solve converged "
                             "to tol_rel %g, per second of the step" % args.ref_tol_rel),
        "counted": int(acc.sum()),
        "converged": int((st == 0).sum()),
        "converged_per_s": int((st == 0).sum()) / (ms_per_step / 1e3),
        "unverified_no_fp64_reference": int(((st == 0) & (ref_st != 0)).sum()),
        "rejected_beyond_1e-4": int((both & ~acc).sum()),
        "fp64_reference": {"tol_rel": args.ref_tol_rel, "seconds": t_ref, "groups": ref_groups,
                           "status_counts": np.bincount(ref_st, minlength=4).tolist()},
        "all_rves_per_s": batch.n_rve / (ms_per_step / 1e3),
        "status_counts": np.bincount(st, minlength=4).tolist(),
        "iters_median": float(np.median(iters)),
        "iters_total": int(iters.sum()),
        "iters_share_on_n_max_rves": float(iters[at_cap].sum() / max(iters.sum(), 1)),
        "element_updates_per_s": elem_updates / (ms_per_step / 1e3),
        "relax_kernel_ms": relax_ms,
        "first_solve_ms_host_order": first_ms[0] if first_ms else None,
        "kernel_groups": groups,
        "group_ms": [float(x) for x in g_ms],
        "stress_kernel_ms": stress_ms,
    }
    log(f"value {value:.1f}/s: {int(acc.sum())} of {int((st == 0).sum())} converged RVEs verified within 1e-4 "
        f"({int(((st == 0) & (ref_st != 0)).sum())} without an FP64 reference, {int((both & ~acc).sum())} beyond 1e-4)")

    # ---------------- tangent dsigma/dF (adjoint CG) on the converged states
    if not args.no_tangent:
        C, ct = b.tangent(like=Fd)   # first call allocates the workspace
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.tangent_steps):
            C, ct = b.tangent(like=Fd)
        e1.record()
        torch.cuda.synchronize()
        t_ms = e0.elapsed_time(e1) / args.tangent_steps
        it = b.tangent_iters()
        ct = ct.cpu().numpy()
        ok = ct == 0
        # algorithmic bytes: one pass over the network per block iteration of
        # the nine right-hand sides, 20 B per fiber, plus 24 B per free node
        # and right-hand side (p, r, Ap, x of a blocked CG): with it_r inner
        # iterations summed over an RVE's nine right-hand sides, it_r / 9
        # block iterations of 20 N_f + 216 N_free bytes
        tan_bytes = float(((it / 9.0) * (20 * nfib + 216 * nfree)).sum())
        out["tangent"] = {
            "workload": "dsigma/dF (9 right-hand sides) of every RVE of the batch at the mixed-precision state",
            "tangents_per_s": int(ok.sum()) / (t_ms / 1e3),
            "ms": t_ms,
            "cg_status_counts": np.bincount(ct, minlength=7).tolist(),
            "inner_iters_per_rhs_median": float(np.median(it[ok] / 9)) if ok.any() else None,
            "roofline": {"bound": "hbm", "achieved": tan_bytes / (t_ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": tan_bytes / (t_ms / 1e3) / PEAK_HBM,
                         "traffic": measured_traffic("tangent"),
                         "kernel": "all tangent launches of one call",
                         "algorithmic_bytes_per_launch": tan_bytes,
                         "bytes_per_unit": "20 per fiber + 216 per free node per block iteration of 9 RHS"},
        }
        log(f"tangent: {t_ms:.1f} ms, status {np.bincount(ct, minlength=7).tolist()}, "
            f"{out['tangent']['roofline']['achieved']:.0f} GB/s algorithmic")
    b.close()

    # ---------------- side lines on the same batch: kinetic damping, stagnation stop
    def side_line(name, bb, note, ok_status=(0,), ref=None):
        bb.profile(True)
        ms, s, stt, itt, _ = timed_solves(bb, Fd, args.steps, args.warmup)
        a, bo, _ = accurate(s, stt, ok_status)
        bb.close()
        line = {"workload": note, "ms_per_step": ms, "solves_per_s": int(a.sum()) / (ms / 1e3),
                "counted": int(a.sum()), "converged": int((stt == 0).sum()),
                "converged_per_s": int((stt == 0).sum()) / (ms / 1e3),
                "status_counts": np.bincount(stt, minlength=9).tolist(),
                "iters_median": float(np.median(itt)),
                "iters_share_on_n_max_rves": float(itt[stt == 1].sum() / max(itt.sum(), 1))}
        if ref is not None:
            # the same count against an FP64 reference of the same scheme
            rs, rst = ref
            a2 = np.isin(stt, ok_status) & (rst == 0) & (rel_err(s, rs) <= 1e-4)
            line["counted_vs_same_scheme_fp64"] = int(a2.sum())
            line["solves_per_s_vs_same_scheme_fp64"] = int(a2.sum()) / (ms / 1e3)
        log(f"{name}: {ms:.1f} ms/step, status {np.bincount(stt, minlength=9).tolist()}, counted {int(a.sum())}"
            + (f" ({line['counted_vs_same_scheme_fp64']} against the same scheme in FP64)" if ref is not None else ""))
        return line

    if not args.no_kinetic:
        bkr = rb.Batch(batch, precision=rb.FP64, damping=rb.DAMP_KINETIC, **dict(common, tol_rel=args.ref_tol_rel))
        ks, kst = bkr.solve(Fd)
        torch.cuda.synchronize()
        kref = (ks.cpu().numpy(), kst.cpu().numpy())
        bkr.close()
        bk = rb.Batch(batch, precision=rb.MIXED, damping=rb.DAMP_KINETIC, **common)
        out["kinetic_damping"] = side_line("kinetic", bk, "same batch and tolerance, kinetic damping (velocities "
                                           "zeroed at kinetic-energy peaks); counted against the viscous FP64 "
                                           "reference, and against a kinetic FP64 solve at the same tol_rel",
                                           ref=kref)
    # iteration cap: the same viscous solve stopped at a lower n_max (the yield
    # of converged RVEs against the time spent on RVEs that never converge)
    out["n_max_tradeoff"] = []
    for cap in args.cap_lines:
        if cap >= args.n_max:
            continue
        bc = rb.Batch(batch, precision=rb.MIXED, **dict(common, n_max=cap))
        out["n_max_tradeoff"].append(dict(side_line(f"n_max {cap}", bc, f"same batch and options, n_max {cap}"),
                                          n_max=cap))
    if not args.no_floor:
        bf = rb.Batch(batch, precision=rb.MIXED, floor_tol_rel=3e-5, stall_checks=32, **dict(common, tol_rel=1e-8))
        out["floor_stop"] = side_line("floor stop", bf, "same batch, tol_rel 1e-8 with the stagnation stop "
                                      "(floor_tol_rel 3e-5, 32 tests); counted: status 0 or 8 within 1e-4",
                                      ok_status=(0, 8))

    # ---------------- FP64 batched (same batch, same tolerance): the plain FP64 speed baseline
    if not args.no_fp64:
        b64 = rb.Batch(batch, precision=rb.FP64, **common)
        log(f"fp64 kernel groups: {b64.describe()}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s64, st64 = b64.solve(Fd)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        s64, st64 = s64.cpu().numpy(), st64.cpu().numpy()
        a64, _, _ = accurate(s64, st64)
        out["fp64_batched"] = {"seconds": t64, "groups": b64.describe(), "counted": int(a64.sum()),
                               "solves_per_s": int(a64.sum()) / t64,
                               "status_counts": np.bincount(st64, minlength=4).tolist()}
        out["mixed_vs_fp64_batched_speedup"] = value / max(out["fp64_batched"]["solves_per_s"], 1e-30)
        log(f"fp64 batched: {t64:.2f}s, counted {int(a64.sum())}; mixed/fp64 {out['mixed_vs_fp64_batched_speedup']:.2f}x")
        b64.close()

    # ---------------- naive FP64, one RVE at a time (a few RVEs, extrapolated per fiber evaluation)
    if not args.no_naive and args.naive_sample > 0:
        idx = np.arange(args.naive_sample)
        sub = batch.subset(idx)
        bn = rb.Batch(sub, precision=rb.FP64, engine=rb.ENGINE_NAIVE, **common)
        t1 = time.perf_counter()
        sn, stn, sts = bn.solve(F[idx], stats=True)
        tn = time.perf_counter() - t1
        eu_sub = float((sts["iters"] * nfib[idx]).sum())
        naive_batch_s = tn / max(eu_sub, 1.0) * elem_updates
        out["naive_fp64"] = {"sample": f"{args.naive_sample} RVEs, {tn:.1f}s, extrapolated per fiber evaluation "
                                       "to the batch's fiber evaluations",
                             "batch_seconds_extrapolated": naive_batch_s,
                             "speedup_of_mixed_batched": naive_batch_s / (ms_per_step / 1e3)}
        log(f"naive: {tn:.1f}s for {args.naive_sample} RVEs -> batch {naive_batch_s:.0f}s, "
            f"speedup {naive_batch_s / (ms_per_step / 1e3):.0f}x")
        bn.close()

    # ---------------- roofline of the dominant kernel (relaxation)
    out["roofline"] = {
        "bound": "alu",
        "achieved": flop_rate / 1e12,
        "peak": PEAK_FP32_PUBLISHED / 1e12,
        "unit": "TFLOP/s",
        "frac": flop_rate / PEAK_FP32_PUBLISHED,
        "attainable_peak": PEAK_FP32_NONPACKED / 1e12,
        "attainable_frac": flop_rate / PEAK_FP32_NONPACKED,
        "traffic": measured_traffic("relax_cfg2"),
        "kernel": dom_name,
        "kernel_ms": dom_ms,
        "span": "relaxation of the whole batch (all launch groups, first start to join)",
        "rves_in_kernel": int(batch.n_rve),
        "groups": group_lines,
        "algorithmic_flops_per_launch": alg_flops,
        "flops_per_unit": "53 per fiber-iteration + 40 per free-node-iteration",
        "peak_note": "published FP32 vector peak (packed FMA); attainable_* is against the 78.6 TFLOP/s of "
                     "unpacked FP32, the library being compiled without packed FP32 instructions",
        "hbm_equivalent": {"achieved": alg_bytes / (dom_ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                           "frac": alg_bytes / (dom_ms / 1e3) / PEAK_HBM, "algorithmic_bytes_per_launch": alg_bytes,
                           "bytes_per_unit": "20 per fiber-iteration + 52 per free-node-iteration"},
    }

    # ---------------- large RVEs (2000 seeds): the HBM-streamed regime
    if args.cfg3_rves > 0:
        t3 = time.time()
        b3net, F3 = load_or_make(3, args.cfg3_rves, args.cache3)
        nf3 = np.diff(b3net.fib_off)
        nfr3 = np.array([int((b3net.is_bnd[b3net.node_off[r]:b3net.node_off[r + 1]] == 0).sum())
                         for r in range(b3net.n_rve)])
        log(f"large RVEs ready in {time.time() - t3:.1f}s: {b3net.n_rve} RVEs, mean {nf3.mean():.0f} fibers")
        F3d = torch.tensor(F3, device=dev)
        b3 = rb.Batch(b3net, precision=rb.MIXED, **common)
        b3.profile(True)
        ms3, s3, st3, it3, gms3 = timed_solves(b3, F3d, 1, 1)
        bytes3 = float((it3 * (20 * nf3 + 52 * nfr3)).sum())
        rate3 = bytes3 / (ms3 / 1e3)
        out["large_rves"] = {
            "workload": "%d Voronoi RVEs of 2000 seeds (mean %d fibers), exp fibers, uniaxial F, mixed precision"
                        % (b3net.n_rve, nf3.mean()),
            "ms_per_solve": ms3, "groups": b3.describe(), "group_ms": [float(x) for x in gms3],
            "status_counts": np.bincount(st3, minlength=4).tolist(),
            "converged_per_s": int((st3 == 0).sum()) / (ms3 / 1e3),
            "element_updates_per_s": float((it3 * nf3).sum()) / (ms3 / 1e3),
            "roofline": {"bound": "hbm", "achieved": rate3 / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": rate3 / PEAK_HBM, "traffic": measured_traffic("relax_cfg3"),
                         "algorithmic_bytes_per_launch": bytes3,
                         "bytes_per_unit": "20 per fiber-iteration + 52 per free-node-iteration"},
        }
        log(f"large RVEs: {ms3:.0f} ms, groups {b3.describe()}, status {np.bincount(st3, minlength=4).tolist()}, "
            f"{rate3 / 1e9:.0f} GB/s algorithmic ({rate3 / PEAK_HBM:.2f} of peak)")
        b3.close()
        if args.cfg3_streamed:
            # the same workload on the streamed kernel (every array in global
            # memory, fiber forces written and gathered): one timed solve
            b3s = rb.Batch(b3net, precision=rb.MIXED, **dict(common, engine=rb.ENGINE_STREAMED))
            b3s.profile(True)
            ms3s, s3s, st3s, it3s, _ = timed_solves(b3s, F3d, 1, 0)
            both3 = (st3 == 0) & (st3s == 0)
            out["large_rves"]["streamed_kernel"] = {
                "ms_per_solve": ms3s, "groups": b3s.describe(),
                "status_counts": np.bincount(st3s, minlength=4).tolist(),
                "speedup_of_default": ms3s / ms3,
                "sigma_max_rel_diff_both_converged": float(rel_err(s3, s3s)[both3].max()) if both3.any() else None}
            log(f"large RVEs on the streamed kernel: {ms3s:.0f} ms ({ms3s / ms3:.2f}x the default engine)")
            b3s.close()

    # ---------------- CPU oracle on a bounded sample
    if not args.no_cpu and args.cpu_sample > 0:
        import oracle
        idx = np.arange(args.cpu_sample)
        sub = batch.subset(idx)
        nproc = os.cpu_count() or 1
        threads = min(nproc, 16)
        o = oracle.make_opts(law=oracle.EXP, alpha=args.alpha, tol_abs=0.0, tol_rel=args.tol_rel,
                             n_max=args.n_max, mass=args.mass)
        t1 = time.perf_counter()
        ref = oracle.solve_batch(sub, F[idx], args.c, o, threads=threads)
        tc = time.perf_counter() - t1
        n_ok = int((ref["status"] == 0).sum())
        out["cpu_baseline"] = {"value": n_ok / tc, "unit": "RVE solves/s", "cores": threads, "kind": "oracle",
                               "sample": f"first {args.cpu_sample} RVEs of the batch, same options (tol_rel "
                                         f"{args.tol_rel:g}); {n_ok} converged in {tc:.1f}s; value counts "
                                         f"converged RVEs",
                               "nproc": nproc, "cpu_model": cpu_model()}
        log(f"oracle: {tc:.1f}s on {threads} threads ({nproc} cpus, {cpu_model()})")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
