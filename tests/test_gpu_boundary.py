"""Boundary items of the C ABI on the GPU, each against the oracle or its
contract: the reference start (RVE_INIT_REFERENCE), caller-given rest
lengths (rve_net_desc.L0), the state generation counter and the autograd
guard built on it, RVE_EWORKSPACE, the admission of kernel builds (none that
uses private memory is chosen), and the tangent at a mixed-precision state.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_09427_amd import synth
from tests.gpu_common import log, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4)])
def test_reference_start_matches_oracle(rb, precision, tol):
    """Free nodes start at Xm (Algorithm "Dynamic Relaxation" sets the free
    displacements to zero): linear fibers, the 100-seed RVE, F = diag(1.1, 1, 1)."""
    log(f"reference start precision={precision}")
    batch, F = synth.make_config_batch(1)
    o = oracle.make_opts(law=oracle.LINEAR, alpha=0.9, tol_abs=1e-10 if precision == 0 else 0.0,
                         tol_rel=0.0 if precision == 0 else 1e-6, init=oracle.INIT_REFERENCE)
    ref = oracle.solve(batch.network(0), F[0], 2.0, o)
    b = rb.Batch(batch, precision=precision, law=rb.LAW_LINEAR, alpha=0.9, c=2.0, init=rb.INIT_REFERENCE,
                 tol_abs=1e-10 if precision == 0 else 0.0, tol_rel=0.0 if precision == 0 else 1e-6)
    sig, st, stats = b.solve(F, stats=True)
    affine = rb.Batch(batch, precision=precision, law=rb.LAW_LINEAR, alpha=0.9, c=2.0,
                      tol_abs=1e-10 if precision == 0 else 0.0, tol_rel=0.0 if precision == 0 else 1e-6)
    _, _, st_aff = affine.solve(F, stats=True)
    err = rel_err(sig, ref["sigma"][None])[0]
    log(f"  status {st[0]} iters gpu {stats['iters'][0]} oracle {ref['iters']} (affine start {st_aff['iters'][0]}), "
        f"err {err:.2e}")
    assert st[0] == 0 and ref["status"] == 0
    assert stats["iters"][0] != st_aff["iters"][0]     # a different start, a different trajectory
    assert err <= tol
    if precision == 0:
        assert abs(int(stats["iters"][0]) - ref["iters"]) <= max(5, ref["iters"] // 100)
    b.close()
    affine.close()


def test_given_rest_lengths_match_oracle(rb):
    """Rest lengths 3% below the reference chords: a pre-stressed network
    that carries stress at F = I; GPU and oracle relax it to the same state."""
    log("given L0")
    nets = [synth.voronoi_network(40, [41, k, 0]) for k in range(3)]
    batch = synth.pack(nets)
    L0 = [0.97 * oracle.rest_lengths(n.X, n.fib) for n in nets]
    F = np.stack([np.eye(3), np.diag([1.05, 1.0, 0.98]), np.eye(3) + 0.02 * np.ones((3, 3))])
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-9, n_max=200000)
    for prec, tol in ((0, 1e-5), (1, 1e-4)):
        b = rb.Batch(batch, precision=prec, law=rb.LAW_EXP, alpha=0.5, c=2.0, tol_abs=0.0,
                     tol_rel=1e-9 if prec == 0 else 1e-5, n_max=200000, L0=np.concatenate(L0))
        sig, st = b.solve(F)
        for k, net in enumerate(nets):
            ref = oracle.solve(net, F[k], 2.0, o, L0=L0[k])
            err = rel_err(sig[k:k + 1], ref["sigma"][None])[0]
            log(f"  precision {prec} RVE {k}: status {st[k]} / {ref['status']}, |sigma| "
                f"{np.abs(ref['sigma']).max():.3e}, err {err:.2e}")
            assert st[k] == 0 and ref["status"] == 0
            assert np.abs(ref["sigma"]).max() > 1e-3      # pre-stressed: stress at F = I too
            assert err <= tol
        b.close()


def test_generation_counter_and_autograd_guard(rb):
    import torch
    from paper_2306_09427_amd.autograd import rve_stress
    log("generation / autograd guard")
    batch, F = synth.make_config_batch(2, idx=[0, 1, 2, 3])
    b = rb.Batch(batch, precision=rb.FP64, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-8,
                 n_max=100000)
    g0 = b.generation()
    b.solve(F)
    assert b.generation() == g0 + 1
    Ft = torch.tensor(F, device="cuda", requires_grad=True)
    sig, st = rve_stress(Ft, b)
    g1 = b.generation()
    sig.sum().backward()                      # unchanged state: backward runs
    # RVEs whose relaxation did not converge have no adjoint (NaN gradient)
    conv = st == 0
    assert Ft.grad is not None and bool(conv.any()) and torch.isfinite(Ft.grad[conv]).all()
    for change in ("solve", "import", "opts"):
        Ft.grad = None
        sig, st = rve_stress(Ft, b)
        if change == "solve":
            b.solve(F)
        elif change == "import":
            Fx, hx, sx = b.export_state()
            b.import_state(Fx, hx, sx)
        else:
            b.set_opts(precision=rb.FP64, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-8,
                       n_max=100000)
        with pytest.raises(RuntimeError, match="changed"):
            sig.sum().backward()
        log(f"  backward refused after a direct {change}")
    assert b.generation() > g1
    b.close()


def test_workspace_errors_use_their_code(rb):
    import torch
    batch, F = synth.make_config_batch(2, idx=[0, 1])
    b = rb.Batch(batch, precision=rb.MIXED, law=rb.LAW_EXP, alpha=0.5, c=2.0, tol_rel=1e-5, tol_abs=0.0)
    need = b.workspace_size()
    small = torch.empty(need // 2 + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(rb.RVEError) as e:
        b.bind_workspace(small)
    assert e.value.code == rb.EWORKSPACE
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    off = (256 - big.data_ptr() % 256) % 256 + 8
    rc = rb.lib().rve_batch_bind_workspace(b._h, C.c_void_p(big.data_ptr() + off), need)
    assert rc == rb.EWORKSPACE, rc
    b.close()


def test_no_build_with_private_memory_is_chosen(rb):
    """The kernel groups of FP64 and mixed batches of every size class use
    only builds without private memory (the FP64 4/2-slot builds of 768 and
    1024 threads, the FP64 6/3-slot build of 1024 threads and the 1024-thread
    FP64 streamed build use some; tests/test_kernel_resources_cpu.py).  Every
    FP32 resident build fits its register budget, so the mixed batch takes
    the 6/3-slot 1024-thread build for its RVEs of 4097-6144 fibers."""
    idx = [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]
    batch, F = synth.make_config_batch(5, idx=idx)
    excluded = {0: ("resident(768,4,2)", "resident(1024,4,2)", "resident(1024,6,3)"), 1: ()}
    for prec in (0, 1):
        for kin in (rb.DAMP_VISCOUS, rb.DAMP_KINETIC):
            b = rb.Batch(batch, precision=prec, law=rb.LAW_EXP, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5,
                         n_max=200, damping=kin)
            d = b.describe()
            log(f"  precision {prec} damping {kin}: {d}")
            assert not any(x in d for x in excluded[prec]), d
            if prec == 1:
                assert "resident(1024,6,3)" in d, d
            sig, st = b.solve(F)
            assert np.all(np.isin(st, (0, 1)))
            b.close()


def test_tangent_at_mixed_state_matches_exact_linearisation(rb):
    """Config-4 RVEs (300 seeds, F = I + 0.05 G): the adjoint tangent at the
    mixed-precision state (FP32 operator products, FP64 dot products and
    refinement) against the oracle's exact dense linearisation at its own
    FP64 state.  Tolerance 1e-3 of max |C|: the two states differ by the
    mixed solve's stopping error (sigma within 1e-4), which the tangent sees
    as a state perturbation; RVEs whose K_ff is not positive definite at
    the oracle's state (no unique linearisation) are skipped and counted."""
    log("tangent at the mixed state, config 4")
    idx = np.array([0, 1, 2, 3, 4, 5])
    batch, F = synth.make_config_batch(4, idx=idx)
    o = oracle.make_opts(law=oracle.EXP, alpha=0.5, tol_abs=0.0, tol_rel=1e-10, n_max=400000)
    ref = oracle.solve_batch(batch, F, 0.1, o)
    b = rb.Batch(batch, precision=rb.MIXED, law=rb.LAW_EXP, mass=1, alpha=0.5, c=0.1, tol_abs=0.0, tol_rel=1e-5,
                 n_max=400000, check_every=8, cg_tol=1e-7)
    sig, st = b.solve(F)
    Cm, tst = b.tangent()
    checked = skipped = 0
    for k in range(len(idx)):
        if st[k] != 0 or ref["status"][k] != 0:
            continue
        net = batch.network(k)
        x = ref["x"][batch.node_off[k]:batch.node_off[k + 1]]
        K = oracle.stiffness_dense(x, net.fib, oracle.rest_lengths(net.X, net.fib), o)
        fr = np.repeat(net.is_bnd == 0, 3)
        try:
            np.linalg.cholesky(K[np.ix_(fr, fr)])
        except np.linalg.LinAlgError:
            skipped += 1
            continue
        Cr = dense.tangent_forward(net, F[k], x, o)
        e_sig = rel_err(sig[k:k + 1], ref["sigma"][k:k + 1])[0]
        err = np.abs(Cm[k] - Cr).max() / np.abs(Cr).max()
        log(f"  RVE {k}: tangent status {tst[k]}, sigma err {e_sig:.1e}, tangent err {err:.2e}")
        assert tst[k] == 0
        assert err <= 1e-3
        checked += 1
    log(f"  checked {checked}, skipped (K_ff not positive definite at the oracle state) {skipped}")
    assert checked >= 3
    b.close()
