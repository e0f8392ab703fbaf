"""GPU tangent dsigma/dF (adjoint CG) and VJP against the oracle.

Reference: the oracle's exact linearisation at its own converged state (dense
K_ff solve), itself pinned to central finite differences of relaxed stresses
on small networks.  Tolerance: max |C_gpu - C_ref| <= 1e-5 max |C_ref| (the
inner solves use FP32 products inside FP64 iterative refinement to
cg_tol = 1e-9, and both states are converged to tol_rel = 1e-11).
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_09427_amd import synth
from tests.gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    return require_gpu()


def _solve_both(rb, batch, F, c=2.0, alpha=0.5, tol_rel=1e-11):
    o = oracle.make_opts(law=oracle.EXP, alpha=alpha, tol_abs=0.0, tol_rel=tol_rel, n_max=400000)
    ref = oracle.solve_batch(batch, F, c, o)
    b = rb.Batch(batch, precision=rb.FP64, law=rb.LAW_EXP, alpha=alpha, c=c, tol_abs=0.0, tol_rel=tol_rel,
                 n_max=400000, cg_tol=1e-9)
    sig, st = b.solve(F)
    return b, sig, st, ref, o


def _stable_dense_tangent(batch, k, ref, F, o):
    net = batch.network(k)
    x = ref["x"][batch.node_off[k]:batch.node_off[k + 1]]
    L0 = oracle.rest_lengths(net.X, net.fib)
    K = oracle.stiffness_dense(x, net.fib, L0, o)
    fr = np.repeat(net.is_bnd == 0, 3)
    try:
        np.linalg.cholesky(K[np.ix_(fr, fr)])
    except np.linalg.LinAlgError:
        return None
    return dense.tangent_forward(net, F[k], x, o)


def test_tangent_small_networks(rb):
    log("tangent small networks")
    nets = [synth.voronoi_network(15, [15, s, 0]) for s in range(8)]
    nets = [n for n in nets if n.n_free > 0]
    batch = synth.pack(nets)
    F = np.tile(np.array([[1.2, 0.04, 0.0], [0.0, 1.12, 0.03], [0.02, 0.0, 1.1]]), (len(nets), 1, 1))
    b, sig, st, ref, o = _solve_both(rb, batch, F)
    C, tst = b.tangent()
    checked = 0
    for k in range(len(nets)):
        if st[k] != 0 or ref["status"][k] != 0:
            continue
        Cr = _stable_dense_tangent(batch, k, ref, F, o)
        if Cr is None:
            continue
        assert tst[k] == 0
        err = np.abs(C[k] - Cr).max() / np.abs(Cr).max()
        log(f"  rve {k}: rel err {err:.2e}")
        assert err <= 1e-5
        checked += 1
    assert checked >= 3
    b.close()


def test_tangent_config4_subset(rb):
    """Four 300-seed RVEs of the tangent workload (F = I + 0.05 G)."""
    log("tangent config4 subset")
    idx = np.array([0, 2, 7, 13])
    batch, F = synth.make_config_batch(4, idx=idx)
    b, sig, st, ref, o = _solve_both(rb, batch, F)
    C, tst = b.tangent()
    checked = 0
    for k in range(len(idx)):
        if st[k] != 0 or ref["status"][k] != 0:
            continue
        Cr = _stable_dense_tangent(batch, k, ref, F, o)
        if Cr is None:
            continue
        err = np.abs(C[k] - Cr).max() / np.abs(Cr).max()
        log(f"  rve {idx[k]}: cg status {tst[k]} rel err {err:.2e}")
        assert tst[k] == 0 and err <= 1e-5
        checked += 1
    assert checked >= 3
    b.close()


def test_vjp_is_tangent_contraction_and_autograd(rb):
    import torch
    from paper_2306_09427_amd.autograd import rve_stress
    log("vjp / autograd")
    batch, F = synth.make_config_batch(4, idx=[0, 2, 7])
    b, sig, st, ref, o = _solve_both(rb, batch, F)
    C, tst = b.tangent()
    g = np.random.default_rng(3).standard_normal((3, 3, 3))
    gF, vst = b.vjp(g)
    expect = np.einsum("rij,rijkl->rkl", g, C.reshape(3, 3, 3, 3, 3))
    ok = (st == 0) & (tst == 0) & (vst == 0)
    assert ok.sum() >= 2
    np.testing.assert_allclose(gF[ok], expect[ok], atol=1e-6 * np.abs(expect[ok]).max())
    Ft = torch.tensor(F, device="cuda", requires_grad=True)
    s_t, st_t = rve_stress(Ft, b)
    loss = (s_t * torch.tensor(g, device="cuda")).sum()
    loss.backward()
    np.testing.assert_allclose(Ft.grad.cpu().numpy()[ok], expect[ok], atol=1e-6 * np.abs(expect[ok]).max())
    b.close()


def test_tangent_matches_gpu_central_differences(rb):
    """Central differences in F (h = 1e-6) of warm-started FP64 GPU relaxations."""
    log("tangent vs GPU FD")
    batch, F = synth.make_config_batch(4, idx=[0])
    b, sig, st, ref, o = _solve_both(rb, batch, F, tol_rel=1e-12)
    assert st[0] == 0
    C, tst = b.tangent()
    h = 1e-6
    fd = np.zeros((9, 9))
    base_h = None
    for col in range(9):
        sg = []
        for sgn in (1.0, -1.0):
            b.set_opts(precision=rb.FP64, law=rb.LAW_EXP, alpha=0.5, c=2.0, tol_abs=0.0, tol_rel=1e-12, n_max=400000)
            b.solve(F)                                   # back to the base state
            b.set_opts(precision=rb.FP64, law=rb.LAW_EXP, alpha=0.5, c=2.0, tol_abs=0.0, tol_rel=1e-12, n_max=400000,
                       init=rb.INIT_WARM)
            Fp = F.copy()
            Fp[0].reshape(9)[col] += sgn * h
            s, stp = b.solve(Fp)
            assert stp[0] == 0
            sg.append(s[0])
        fd[:, col] = ((sg[0] - sg[1]) / (2 * h)).ravel()
    err = np.abs(fd - C[0]).max() / np.abs(C[0]).max()
    log(f"  FD vs adjoint rel err {err:.2e}")
    assert err <= 1e-4
    b.close()
