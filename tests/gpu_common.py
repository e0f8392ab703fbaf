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


def grade_parity(b, batch, F, sig, st, ref_sigma, ref_status, tol, opts, label, ref_x=None, residual_rel=None,
                 max_check=64):
    """Grade GPU stresses against the oracle's, RVE by RVE, with no allowance.

    For every RVE converged on both sides: within `tol` (relative, max-norm)
    of the oracle's stress, or else a different equilibrium that is checked
    on its own with the oracle's arithmetic: at the GPU's positions the FP64
    free-node residual is at most residual_rel |f_bnd| (an equilibrium of
    the same network under the same F) and the oracle's boundary-reaction
    stress of that state equals the GPU's stress within `tol`.  Such RVEs
    are counted and logged (with the stability of both states where the
    dense check fits), never passed silently; an RVE that is neither fails.
    Returns dict(agree, different, both)."""
    import oracle
    from oracle.stability import equilibrium, is_stable
    residual_rel = residual_rel if residual_rel is not None else 10 * max(tol, 1e-8)
    sig = np.asarray(sig).reshape(len(st), 3, 3)
    both = (np.asarray(st) == 0) & (np.asarray(ref_status) == 0)
    err = rel_err(sig, np.asarray(ref_sigma).reshape(len(st), 3, 3))
    diff = np.where(both & ~(err <= tol))[0]
    log(f"  [{label}] converged both {int(both.sum())}, within {tol:g}: {int((both & (err <= tol)).sum())}, "
        f"max err {err[both].max() if both.any() else 0:.2e}, differing {len(diff)}")
    assert len(diff) <= max_check, f"{len(diff)} RVEs differ (more than can be checked)"
    bad = []
    stable_both = 0
    for r in diff:
        net = batch.network(int(r))
        Fr = np.asarray(F).reshape(-1, 3, 3)[r]
        x = b.positions(int(r))
        R, Fb, s_x = equilibrium(net, Fr, x, opts)
        e_state = rel_err(sig[r][None], s_x[None])[0]
        ok = R <= residual_rel * Fb and e_state <= tol
        sg = is_stable(net, x, opts)
        so = is_stable(net, ref_x[r], opts) if ref_x is not None else None
        stable_both += int(bool(sg) and bool(so))
        log(f"    RVE {r}: err vs oracle {err[r]:.2e}; GPU state |f_free|/|f_bnd| {R / max(Fb, 1e-300):.1e}, "
            f"stress of the state {e_state:.1e}, stable gpu={sg} oracle={so} -> "
            f"{'different equilibrium' if ok else 'FAIL'}")
        if not ok:
            bad.append(int(r))
    log(f"  [{label}] different equilibria {len(diff) - len(bad)} (both states stable: {stable_both}), failures {bad}")
    assert not bad, f"RVEs {bad} differ from the oracle and their GPU state is not an equilibrium"
    return dict(agree=int((both & (err <= tol)).sum()), different=len(diff), both=int(both.sum()))
