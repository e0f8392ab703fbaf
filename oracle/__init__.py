"""FP64 CPU oracle for the fiber-network RVE relaxation (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports it, and it imports nothing from the product path.

``dr_oracle.c`` restates the relaxation, the truss force law and the
boundary-reaction stress from the paper (Section 2: affine boundary condition
and homogenized Cauchy stress as a boundary integral of traction times
position; Section 3.2: the dynamic-relaxation algorithm).  ``dense.py`` holds
the small dense-matrix checks: brute-force Newton and the exact linearised
tangent dsigma/dF.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, LOAD_PATH, SRC, build

LINEAR, EXP = 0, 1
INIT_AFFINE, INIT_REFERENCE, INIT_GIVEN = 0, 1, 2
MASS_LUMPED, MASS_SCALED = 0, 1
CONVERGED, MAXITER, NONFINITE, BAD_F = 0, 1, 2, 3
ENERGY = 7
STAGNATED = 8
DAMP_VISCOUS, DAMP_KINETIC, DAMP_ADAPTIVE = 0, 1, 2


class Opts(C.Structure):
    _fields_ = [("law", C.c_int32), ("init", C.c_int32), ("mass", C.c_int32), ("pad_", C.c_int32),
                ("EA", C.c_double), ("B", C.c_double),
                ("rhoA", C.c_double), ("alpha", C.c_double), ("tol_abs", C.c_double),
                ("tol_rel", C.c_double), ("n_max", C.c_int64), ("floor_tol_rel", C.c_double),
                ("stall_checks", C.c_int32), ("pad2_", C.c_int32)]


def make_opts(law=EXP, EA=1.0, B=10.0, rhoA=1.0, alpha=0.9, tol_abs=1e-10, tol_rel=0.0,
              n_max=1_000_000, init=INIT_AFFINE, mass=MASS_LUMPED, floor_tol_rel=0.0, stall_checks=16) -> Opts:
    return Opts(int(law), int(init), int(mass), 0, float(EA), float(B), float(rhoA), float(alpha),
                float(tol_abs), float(tol_rel), int(n_max), float(floor_tol_rel), int(stall_checks), 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LOAD_PATH == LIB and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = C.CDLL(LOAD_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        L.or_forces.argtypes = [i64, i64, P, P, P, C.POINTER(Opts), P, P, P]
        L.or_stiffness_dense.argtypes = [i64, i64, P, P, P, C.POINTER(Opts), P]
        L.or_stress.argtypes = [i64, P, P, P, P, C.c_double, P]
        L.or_rest_lengths.argtypes = [i64, P, P, P]
        L.or_solve.argtypes = [i64, i64, P, P, P, P, C.c_double, P, C.c_double, C.POINTER(Opts),
                               P, P, P, P, P]
        L.or_solve.restype = C.c_int
        L.or_solve_batch.argtypes = [i64, P, P, P, P, P, P, P, P, C.POINTER(Opts), C.c_int32,
                                     P, P, P, P, P, P]
        L.or_solve_variant.argtypes = [i64, i64, P, P, P, C.c_double, P, C.c_double, C.POINTER(Opts),
                                       C.c_int32, C.c_int32, C.c_double, P, P, P, P, P, P, P]
        L.or_solve_variant.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def rest_lengths(X, fib):
    X = _f64(X); fib = np.ascontiguousarray(fib, np.int32)
    L0 = np.empty(len(fib))
    lib().or_rest_lengths(len(fib), _p(X), _p(fib), _p(L0))
    return L0


def forces(x, fib, L0, opts):
    """Internal nodal forces, Gershgorin sums G and stored energy at positions x."""
    x = _f64(x); fib = np.ascontiguousarray(fib, np.int32); L0 = _f64(L0)
    n = len(x)
    f = np.empty((n, 3)); G = np.empty(n); W = C.c_double(0.0)
    lib().or_forces(n, len(fib), _p(x), _p(fib), _p(L0), C.byref(opts), _p(f), _p(G), C.byref(W))
    return f, G, W.value


def stiffness_dense(x, fib, L0, opts):
    x = _f64(x); fib = np.ascontiguousarray(fib, np.int32); L0 = _f64(L0)
    n = len(x)
    K = np.empty((3 * n, 3 * n))
    lib().or_stiffness_dense(n, len(fib), _p(x), _p(fib), _p(L0), C.byref(opts), _p(K))
    return K


def stress(x, f, is_bnd, F, V0=1.0):
    x = _f64(x); f = _f64(f); F = _f64(F); ib = np.ascontiguousarray(is_bnd, np.uint8)
    s = np.empty(9)
    lib().or_stress(len(x), _p(x), _p(f), _p(ib), _p(F), float(V0), _p(s))
    return s.reshape(3, 3)


def solve(net, F, c, opts, x0=None, V0=1.0, L0=None):
    """Relax one network under F.  Returns dict(sigma, x, iters, R, D, status)."""
    X = _f64(net.X); ib = np.ascontiguousarray(net.is_bnd, np.uint8)
    fib = np.ascontiguousarray(net.fib, np.int32); F = _f64(F)
    x = np.zeros_like(X) if x0 is None else _f64(x0).copy()
    sig = np.empty(9); it = C.c_int64(0); R = C.c_double(0); D = C.c_double(0)
    L0a = None if L0 is None else _f64(L0)
    st = lib().or_solve(len(X), len(fib), _p(X), _p(ib), _p(fib), _p(L0a), float(V0), _p(F), float(c),
                        C.byref(opts), _p(x), _p(sig), C.byref(it), C.byref(R), C.byref(D))
    return dict(sigma=sig.reshape(3, 3), x=x, iters=it.value, R=R.value, D=D.value, status=st)


def solve_batch(batch, F, c, opts, threads=None, V0=None):
    """Relax every RVE of a packed batch (one RVE per thread at a time)."""
    R_ = batch.n_rve
    F = _f64(F).reshape(R_, 9)
    c = _f64(np.broadcast_to(np.asarray(c, dtype=np.float64), (R_,)))
    V0a = None if V0 is None else _f64(np.broadcast_to(V0, (R_,)))
    x = np.zeros_like(batch.X)
    sig = np.empty((R_, 9)); iters = np.empty(R_, np.int64)
    Rr = np.empty(R_); Dd = np.empty(R_); st = np.empty(R_, np.int32)
    if threads is None:
        threads = os.cpu_count() or 1
    lib().or_solve_batch(R_, _p(batch.node_off), _p(batch.fib_off), _p(_f64(batch.X)),
                         _p(np.ascontiguousarray(batch.is_bnd, np.uint8)),
                         _p(np.ascontiguousarray(batch.fib, np.int32)), _p(V0a), _p(F), _p(c),
                         C.byref(opts), int(threads), _p(x), _p(sig), _p(iters), _p(Rr), _p(Dd), _p(st))
    return dict(sigma=sig.reshape(R_, 3, 3), x=x, iters=iters, R=Rr, D=Dd, status=st)


def solve_variant(net, F, c, opts, damping=DAMP_VISCOUS, energy_check=False, energy_tol=0.05, x0=None, V0=1.0):
    """Relax one network with a damping variant (viscous / kinetic / adaptive)
    and the optional energy-balance check (dr_oracle.c, or_solve_variant).
    Returns dict(sigma, x, iters, R, D, c, energy, status)."""
    X = _f64(net.X); ib = np.ascontiguousarray(net.is_bnd, np.uint8)
    fib = np.ascontiguousarray(net.fib, np.int32); F = _f64(F)
    x = np.zeros_like(X) if x0 is None else _f64(x0).copy()
    sig = np.empty(9); it = C.c_int64(0); R = C.c_double(0); D = C.c_double(0)
    cf = C.c_double(0); e = C.c_double(0)
    st = lib().or_solve_variant(len(X), len(fib), _p(X), _p(ib), _p(fib), float(V0), _p(F), float(c),
                                C.byref(opts), int(damping), int(bool(energy_check)), float(energy_tol), _p(x),
                                _p(sig), C.byref(it), C.byref(R), C.byref(D), C.byref(cf), C.byref(e))
    return dict(sigma=sig.reshape(3, 3), x=x, iters=it.value, R=R.value, D=D.value, c=cf.value,
                energy=e.value, status=st)


def solve_variant_batch(batch, F, c, opts, damping=DAMP_VISCOUS, energy_check=False, energy_tol=0.05,
                        threads=None):
    """solve_variant over every RVE of a packed batch (RVEs spread over threads)."""
    from concurrent.futures import ThreadPoolExecutor
    R_ = batch.n_rve
    F = _f64(F).reshape(R_, 3, 3)
    c = np.broadcast_to(np.asarray(c, dtype=np.float64), (R_,))
    with ThreadPoolExecutor(max_workers=threads or os.cpu_count() or 1) as ex:
        outs = list(ex.map(lambda r: solve_variant(batch.network(r), F[r], c[r], opts, damping, energy_check,
                                                   energy_tol), range(R_)))
    keys = ("iters", "R", "D", "c", "energy", "status")
    res = {k: np.array([o[k] for o in outs]) for k in keys}
    res["status"] = res["status"].astype(np.int32)
    res["sigma"] = np.array([o["sigma"] for o in outs])
    res["x"] = np.concatenate([o["x"] for o in outs]) if outs else np.zeros((0, 3))
    return res
