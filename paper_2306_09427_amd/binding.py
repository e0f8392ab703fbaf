"""ctypes binding of librvebatch.so (argument marshalling only).

Every step of the relaxation, the stress and the tangent runs in the HIP
library; this module converts numpy arrays / torch tensors to pointers and
option structs.  Importing it does not touch the GPU; creating a Batch does.
If the library is missing, loading fails with an error (there is no CPU
fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librvebatch.so")

FP64, MIXED = 0, 1
LAW_LINEAR, LAW_EXP = 0, 1
MASS_LUMPED, MASS_SCALED = 0, 1
INIT_AFFINE, INIT_REFERENCE, INIT_WARM = 0, 1, 2
ENGINE_AUTO, ENGINE_STREAMED, ENGINE_NAIVE, ENGINE_TEAM, ENGINE_INCIDENCE = 0, 1, 2, 3, 4
GROUP_STREAMED, GROUP_INCIDENCE, GROUP_INCIDENCE_GLOBAL = -1, -100, -101
PTR_HOST, PTR_DEVICE = 0, 1
ST_CONVERGED, ST_MAXITER, ST_NONFINITE, ST_BAD_F, ST_NO_STATE, ST_CG_MAXITER, ST_CG_INDEFINITE, ST_ENERGY = range(8)
ST_STAGNATED = 8
DAMP_VISCOUS, DAMP_KINETIC, DAMP_ADAPTIVE = 0, 1, 2
ORDER_AUTO, ORDER_HOST, ORDER_COST = 0, 1, 2
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EWORKSPACE = 0, -22, -12, -5, -3, -28

EXPORTS = ["rve_version", "rve_last_error", "rve_default_opts", "rve_batch_create", "rve_batch_set_opts",
           "rve_batch_set_stream", "rve_batch_sizes", "rve_batch_solve", "rve_batch_tangent", "rve_batch_vjp",
           "rve_batch_positions", "rve_batch_destroy", "rve_batch_profile", "rve_batch_kernel_ms",
           "rve_batch_autotune", "rve_batch_describe", "rve_batch_groups", "rve_batch_tangent_iters", "rve_batch_orientation",
           "rve_batch_fd_tangent", "rve_batch_export_state", "rve_batch_import_state",
           "rve_batch_workspace_size", "rve_batch_bind_workspace", "rve_batch_damping_stats",
           "rve_batch_generation", "rve_check_indexing", "rve_batch_team_spin_limit", "rve_batch_solve_static"]


class NetDesc(C.Structure):
    _fields_ = [("n_rve", C.c_int64), ("node_off", C.c_void_p), ("fib_off", C.c_void_p), ("X", C.c_void_p),
                ("is_bnd", C.c_void_p), ("fib", C.c_void_p), ("V0", C.c_void_p), ("L0", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("law", C.c_int32), ("mass", C.c_int32), ("init", C.c_int32),
                ("EA", C.c_double), ("B", C.c_double), ("rhoA", C.c_double), ("alpha", C.c_double),
                ("c", C.c_double), ("c_per_rve", C.c_void_p), ("tol_abs", C.c_double), ("tol_rel", C.c_double),
                ("n_max", C.c_int64), ("check_every", C.c_int32), ("engine", C.c_int32),
                ("threads_per_rve", C.c_int32), ("cg_tol", C.c_double), ("cg_max_iter", C.c_int64),
                ("stream", C.c_void_p), ("damping", C.c_int32), ("energy_check", C.c_int32),
                ("energy_tol", C.c_double), ("floor_tol_rel", C.c_double), ("stall_checks", C.c_int32),
                ("tangent_rhs", C.c_int32), ("work_order", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_void_p), ("R", C.c_void_p), ("D", C.c_void_p), ("Fb", C.c_void_p)]


class RVEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rvebatch error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load librvebatch.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        # The library links the system HIP runtime while torch carries its
        # own copy; torch's copy finds no GPU once the other one has opened
        # the device, so let torch open it first when torch is installed.
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.rve_version.restype = C.c_int
        L.rve_last_error.restype = C.c_char_p
        L.rve_default_opts.argtypes = [C.POINTER(Opts)]
        L.rve_batch_create.argtypes = [C.POINTER(NetDesc), C.POINTER(Opts), C.POINTER(P)]
        L.rve_batch_set_opts.argtypes = [P, C.POINTER(Opts)]
        L.rve_batch_set_stream.argtypes = [P, P]
        L.rve_batch_sizes.argtypes = [P, P, P, P]
        L.rve_batch_solve.argtypes = [P, P, P, P, C.POINTER(Stats), C.c_int32]
        L.rve_batch_tangent.argtypes = [P, P, P, C.c_int32]
        L.rve_batch_vjp.argtypes = [P, P, P, P, C.c_int32]
        L.rve_batch_positions.argtypes = [P, C.c_int64, P]
        L.rve_batch_profile.argtypes = [P, C.c_int]
        L.rve_batch_kernel_ms.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.rve_batch_autotune.argtypes = [P, P, C.c_int32, C.c_int32]
        L.rve_batch_describe.argtypes = [P, C.c_char_p, C.c_size_t]
        L.rve_batch_groups.argtypes = [P, P, P, P, C.c_int32, P]
        L.rve_batch_tangent_iters.argtypes = [P, P, C.c_int32]
        L.rve_batch_orientation.argtypes = [P, P, P, P, C.c_int32]
        L.rve_batch_fd_tangent.argtypes = [P, C.c_double, P, P, P, C.c_int32]
        L.rve_batch_export_state.argtypes = [P, P, P, P, C.c_int32]
        L.rve_batch_import_state.argtypes = [P, P, P, P, P, C.c_int32]
        L.rve_batch_workspace_size.argtypes = [P, C.POINTER(C.c_size_t)]
        L.rve_batch_bind_workspace.argtypes = [P, P, C.c_size_t]
        L.rve_batch_damping_stats.argtypes = [P, P, P, C.c_int32]
        L.rve_batch_generation.argtypes = [P, C.POINTER(C.c_uint64)]
        L.rve_batch_solve_static.argtypes = [P, P, P, P, C.c_int32]
        L.rve_check_indexing.argtypes = [C.POINTER(NetDesc), C.c_int32, C.c_int32]
        L.rve_batch_team_spin_limit.argtypes = [P, C.c_int64]
        L.rve_batch_destroy.argtypes = [P]
        L.rve_batch_destroy.restype = None
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rve_last_error().decode()


def _check(rc):
    if rc != OK:
        raise RVEError(rc, last_error())


def make_opts(precision=FP64, law=LAW_EXP, mass=MASS_LUMPED, init=INIT_AFFINE, EA=1.0, B=10.0, rhoA=1.0,
              alpha=0.9, c=2.0, tol_abs=1e-10, tol_rel=0.0, n_max=1_000_000, check_every=1,
              engine=ENGINE_AUTO, threads_per_rve=0, cg_tol=1e-6, cg_max_iter=0, damping=DAMP_VISCOUS,
              energy_check=False, energy_tol=0.05, floor_tol_rel=0.0, stall_checks=16, tangent_rhs=0,
              work_order=0) -> Opts:
    o = Opts()
    lib().rve_default_opts(C.byref(o))
    o.precision, o.law, o.mass, o.init = int(precision), int(law), int(mass), int(init)
    o.EA, o.B, o.rhoA, o.alpha, o.c = float(EA), float(B), float(rhoA), float(alpha), float(c)
    o.tol_abs, o.tol_rel, o.n_max, o.check_every = float(tol_abs), float(tol_rel), int(n_max), int(check_every)
    o.engine, o.threads_per_rve = int(engine), int(threads_per_rve)
    o.cg_tol, o.cg_max_iter = float(cg_tol), int(cg_max_iter)
    o.damping, o.energy_check, o.energy_tol = int(damping), int(bool(energy_check)), float(energy_tol)
    o.floor_tol_rel, o.stall_checks = float(floor_tol_rel), int(stall_checks)
    o.tangent_rhs = int(tangent_rhs)
    o.work_order = int(work_order)
    return o


def _ptr(a):
    """Pointer and kind of a numpy array (host) or torch tensor (host or device)."""
    if a is None:
        return None, PTR_HOST
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), (PTR_DEVICE if a.is_cuda else PTR_HOST)
    return a.ctypes.data, PTR_HOST


def net_desc(nets, V0=None, L0=None):
    """NetDesc of a packed batch (node_off, fib_off, X, is_bnd, fib) and the
    arrays it points into (keep them alive while the descriptor is used).
    V0: per-RVE reference volume (None: 1); L0: per-fiber rest length (None:
    the reference chord length)."""
    node_off = np.ascontiguousarray(nets.node_off, np.int64)
    fib_off = np.ascontiguousarray(nets.fib_off, np.int64)
    X = np.ascontiguousarray(nets.X, np.float64)
    ib = np.ascontiguousarray(nets.is_bnd, np.uint8)
    fib = np.ascontiguousarray(nets.fib, np.int32)
    n_rve = int(len(node_off) - 1)
    V0a = None if V0 is None else np.ascontiguousarray(np.broadcast_to(V0, (n_rve,)), np.float64)
    L0a = None if L0 is None else np.ascontiguousarray(L0, np.float64).reshape(int(fib_off[-1]))
    d = NetDesc(n_rve, node_off.ctypes.data, fib_off.ctypes.data, X.ctypes.data, ib.ctypes.data,
                fib.ctypes.data, None if V0a is None else V0a.ctypes.data, None if L0a is None else L0a.ctypes.data)
    return d, (node_off, fib_off, X, ib, fib, V0a, L0a)


def check_indexing(nets, precision=MIXED, plant=0, L0=None):
    """Host replay of the kernels' index arithmetic over a batch (rve_check_indexing); raises on a violation."""
    d, keep = net_desc(nets, None, L0)
    _check(lib().rve_check_indexing(C.byref(d), int(precision), int(plant)))


class Batch:
    """A packed batch of RVE networks resident on the current HIP device."""

    def __init__(self, nets, opts: Opts | None = None, c_per_rve=None, V0=None, L0=None, **kw):
        self._keep = {}
        d, keep = net_desc(nets, V0, L0)
        self.n_rve = int(d.n_rve)
        node_off = keep[0]
        self.opts = opts if opts is not None else make_opts(**kw)
        cpr = None
        if c_per_rve is not None:
            cpr = np.ascontiguousarray(np.broadcast_to(c_per_rve, (self.n_rve,)), np.float64)
            self.opts.c_per_rve = cpr.ctypes.data
        h = C.c_void_p()
        _check(lib().rve_batch_create(C.byref(d), C.byref(self.opts), C.byref(h)))
        self.opts.c_per_rve = None
        self._h = h
        self.node_off = node_off

    def close(self):
        if getattr(self, "_h", None):
            lib().rve_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_opts(self, opts: Opts | None = None, c_per_rve=None, **kw):
        o = opts if opts is not None else make_opts(**kw)
        cpr = None
        if c_per_rve is not None:
            cpr = np.ascontiguousarray(np.broadcast_to(c_per_rve, (self.n_rve,)), np.float64)
            o.c_per_rve = cpr.ctypes.data
        _check(lib().rve_batch_set_opts(self._h, C.byref(o)))
        o.c_per_rve = None
        self.opts = o

    def team_spin_limit(self, polls):
        """Polls of a team barrier before a team gives up (tests of that path)."""
        _check(lib().rve_batch_team_spin_limit(self._h, int(polls)))

    def generation(self):
        """Counter of the state's changes (solve, import, option change)."""
        g = C.c_uint64()
        _check(lib().rve_batch_generation(self._h, C.byref(g)))
        return g.value

    def set_stream(self, stream_handle):
        _check(lib().rve_batch_set_stream(self._h, stream_handle))

    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().rve_batch_sizes(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def _outs(self, F, shape_tail, dtype):
        """Allocate outputs like F (numpy on host, torch on F's device)."""
        if hasattr(F, "data_ptr"):
            import torch
            tdt = {np.float64: torch.float64, np.int32: torch.int32, np.int64: torch.int64}[dtype]
            return torch.empty((self.n_rve, *shape_tail), dtype=tdt, device=F.device)
        return np.empty((self.n_rve, *shape_tail), dtype=dtype)

    def solve(self, F, stats=False):
        """Relax all RVEs under F[R,3,3]; returns sigma[R,3,3], status[R] (and stats)."""
        if hasattr(F, "data_ptr"):
            F = F.contiguous()
            if F.is_cuda:
                import torch
                self.set_stream(C.c_void_p(torch.cuda.current_stream(F.device).cuda_stream))
        else:
            F = np.ascontiguousarray(F, np.float64).reshape(self.n_rve, 3, 3)
        sig = self._outs(F, (3, 3), np.float64)
        st = self._outs(F, (), np.int32)
        fp, kind = _ptr(F)
        S = None
        out = {}
        if stats:
            out = {"iters": self._outs(F, (), np.int64), "R": self._outs(F, (), np.float64),
                   "D": self._outs(F, (), np.float64), "Fb": self._outs(F, (), np.float64)}
            S = Stats(_ptr(out["iters"])[0], _ptr(out["R"])[0], _ptr(out["D"])[0], _ptr(out["Fb"])[0])
        _check(lib().rve_batch_solve(self._h, fp, _ptr(sig)[0], _ptr(st)[0], C.byref(S) if S else None, kind))
        return (sig, st, out) if stats else (sig, st)

    def solve_static(self, F):
        """rve_batch_solve_static: the solve with its work areas in the
        library's fixed device scratch array (no device allocation); returns
        sigma[R,3,3], status[R]."""
        if hasattr(F, "data_ptr"):
            F = F.contiguous()
            if F.is_cuda:
                import torch
                self.set_stream(C.c_void_p(torch.cuda.current_stream(F.device).cuda_stream))
        else:
            F = np.ascontiguousarray(F, np.float64).reshape(self.n_rve, 3, 3)
        sig = self._outs(F, (3, 3), np.float64)
        st = self._outs(F, (), np.int32)
        fp, kind = _ptr(F)
        _check(lib().rve_batch_solve_static(self._h, fp, _ptr(sig)[0], _ptr(st)[0], kind))
        return sig, st

    def tangent(self, like=None):
        """dsigma/dF [R,9,9] at the last solve's state, and status [R]."""
        ref = like if like is not None else np.empty(0)
        ds = self._outs(ref, (9, 9), np.float64)
        st = self._outs(ref, (), np.int32)
        _check(lib().rve_batch_tangent(self._h, _ptr(ds)[0], _ptr(st)[0], _ptr(ds)[1]))
        return ds, st

    def vjp(self, gsigma):
        """g_F[R,3,3] = sum_ij g_ij dsigma_ij/dF at the last solve's state."""
        if hasattr(gsigma, "data_ptr"):
            gsigma = gsigma.contiguous()
        else:
            gsigma = np.ascontiguousarray(gsigma, np.float64)
        gF = self._outs(gsigma, (3, 3), np.float64)
        st = self._outs(gsigma, (), np.int32)
        gp, kind = _ptr(gsigma)
        _check(lib().rve_batch_vjp(self._h, gp, _ptr(gF)[0], _ptr(st)[0], kind))
        return gF, st

    def fd_tangent(self, h=1e-4, like=None):
        """The paper's finite-difference tangent at the last solve's state:
        spatial C [R,6,6], A = dPi/dE [R,6,6] (Mandel) and status [R]."""
        ref = like if like is not None else np.empty(0)
        Cm = self._outs(ref, (6, 6), np.float64)
        Am = self._outs(ref, (6, 6), np.float64)
        st = self._outs(ref, (), np.int32)
        _check(lib().rve_batch_fd_tangent(self._h, float(h), _ptr(Cm)[0], _ptr(Am)[0], _ptr(st)[0], _ptr(Cm)[1]))
        return Cm, Am, st

    def orientation(self, e=(1.0, 0.0, 0.0), like=None):
        """Orientation tensor [R,3,3] and degree of alignment P2 [R] along e at the last solve's state."""
        ref = like if like is not None else np.empty(0)
        om = self._outs(ref, (3, 3), np.float64)
        p2 = self._outs(ref, (), np.float64)
        ev = np.ascontiguousarray(np.asarray(e, dtype=np.float64).reshape(3))
        _check(lib().rve_batch_orientation(self._h, ev.ctypes.data, _ptr(om)[0], _ptr(p2)[0], _ptr(om)[1]))
        return om, p2

    def export_state(self, like=None):
        """(F [R,3,3], h [nodes,3] in the caller's node order, status [R]) of the last solve or import."""
        ref = like if like is not None else np.empty(0)
        Fo = self._outs(ref, (3, 3), np.float64)
        st = self._outs(ref, (), np.int32)
        nn = int(self.node_off[-1])
        if hasattr(ref, "data_ptr"):
            import torch
            h = torch.empty((nn, 3), dtype=torch.float64, device=ref.device)
        else:
            h = np.empty((nn, 3), np.float64)
        _check(lib().rve_batch_export_state(self._h, _ptr(Fo)[0], _ptr(h)[0], _ptr(st)[0], _ptr(Fo)[1]))
        return Fo, h, st

    def import_state(self, F, h, status):
        """Replace the batch's state (F, fluctuation h per caller node, status).
        Returns the stress [R,3,3] re-evaluated at the imported state."""
        nn = int(self.node_off[-1])
        if hasattr(F, "data_ptr"):
            import torch
            F, h, status = F.contiguous(), h.contiguous(), status.contiguous()
            if not (F.device == h.device == status.device):
                raise ValueError("F, h and status must live on one device")
            if F.dtype != torch.float64 or h.dtype != torch.float64 or status.dtype != torch.int32:
                raise ValueError("F and h must be float64, status int32")
            if F.numel() != 9 * self.n_rve or h.numel() != 3 * nn or status.numel() != self.n_rve:
                raise ValueError("F, h or status has the wrong size")
        else:
            F = np.ascontiguousarray(F, np.float64).reshape(self.n_rve, 3, 3)
            h = np.ascontiguousarray(h, np.float64).reshape(nn, 3)
            status = np.ascontiguousarray(status, np.int32).reshape(self.n_rve)
        sig = self._outs(F, (3, 3), np.float64)
        fp, kind = _ptr(F)
        _check(lib().rve_batch_import_state(self._h, fp, _ptr(h)[0], _ptr(status)[0], _ptr(sig)[0], kind))
        return sig

    def damping_stats(self):
        """(final damping coefficient [R], final relative energy balance [R]) of
        the last solve with a damping alternative or the energy check."""
        cf = np.empty(self.n_rve)
        en = np.empty(self.n_rve)
        _check(lib().rve_batch_damping_stats(self._h, cf.ctypes.data, en.ctypes.data, PTR_HOST))
        return cf, en

    def workspace_size(self):
        """Bytes of device memory that cover every on-demand work area of the batch."""
        n = C.c_size_t()
        _check(lib().rve_batch_workspace_size(self._h, C.byref(n)))
        return n.value

    def bind_workspace(self, buf):
        """Carve the batch's work areas from `buf` (a device tensor the caller
        owns; kept referenced here), or return to library-owned areas (None)."""
        if buf is None:
            _check(lib().rve_batch_bind_workspace(self._h, None, 0))
            self._ws = None
            return
        nbytes = buf.numel() * buf.element_size()
        _check(lib().rve_batch_bind_workspace(self._h, buf.data_ptr(), nbytes))
        self._ws = buf

    def tangent_iters(self):
        """Inner CG iterations of the last tangent/vjp call, summed per RVE (host int64 [R])."""
        it = np.zeros(self.n_rve, np.int64)
        _check(lib().rve_batch_tangent_iters(self._h, _ptr(it)[0], 0))
        return it

    def autotune(self, F, n_iter=200):
        """Time every eligible kernel variant per size tier and keep the fastest."""
        if hasattr(F, "data_ptr"):
            F = F.contiguous()
        else:
            F = np.ascontiguousarray(F, np.float64).reshape(self.n_rve, 3, 3)
        p, kind = _ptr(F)
        _check(lib().rve_batch_autotune(self._h, p, kind, int(n_iter)))

    def describe(self):
        buf = C.create_string_buffer(1024)
        _check(lib().rve_batch_describe(self._h, buf, 1024))
        return buf.value.decode()

    def groups(self):
        """(group index per RVE, code per group (resident variant >= 0, -1 streamed, -1 - k team of k,
        -100 incidence, -101 incidence in global mode), ms per group of the last profiled solve)."""
        g = np.empty(self.n_rve, np.int32)
        var = np.empty(16, np.int32)
        ms = np.empty(16)
        n = C.c_int32()
        _check(lib().rve_batch_groups(self._h, g.ctypes.data, var.ctypes.data, ms.ctypes.data, 16, C.byref(n)))
        return g, var[:n.value], ms[:n.value]

    def profile(self, enable=True):
        _check(lib().rve_batch_profile(self._h, 1 if enable else 0))

    def kernel_ms(self):
        """(relaxation ms, stress ms) of the last profiled solve (HIP events)."""
        a, b = C.c_double(), C.c_double()
        _check(lib().rve_batch_kernel_ms(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def positions(self, r):
        nn = int(self.node_off[r + 1] - self.node_off[r])
        x = np.empty((nn, 3))
        _check(lib().rve_batch_positions(self._h, int(r), x.ctypes.data))
        return x
