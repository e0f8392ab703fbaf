"""Incremental FE^2 driver on top of the batched RVE library (Algorithm 1).

The macroscale is a small total-Lagrangian finite-element problem on a box
of unit trilinear hexahedra with 2x2x2 Gauss points; every Gauss point owns
one RVE of the batch (RVE index = 8 * element + Gauss point, elements with
z fastest, then y, then x; Gauss points with zeta fastest).  Each Newton
iteration of a load step sends the Gauss-point deformation gradients to the
microscale in one batched call, receives the Cauchy stresses and the tangents
d sigma / dF, turns them into the first Piola-Kirchhoff stress
P = J sigma F^-T and its derivative dP/dF, assembles the macroscale residual
and stiffness, and solves for the displacement correction (Algorithm 1: the
macro Newton loop around the batched constitutive call; Section 2: the
macroscale deformation gradient drives each RVE).  The updated-Lagrangian
form of the paper (Cauchy stress with the spatial tangent) is the same
linearisation written on the current configuration.

Warm starts: each micro solve starts from the fluctuation left by the
previous one (the last Newton iterate), which is what the paper's
dynamic-relaxation increment does (free displacements start from the last
state).  Load steps that fail (non-finite micro states or no Newton
convergence) are retried with half the increment after restoring the
micro state exported at the last accepted step.

Loading: extension along x with stretch lam, u_x = 0 on x = 0 and
u_x = (lam - 1) L_x on x = L_x, either with symmetry planes u_y = 0 on
y = 0 and u_z = 0 on z = 0 and traction-free lateral faces ("uniaxial",
the paper's tissue test) or with both x faces gripped (u_y = u_z = 0 there,
"clamped"), or every boundary node on the affine map of
F_M = diag(lam, lam_t, lam_t), lam_t = 1 + (lam - 1)/2 ("affine": the
whole box in tension, heterogeneous inside).  A sub-isostatic fiber network
carries almost no load, and has a singular stiffness, until its fibers have
rotated towards the load (the toe region): under uniaxial loading the
first steps see tiny reactions, Gauss points in lateral compression relax
slowly and their tangents do not exist; the affine setup keeps every
network in tension.

Host code (numpy/scipy): the macro problem has a few thousand unknowns; all
microscale work runs in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

GP = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
CORNERS = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=np.float64)


class HexMesh:
    """nx * ny * nz unit cubes; node (ix, iy, iz) has id (ix (ny+1) + iy) (nz+1) + iz."""

    def __init__(self, nx: int, ny: int, nz: int):
        self.nx, self.ny, self.nz = nx, ny, nz
        ix, iy, iz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
        self.X = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
        self.n_nodes = len(self.X)
        nid = lambda a, b, c: (a * (ny + 1) + b) * (nz + 1) + c
        el = []
        for ex in range(nx):
            for ey in range(ny):
                for ez in range(nz):
                    el.append([nid(ex + int(c[0]), ey + int(c[1]), ez + int(c[2])) for c in CORNERS])
        self.elems = np.array(el, dtype=np.int64)          # (nel, 8)
        self.n_elems = len(self.elems)
        # trilinear shape-function gradients at the Gauss points of a unit cube
        dN = []
        for xi in GP:
            for eta in GP:
                for zeta in GP:
                    p = np.array([xi, eta, zeta])
                    w = np.where(CORNERS == 1, p, 1 - p)
                    s = np.where(CORNERS == 1, 1.0, -1.0)
                    dN.append(np.stack([s[:, 0] * w[:, 1] * w[:, 2], w[:, 0] * s[:, 1] * w[:, 2],
                                        w[:, 0] * w[:, 1] * s[:, 2]], axis=1))
        self.dN = np.array(dN)                             # (8 gp, 8 nodes, 3)
        self.w = 1.0 / 8.0                                 # Gauss weight x unit-cube volume
        self.n_gp = 8 * self.n_elems
        self.L = np.array([nx, ny, nz], dtype=np.float64)
        # element-to-global DOF map and the sparsity pattern of K
        edof = (3 * self.elems[:, :, None] + np.arange(3)[None, None, :]).reshape(self.n_elems, 24)
        self.edof = edof
        self._rows = np.repeat(edof, 24, axis=1).ravel()
        self._cols = np.tile(edof, (1, 24)).ravel()

    def deformation_gradients(self, u: np.ndarray) -> np.ndarray:
        """F = I + grad u at every Gauss point, (n_gp, 3, 3)."""
        ue = u[self.elems]                                  # (nel, 8, 3)
        G = np.einsum("eai,gaj->egij", ue, self.dN)
        return (np.eye(3) + G).reshape(self.n_gp, 3, 3)

    def internal_force(self, P: np.ndarray) -> np.ndarray:
        """f_a,i = sum_gp P_iJ dN_a,J w, (n_nodes, 3)."""
        Pe = P.reshape(self.n_elems, 8, 3, 3)
        fe = np.einsum("egij,gaj->eai", Pe, self.dN) * self.w
        f = np.zeros((self.n_nodes, 3))
        np.add.at(f, self.elems, fe)
        return f

    def stiffness(self, A: np.ndarray) -> sp.csr_matrix:
        """K_(a,i),(b,k) = sum_gp dN_a,J A_iJkL dN_b,L w, A as (n_gp, 9, 9) with row 3i+J, column 3k+L."""
        A4 = A.reshape(self.n_elems, 8, 3, 3, 3, 3)
        Ke = np.einsum("gaj,egijkl,gbl->eaibk", self.dN, A4, self.dN, optimize=True) * self.w
        Ke = Ke.reshape(self.n_elems, 24, 24)
        n = 3 * self.n_nodes
        return sp.coo_matrix((Ke.ravel(), (self._rows, self._cols)), shape=(n, n)).tocsr()

    def boundary_dofs(self, lam: float, kind: str = "uniaxial"):
        """Fixed DOFs and their values for extension along x ("uniaxial":
        symmetry planes y = 0 and z = 0; "clamped": both x faces gripped)."""
        X = self.X
        if kind == "affine":
            on = np.zeros(len(X), bool)
            for k in range(3):
                on |= (X[:, k] == 0) | (X[:, k] == self.L[k])
            ids = np.nonzero(on)[0]
            lam_t = 1.0 + 0.5 * (lam - 1.0)
            U = X[ids] * (np.array([lam, lam_t, lam_t]) - 1.0)
            dofs = (3 * ids[:, None] + np.arange(3)[None, :]).ravel()
            return dofs, U.ravel()
        x0, x1 = X[:, 0] == 0, X[:, 0] == self.L[0]
        spec = [(x0, 0, 0.0), (x1, 0, (lam - 1.0) * self.L[0])]
        if kind == "uniaxial":
            spec += [(X[:, 1] == 0, 1, 0.0), (X[:, 2] == 0, 2, 0.0)]
        elif kind == "clamped":
            spec += [(x0, 1, 0.0), (x0, 2, 0.0), (x1, 1, 0.0), (x1, 2, 0.0)]
        else:
            raise ValueError(f"unknown boundary condition {kind!r}")
        dofs, vals = [], []
        for face, comp, val in spec:
            ids = np.nonzero(face)[0]
            dofs.append(3 * ids + comp)
            vals.append(np.full(len(ids), val))
        dofs = np.concatenate(dofs)
        vals = np.concatenate(vals)
        order = np.argsort(dofs, kind="stable")
        dofs, vals = dofs[order], vals[order]
        keep = np.ones(len(dofs), bool)
        keep[1:] = dofs[1:] != dofs[:-1]
        return dofs[keep], vals[keep]


def first_pk(F: np.ndarray, sigma: np.ndarray, dsdF: np.ndarray | None = None):
    """P = J sigma F^-T and, with d sigma / dF (rows 3i+j, columns 3k+l),
    dP_iJ/dF_kL = P_iJ Finv_Lk + J dsigma_ij/dF_kL Finv_Jj - J sigma_ij Finv_Jk Finv_Lj
    as (n, 9, 9) with row 3i+J, column 3k+L."""
    Finv = np.linalg.inv(F)
    J = np.linalg.det(F)
    P = J[:, None, None] * sigma @ np.transpose(Finv, (0, 2, 1))
    if dsdF is None:
        return P, None
    D = dsdF.reshape(-1, 3, 3, 3, 3)
    A = (np.einsum("niJ,nLk->niJkL", P, Finv)
         + J[:, None, None, None, None] * np.einsum("nijkL,nJj->niJkL", D, Finv)
         - J[:, None, None, None, None] * np.einsum("nij,nJk,nLj->niJkL", sigma, Finv, Finv))
    return P, A.reshape(-1, 9, 9)


class GpuMicro:
    """Microscale of the driver: one batch of RVEs, one per Gauss point.

    refine_tangent: with a mixed-precision batch, take the tangent at an FP64
    state instead: the mixed state is exported, imported into an FP64 twin
    batch of the same networks, relaxed further from there (warm start,
    tol_rel refine_tol) and linearised in FP64.  Floppy RVEs that stop at the
    mixed tolerance can sit on the unstable side of a soft mode, where K_ff is
    indefinite and no tangent exists; the FP64 state is usually stable."""

    def __init__(self, nets, warm: bool = True, refine_tangent: bool = False, refine_tol: float = 1e-8, **opts):
        from . import binding as rb
        self.rb = rb
        self.opts = dict(opts)
        self.opts.pop("init", None)   # the driver chooses the start (affine, then warm)
        self.warm = warm
        self.batch = rb.Batch(nets, **self.opts)
        self.has_state = False
        self.warm_now = False
        self.twin = None
        self.last_F = None
        if refine_tangent:
            o = dict(self.opts)
            o.update(precision=rb.FP64, tol_rel=refine_tol, init=rb.INIT_WARM)
            self.twin = rb.Batch(nets, **o)

    def solve(self, F):
        use_warm = self.warm and self.has_state
        if use_warm != self.warm_now:
            o = dict(self.opts)
            o["init"] = self.rb.INIT_WARM if use_warm else self.rb.INIT_AFFINE
            self.batch.set_opts(**o)
            self.warm_now = use_warm
        sig, st, stats = self.batch.solve(F, stats=True)
        self.has_state = True
        self.last_F = F
        return sig, st, stats["iters"]

    def tangent(self):
        if self.twin is None:
            return self.batch.tangent()
        Fe, h, st = self.batch.export_state()
        self.twin.import_state(Fe, h, st)
        self.twin.solve(self.last_F)
        return self.twin.tangent()

    def checkpoint(self):
        return self.batch.export_state() if self.has_state else None

    def restore(self, state):
        if state is None:
            self.has_state = False
        else:
            self.batch.import_state(*state)
            self.has_state = True

    def close(self):
        self.batch.close()
        if self.twin is not None:
            self.twin.close()


@dataclass
class NewtonRecord:
    lam: float
    residual: list = field(default_factory=list)       # |r_free| / |reaction| per iteration
    micro_iters: list = field(default_factory=list)    # summed relaxation iterations per micro solve
    micro_ms: list = field(default_factory=list)
    tangent_ms: list = field(default_factory=list)
    micro_status: list = field(default_factory=list)   # counts of statuses 0..3 per micro solve
    tangent_fallback: list = field(default_factory=list)   # Gauss points whose tangent was replaced
    converged: bool = False
    reason: str = ""                                   # why the step failed


class FE2:
    """Load-stepping Newton solver of the macroscale problem."""

    def __init__(self, mesh: HexMesh, micro, tol: float = 1e-5, max_newton: int = 10, bc: str = "uniaxial",
                 atol: float = 0.0, verbose: bool = False):
        self.mesh = mesh
        self.verbose = verbose
        self.micro = micro
        self.tol = tol
        self.atol = atol
        self.bc = bc
        self.max_newton = max_newton
        self.u = np.zeros((mesh.n_nodes, 3))
        self.lam = 1.0
        self.history: list[NewtonRecord] = []
        self.sigma = None
        self.F = None
        self.status = None
        self.A_last = None

    def _micro_stress(self, u, rec):
        F = self.mesh.deformation_gradients(u)
        t0 = time.perf_counter()
        sig, st, it = self.micro.solve(F)
        rec.micro_ms.append(1e3 * (time.perf_counter() - t0))
        rec.micro_iters.append(int(np.asarray(it).sum()))
        rec.micro_status.append(np.bincount(np.asarray(st), minlength=4)[:4].tolist())
        return F, np.asarray(sig), np.asarray(st)

    def step(self, lam_to: float) -> NewtonRecord:
        """One load step from the current state to stretch lam_to; the state
        moves only if the step converges."""
        m = self.mesh
        rec = NewtonRecord(lam=lam_to)
        dofs, vals = m.boundary_dofs(lam_to, self.bc)
        free = np.ones(3 * m.n_nodes, bool)
        free[dofs] = False
        u = self.u.copy()
        u[:, 0] += (lam_to - self.lam) * m.X[:, 0]        # predictor: affine stretch increment
        if self.bc == "affine":
            u[:, 1:] += 0.5 * (lam_to - self.lam) * m.X[:, 1:]
        u.reshape(-1)[dofs] = vals
        for it in range(self.max_newton + 1):
            F, sig, st = self._micro_stress(u, rec)
            # non-finite, bad F or a failed energy check: no usable stress
            # (n_max and the stagnation stop leave one)
            bad = np.isin(st, (2, 3, 7))
            if bad.any():
                rec.reason = f"{int(bad.sum())} micro states non-finite, with a bad F or an energy-check failure"
                return rec
            P, _ = first_pk(F, sig)
            r = m.internal_force(P).reshape(-1)
            react = np.linalg.norm(r[~free])
            rfree = np.linalg.norm(r[free])
            res = rfree / max(react, 1e-300)
            rec.residual.append(res)
            if self.verbose:
                print(f"stretch {lam_to:.5f} newton {it}: residual {res:.3e}, micro {rec.micro_ms[-1]:.0f} ms, "
                      f"{rec.micro_iters[-1]} relaxation iterations, statuses {rec.micro_status[-1]}", flush=True)
            if res <= self.tol or rfree <= self.atol:
                rec.converged = True
                self.u, self.lam, self.F, self.sigma, self.status = u, lam_to, F, sig, st
                return rec
            if it == self.max_newton:
                rec.reason = f"no convergence in {self.max_newton} Newton iterations"
                return rec
            t0 = time.perf_counter()
            ds, tst = self.micro.tangent()
            rec.tangent_ms.append(1e3 * (time.perf_counter() - t0))
            ds = np.asarray(ds)
            ok = (np.asarray(tst) == 0) & np.isfinite(ds).all(axis=(1, 2))
            if not ok.any():
                rec.reason = "no Gauss point has a tangent"
                return rec
            _, A = first_pk(F, sig, np.where(ok[:, None, None], ds, 0.0))
            # Gauss points without a tangent (no converged state, or K_ff not
            # positive definite there) keep their last tangent, else take the
            # mean of the others: the residual stays exact, only the Newton
            # matrix is approximate
            if self.A_last is None:
                self.A_last = np.broadcast_to(A[ok].mean(axis=0), A.shape).copy()
            A[~ok] = self.A_last[~ok]
            self.A_last = A.copy()
            rec.tangent_fallback.append(int((~ok).sum()))
            K = m.stiffness(A)
            Kff = K[free][:, free]
            du = spla.spsolve(Kff.tocsc(), -r[free])
            u.reshape(-1)[free] += du
        return rec

    def run(self, lam_final: float, n_steps: int, max_cutbacks: int = 4):
        """Load from the current stretch to lam_final in n_steps equal steps,
        halving a failed step (after restoring the micro state of the last
        accepted step) up to max_cutbacks times in a row."""
        dl = (lam_final - self.lam) / n_steps
        cut = 0
        while self.lam < lam_final - 1e-14:
            ckpt = self.micro.checkpoint()
            target = min(self.lam + dl, lam_final)
            rec = self.step(target)
            self.history.append(rec)
            if rec.converged:
                cut = 0
                continue
            cut += 1
            if cut > max_cutbacks:
                raise RuntimeError(f"load step to stretch {target} failed after {max_cutbacks} cutbacks: {rec.reason}")
            self.micro.restore(ckpt)
            dl *= 0.5
        return self.history


def _config5_main(argv=None):
    """FE^2 run on the 16 x 16 x 4 hex mesh with the 8192 RVEs of the
    lognormal-size workload (one per Gauss point): prints a JSON summary."""
    import argparse
    import json

    from . import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--lam", type=float, default=1.1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--cold", action="store_true", help="start every micro solve from the affine state")
    ap.add_argument("--mesh", type=int, nargs=3, default=[16, 16, 4])
    ap.add_argument("--bc", default="affine", choices=["affine", "clamped", "uniaxial"])
    ap.add_argument("--damping", default="viscous", choices=["viscous", "kinetic"])
    args = ap.parse_args(argv)
    mesh = HexMesh(*args.mesh)
    t0 = time.perf_counter()
    batch, _ = synth.make_config_batch(5, idx=np.arange(mesh.n_gp))
    gen_s = time.perf_counter() - t0
    from . import binding as rb
    micro = GpuMicro(batch, warm=not args.cold, precision=rb.MIXED, law=rb.LAW_EXP, mass=rb.MASS_SCALED, alpha=0.5,
                     c=0.1, tol_abs=0.0, tol_rel=1e-5, n_max=100000, check_every=8, cg_tol=1e-6,
                     damping=rb.DAMP_KINETIC if args.damping == "kinetic" else rb.DAMP_VISCOUS)
    drv = FE2(mesh, micro, tol=args.tol, bc=args.bc, verbose=True)
    t0 = time.perf_counter()
    hist = drv.run(args.lam, args.steps)
    wall = time.perf_counter() - t0
    micro.close()
    out = {"mesh": args.mesh, "bc": args.bc, "damping": args.damping, "rves": mesh.n_gp, "lam": args.lam, "steps": args.steps, "warm": not args.cold,
           "generation_s": round(gen_s, 1), "wall_s": round(wall, 2),
           "micro_solve_s": round(sum(sum(h.micro_ms) for h in hist) / 1e3, 2),
           "tangent_s": round(sum(sum(h.tangent_ms) for h in hist) / 1e3, 2),
           "micro_iters_total": int(sum(sum(h.micro_iters) for h in hist)),
           "steps_detail": [{"lam": h.lam, "converged": h.converged, "residual": [float(f"{x:.3e}") for x in h.residual],
                             "micro_ms": [round(x) for x in h.micro_ms], "micro_iters": h.micro_iters,
                             "status": h.micro_status, "tangent_fallback": h.tangent_fallback} for h in hist],
           "mean_sigma_xx": float(drv.sigma[:, 0, 0].mean()) if drv.sigma is not None else None}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    _config5_main()
