"""Seeded synthetic inputs: Voronoi fiber networks and deformation gradients.

This module only produces geometry, topology and loading.  It holds none of
the relaxation, force, stress or tangent arithmetic, so both the CPU oracle
(under ``oracle/``) and the HIP path consume the same inputs without sharing
any of the method's code.

Network recipe (the paper's RVEs are Voronoi fiber networks clipped to a
cube; the RVE libraries themselves are not available, so these stand in):

1. ``n_seeds`` points uniform in the unit cube, plus 26 far padding seeds on
   the grid {-50, 0.5, 51}^3 (centre excluded) so that every Voronoi edge
   near the cube is finite without changing the diagram inside it.
2. Every finite ridge-polygon edge of the diagram, deduplicated.
3. Each edge is clipped to [0, 1]^3 (Liang-Barsky).  A clip point becomes a
   boundary node (degree 1, lies on a cube face); Voronoi vertices inside the
   cube become free nodes.  Empty segments are dropped.
4. Short-fiber merge: fibers shorter than ``merge_frac`` x mean length are
   contracted, shortest first.  A contraction that touches a boundary node
   keeps the boundary node; two free nodes merge at the midpoint; a short
   fiber between two boundary nodes is dropped.  Parallel fibers and
   self-loops created by a merge are removed.
5. Connected components with no boundary node are dropped, and so are
   isolated nodes.

Random streams: ``numpy.random.default_rng([config_id, rve_index, stream])``
with stream 0 for seed points, 1 for F and 2 for the seed count.
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Network", "Batch", "voronoi_network", "lattice_network", "chain_network",
    "single_fiber_network", "pack", "F_config1", "F_sym_perturbed",
    "F_uniaxial", "seed_count", "hex_mesh_F", "make_config_batch",
]

_PAD = np.array([[a, b, c] for a in (-50.0, 0.5, 51.0) for b in (-50.0, 0.5, 51.0)
                 for c in (-50.0, 0.5, 51.0) if not (a == 0.5 and b == 0.5 and c == 0.5)])


@dataclass
class Network:
    """One RVE: node coordinates X (reference configuration, unit cube),
    boundary flags and fiber connectivity (pairs of local node ids)."""
    X: np.ndarray        # (n_nodes, 3) float64
    is_bnd: np.ndarray   # (n_nodes,) uint8, 1 = node on the cube boundary
    fib: np.ndarray      # (n_fib, 2) int32

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_fib(self) -> int:
        return int(self.fib.shape[0])

    @property
    def n_free(self) -> int:
        return int(self.n_nodes - int(self.is_bnd.sum()))


@dataclass
class Batch:
    """Ragged batch in the packed (row-offset + values) layout."""
    node_off: np.ndarray  # (R+1,) int64
    fib_off: np.ndarray   # (R+1,) int64
    X: np.ndarray         # (sum nodes, 3) float64
    is_bnd: np.ndarray    # (sum nodes,) uint8
    fib: np.ndarray       # (sum fibers, 2) int32, ids local to each RVE

    @property
    def n_rve(self) -> int:
        return int(self.node_off.shape[0] - 1)

    def network(self, r: int) -> Network:
        a, b = int(self.node_off[r]), int(self.node_off[r + 1])
        c, d = int(self.fib_off[r]), int(self.fib_off[r + 1])
        return Network(self.X[a:b], self.is_bnd[a:b], self.fib[c:d])

    def subset(self, idx) -> "Batch":
        return pack([self.network(int(r)) for r in idx])


def pack(nets) -> Batch:
    nets = list(nets)
    nn = np.array([n.n_nodes for n in nets], dtype=np.int64)
    nf = np.array([n.n_fib for n in nets], dtype=np.int64)
    node_off = np.concatenate([[0], np.cumsum(nn)]).astype(np.int64)
    fib_off = np.concatenate([[0], np.cumsum(nf)]).astype(np.int64)
    if nets:
        X = np.ascontiguousarray(np.concatenate([n.X for n in nets]), dtype=np.float64)
        ib = np.ascontiguousarray(np.concatenate([n.is_bnd for n in nets]), dtype=np.uint8)
        fb = np.ascontiguousarray(np.concatenate([n.fib for n in nets]), dtype=np.int32)
    else:
        X = np.zeros((0, 3)); ib = np.zeros(0, np.uint8); fb = np.zeros((0, 2), np.int32)
    return Batch(node_off, fib_off, X, ib, fb)


# --------------------------------------------------------------------------
# Voronoi networks
# --------------------------------------------------------------------------
def _ridge_edges(vor) -> np.ndarray:
    """Unique finite edges (i < j) of all ridge polygons."""
    rv = vor.ridge_vertices
    lens = np.fromiter((len(r) for r in rv), dtype=np.int64, count=len(rv))
    flat = np.fromiter((v for r in rv for v in r), dtype=np.int64, count=int(lens.sum()))
    start = np.concatenate([[0], np.cumsum(lens)[:-1]])
    nxt = np.arange(flat.size) + 1
    last = start + lens - 1
    nxt[last] = start                          # close each polygon
    a, b = flat, flat[nxt]
    ok = (a >= 0) & (b >= 0)
    a, b = a[ok], b[ok]
    e = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)
    e = e[e[:, 0] != e[:, 1]]
    return np.unique(e, axis=0)


def _clip_unit_cube(P0: np.ndarray, P1: np.ndarray):
    """Liang-Barsky clip of segments P0->P1 to [0,1]^3.
    Returns (t0, t1, keep) with the kept part being P0 + t*(P1-P0), t in [t0,t1]."""
    d = P1 - P0
    t0 = np.zeros(len(P0)); t1 = np.ones(len(P0))
    keep = np.ones(len(P0), dtype=bool)
    for k in range(3):
        for p, q in ((-d[:, k], P0[:, k]), (d[:, k], 1.0 - P0[:, k])):
            par = p == 0.0
            keep &= ~(par & (q < 0.0))
            with np.errstate(divide="ignore", invalid="ignore"):
                r = np.where(par, 0.0, q / np.where(par, 1.0, p))
            neg = (p < 0.0)
            pos = (p > 0.0)
            t0 = np.where(neg, np.maximum(t0, r), t0)
            t1 = np.where(pos, np.minimum(t1, r), t1)
    keep &= t0 < t1
    return t0, t1, keep


def _components_with_boundary(n_nodes, fib, is_bnd):
    """Mask of nodes in a connected component that touches the boundary."""
    parent = np.arange(n_nodes)

    def find(x):
        root = x
        while parent[root] != root:
            root = parent[root]
        while parent[x] != root:
            parent[x], x = root, parent[x]
        return root

    for a, b in fib:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    roots = np.array([find(i) for i in range(n_nodes)])
    good_roots = np.unique(roots[is_bnd.astype(bool)])
    return np.isin(roots, good_roots)


def _merge_short(X, is_bnd, fib, frac):
    """Contract fibers shorter than frac * mean length, shortest first."""
    if frac <= 0.0 or len(fib) == 0:
        return X, is_bnd, fib
    X = X.copy()
    L = np.linalg.norm(X[fib[:, 1]] - X[fib[:, 0]], axis=1)
    thr = frac * L.mean()
    alias = np.arange(len(X))

    def rep(i):
        while alias[i] != i:
            alias[i] = alias[alias[i]]
            i = alias[i]
        return i

    drop = np.zeros(len(fib), dtype=bool)
    changed = True
    while changed:
        changed = False
        a = np.array([rep(i) for i in fib[:, 0]])
        b = np.array([rep(i) for i in fib[:, 1]])
        L = np.linalg.norm(X[b] - X[a], axis=1)
        live = (~drop) & (a != b)
        cand = np.where(live & (L < thr))[0]
        if cand.size == 0:
            break
        order = cand[np.argsort(L[cand], kind="stable")]
        touched = set()
        for f in order:
            ia, ib = rep(int(fib[f, 0])), rep(int(fib[f, 1]))
            if ia == ib or ia in touched or ib in touched:
                continue
            ba, bb = bool(is_bnd[ia]), bool(is_bnd[ib])
            if ba and bb:
                drop[f] = True
            elif ba:
                alias[ib] = ia
            elif bb:
                alias[ia] = ib
            else:
                X[ia] = 0.5 * (X[ia] + X[ib])
                alias[ib] = ia
            touched.add(ia); touched.add(ib)
            changed = True
    a = np.array([rep(i) for i in fib[:, 0]], dtype=np.int64)
    b = np.array([rep(i) for i in fib[:, 1]], dtype=np.int64)
    ok = (~drop) & (a != b)
    e = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)[ok]
    e = np.unique(e, axis=0)
    return X, is_bnd, e


def voronoi_network(n_seeds: int, rng_key, merge_frac: float = 0.05) -> Network:
    """Voronoi fiber network from ``n_seeds`` uniform seeds in the unit cube."""
    from scipy.spatial import Voronoi
    rng = np.random.default_rng(rng_key)
    pts = rng.random((int(n_seeds), 3))
    vor = Voronoi(np.vstack([pts, _PAD]))
    V = vor.vertices
    E = _ridge_edges(vor)
    P0, P1 = V[E[:, 0]], V[E[:, 1]]
    t0, t1, keep = _clip_unit_cube(P0, P1)
    E, P0, P1, t0, t1 = E[keep], P0[keep], P1[keep], t0[keep], t1[keep]
    d = P1 - P0
    seg_len = np.linalg.norm(d, axis=1) * (t1 - t0)
    ok = seg_len > 1e-12
    E, P0, d, t0, t1 = E[ok], P0[ok], d[ok], t0[ok], t1[ok]
    # Voronoi vertices strictly used inside the cube become free nodes.
    in0 = t0 <= 0.0
    in1 = t1 >= 1.0
    used = np.unique(np.concatenate([E[in0, 0], E[in1, 1]]))
    vid = -np.ones(len(V), dtype=np.int64)
    vid[used] = np.arange(len(used))
    Xf = V[used]
    nb0 = int((~in0).sum()); nb1 = int((~in1).sum())
    Xb0 = P0[~in0] + t0[~in0, None] * d[~in0]
    Xb1 = P0[~in1] + t1[~in1, None] * d[~in1]
    Xb = np.clip(np.vstack([Xb0, Xb1]), 0.0, 1.0)
    nf = len(used)
    ia = np.empty(len(E), dtype=np.int64)
    ib = np.empty(len(E), dtype=np.int64)
    ia[in0] = vid[E[in0, 0]]
    ia[~in0] = nf + np.arange(nb0)
    ib[in1] = vid[E[in1, 1]]
    ib[~in1] = nf + nb0 + np.arange(nb1)
    X = np.vstack([Xf, Xb])
    is_bnd = np.concatenate([np.zeros(nf, np.uint8), np.ones(nb0 + nb1, np.uint8)])
    fib = np.stack([ia, ib], axis=1)
    X, is_bnd, fib = _merge_short(X, is_bnd, fib, merge_frac)
    return _finalize(X, is_bnd, fib)


def _finalize(X, is_bnd, fib) -> Network:
    """Drop floating components and unused nodes, relabel densely."""
    n = len(X)
    keep_node = _components_with_boundary(n, fib, is_bnd)
    deg = np.bincount(fib.ravel(), minlength=n)
    keep_node &= deg > 0
    fib = fib[keep_node[fib[:, 0]] & keep_node[fib[:, 1]]]
    new = -np.ones(n, dtype=np.int64)
    new[keep_node] = np.arange(int(keep_node.sum()))
    return Network(np.ascontiguousarray(X[keep_node], dtype=np.float64),
                   np.ascontiguousarray(is_bnd[keep_node], dtype=np.uint8),
                   np.ascontiguousarray(new[fib], dtype=np.int32))


# --------------------------------------------------------------------------
# Small structured networks (closed-form test cases)
# --------------------------------------------------------------------------
def single_fiber_network(Xa, Xb) -> Network:
    X = np.array([Xa, Xb], dtype=np.float64)
    return Network(X, np.ones(2, np.uint8), np.array([[0, 1]], np.int32))


def chain_network(points, bnd_ends=True) -> Network:
    """Chain of fibers through ``points``; the two end points are boundary nodes."""
    X = np.asarray(points, dtype=np.float64)
    n = len(X)
    ib = np.zeros(n, np.uint8)
    if bnd_ends:
        ib[0] = ib[-1] = 1
    fib = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).astype(np.int32)
    return Network(X, ib, fib)


def lattice_network(n: int) -> Network:
    """Regular n^3-cell cubic lattice of axis-aligned fibers spanning [0,1]^3.
    Nodes on the cube faces are boundary nodes."""
    g = np.arange(n + 1) / n
    I, J, K = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    idx = (I * (n + 1) + J) * (n + 1) + K
    X = np.stack([g[I.ravel()], g[J.ravel()], g[K.ravel()]], axis=1)
    on_face = lambda a: (a == 0) | (a == n)
    ib = (on_face(I) | on_face(J) | on_face(K)).ravel().astype(np.uint8)
    fibs = []
    fibs.append(np.stack([idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()], 1))
    fibs.append(np.stack([idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()], 1))
    fibs.append(np.stack([idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()], 1))
    return Network(X, ib, np.concatenate(fibs).astype(np.int32))


# --------------------------------------------------------------------------
# Deformation gradients
# --------------------------------------------------------------------------
def F_config1() -> np.ndarray:
    return np.diag([1.1, 1.0, 1.0]).reshape(1, 3, 3)


def F_sym_perturbed(config_id: int, n: int, amp: float) -> np.ndarray:
    """F = I + amp*G, G symmetric; its 6 upper entries are N(0,1) clipped to [-1,1]."""
    out = np.empty((n, 3, 3))
    iu = np.triu_indices(3)
    for r in range(n):
        g = np.clip(np.random.default_rng([config_id, r, 1]).standard_normal(6), -1.0, 1.0)
        G = np.zeros((3, 3)); G[iu] = g; G = G + np.triu(G, 1).T
        out[r] = np.eye(3) + amp * G
    return out


def F_uniaxial(config_id: int, n: int, lo: float = 1.0, hi: float = 1.3) -> np.ndarray:
    """F = diag(lam, lam^-1/2, lam^-1/2), lam ~ U[lo, hi]."""
    out = np.zeros((n, 3, 3))
    for r in range(n):
        lam = np.random.default_rng([config_id, r, 1]).uniform(lo, hi)
        out[r] = np.diag([lam, lam ** -0.5, lam ** -0.5])
    return out


def seed_count(config_id: int, r: int) -> int:
    rng = np.random.default_rng([config_id, r, 2])
    if config_id == 2:
        return int(rng.integers(200, 401))
    if config_id == 5:
        return int(np.clip(round(rng.lognormal(np.log(400.0), 0.8)), 100, 3000))
    return {1: 100, 3: 2000, 4: 300}[config_id]


def hex_mesh_u(X, lam=1.1, amp=0.02, seed=5) -> np.ndarray:
    """Displacement field of the hex-mesh workload at points X (n, 3):
    u = (F_M - I) X + w(X), F_M = diag(lam, lam^-1/2, lam^-1/2),
    w = amp * sum of 8 sinusoids with random direction, phase and wavelength
    in [4, 16]."""
    rng = np.random.default_rng([seed, 0, 3])
    FM = np.diag([lam, lam ** -0.5, lam ** -0.5])
    dirs = rng.standard_normal((8, 3)); dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pol = rng.standard_normal((8, 3)); pol /= np.linalg.norm(pol, axis=1, keepdims=True)
    wl = rng.uniform(4.0, 16.0, 8); ph = rng.uniform(0, 2 * np.pi, 8)
    kvec = dirs * (2 * np.pi / wl)[:, None]
    X = np.asarray(X, dtype=np.float64)
    return X @ (FM - np.eye(3)).T + amp * np.sin(X @ kvec.T + ph) @ pol


def hex_mesh_F(nx=16, ny=16, nz=4, lam=1.1, amp=0.02, seed=5) -> np.ndarray:
    """Deformation gradients at the 2x2x2 Gauss points of an nx*ny*nz mesh of
    unit trilinear hexes under the displacement field of hex_mesh_u.
    Returns (nx*ny*nz*8, 3, 3)."""

    def u_of(X):
        return hex_mesh_u(X, lam, amp, seed)

    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=np.float64)
    out = []
    for ex in range(nx):
        for ey in range(ny):
            for ez in range(nz):
                org = np.array([ex, ey, ez], dtype=np.float64)
                uI = u_of(org + corners)                     # (8,3)
                for xi in gp:
                    for eta in gp:
                        for zeta in gp:
                            p = np.array([xi, eta, zeta])
                            # trilinear shape-function gradients on a unit hex
                            w = np.where(corners == 1, p, 1 - p)   # (8,3)
                            s = np.where(corners == 1, 1.0, -1.0)
                            dN = np.stack([s[:, 0] * w[:, 1] * w[:, 2],
                                           w[:, 0] * s[:, 1] * w[:, 2],
                                           w[:, 0] * w[:, 1] * s[:, 2]], axis=1)
                            out.append(np.eye(3) + uI.T @ dN)
    return np.array(out)


# --------------------------------------------------------------------------
# Whole configurations
# --------------------------------------------------------------------------
def _gen_one(args):
    cfg, r = args
    return voronoi_network(seed_count(cfg, r), [cfg, r, 0])


def make_config_batch(config_id: int, n_rve: int | None = None, idx=None, workers: int | None = None):
    """Networks and F for one of the five workloads.

    1: one 100-seed RVE, F = diag(1.1, 1, 1).
    2: 4096 RVEs, seeds ~ U{200..400}, F = I + 0.1 G.
    3: 512 RVEs, 2000 seeds, F = diag(lam, lam^-1/2, lam^-1/2), lam ~ U[1, 1.3].
    4: 1024 RVEs, 300 seeds, F = I + 0.05 G.
    5: 8192 RVEs, seeds lognormal(median 400, sigma 0.8) clipped to [100, 3000],
       F from a 16x16x4 hex mesh under uniaxial extension.
    ``idx`` selects a subset of RVE indices (same networks and F as in the full set).
    """
    full = {1: 1, 2: 4096, 3: 512, 4: 1024, 5: 8192}[config_id]
    if idx is None:
        idx = np.arange(full if n_rve is None else n_rve)
    idx = np.asarray(idx, dtype=np.int64)
    jobs = [(config_id, int(r)) for r in idx]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers > 1 and len(jobs) > 8:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            nets = pool.map(_gen_one, jobs, chunksize=max(1, len(jobs) // (4 * workers)))
    else:
        nets = [_gen_one(j) for j in jobs]
    if config_id == 1:
        F = F_config1()
    elif config_id == 2:
        F = F_sym_perturbed(2, int(idx.max()) + 1, 0.1)[idx]
    elif config_id == 3:
        F = F_uniaxial(3, int(idx.max()) + 1)[idx]
    elif config_id == 4:
        F = F_sym_perturbed(4, int(idx.max()) + 1, 0.05)[idx]
    else:
        F = hex_mesh_F()[idx]
    return pack(nets), np.ascontiguousarray(F)
