"""Seeded synthetic graph workloads and right-hand sides.

This module only draws inputs: edge lists, weights and right-hand sides.  It
holds none of the solver's arithmetic, so the CPU oracle and the HIP path can
both be fed from it without sharing any method code.

Workloads (one per benchmark configuration):

* ``grid2d``   -- 2-D 5-point grid, ids ``i + nx*j``, unit weights.
* ``chung_lu`` -- power-law graph with expected degrees ``phi_i ~ (i+i0)^(-1/(beta-1))``,
  ``beta = 2.1``, mean degree 16, cutoff ``sqrt(16*n0)``; endpoints drawn i.i.d.
  proportional to ``phi``; self-loops dropped, duplicates merged, largest
  connected component kept; weights U[0.1, 1].
* ``grid3d_aniso`` -- 3-D 7-point grid with direction weights (x:1, y:1e-2,
  z:1e-4) times log-uniform[0.5, 2] noise per edge.
* ``graph_batch`` -- many uneven graphs (2-D grid / Erdos-Renyi mean degree 8 /
  random geometric), sizes log-uniform in [1e3, 2e5], weights U[0.1, 1].
* ``rgg``      -- random geometric graph in the unit square, radius
  ``sqrt(12/(pi n))``, weights ``exp(-d^2/r^2)``, largest component kept.
* ``grid2d_periodic`` -- the periodic 5-point Poisson grid of the geometric
  multigrid experiment, ids ``i + side*j``, unit weights.

Every draw comes from ``numpy.random.default_rng(seed)`` with a fixed seed per
workload and stream, so the same call gives byte-identical arrays everywhere.
Node ids after taking a largest component are relabelled by ascending original
id.  Right-hand sides are projected to zero sum (the system needs a zero-sum
b, Section 1 of the paper, eq. linsys).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEEDS = {"grid2d": 101, "chung_lu": 102, "grid3d_aniso": 103,
         "graph_batch": 104, "rgg": 105, "lgm": 106, "negative": 107}
# independent random streams per workload
_S_GRAPH, _S_WEIGHT, _S_RHS, _S_LABEL = 0, 1, 2, 4


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


@dataclasses.dataclass
class Graph:
    """Undirected weighted graph as a COO edge list (each edge once)."""
    name: str
    n: int
    eu: np.ndarray  # int32 [m]
    ev: np.ndarray  # int32 [m]
    w: np.ndarray   # float64 [m]
    coords: np.ndarray | None = None

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])


def _largest_component(n, eu, ev, w, coords=None):
    """Keep the largest connected component, relabelled by ascending id."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    a = sp.coo_matrix((np.ones(eu.shape[0]), (eu, ev)), shape=(n, n))
    ncomp, lab = connected_components(a, directed=False)
    if ncomp == 1:
        return n, eu, ev, w, coords
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = np.full(n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    em = keep[eu] & keep[ev]
    eu2 = newid[eu[em]].astype(np.int32)
    ev2 = newid[ev[em]].astype(np.int32)
    c2 = coords[keep] if coords is not None else None
    return int(keep.sum()), eu2, ev2, w[em], c2


def grid2d(nx: int = 64, ny: int | None = None, seed: int = SEEDS["grid2d"],
           weights: str = "unit") -> Graph:
    ny = nx if ny is None else ny
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)  # id = i + nx*j
    h_u, h_v = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    v_u, v_v = idx[:-1, :].ravel(), idx[1:, :].ravel()
    eu = np.concatenate([h_u, v_u]).astype(np.int32)
    ev = np.concatenate([h_v, v_v]).astype(np.int32)
    if weights == "unit":
        w = np.ones(eu.shape[0])
    else:
        w = _rng(seed, _S_WEIGHT).uniform(0.1, 1.0, eu.shape[0])
    return Graph(f"grid2d_{nx}x{ny}", nx * ny, eu, ev, w)


def grid2d_periodic(side: int = 1024) -> Graph:
    """Periodic side x side 5-point grid, unit weights: edges (i, j)-(i+1, j)
    and (i, j)-(i, j+1), indices mod side."""
    u = np.arange(side * side, dtype=np.int64)
    i, j = u % side, u // side
    eu = np.concatenate([u, u]).astype(np.int32)
    ev = np.concatenate([(i + 1) % side + side * j, i + side * ((j + 1) % side)]).astype(np.int32)
    return Graph(f"grid2d_periodic_{side}", side * side, eu, ev, np.ones(eu.shape[0]))


# Grid Laplacians with negative weights (the grid table of the paper's
# numerical results, cases a-d): off-diagonal stencil entries as printed
# (normalised), w = -entry, for the neighbour offsets (dx, dy) with dx >= 0
# listed once; Neumann boundaries, i.e. the graph Laplacian of these weights.
STENCILS = {
    "a": [(1, 0, 1.0), (0, 1, 1.0)],                                   # 5-point
    "b": [(1, 0, 16.0), (0, 1, 16.0), (2, 0, -1.0), (0, 2, -1.0)],     # fourth order
    "c": [(1, 0, 0.2525), (0, 1, 0.2525), (1, 1, -0.12375), (1, -1, 0.12375)],  # rotated, agnostic U_xy
    "d": [(1, 0, 0.5), (0, 1, 0.5), (1, 1, -0.2475)],                  # rotated, NE-SW U_xy
}


def grid_stencil(side: int = 1024, case: str = "b") -> Graph:
    """side x side grid, id = i + side*j, one edge per in-grid neighbour
    offset of the case's stencil with its (possibly negative) weight."""
    idx = np.arange(side * side, dtype=np.int64).reshape(side, side)  # [j, i]
    eu, ev, w = [], [], []
    for dx, dy, wt in STENCILS[case]:
        j0, j1 = max(0, -dy), side - max(0, dy)
        i1 = side - dx
        a = idx[j0:j1, 0:i1].ravel()
        b = idx[j0 + dy:j1 + dy, dx:i1 + dx].ravel()
        eu.append(a)
        ev.append(b)
        w.append(np.full(a.shape[0], wt))
    eu = np.concatenate(eu).astype(np.int32)
    ev = np.concatenate(ev).astype(np.int32)
    return Graph(f"grid_stencil_{case}_{side}", side * side, eu, ev, np.concatenate(w))


def grid3d_aniso(nside: int = 128, seed: int = SEEDS["grid3d_aniso"]) -> Graph:
    n = nside ** 3
    idx = np.arange(n, dtype=np.int64).reshape(nside, nside, nside)  # [z,y,x]
    parts_u, parts_v, parts_s = [], [], []
    for axis, scale in ((2, 1.0), (1, 1e-2), (0, 1e-4)):
        sl_a = [slice(None)] * 3
        sl_b = [slice(None)] * 3
        sl_a[axis] = slice(None, -1)
        sl_b[axis] = slice(1, None)
        u = idx[tuple(sl_a)].ravel()
        v = idx[tuple(sl_b)].ravel()
        parts_u.append(u)
        parts_v.append(v)
        parts_s.append(np.full(u.shape[0], scale))
    eu = np.concatenate(parts_u).astype(np.int32)
    ev = np.concatenate(parts_v).astype(np.int32)
    noise = np.exp(_rng(seed, _S_WEIGHT).uniform(math.log(0.5), math.log(2.0), eu.shape[0]))
    w = np.concatenate(parts_s) * noise
    return Graph(f"grid3d_aniso_{nside}", n, eu, ev, w)


def chung_lu(n0: int = 1 << 20, mean_deg: float = 16.0, beta: float = 2.1,
             seed: int = SEEDS["chung_lu"]) -> Graph:
    """Chung-Lu power law: phi_i = c (i + i0)^(-1/(beta-1))."""
    expo = 1.0 / (beta - 1.0)
    phi_max = math.sqrt(mean_deg * n0)
    i = np.arange(n0, dtype=np.float64)

    def mean_for(i0):
        c = phi_max * i0 ** expo
        return float(np.mean(c * (i + i0) ** (-expo)))

    lo, hi = 1e-6, float(n0)  # the mean grows with i0
    for _ in range(60):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) > mean_deg:
            hi = mid
        else:
            lo = mid
    i0 = math.sqrt(lo * hi)
    phi = phi_max * i0 ** expo * (i + i0) ** (-expo)
    cdf = np.cumsum(phi)
    cdf /= cdf[-1]
    npairs = int(round(mean_deg * n0 / 2))
    rng = _rng(seed, _S_GRAPH)
    a = np.searchsorted(cdf, rng.random(npairs), side="right")
    b = np.searchsorted(cdf, rng.random(npairs), side="right")
    a = np.minimum(a, n0 - 1)
    b = np.minimum(b, n0 - 1)
    keep = a != b
    lo_, hi_ = np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])
    key = np.unique(lo_.astype(np.int64) * n0 + hi_)
    eu = (key // n0).astype(np.int32)
    ev = (key % n0).astype(np.int32)
    n, eu, ev, _, _ = _largest_component(n0, eu, ev, np.ones(eu.shape[0]))
    w = _rng(seed, _S_WEIGHT).uniform(0.1, 1.0, eu.shape[0])
    return Graph(f"chung_lu_{n0}", n, eu, ev, w)


def _rgg_edges(pts: np.ndarray, r: float):
    from scipy.spatial import cKDTree
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    if pairs.shape[0] == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    lo_, hi_ = pairs.min(axis=1), pairs.max(axis=1)
    key = np.unique(lo_ * pts.shape[0] + hi_)
    return (key // pts.shape[0]).astype(np.int32), (key % pts.shape[0]).astype(np.int32)


def rgg(npts: int = 1 << 20, seed: int = SEEDS["rgg"], weights: str = "gauss") -> Graph:
    """Random geometric graph, radius sqrt(12/(pi n)) (mean degree ~12)."""
    pts = _rng(seed, _S_GRAPH).random((npts, 2))
    r = math.sqrt(12.0 / (math.pi * npts))
    eu, ev = _rgg_edges(pts, r)
    d2 = np.sum((pts[eu] - pts[ev]) ** 2, axis=1)
    if weights == "gauss":
        w = np.exp(-d2 / (r * r))
    else:
        w = _rng(seed, _S_WEIGHT).uniform(0.1, 1.0, eu.shape[0])
    n, eu, ev, w, pts2 = _largest_component(npts, eu, ev, w, pts)
    return Graph(f"rgg_{npts}", n, eu, ev, w, coords=pts2)


def erdos_renyi(n: int, mean_deg: float, seed: int) -> Graph:
    """G(n, p) with p = mean_deg/(n-1): the edge count is Binomial(N, p) and the
    edges are a uniformly random set of that many distinct pairs."""
    rng = _rng(seed, _S_GRAPH)
    npair = n * (n - 1) // 2
    p = mean_deg / (n - 1)
    m = int(rng.binomial(npair, p))
    keys = np.zeros(0, np.int64)
    while keys.shape[0] < m:
        a = rng.integers(0, n, 2 * m + 16)
        b = rng.integers(0, n, 2 * m + 16)
        ok = a != b
        k = np.minimum(a[ok], b[ok]) * n + np.maximum(a[ok], b[ok])
        keys = np.unique(np.concatenate([keys, k]))
    keys = rng.permutation(keys)[:m]
    keys.sort()
    eu = (keys // n).astype(np.int32)
    ev = (keys % n).astype(np.int32)
    n2, eu, ev, _, _ = _largest_component(n, eu, ev, np.ones(m))
    w = _rng(seed, _S_WEIGHT).uniform(0.1, 1.0, eu.shape[0])
    return Graph(f"er_{n}", n2, eu, ev, w)


def er_with_hubs(n: int, mean_deg: float, hub_degrees, seed: int) -> Graph:
    """G(n, p) background plus hubs: node i (i < len(hub_degrees)) joined to
    hub_degrees[i] distinct random other nodes (a test input with rows far
    longer than a relaxation chunk)."""
    g = erdos_renyi(n, mean_deg, seed)
    rng = _rng(seed, _S_LABEL + 1)
    eu, ev = [g.eu.astype(np.int64)], [g.ev.astype(np.int64)]
    for h, d in enumerate(hub_degrees):
        nb = rng.choice(np.arange(len(hub_degrees), g.n), size=int(d), replace=False)
        eu.append(np.full(nb.shape[0], h, np.int64))
        ev.append(nb)
    a, b = np.concatenate(eu), np.concatenate(ev)
    key = np.unique(np.minimum(a, b) * g.n + np.maximum(a, b))
    eu2 = (key // g.n).astype(np.int32)
    ev2 = (key % g.n).astype(np.int32)
    w = _rng(seed, _S_WEIGHT + 8).uniform(0.1, 1.0, eu2.shape[0])
    return Graph(f"er_hubs_{n}", g.n, eu2, ev2, w)


def graph_batch(count: int = 256, nmin: float = 1e3, nmax: float = 2e5,
                seed: int = SEEDS["graph_batch"]) -> list[Graph]:
    """Uneven batch: type g mod 3 in {2-D grid, ER(mean deg 8), RGG}."""
    sizes = np.rint(np.exp(_rng(seed, _S_GRAPH).uniform(math.log(nmin), math.log(nmax), count)))
    out = []
    for g in range(count):
        ng = int(sizes[g])
        sub = seed * 1000 + g
        if g % 3 == 0:
            side = max(2, int(round(math.sqrt(ng))))
            out.append(grid2d(side, side, seed=sub, weights="uniform"))
        elif g % 3 == 1:
            out.append(erdos_renyi(ng, 8.0, sub))
        else:
            out.append(rgg(ng, seed=sub, weights="uniform"))
    return out


def rhs_normal(n: int, k: int = 1, seed: int = 0) -> np.ndarray:
    """N(0,1) right-hand sides, each column projected to zero sum.
    Shape [n] for k == 1, else [n, k] row-major (RHS index fastest)."""
    b = _rng(seed, _S_RHS).standard_normal((n, k))
    b -= b.mean(axis=0, keepdims=True)
    return b[:, 0].copy() if k == 1 else np.ascontiguousarray(b)


def label_split(n: int, frac: float = 0.01, seed: int = SEEDS["rgg"]):
    """Disjoint seeded labelled and held-out node sets (each ~frac*n nodes)."""
    perm = _rng(seed, _S_LABEL).permutation(n)
    k = max(1, int(round(frac * n)))
    return np.sort(perm[:k]), np.sort(perm[k:2 * k])


def rhs_labels(n: int, labelled: np.ndarray, seed: int = SEEDS["rgg"]) -> np.ndarray:
    """b = +/-1 (Rademacher) on the labelled nodes, then zero-mean."""
    b = np.zeros(n)
    b[labelled] = np.where(_rng(seed, _S_RHS).random(labelled.shape[0]) < 0.5, -1.0, 1.0)
    return b - b.mean()


def config(name: str):
    """Full-size inputs of a named benchmark configuration."""
    if name == "grid2d_64":
        g = grid2d(64)
        return g, rhs_normal(g.n, 1, SEEDS["grid2d"])
    if name == "chung_lu_2p20":
        g = chung_lu()
        return g, rhs_normal(g.n, 1, SEEDS["chung_lu"])
    if name == "grid3d_128_k32":
        g = grid3d_aniso(128)
        return g, rhs_normal(g.n, 32, SEEDS["grid3d_aniso"])
    if name == "negative_grid_1024":
        g = grid_stencil(1024, "b")
        return g, rhs_normal(g.n, 1, SEEDS["negative"])
    if name == "lgm_1024":
        g = grid2d_periodic(1024)
        return g, rhs_normal(g.n, 1, SEEDS["lgm"])
    if name == "rgg_2p20":
        g = rgg()
        lab, _ = label_split(g.n)
        return g, rhs_labels(g.n, lab)
    raise KeyError(name)
