"""Seeded synthetic inputs: graphs (symmetric CSR adjacency) and right-hand sides.

This module only makes inputs. It holds none of the solver's arithmetic and is
shared by the CPU oracle tests and the GPU path so that both see identical
bytes. Every generator is deterministic in its seed (numpy PCG64).

Graph format (what every solver entry point takes): a weighted, undirected,
connected graph as the CSR of its adjacency matrix ``A`` with both directions
stored, columns strictly increasing within each row, no diagonal entries and
strictly positive weights:

* ``row_ptr``: int64[n+1]
* ``col``: int32[nnz]
* ``w``: float64[nnz]

Recipes follow the workloads the paper evaluates on (Section 4): regular grids
stand in for high-diameter graphs, R-MAT and Chung-Lu graphs for the
power-law social graphs of the strong-scaling study.
"""

from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Graph",
    "from_edges",
    "grid2d",
    "grid3d",
    "path",
    "cycle",
    "star",
    "complete",
    "gnp",
    "rmat",
    "chung_lu",
    "rhs",
    "config_graph",
    "config_rhs",
    "CONFIGS",
    "serving_pool",
    "serving_requests",
]


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    w: np.ndarray  # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def copy(self) -> "Graph":
        return Graph(self.n, self.row_ptr.copy(), self.col.copy(), self.w.copy(), self.name)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def from_edges(n, u, v, w=None, name=""):
    """Build the symmetric CSR from undirected edges (u_k, v_k, w_k).

    Self-loops are dropped, duplicate pairs keep their first weight, both
    directions are stored.  ``w=None`` gives unit weights.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(u.shape[0], dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    keep = u != v
    u, v, w = u[keep], v[keep], w[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * np.int64(n) + b
    key, first = np.unique(key, return_index=True)
    w = w[first]
    a = key // n
    b = key % n
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    # (row, col) pairs are distinct, so ordering by the combined key is the
    # row-major order
    order = np.argsort(rows * np.int64(n) + cols)
    rows, cols, ww = rows[order], cols[order], ww[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(int(n), row_ptr, cols.astype(np.int32), ww.astype(np.float64), name)


def _undirected_pairs(g: Graph):
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col.astype(np.int64)
    m = rows < cols
    return rows[m], cols[m], g.w[m]


def _with_weights(g: Graph, weights: str, rng) -> Graph:
    """Assign one weight per undirected edge (in (u<v) sorted order)."""
    if weights == "unit":
        return g
    a, b, _ = _undirected_pairs(g)
    m = a.shape[0]
    if weights == "uniform01":
        # U(0,1]: 1 - U[0,1)
        w = 1.0 - rng.random(m)
    elif weights == "loguniform":
        # 10^U(-3,3): log-uniform in [1e-3, 1e3]
        w = np.power(10.0, rng.uniform(-3.0, 3.0, m))
    else:
        raise ValueError(f"unknown weights {weights!r}")
    return from_edges(g.n, a, b, w, g.name)


def grid2d(nx, ny, weights="unit", seed=0):
    """5-point grid graph nx x ny; vertex (x, y) has id y*nx + x."""
    idx = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    g = from_edges(nx * ny, u, v, None, f"grid2d_{nx}x{ny}")
    return _with_weights(g, weights, _rng(seed))


def grid3d(nx, ny, nz, weights="unit", seed=0):
    """7-point grid graph; vertex (x, y, z) has id (z*ny + y)*nx + x."""
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    u = np.concatenate(
        [idx[:, :, :-1].ravel(), idx[:, :-1, :].ravel(), idx[:-1, :, :].ravel()]
    )
    v = np.concatenate(
        [idx[:, :, 1:].ravel(), idx[:, 1:, :].ravel(), idx[1:, :, :].ravel()]
    )
    g = from_edges(nx * ny * nz, u, v, None, f"grid3d_{nx}x{ny}x{nz}")
    return _with_weights(g, weights, _rng(seed))


def path(n, w=None):
    u = np.arange(n - 1)
    return from_edges(n, u, u + 1, w, f"path_{n}")


def cycle(n, w=None):
    u = np.arange(n)
    return from_edges(n, u, (u + 1) % n, w, f"cycle_{n}")


def star(m, w=None):
    """Star K_{1,m}: hub 0 joined to leaves 1..m."""
    return from_edges(m + 1, np.zeros(m, dtype=np.int64), np.arange(1, m + 1), w, f"star_{m}")


def complete(n, w=None):
    a, b = np.triu_indices(n, 1)
    return from_edges(n, a, b, w, f"complete_{n}")


def largest_component(g: Graph) -> Graph:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    if g.n == 0:
        return g
    mat = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    ncomp, labels = connected_components(mat, directed=False)
    if ncomp == 1:
        return g
    big = np.argmax(np.bincount(labels))
    keep = labels == big
    new_id = -np.ones(g.n, dtype=np.int64)
    new_id[keep] = np.arange(int(keep.sum()))
    a, b, w = _undirected_pairs(g)
    m = keep[a] & keep[b]
    return from_edges(int(keep.sum()), new_id[a[m]], new_id[b[m]], w[m], g.name)


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Vertex i becomes perm[i]."""
    a, b, w = _undirected_pairs(g)
    return from_edges(g.n, perm[a], perm[b], w, g.name)


def gnp(n, p, seed=0, weights="uniform01"):
    """Erdos-Renyi G(n, p), largest connected component."""
    rng = _rng(seed)
    a, b = np.triu_indices(n, 1)
    m = rng.random(a.shape[0]) < p
    g = from_edges(n, a[m], b[m], None, f"gnp_{n}_{p}")
    g = largest_component(g)
    return _with_weights(g, weights, rng)


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, d=0.05, seed=2,
         weights="uniform01", permute=True):
    """R-MAT graph (Chakrabarti, Zhan & Faloutsos 2004).

    edge_factor * 2^scale directed samples; each picks one quadrant per bit
    with probabilities (a, b, c, d).  Symmetrized, duplicates merged, loops
    dropped, largest connected component kept, vertices relabelled by a
    seeded permutation (Graph500 practice), then weights per undirected edge.
    """
    rng = _rng(seed)
    n = 1 << scale
    m = edge_factor * n
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for bit in range(scale):
        r = rng.random(m)
        ubit = r >= ab  # quadrants c, d
        vbit = ((r >= a) & (r < ab)) | (r >= abc)  # quadrants b, d
        u |= ubit.astype(np.int64) << bit
        v |= vbit.astype(np.int64) << bit
        del r, ubit, vbit
    g = from_edges(n, u, v, None, f"rmat_s{scale}_ef{edge_factor}")
    del u, v
    g = largest_component(g)
    if permute:
        g = relabel(g, rng.permutation(g.n))
    return _with_weights(g, weights, rng)


def _chung_lu_offset(n, alpha, mean_deg, max_deg):
    """i0 such that w_i = c (i+i0)^-alpha has mean mean_deg and w_0 = max_deg."""
    i = np.arange(n, dtype=np.float64)

    def ratio(i0):
        t = np.power(i + i0, -alpha)
        return t[0] / t.mean()

    target = max_deg / mean_deg
    lo, hi = 1e-6, float(n)
    for _ in range(200):  # ratio decreases as i0 grows
        mid = np.sqrt(lo * hi)
        if mid == lo or mid == hi:  # converged: later steps would not move lo or hi
            break
        if ratio(mid) > target:
            lo = mid
        else:
            hi = mid
    i0 = np.sqrt(lo * hi)
    t = np.power(i + i0, -alpha)
    return t * (mean_deg / t.mean())


def _sorted_search(cdf, r):
    """np.searchsorted(cdf, r, side="right"), computed on sorted queries
    (cache-friendly) and returned in the queries' order."""
    order = np.argsort(r)
    out = np.empty(r.shape[0], dtype=np.int64)
    out[order] = np.searchsorted(cdf, r[order], side="right")
    return out


def chung_lu(n, gamma=2.1, mean_deg=16.0, max_deg=1e5, seed=6, weights="uniform01"):
    """Chung-Lu power-law graph.

    Expected degrees w_i proportional to (i + i0)^(-1/(gamma-1)), scaled to
    mean ``mean_deg`` with the largest equal to ``max_deg``.  n*mean_deg/2
    edges are sampled with both endpoints drawn proportional to w; loops are
    dropped, duplicates merged, the largest connected component kept.
    """
    rng = _rng(seed)
    wexp = _chung_lu_offset(n, 1.0 / (gamma - 1.0), mean_deg, max_deg)
    cdf = np.cumsum(wexp)
    cdf /= cdf[-1]
    m = int(n * mean_deg / 2)
    u = _sorted_search(cdf, rng.random(m))
    v = _sorted_search(cdf, rng.random(m))
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    g = from_edges(n, u, v, None, f"chunglu_{n}_g{gamma}")
    del u, v
    g = largest_component(g)
    return _with_weights(g, weights, rng)


def rhs(n, k=1, seed=1):
    """k right-hand sides ~ N(0,1), row-major float64 array of shape (n, k).

    Not projected: the solver removes the constant component itself.
    """
    return _rng(seed).standard_normal((n, k))


# The evaluation workloads (graph recipe, RHS count, precision); the serving
# pool is built by serving_pool below.
CONFIGS = {
    "grid2d_64": dict(graph=("grid2d", dict(nx=64, ny=64)), k=1, rhs_seed=1, precision="fp64"),
    "rmat_s18": dict(graph=("rmat", dict(scale=18, edge_factor=16, seed=2)), k=1, rhs_seed=3,
                     precision="fp64"),
    "grid3d_128_loguniform": dict(
        graph=("grid3d", dict(nx=128, ny=128, nz=128, weights="loguniform", seed=4)),
        k=32, rhs_seed=5, precision="mixed"),
    "chunglu_4m": dict(graph=("chung_lu", dict(n=4 << 20, gamma=2.1, mean_deg=16.0, max_deg=1e5,
                                                seed=6)), k=16, rhs_seed=6, precision="mixed"),
}


def serving_pool(count=64, n_min=1e3, n_max=1e6, seed=7):
    """The serving workload's pool: `count` graphs with vertex counts
    log-uniform in [n_min, n_max], cycling through 2D and 3D grids (unit
    weights) and R-MAT graphs (edge factor 16, U(0,1]); each graph has its own
    seed derived from `seed`."""
    rng = _rng(seed)
    pool = []
    for i in range(count):
        n = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        gseed = int(rng.integers(1, 2**31))
        kind = i % 3
        if kind == 0:
            side = max(2, int(round(np.sqrt(n))))
            g = grid2d(side, side)
        elif kind == 1:
            side = max(2, int(round(n ** (1.0 / 3.0))))
            g = grid3d(side, side, side)
        else:
            g = rmat(max(8, int(round(np.log2(n)))), 16, seed=gseed)
        g.name = f"pool{i}_{g.name}"
        pool.append(g)
    return pool


def serving_requests(pool_sizes, count, seed=7, k_max=8):
    """`count` requests (graph index, RHS count in 1..k_max, RHS seed),
    graphs drawn uniformly from the pool."""
    rng = _rng(seed + 1)
    g = rng.integers(0, len(pool_sizes), count)
    k = rng.integers(1, k_max + 1, count)
    return [(int(g[i]), int(k[i]), 1000 + i) for i in range(count)]


def config_graph(name, **override):
    kind, kw = CONFIGS[name]["graph"]
    kw = dict(kw)
    kw.update(override)
    g = globals()[kind](**kw)
    g.name = name
    return g


def config_rhs(name, n, k=None):
    cfg = CONFIGS[name]
    return rhs(n, cfg["k"] if k is None else k, cfg["rhs_seed"])
