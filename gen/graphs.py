"""Seeded synthetic task graphs and mappings.

This module only *produces inputs*: task graphs in CSR form (both directions of
every undirected edge stored, as the CSR description of the paper's Section 3.4
requires), vertex/edge weights and initial mappings.  It contains none of the
mapping method's arithmetic and is shared by the CPU oracle tests and the GPU
path alike.

The shapes follow the workloads the paper evaluates on (Section 5, Table 1):
mesh-like graphs (2-D grids and random geometric graphs) and skewed power-law
graphs (R-MAT), with integer vertex and edge weights.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Graph",
    "from_edges",
    "grid2d",
    "rgg",
    "rmat",
    "random_balanced_mapping",
    "random_mapping",
    "shuffle_rows",
    "path_graph",
    "rmat_n",
    "rgg_radius",
    "delaunay",
]


@dataclasses.dataclass
class Graph:
    """Undirected weighted graph in CSR form.

    xadj   int64[n+1]  row offsets
    adjncy int32[nnz]  neighbour ids; every edge {u,v} appears in both rows
    adjwgt int32[nnz]  edge weights (> 0), symmetric
    vwgt   int32[n]    vertex weights (> 0)
    """

    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray
    vwgt: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xadj.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.adjncy.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.xadj)


def from_edges(n: int, u, v, w, vwgt) -> Graph:
    """Build a symmetric CSR from an undirected edge list.

    The list must hold each unordered pair once with u != v.  Rows come out
    sorted by neighbour id.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.asarray(w, dtype=np.int32)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    wt = np.concatenate([w, w])
    order = np.argsort(src * np.int64(n) + dst, kind="stable")
    src = src[order]
    dst = dst[order].astype(np.int32)
    wt = wt[order]
    counts = np.bincount(src, minlength=n).astype(np.int64)
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=xadj[1:])
    return Graph(xadj, np.ascontiguousarray(dst), np.ascontiguousarray(wt),
                 np.ascontiguousarray(np.asarray(vwgt, dtype=np.int32)))


def grid2d(rows: int, cols: int, name: str = "") -> Graph:
    """rows x cols 4-neighbour grid, row-major ids, unit weights."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    hu = ids[:, :-1].ravel()
    hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel()
    vv = ids[1:, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hv, vv])
    n = rows * cols
    return from_edges(n, u, v, np.ones(u.shape[0], np.int32),
                      np.ones(n, np.int32))._replace_name(name or f"grid{rows}x{cols}")


def path_graph(n: int, w: int = 1) -> Graph:
    u = np.arange(n - 1)
    return from_edges(n, u, u + 1, np.full(n - 1, w, np.int32), np.ones(n, np.int32))


def rgg(n: int, seed: int, mean_deg: float = 8.0, wmax: int = 10,
        name: str = "") -> Graph:
    """Random geometric graph in the unit square.

    Points are uniform in [0,1)^2; two points are joined when their distance is
    below r with n*pi*r^2 = mean_deg.  Vertex ids are ordered by grid cell
    (cell side >= r, row-major over cells) and then by draw index, so that ids
    carry spatial locality.  Unit vertex weights, edge weights uniform in
    {1..wmax}.
    """
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    r = float(np.sqrt(mean_deg / (np.pi * n)))
    ncell = max(1, int(np.floor(1.0 / r)))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((np.arange(n), cx, cy))
    pts = pts[order]
    tree = cKDTree(pts)
    pairs = tree.query_pairs(r * (1 - 1e-12), output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    key = pairs[:, 0].astype(np.int64) * n + pairs[:, 1]
    pairs = pairs[np.argsort(key, kind="stable")]
    w = rng.integers(1, wmax + 1, size=pairs.shape[0], dtype=np.int32)
    g = from_edges(n, pairs[:, 0], pairs[:, 1], w, np.ones(n, np.int32))
    g.name = name or f"rgg{n}"
    return g


def _log(msg):
    import sys
    print(f"[gen] {msg}", file=sys.stderr, flush=True)


def _cell_order(pts: np.ndarray, cell: float) -> np.ndarray:
    """Permutation sorting points by grid cell (side `cell`, row-major over
    cells), then by draw index: ids that carry spatial locality."""
    n = pts.shape[0]
    ncell = max(1, int(np.floor(1.0 / cell)))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    return np.lexsort((np.arange(n), cx, cy))


def rgg_radius(n: int, seed: int, radius: float, strips: int = 1, name: str = "") -> Graph:
    """Random geometric graph in the unit square with a given connection
    radius (the paper's rgg23/rgg24 use 0.55 * sqrt(ln n / n)).  Unit vertex
    and edge weights; ids ordered by grid cell (side >= radius).  Pairs are
    found strip by strip along x (each strip's tree also holds the points
    within `radius` to its right), which gives exactly the pairs of a global
    query."""
    from scipy.spatial import cKDTree

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    pts = pts[_cell_order(pts, radius)]
    r = radius * (1 - 1e-12)
    us, vs = [], []
    edges = np.linspace(0.0, 1.0, strips + 1)
    for k in range(strips):
        lo, hi = edges[k], edges[k + 1]
        core = np.nonzero((pts[:, 0] >= lo) & ((pts[:, 0] < hi) | (k == strips - 1)))[0]
        ext = np.nonzero((pts[:, 0] >= lo) & (pts[:, 0] < hi + radius))[0]
        tree_core = cKDTree(pts[core])
        tree_ext = cKDTree(pts[ext])
        res = tree_core.query_ball_tree(tree_ext, r)
        cnt = np.fromiter((len(x) for x in res), dtype=np.int64, count=len(res))
        a = np.repeat(core, cnt)
        b = ext[np.fromiter((j for x in res for j in x), dtype=np.int64, count=int(cnt.sum()))]
        # a pair inside the core is seen from both ends (keep the smaller id
        # first); a pair reaching right of the core only from its core end
        b_core = (pts[b, 0] < hi) | (k == strips - 1)
        keep = np.where(b_core, a < b, True)
        lo_id = np.minimum(a, b)
        b = np.maximum(a, b)
        a = lo_id
        us.append(a[keep])
        vs.append(b[keep])
        if strips > 1:
            _log(f"rgg strip {k + 1}/{strips}: {int(keep.sum())} pairs")
    u = np.concatenate(us)
    v = np.concatenate(vs)
    key = u * n + v
    order = np.argsort(key, kind="stable")
    u, v = u[order], v[order]
    g = from_edges(n, u, v, np.ones(u.shape[0], np.int32), np.ones(n, np.int32))
    g.name = name or f"rgg{n}"
    return g


def delaunay(n: int, seed: int, strips: int = 1, name: str = "") -> Graph:
    """Delaunay triangulation of n uniform points in the unit square (the
    paper's del23/del24).  Unit vertex and edge weights; ids ordered by grid
    cell (side 1/sqrt(n)).  With strips > 1 the points are triangulated per
    vertical strip plus a margin of 32/sqrt(n) on each side, and an edge is
    kept by the strip that holds its smaller-x endpoint in its core.  The
    result equals the global triangulation except for a few long edges of
    the convex hull along the square's top and bottom sides (at n = 2^18
    and 8 strips: 21 of 786 402 global edges missing, 2 hull edges added;
    the tests check this bound)."""
    from scipy.spatial import Delaunay

    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.random((n, 2))
    pts = pts[_cell_order(pts, 1.0 / np.sqrt(n))]
    margin = 32.0 / np.sqrt(n) if strips > 1 else 0.0
    edges = np.linspace(0.0, 1.0, strips + 1)
    keys = []
    for k in range(strips):
        lo, hi = edges[k], edges[k + 1]
        sel = np.nonzero((pts[:, 0] >= lo - margin) & (pts[:, 0] < hi + margin))[0]
        tri = Delaunay(pts[sel]).simplices
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]])
        a = sel[e[:, 0]]
        b = sel[e[:, 1]]
        lo_id = np.minimum(a, b)
        hi_id = np.maximum(a, b)
        # owner strip: the one whose core holds the endpoint with smaller x
        xa, xb = pts[lo_id, 0], pts[hi_id, 0]
        xm = np.minimum(xa, xb)
        own = (xm >= lo) & ((xm < hi) | (k == strips - 1))
        keys.append(np.unique(lo_id[own].astype(np.int64) * n + hi_id[own]))
        if strips > 1:
            _log(f"delaunay strip {k + 1}/{strips}: {len(sel)} points")
    key = np.unique(np.concatenate(keys))
    u = key // n
    v = key % n
    g = from_edges(n, u, v, np.ones(u.shape[0], np.int32), np.ones(n, np.int32))
    g.name = name or f"del{n}"
    return g


def rmat(scale: int, draws: int, seed: int,
         probs=(0.57, 0.19, 0.19, 0.05), wmax: int = 10, cmax: int = 4,
         name: str = "") -> Graph:
    """R-MAT graph on 2^scale vertices from `draws` edge draws.

    Each draw descends `scale` quadrant levels with probabilities (a, b, c, d),
    no noise and no relabelling.  Self-loops are dropped; duplicate undirected
    pairs are merged with their weights summed (each draw carries a weight
    uniform in {1..wmax}).  Vertex weights are uniform in {1..cmax}.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << scale
    a, b, c, _ = probs
    t1, t2, t3 = a, a + b, a + b + c
    src = np.zeros(draws, dtype=np.int64)
    dst = np.zeros(draws, dtype=np.int64)
    chunk = 1 << 22
    for level in range(scale):
        bit = np.int64(1) << np.int64(scale - 1 - level)
        for s in range(0, draws, chunk):
            e = min(draws, s + chunk)
            x = rng.random(e - s)
            down = x >= t2          # quadrants c, d: source bit set
            right = ((x >= t1) & (x < t2)) | (x >= t3)   # quadrants b, d
            src[s:e] += down * bit
            dst[s:e] += right * bit
    w = rng.integers(1, wmax + 1, size=draws, dtype=np.int64)
    keep = src != dst
    src, dst, w = src[keep], dst[keep], w[keep]
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    key = lo * n + hi
    del src, dst, lo, hi
    uniq, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=w).astype(np.int64)
    del inv, key, w
    if wsum.max(initial=0) > np.iinfo(np.int32).max:
        raise OverflowError("merged edge weight exceeds int32")
    u = uniq // n
    v = uniq % n
    vwgt = rng.integers(1, cmax + 1, size=n, dtype=np.int32)
    g = from_edges(n, u, v, wsum.astype(np.int32), vwgt)
    g.name = name or f"rmat{scale}"
    return g


def rmat_n(n: int, draws: int, seed: int, probs=(0.57, 0.19, 0.19, 0.05), wmax: int = 10,
           cmax: int = 4, name: str = "") -> Graph:
    """R-MAT on n vertices (n need not be a power of two): quadrant descent over
    ceil(log2 n) levels, draws with an endpoint >= n are dropped and replaced
    by further draws until `draws` draws are in range; then as rmat()."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = max(1, int(np.ceil(np.log2(max(n, 2)))))
    a, b, c, _ = probs
    t1, t2, t3 = a, a + b, a + b + c
    src_all, dst_all = [], []
    have = 0
    while have < draws:
        m = int((draws - have) * (2 ** scale) / n * 1.2) + 64
        src = np.zeros(m, dtype=np.int64)
        dst = np.zeros(m, dtype=np.int64)
        for level in range(scale):
            bit = np.int64(1) << np.int64(scale - 1 - level)
            x = rng.random(m)
            src += (x >= t2) * bit
            dst += (((x >= t1) & (x < t2)) | (x >= t3)) * bit
        ok = (src < n) & (dst < n)
        src_all.append(src[ok])
        dst_all.append(dst[ok])
        have += int(ok.sum())
    src = np.concatenate(src_all)[:draws]
    dst = np.concatenate(dst_all)[:draws]
    w = rng.integers(1, wmax + 1, size=draws, dtype=np.int64)
    keep = src != dst
    src, dst, w = src[keep], dst[keep], w[keep]
    key = np.minimum(src, dst) * n + np.maximum(src, dst)
    uniq, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=w).astype(np.int64)
    vwgt = rng.integers(1, cmax + 1, size=n, dtype=np.int32)
    g = from_edges(n, uniq // n, uniq % n, wsum.astype(np.int32), vwgt)
    g.name = name or f"rmat_n{n}"
    return g


def random_balanced_mapping(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded random mapping with block sizes differing by at most one:
    a uniform random permutation perm, and block(perm[i]) = i mod k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(n)
    part = np.empty(n, dtype=np.int32)
    part[perm] = (np.arange(n) % k).astype(np.int32)
    return part


def random_mapping(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded uniform random block per vertex (usually imbalanced)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, k, size=n, dtype=np.int32)


def shuffle_rows(g: Graph, seed: int) -> Graph:
    """Same graph with the entries of every CSR row permuted at random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = g.n
    rowid = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.xadj))
    order = np.lexsort((rng.random(g.nnz), rowid))
    return Graph(g.xadj.copy(), g.adjncy[order].copy(), g.adjwgt[order].copy(),
                 g.vwgt.copy(), g.name + "-shuffled")


def _replace_name(self: Graph, name: str) -> Graph:
    self.name = name
    return self


Graph._replace_name = _replace_name
