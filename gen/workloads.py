"""Named synthetic workloads (inputs only).

Each workload is a task graph plus a machine hierarchy a = a_1:...:a_l
(a_1 innermost: PEs per processor), level distances d = d_1:...:d_l and an
imbalance eps, following the experimental setup of Section 5 of the paper
(d = 1:10:100, eps = 3 %, hierarchies 4:8:{1..6}).  The graphs stand in for
the paper's instance set (Table 1), which is not available here; rgg23/24
and del23/24 follow its description of those four instances.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from . import graphs


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: str          # "grid" | "rgg" | "rmat"
    size: tuple        # grid: (rows, cols); rgg: (n,); rmat: (scale, draws)
    a: tuple
    d: tuple
    eps: float = 0.03
    gseed: int = 0

    @property
    def k(self) -> int:
        return int(np.prod(self.a))

    def graph(self) -> graphs.Graph:
        return _build(self.kind, self.size, self.gseed)

    def describe(self) -> dict:
        return {"workload": self.name, "kind": self.kind, "size": list(self.size),
                "hierarchy": ":".join(map(str, self.a)),
                "distance": ":".join(map(str, self.d)), "eps": self.eps,
                "k": self.k, "graph_seed": self.gseed}


def paper_radius(n: int) -> float:
    """Connection radius of the paper's rgg23/rgg24: 0.55 sqrt(ln n / n)."""
    return 0.55 * float(np.sqrt(np.log(n) / n))


@functools.lru_cache(maxsize=4)
def _build(kind, size, gseed):
    if kind == "grid":
        return graphs.grid2d(*size)
    if kind == "rgg":
        return graphs.rgg(size[0], gseed)
    if kind == "rmat":
        return graphs.rmat(size[0], size[1], gseed)
    if kind == "rggp":
        n = size[0]
        return graphs.rgg_radius(n, gseed, paper_radius(n), strips=max(1, n >> 20))
    if kind == "del":
        n = size[0]
        return graphs.delaunay(n, gseed, strips=max(1, n >> 20))
    raise ValueError(kind)


D3 = (1, 10, 100)

WORKLOADS = {
    # 64x64 4-neighbour grid, unit weights, 2:2:4 (k = 16)
    "grid64": Workload("grid64", "grid", (64, 64), (2, 2, 4), D3),
    # random geometric graph, n = 2^20, mean degree 8, w ~ U{1..10}, 4:8:8 (k = 256)
    "rgg20": Workload("rgg20", "rgg", (1 << 20,), (4, 8, 8), D3, gseed=0xC2),
    # R-MAT, n = 2^22, 2^25 draws, c ~ U{1..4}, w ~ U{1..10}, 4:16:8 (k = 512)
    "rmat22": Workload("rmat22", "rmat", (22, 1 << 25), (4, 16, 8), D3, gseed=0xC3),
    # scaled-down shapes of the two large workloads, for fast parity runs
    "rgg14": Workload("rgg14", "rgg", (1 << 14,), (4, 8, 8), D3, gseed=0xC2),
    "rgg17": Workload("rgg17", "rgg", (1 << 17,), (4, 8, 8), D3, gseed=0xC2),
    "rmat14": Workload("rmat14", "rmat", (14, 1 << 17), (4, 16, 8), D3, gseed=0xC3),
    "rmat17": Workload("rmat17", "rmat", (17, 1 << 20), (4, 16, 8), D3, gseed=0xC3),
    # stand-ins of the paper's largest mesh instances (unit weights, radius
    # 0.55 sqrt(ln n / n) resp. Delaunay), hierarchy 4:8:6 (k = 192)
    "rgg23": Workload("rgg23", "rggp", (1 << 23,), (4, 8, 6), D3, gseed=0xC6),
    "rgg24": Workload("rgg24", "rggp", (1 << 24,), (4, 8, 6), D3, gseed=0xC6),
    "del23": Workload("del23", "del", (1 << 23,), (4, 8, 6), D3, gseed=0xC7),
    "del24": Workload("del24", "del", (1 << 24,), (4, 8, 6), D3, gseed=0xC7),
    # the same shapes at 2^16 for parity runs
    "rgg16p": Workload("rgg16p", "rggp", (1 << 16,), (4, 8, 6), D3, gseed=0xC6),
    "del16": Workload("del16", "del", (1 << 16,), (4, 8, 6), D3, gseed=0xC7),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]


# ---------------------------------------------------------------------------
# many instances: the batched workload and the served request stream
# ---------------------------------------------------------------------------
BATCH_HIERARCHIES = [(2, 2, 4), (4, 4, 8), (4, 8, 8)]


@dataclasses.dataclass
class Instance:
    name: str
    graph: graphs.Graph
    a: tuple
    d: tuple
    eps: float
    seed: int


def _member_rng(base: int, index: int):
    return np.random.Generator(np.random.PCG64([base, index]))


def instance(kind: str, n: int, a, seed: int, name: str) -> Instance:
    if kind == "grid":
        r = max(1, int(np.floor(np.sqrt(n))))
        g = graphs.grid2d(r, max(1, n // r))
    elif kind == "rgg":
        g = graphs.rgg(n, seed)
    else:
        g = graphs.rmat_n(n, 8 * n, seed)
    return Instance(name, g, tuple(a), D3, 0.03, 1)


def batch_spec(i: int, base_seed: int = 0xC4, log2_lo: float = 10.0, log2_hi: float = 16.0):
    """Member i of the batched workload, unbuilt: (kind, n, a, graph_seed,
    seed) with n = floor(2^U(lo,hi)), kind grid / rgg / rmat with probability
    1/3 each, hierarchy drawn from 2:2:4, 4:4:8, 4:8:8."""
    rng = _member_rng(base_seed, i)
    n = int(np.floor(2.0 ** rng.uniform(log2_lo, log2_hi)))
    kind = ["grid", "rgg", "rmat"][int(rng.integers(0, 3))]
    a = BATCH_HIERARCHIES[int(rng.integers(0, 3))]
    gseed = int(rng.integers(0, 2 ** 31))
    return kind, n, a, gseed, 1 + int(rng.integers(0, 5))


def batch_member(i: int, base_seed: int = 0xC4, log2_lo: float = 10.0,
                 log2_hi: float = 16.0) -> Instance:
    kind, n, a, gseed, seed = batch_spec(i, base_seed, log2_lo, log2_hi)
    inst = instance(kind, n, a, gseed, f"{kind}{n}")
    inst.seed = seed
    return inst


def batch_members(count: int = 512, base_seed: int = 0xC4, log2_lo: float = 10.0,
                  log2_hi: float = 16.0):
    """Instances of the batched workload (batch_spec), distances 1:10:100,
    eps 3 %; everything derived from (base_seed, index)."""
    return [batch_member(i, base_seed, log2_lo, log2_hi) for i in range(count)]


def serve_arrivals(count: int, qps: float, base_seed: int = 0xC5):
    """Arrival times (seconds) of serve_stream(count, qps, base_seed), without
    building the graphs."""
    t, out = 0.0, []
    for i in range(count):
        t += float(_member_rng(base_seed, i).exponential(1.0 / qps))
        out.append(t)
    return out


def serve_stream(count: int, qps: float, base_seed: int = 0xC5, log2_lo: float = 12.0,
                 log2_hi: float = 20.0):
    """Requests of the served workload: exponential inter-arrival times at
    `qps`, n = floor(2^U(lo,hi)), rgg or rmat 1/2 each, hierarchy 4:8:8 or
    4:16:8 1/2 each.  Returns (arrival_seconds, Instance) pairs."""
    out = []
    t = 0.0
    for i in range(count):
        rng = _member_rng(base_seed, i)
        t += float(rng.exponential(1.0 / qps))
        n = int(np.floor(2.0 ** rng.uniform(log2_lo, log2_hi)))
        kind = "rgg" if rng.integers(0, 2) == 0 else "rmat"
        a = (4, 8, 8) if rng.integers(0, 2) == 0 else (4, 16, 8)
        gseed = int(rng.integers(0, 2 ** 31))
        inst = instance(kind, n, a, gseed, f"{kind}{n}")
        inst.seed = 1 + int(rng.integers(0, 5))
        out.append((t, inst))
    return out


SERVE_HIERARCHIES = ((4, 8, 8), (4, 16, 8))


def serve_pool_spec(pool: int, base_seed: int = 0xC5, log2_lo: float = 12.0,
                    log2_hi: float = 20.0):
    """The resident graphs of the pooled served workload, as (kind, n,
    graph_seed, name) tuples: n = floor(2^U(lo,hi)), rgg or rmat 1/2 each;
    instance(kind, n, a, graph_seed, name) builds one (a is per request)."""
    out = []
    for i in range(pool):
        rng = _member_rng(base_seed ^ 0x9001, i)
        n = int(np.floor(2.0 ** rng.uniform(log2_lo, log2_hi)))
        kind = "rgg" if rng.integers(0, 2) == 0 else "rmat"
        out.append((kind, n, int(rng.integers(0, 2 ** 31)), f"{kind}{n}"))
    return out


def serve_requests(count: int, pool: int, base_seed: int = 0xC5):
    """Requests of the pooled served workload: request i maps pool graph
    `graph` (uniform over the pool) onto hierarchy 4:8:8 or 4:16:8 (1/2
    each) with seed 1..5; arrival times come from serve_arrivals(count, qps,
    base_seed).  Returns (graph_index, a, seed) triples."""
    out = []
    for i in range(count):
        rng = _member_rng(base_seed ^ 0x9002, i)
        out.append((int(rng.integers(0, pool)),
                    SERVE_HIERARCHIES[int(rng.integers(0, 2))],
                    1 + int(rng.integers(0, 5))))
    return out
