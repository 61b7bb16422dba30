"""Named synthetic workloads (inputs only).

Each workload is a task graph plus a machine hierarchy a = a_1:...:a_l
(a_1 innermost: PEs per processor), level distances d = d_1:...:d_l and an
imbalance eps, following the experimental setup of Section 5 of the paper
(d = 1:10:100, eps = 3 %).  The graphs stand in for the paper's instance set
(Table 1), which is not available here.
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


@functools.lru_cache(maxsize=4)
def _build(kind, size, gseed):
    if kind == "grid":
        return graphs.grid2d(*size)
    if kind == "rgg":
        return graphs.rgg(size[0], gseed)
    if kind == "rmat":
        return graphs.rmat(size[0], size[1], gseed)
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
}


def get(name: str) -> Workload:
    return WORKLOADS[name]
