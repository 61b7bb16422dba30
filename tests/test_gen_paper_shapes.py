"""The stand-ins of the paper's rgg23/rgg24 and del23/del24 (Section 5:
random geometric graphs with radius 0.55 sqrt(ln n / n); Delaunay
triangulations of uniform points) are built strip by strip at full size.
These CPU tests check the strip construction against a single global
construction on smaller point sets."""
import numpy as np

from gen import graphs, workloads


def edge_set(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    m = src < g.adjncy
    return set((src[m] * g.n + g.adjncy[m]).tolist())


def test_rgg_strips_equal_global_query():
    n = 1 << 16
    r = workloads.paper_radius(n)
    a = graphs.rgg_radius(n, 11, r, strips=1)
    b = graphs.rgg_radius(n, 11, r, strips=8)
    assert np.array_equal(a.xadj, b.xadj) and np.array_equal(a.adjncy, b.adjncy)
    # radius rule: mean degree n * pi * r^2 = 0.3025 * pi * ln n, up to sampling
    # noise and the square's boundary
    mean = a.nnz / n
    want = 0.3025 * np.pi * np.log(n)
    assert 0.9 * want < mean < want


def test_delaunay_strips_match_global_up_to_hull_edges():
    n = 1 << 16
    a = graphs.delaunay(n, 13, strips=1)
    b = graphs.delaunay(n, 13, strips=8)
    ea, eb = edge_set(a), edge_set(b)
    # planar triangulation of points in general position: 3n - 3 - h edges
    assert 3 * n - 3 - 2000 < len(ea) <= 3 * n - 6
    # the strip construction differs only in a few long hull edges
    assert len(ea - eb) <= 64 and len(eb - ea) <= 64
    rng = np.random.Generator(np.random.PCG64(13))
    pts = rng.random((n, 2))
    pts = pts[graphs._cell_order(pts, 1.0 / np.sqrt(n))]
    for k in (ea ^ eb):
        u, v = divmod(k, n)
        # both ends on the bottom or top side of the square
        ys = pts[[u, v], 1]
        assert np.all(ys < 0.01) or np.all(ys > 0.99)


def test_paper_shape_workloads_registered():
    for name, n in (("rgg23", 1 << 23), ("rgg24", 1 << 24), ("del23", 1 << 23),
                    ("del24", 1 << 24)):
        w = workloads.get(name)
        assert w.size == (n,) and w.a == (4, 8, 6) and w.d == (1, 10, 100) and w.eps == 0.03
