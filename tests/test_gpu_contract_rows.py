"""Row-local contraction against the oracle.

Levels with at least contract_rows_min_nnz arcs, whose coarse rows above 64
staged arcs hold at most contract_rows_long_pct percent of them, stage every
coarse row at the offset of its upper bound deg(v) + deg(M(v)) and merge
rows of at most 64 arcs on lane groups, of at most 512 on one wave (up to
eight per lane), of at most 2048 in LDS, and radix-sort only the arcs of
longer rows.  The launch parameters set to 1 and 100 send every level of
these small graphs there.  Cases: matchings from the matcher, no matching
at all, a matching whose pairs hold only each other (every arc a self
loop), rows at every size boundary (64 / 65, 128 / 129, 256 / 257,
512 / 513, 2048 / 2049 staged arcs), two matched hubs with common
neighbours (every merged arc the sum of two, runs across lanes), hubs above
512 arcs (with and without the one-wave class for 65..512), isolated
vertices, and malformed matchings (refused)."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_12196_amd as pm
    pm.lib()
    return pm


@pytest.fixture(scope="module", autouse=True)
def force_path(pm):
    with pm.tuned(contract_rows_min_nnz=1, contract_rows_long_pct=100):
        yield


def t32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.int32))).cuda()


def host(x):
    return x.cpu().numpy()


def dense(n=3000, deg=150, seed=4):
    """Random graph with most degrees in 65..512 and eight hubs above 512."""
    rng = np.random.default_rng(seed)
    m = n * deg // 2
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    hubs = rng.integers(0, n, 8)
    u = np.concatenate([u, np.repeat(hubs, 700)])
    v = np.concatenate([v, rng.integers(0, n, 8 * 700)])
    return simple(n, u, v, rng)


def simple(n, u, v, rng):
    keep = u != v
    lo, hi = np.minimum(u[keep], v[keep]), np.maximum(u[keep], v[keep])
    uv = np.unique(np.stack([lo, hi], 1), axis=0)
    w = rng.integers(1, 11, uv.shape[0])
    return gen.from_edges(n, uv[:, 0], uv[:, 1], w, rng.integers(1, 5, n))


def sparse_with_isolated(n=5000, m=9000, seed=8):
    """Random sparse graph on the first 80 % of the ids: the rest isolated."""
    rng = np.random.default_rng(seed)
    k = int(n * 0.8)
    return simple(n, rng.integers(0, k, m), rng.integers(0, k, m), rng)


def star(leaves=3000, seed=2):
    rng = np.random.default_rng(seed)
    u = np.zeros(leaves, np.int64)
    v = np.arange(1, leaves + 1)
    return gen.from_edges(leaves + 1, u, v, rng.integers(1, 11, leaves), np.ones(leaves + 1))


def boundary_rows(seed=3):
    """Vertices 0..3 with degrees 40, 24, 40, 25 into a pool of 200 others:
    the pairs (0, 1) and (2, 3), joined by an edge, give coarse rows of 64 and
    65 staged arcs."""
    rng = np.random.default_rng(seed)
    pool = 4 + np.arange(200)
    us, vs = [0, 2], [1, 3]
    for x, d in ((0, 39), (1, 23), (2, 39), (3, 24)):
        nb = rng.choice(pool, d, replace=False)
        us += [x] * d
        vs += list(nb)
    # a sparse background among the pool
    bu = rng.integers(4, 204, 300)
    bv = rng.integers(4, 204, 300)
    g = simple(204, np.concatenate([us, bu]), np.concatenate([vs, bv]), rng)
    deg = np.diff(g.xadj)
    assert deg[0] + deg[1] == 64 and deg[2] + deg[3] == 65
    match = np.arange(204, dtype=np.int32)
    match[[0, 1, 2, 3]] = [1, 0, 3, 2]
    return g, match


def hub_pairs(total, seed=9):
    """Hubs 0, 1 (staged row of `total` arcs) and hubs 2, 3 (total + 1) over a
    pool of leaves with large overlaps, each pair joined by an edge and
    matched."""
    rng = np.random.default_rng(seed + total)
    leaves = max(total, 200)
    pool = 4 + np.arange(leaves)
    a = total // 2 + 3
    us, vs = [0, 2], [1, 3]
    for x, d in ((0, a - 1), (1, total - a - 1), (2, a - 1), (3, total - a)):
        nb = rng.choice(pool, d, replace=False)
        us += [x] * d
        vs += list(nb)
    g = simple(leaves + 4, np.asarray(us), np.asarray(vs), rng)
    deg = np.diff(g.xadj)
    assert deg[0] + deg[1] == total and deg[2] + deg[3] == total + 1
    match = np.arange(leaves + 4, dtype=np.int32)
    match[[0, 1, 2, 3]] = [1, 0, 3, 2]
    return g, match


def twin_hubs(leaves=6000, seed=10):
    """Hubs 0 and 1 joined and sharing every leaf, matched: one coarse row of
    2 * 6001 staged arcs whose merged arcs each add two weights."""
    rng = np.random.default_rng(seed)
    lv = 2 + np.arange(leaves)
    u = np.concatenate([[0], np.zeros(leaves, np.int64), np.ones(leaves, np.int64)])
    v = np.concatenate([[1], lv, lv])
    g = gen.from_edges(leaves + 2, u, v, rng.integers(1, 11, u.shape[0]),
                       rng.integers(1, 5, leaves + 2))
    match = np.arange(leaves + 2, dtype=np.int32)
    match[[0, 1]] = [1, 0]
    return g, match


def pairs_only(n=4000, seed=5):
    """A perfect matching graph matched along its own edges: no coarse arc."""
    rng = np.random.default_rng(seed)
    u = np.arange(0, n, 2)
    g = gen.from_edges(n, u, u + 1, rng.integers(1, 11, n // 2), np.ones(n))
    match = np.arange(n, dtype=np.int32) ^ 1
    return g, match


def check(pm, pmo, g, match_h):
    dg = pm.DeviceGraph.from_host(g)
    nc_h, cmap_h = pmo.coarse_map(match_h)
    cx_h, ca_h, cw_h, cv_h = pmo.contract(g, cmap_h, nc_h)
    cmap_d, cg = pm.pm_contract(dg, t32(match_h))
    assert np.array_equal(host(cmap_d), cmap_h)
    assert np.array_equal(host(cg.xadj), cx_h)
    assert np.array_equal(host(cg.adjncy), ca_h)
    assert np.array_equal(host(cg.adjwgt), cw_h)
    assert np.array_equal(host(cg.vwgt), cv_h)


def matched(pm, pmo, g, k=16, eps=0.03, seed=5):
    lm = pmo.lmax(int(g.vwgt.sum()), k, eps)
    rounds_h, match_h = pmo.hem(g, lm, seed, level=1)
    return match_h


GRAPHS = {
    "grid64": lambda: gen.get("grid64").graph(),
    "rgg14": lambda: gen.get("rgg14").graph(),
    "rmat14": lambda: gen.get("rmat14").graph(),
    "del16": lambda: gen.get("del16").graph(),
    "dense": dense,
    "isolated": sparse_with_isolated,
    "star": star,
    "star6000": lambda: star(leaves=6000, seed=12),
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


@pytest.mark.parametrize("wmin", [1, 8192])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_contract_rows_matched(pm, pmo, name, wmin):
    g = graph(name)
    say("contract rows, matched", name, wmin)
    with pm.tuned(wave_min_count=wmin):
        check(pm, pmo, g, matched(pm, pmo, g))


def test_contract_rows_twin_hubs_wave(pm, pmo):
    """Twin hubs of 150 leaves: one row of 302 staged arcs on one wave, every
    merged arc the sum of two, runs crossing lane boundaries."""
    g, match = twin_hubs(leaves=150, seed=11)
    say("contract rows, twin hubs on one wave")
    check(pm, pmo, g, match)


@pytest.mark.parametrize("name", ["rmat14", "dense", "star", "isolated"])
def test_contract_rows_unmatched(pm, pmo, name):
    g = graph(name)
    say("contract rows, identity matching", name)
    check(pm, pmo, g, np.arange(g.n, dtype=np.int32))


def test_contract_rows_boundary_64_65(pm, pmo):
    g, match = boundary_rows()
    say("contract rows, 64 / 65 staged arcs")
    check(pm, pmo, g, match)


@pytest.mark.parametrize("total", [128, 256, 512, 2048])
def test_contract_rows_size_boundaries(pm, pmo, total):
    """Rows of exactly 128 / 256 / 512 staged arcs and one more (two, four,
    eight arcs per lane on one wave, then the workgroup), 2048 and 2049 (the
    workgroup, then the radix sort)."""
    g, match = hub_pairs(total)
    say("contract rows, staged arcs", total, total + 1)
    check(pm, pmo, g, match)


def test_contract_rows_sorted_path_sums(pm, pmo):
    g, match = twin_hubs()
    say("contract rows, matched hubs above 2048")
    check(pm, pmo, g, match)


def test_contract_rows_all_self_loops(pm, pmo):
    g, match = pairs_only()
    say("contract rows, only self loops")
    check(pm, pmo, g, match)
    cmap_d, cg = pm.pm_contract(pm.DeviceGraph.from_host(g), t32(match))
    assert cg.nnz == 0 and cg.n == g.n // 2


def test_contract_rows_equal_sorted_path(pm, pmo):
    """The two contraction paths give the same coarse graph on a matching of
    the matcher, level after level of rmat14."""
    g = graph("rmat14")
    for lvl in range(4):
        say("contract rows vs sorted path, level", lvl)
        match_h = matched(pm, pmo, g, seed=lvl + 1)
        dg = pm.DeviceGraph.from_host(g)
        cmap_a, ga = pm.pm_contract(dg, t32(match_h))
        with pm.tuned(contract_rows_min_nnz=2**31 - 1):
            cmap_b, gb = pm.pm_contract(dg, t32(match_h))
        for x, y in ((cmap_a, cmap_b), (ga.xadj, gb.xadj), (ga.adjncy, gb.adjncy),
                     (ga.adjwgt, gb.adjwgt), (ga.vwgt, gb.vwgt)):
            assert np.array_equal(host(x), host(y))
        nc_h, cmap_h = pmo.coarse_map(match_h)
        g = gen.Graph(*pmo.contract(g, cmap_h, nc_h))


@pytest.mark.parametrize("pct", [0, 12, 30, 50, 70, 90])
@pytest.mark.parametrize("name", ["rmat14", "dense"])
def test_contract_long_share_limit(pm, pmo, name, pct):
    """Share limits below 100 % send a level to the sort either from the fine
    classes alone or after the row pre-pass; the result is the same."""
    g = graph(name)
    say("contract rows, long-row share limit", name, pct)
    with pm.tuned(contract_rows_long_pct=pct):
        check(pm, pmo, g, matched(pm, pmo, g))


@pytest.mark.parametrize("bad", ["one_way", "out_of_range", "negative"])
def test_contract_refuses_malformed_matching(pm, bad):
    g = graph("rgg14")
    m = np.arange(g.n, dtype=np.int32)
    if bad == "one_way":
        m[0] = 1            # 1 still points to itself
    elif bad == "out_of_range":
        m[5] = g.n
    else:
        m[7] = -2
    say("contract refuses", bad)
    with pytest.raises(pm.PmError) as e:
        pm.pm_contract(pm.DeviceGraph.from_host(g), t32(m))
    assert e.value.code == pm.PM_EINVAL


@pytest.mark.parametrize("name,a,d", [("rmat14", (4, 16, 8), (1, 10, 100)),
                                      ("del16", (4, 8, 8), (1, 10, 100))])
def test_map_parity_contract_rows(pm, pmo, name, a, d):
    g = graph(name)
    say("map with row-local contraction", name)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 1)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 1)
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert np.array_equal(host(part_d), part_h)
