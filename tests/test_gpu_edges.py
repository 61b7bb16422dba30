"""Edge cases of the C ABI on the GPU: empty and degenerate graphs, trivial
hierarchies, hub rows, and every error path (bad arguments are rejected by
the host or by the library's own bounds-checked validation kernels)."""
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


def host(x):
    return x.cpu().numpy()


def empty_graph(n):
    return gen.Graph(np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                     np.ones(n, np.int32))


def star(n_leaves, w=1):
    u = np.zeros(n_leaves, np.int64)
    v = np.arange(1, n_leaves + 1)
    return gen.from_edges(n_leaves + 1, u, v, np.full(n_leaves, w), np.ones(n_leaves + 1))


@pytest.mark.parametrize("n", [0, 1, 5, 300])
def test_graphs_without_edges(pm, pmo, n):
    say("no edges n =", n)
    g = empty_graph(n)
    a, d = (2, 2), (1, 10)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 1)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 1)
    assert rc_d == rc_h
    assert np.array_equal(host(part_d), part_h)
    assert st_d.j_final == 0


def test_single_pe_hierarchy(pm, pmo):
    say("k = 1")
    w = gen.get("rgg14")
    g = w.graph()
    rc, part, st = pm.pm_map(pm.DeviceGraph.from_host(g), (1,), (5,), 0.03, 1)
    assert rc == 0 and (host(part) == 0).all() and st.j_final == 0


def test_degenerate_levels(pm, pmo):
    say("degenerate hierarchy levels 4:1:8 and 1:4")
    g = gen.get("rmat14").graph()
    for a, d in [((4, 1, 8), (1, 10, 100)), ((1, 4), (3, 7))]:
        rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 2)
        rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 2)
        assert rc_d == rc_h and np.array_equal(host(part_d), part_h)


@pytest.mark.parametrize("leaves", [70, 5000, 70000])
def test_hub_rows(pm, pmo, leaves):
    say("star with", leaves, "leaves")
    g = star(leaves, w=3)
    a, d = (4, 4), (1, 10)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 1)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 1)
    assert rc_d == rc_h and np.array_equal(host(part_d), part_h)


def test_ragged_degree_mix(pm, pmo):
    """Degrees straddling every lane-group boundary (8/16/32/64) in one graph."""
    say("ragged degree mix")
    rng = np.random.Generator(np.random.PCG64(3))
    n = 3000
    pairs = set()
    for v in range(n):
        deg = int(rng.choice([0, 1, 7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 130]))
        for u in rng.integers(0, n, size=deg):
            if u != v:
                pairs.add((min(u, v), max(u, v)))
    e = np.array(sorted(pairs))
    g = gen.from_edges(n, e[:, 0], e[:, 1], rng.integers(1, 9, size=len(e)),
                       rng.integers(1, 4, size=n))
    a, d = (2, 3, 4), (1, 10, 100)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 4)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 4)
    assert rc_d == rc_h and np.array_equal(host(part_d), part_h)


def test_infeasible_instance_warns(pm, pmo):
    """eps = 0 with one vertex heavier than the average block: no balanced
    mapping exists; the least-imbalanced mapping comes back with a warning."""
    say("infeasible instance")
    g = gen.path_graph(40)
    g.vwgt[0] = 50
    a, d = (2, 2), (1, 10)
    rc_h, part_h, _ = pmo.map_graph(g, a, d, 0.0, 1)
    rc_d, part_d, _ = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.0, 1)
    assert rc_h == rc_d == pm.PM_WARN_IMBALANCED
    assert np.array_equal(host(part_d), part_h)


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------

def test_bad_hierarchies_rejected(pm):
    import torch
    say("bad hierarchies")
    g = pm.DeviceGraph.from_host(gen.grid2d(8, 8))
    part = torch.zeros(64, dtype=torch.int32, device="cuda")
    for a, d in [((0, 2), (1, 1)), ((2, 2), (1, -1)), ((1 << 14,), (1,)),
                 ((2,) * 14, (1,) * 14)]:
        with pytest.raises((pm.PmError, ValueError)):
            pm.pm_comm_cost(g, a, d, part)


def test_mapping_out_of_range_rejected(pm):
    import torch
    say("ids out of range")
    g = pm.DeviceGraph.from_host(gen.grid2d(8, 8))
    for bad in (-1, 4):
        part = torch.zeros(64, dtype=torch.int32, device="cuda")
        part[5] = bad
        with pytest.raises(pm.PmError) as e:
            pm.pm_refine(g, (2, 2), (1, 10), 0.03, 1, part)
        assert e.value.code == pm.PM_EINVAL
        with pytest.raises(pm.PmError):
            pm.pm_comm_cost(g, (2, 2), (1, 10), part)


@pytest.mark.parametrize("defect", ["asym", "selfloop", "range", "weight", "xadj"])
def test_malformed_graph_rejected_with_validation(pm, defect):
    import torch
    say("malformed graph", defect)
    g = gen.grid2d(8, 8)
    xadj, adj, w, vw = g.xadj.copy(), g.adjncy.copy(), g.adjwgt.copy(), g.vwgt.copy()
    if defect == "asym":
        w[3] = 7
    elif defect == "selfloop":
        adj[0] = 0
    elif defect == "range":
        adj[0] = 64
    elif defect == "weight":
        w[0] = 0
        w[np.nonzero(adj == 0)[0][0]] = 0
    elif defect == "xadj":
        xadj[10] = xadj[11] + 1
    dg = pm.DeviceGraph.from_host(gen.Graph(xadj, adj, w, vw))
    part = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(pm.PmError) as e:
        pm.pm_map(dg, (2, 2), (1, 10), 0.03, 1, part=part, validate=True)
    assert e.value.code == pm.PM_EGRAPH


def test_weight_overflow_rejected(pm):
    say("weight overflow")
    g = gen.path_graph(4)
    g.vwgt[:] = 2 ** 30
    with pytest.raises(pm.PmError) as e:
        pm.pm_map(pm.DeviceGraph.from_host(g), (2,), (1,), 0.03, 1)
    assert e.value.code == pm.PM_EOVERFLOW


@pytest.mark.parametrize("a,d", [((8, 32, 32), (1, 10, 100)),      # 2^13 codes, k = 8192
                                 ((5, 30, 25), (1, 3, 9))])         # 13 code bits, k = 3750
def test_largest_hierarchy(pm, pmo, a, d):
    """The largest hierarchy the block codes allow (13 bits): histograms of
    8192 entries, no per-wave slices; J, one label-propagation round and the
    whole map against the oracle."""
    import torch
    g = gen.get("rgg14").graph()
    k = int(np.prod(a))
    dg = pm.DeviceGraph.from_host(g)
    part = gen.random_mapping(g.n, k, 4)
    pd = torch.from_numpy(part.astype(np.int32)).cuda()
    say("largest hierarchy J", a)
    assert pm.pm_comm_cost(dg, a, d, pd) == pmo.comm_cost(g, part, a, d)
    say("largest hierarchy lp round", a)
    lock = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
    p_h, l_h, t_h, g_h, m_h = pmo.lp_round(g, a, d, part, np.zeros(g.n, np.uint8))
    t_d, g_d, m_d = pm.pm_lp_round(dg, a, d, pd, lock)
    assert np.array_equal(host(g_d), g_h) and np.array_equal(host(m_d), m_h)
    assert np.array_equal(host(pd), p_h)
    say("largest hierarchy map", a)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 1)
    rc_d, part_d, st_d = pm.pm_map(dg, a, d, 0.03, 1)
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert np.array_equal(host(part_d), part_h)
