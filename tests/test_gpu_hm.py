"""Hierarchical multisection on the GPU (Section 4.1, Algorithms 1 and 2):
the induced subgraphs of a partition and the whole recursion, exactly as the
oracle computes them."""
import sys

import numpy as np
import pytest

import gen
from gen.graphs import Graph

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


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def t32(torch_mod, x):
    return torch_mod.from_numpy(np.ascontiguousarray(np.asarray(x, np.int32))).cuda()


def host(x):
    return x.cpu().numpy()


def weighted(g, seed):
    """The same graph with vertex weights in [1, 9]."""
    rng = np.random.default_rng(seed)
    vw = rng.integers(1, 10, g.n).astype(np.int32)
    return Graph(g.xadj, g.adjncy, g.adjwgt, vw, g.name + "-w")


def ragged(n, seed):
    """A sparse random graph whose size is no multiple of the tile."""
    rng = np.random.default_rng(seed)
    m = 3 * n
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    keep = u != v
    u, v = np.minimum(u[keep], v[keep]), np.maximum(u[keep], v[keep])
    uv = np.unique(np.stack([u, v], 1), axis=0)
    w = rng.integers(1, 5, uv.shape[0])
    return gen.from_edges(n, uv[:, 0], uv[:, 1], w, rng.integers(1, 4, n))


def compare_subgraphs(got, want, n, parts):
    assert np.array_equal(host(got["vstart"]), want["vstart"])
    assert np.array_equal(host(got["estart"]), want["estart"])
    assert np.array_equal(host(got["order"]), want["order"][:n])
    assert np.array_equal(host(got["xadj"]), want["xadj"][: n + parts])
    assert np.array_equal(host(got["adjncy"]), want["adjncy"])
    assert np.array_equal(host(got["adjwgt"]), want["adjwgt"])
    assert np.array_equal(host(got["vwgt"]), want["vwgt"][:n])


SUB_CASES = [("grid64", 5, "random4"),     # block 4 stays empty
             ("rgg14", 16, "mapped"),
             ("rmat14", 7, "random"),
             ("rgg14w", 3, "random"),
             ("ragged", 11, "random"),
             ("ragged", 1, "random"),
             ("rmat14", 300, "random")]    # more blocks than a tile's worth


def sub_graph(name):
    if name == "rgg14w":
        return weighted(gen.get("rgg14").graph(), 5)
    if name == "ragged":
        return ragged(4099, 9)
    return gen.get(name).graph()


@pytest.mark.parametrize("name,parts,how", SUB_CASES)
def test_subgraphs_parity(pm, pmo, torch_mod, name, parts, how):
    g = sub_graph(name)
    rng = np.random.default_rng(parts * 131 + g.n)
    if how == "mapped":
        _, part, _ = pmo.map_graph(g, (parts,), (1,), 0.03, 2)
    elif how == "random4":
        part = rng.integers(0, parts - 1, g.n)
    else:
        part = rng.integers(0, parts, g.n)
    part = np.asarray(part, np.int32)
    say("subgraphs", name, g.n, parts, how)
    want = pmo.subgraphs(g, part, parts)
    dg = pm.DeviceGraph.from_host(g)
    got = pm.pm_subgraphs(dg, t32(torch_mod, part), parts)
    compare_subgraphs(got, want, g.n, parts)


def test_subgraphs_of_empty_graph(pm, pmo, torch_mod):
    g = gen.from_edges(0, [], [], [], [])
    dg = pm.DeviceGraph.from_host(g)
    part = torch_mod.empty(0, dtype=torch_mod.int32, device="cuda")
    got = pm.pm_subgraphs(dg, part, 3)
    assert host(got["vstart"]).tolist() == [0, 0, 0, 0]
    assert host(got["estart"]).tolist() == [0, 0, 0, 0]
    assert host(got["xadj"]).tolist() == [0, 0, 0]
    assert got["adjncy"].numel() == 0 and got["order"].numel() == 0


def test_subgraphs_reject_ids_out_of_range(pm, torch_mod):
    g = gen.get("grid64").graph()
    dg = pm.DeviceGraph.from_host(g)
    for bad in (-1, 4):
        part = np.zeros(g.n, np.int32)
        part[g.n - 1] = bad
        say("subgraphs bad id", bad)
        with pytest.raises(pm.PmError) as e:
            pm.pm_subgraphs(dg, t32(torch_mod, part), 4)
        assert e.value.code == pm.PM_EINVAL
    with pytest.raises(pm.PmError):
        pm.pm_subgraphs(dg, t32(torch_mod, np.zeros(g.n)), 0)


HM_CASES = [("rgg14", (4, 8, 8), (1, 10, 100)),
            ("rmat14", (4, 16, 8), (1, 10, 100)),
            ("grid64", (2, 2, 4), (1, 10, 100)),
            ("rgg14", (4, 8, 3), (1, 10, 100)),
            ("rgg14w", (2, 3, 5), (1, 5, 25)),
            ("ragged", (3, 4), (1, 20)),
            ("rgg16p", (4, 8, 6), (1, 10, 100)),
            ("del16", (4, 8, 6), (1, 10, 100))]


@pytest.mark.parametrize("name,a,d", HM_CASES)
def test_hm_parity(pm, pmo, name, a, d):
    g = sub_graph(name) if name in ("rgg14w", "ragged") else gen.get(name).graph()
    say("hm", name, g.n, a)
    rc_o, part_o = pmo.hm(g, a, 0.03, 1)
    dg = pm.DeviceGraph.from_host(g)
    rc, part, j, calls = pm.pm_map_hm(dg, a, d, 0.03, 1)
    assert rc == rc_o
    assert np.array_equal(host(part), part_o)
    assert j == pmo.comm_cost(g, part_o, a, d)
    # one partitioning call per non-empty subgraph, at most 1 + a_l + a_l a_{l-1} ...
    bound = sum(int(np.prod(a[len(a) - i:])) for i in range(len(a)))
    assert 1 <= calls <= bound


def test_hm_does_not_depend_on_worker_count(pm):
    g = gen.get("rmat14").graph()
    dg = pm.DeviceGraph.from_host(g)
    say("hm workers 1 vs 8")
    r1 = pm.pm_map_hm(dg, (4, 8, 8), (1, 10, 100), 0.03, 7, workers=1)
    r8 = pm.pm_map_hm(dg, (4, 8, 8), (1, 10, 100), 0.03, 7, workers=8)
    assert r1[0] == r8[0] and r1[2] == r8[2] and r1[3] == r8[3]
    assert np.array_equal(host(r1[1]), host(r8[1]))


def test_hm_with_one_level_is_the_mapper(pm):
    g = gen.get("rgg14").graph()
    dg = pm.DeviceGraph.from_host(g)
    say("hm one level")
    rc, part, j, calls = pm.pm_map_hm(dg, (16,), (1,), 0.03, 3)
    rc2, part2, st = pm.pm_map(dg, (16,), (1,), 0.03, 3)
    assert calls == 1 and rc == rc2 and j == st.j_final
    assert np.array_equal(host(part), host(part2))


def test_hm_rejects_bad_hierarchies(pm):
    g = gen.get("grid64").graph()
    dg = pm.DeviceGraph.from_host(g)
    with pytest.raises(pm.PmError) as e:
        pm.pm_map_hm(dg, (1 << 14,), (1,), 0.03, 1)
    assert e.value.code == pm.PM_EOVERFLOW
    with pytest.raises(pm.PmError) as e:
        pm.pm_map_hm(dg, (0, 4), (1, 10), 0.03, 1)
    assert e.value.code == pm.PM_EINVAL
