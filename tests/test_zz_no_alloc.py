"""The entry point that allocates nothing (pm_comm_cost_noalloc), called
through the C ABI, against pm_comm_cost on the same inputs: two calls in a
row, the second on a smaller graph (the shared scratch keeps the first
call's partial sums), a graph larger than 4096 workgroups' worth of
vertices (the grid walks the rest), a graph of one vertex, an empty graph,
and a mapping with an id outside [0,k)."""
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


def t32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.int32))).cuda()


def test_noalloc_equals_comm_cost_twice_then_smaller(pm, pmo):
    cases = [("rgg17", (4, 8, 8), (1, 10, 100), 3), ("rmat14", (4, 16, 8), (1, 10, 100), 5),
             ("grid64", (2, 2, 4), (1, 10, 100), 7), ("rgg14", (4, 8, 3), (2, 7, 50), 9)]
    for name, a, d, seed in cases:
        g = gen.get(name).graph()
        dg = pm.DeviceGraph.from_host(g)
        part = gen.random_mapping(g.n, int(np.prod(a)), seed)
        pd = t32(part)
        say("noalloc", name, a)
        ref = pm.pm_comm_cost(dg, a, d, pd)
        assert ref == pmo.comm_cost(g, part, a, d)
        for rep in range(2):
            assert pm.pm_comm_cost_noalloc(dg, a, d, pd) == ref, (name, rep)


def test_noalloc_beyond_one_pass_of_the_grid(pm):
    # 2^21 vertices: more than 4096 workgroups of 256 vertices, so every
    # workgroup walks two chunks
    say("noalloc rgg20 x2")
    w = gen.get("rgg20")
    g = w.graph()
    dg = pm.DeviceGraph.from_host(g)
    part = t32(gen.random_mapping(g.n, w.k, 1))
    assert pm.pm_comm_cost_noalloc(dg, w.a, w.d, part) == pm.pm_comm_cost(dg, w.a, w.d, part)
    g2 = gen.rmat(21, 1 << 23, 0xC3, name="rmat21")
    dg2 = pm.DeviceGraph.from_host(g2)
    part2 = t32(gen.random_mapping(g2.n, 512, 2))
    say("noalloc rmat21", g2.n)
    ref = pm.pm_comm_cost(dg2, (4, 16, 8), (1, 10, 100), part2)
    assert pm.pm_comm_cost_noalloc(dg2, (4, 16, 8), (1, 10, 100), part2) == ref
    # and a small graph right after: the scratch still holds the big call's sums
    say("noalloc grid64 after rmat21")
    g3 = gen.get("grid64").graph()
    dg3 = pm.DeviceGraph.from_host(g3)
    part3 = t32(gen.random_mapping(g3.n, 16, 4))
    assert pm.pm_comm_cost_noalloc(dg3, (2, 2, 4), (1, 10, 100), part3) == \
        pm.pm_comm_cost(dg3, (2, 2, 4), (1, 10, 100), part3)


def test_noalloc_edge_cases(pm):
    say("noalloc edge cases")
    g1 = gen.from_edges(1, [], [], [], [3])
    dg1 = pm.DeviceGraph.from_host(g1)
    assert pm.pm_comm_cost_noalloc(dg1, (4,), (1,), t32([2])) == 0
    g0 = gen.from_edges(0, [], [], [], [])
    dg0 = pm.DeviceGraph.from_host(g0)
    assert pm.pm_comm_cost_noalloc(dg0, (4,), (1,), t32(np.zeros(0, np.int32))) == 0
    g = gen.get("grid64").graph()
    dg = pm.DeviceGraph.from_host(g)
    part = gen.random_mapping(g.n, 16, 3)
    part[100] = 16  # outside [0,16)
    with pytest.raises(pm.PmError) as e:
        pm.pm_comm_cost_noalloc(dg, (2, 2, 4), (1, 10, 100), t32(part))
    assert e.value.code == pm.PM_EINVAL
    part[100] = 3
    assert pm.pm_comm_cost_noalloc(dg, (2, 2, 4), (1, 10, 100), t32(part)) == \
        pm.pm_comm_cost(dg, (2, 2, 4), (1, 10, 100), t32(part))
