"""Rebalancing rounds that tile only the vertices of overloaded blocks (used
on large levels) against the oracle, through refinement and the whole map.
The launch parameter reb_compact_min_n=1 turns the compaction on for the
small graphs here; the full-size rgg20 parity tests cover it at its own
threshold."""
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
    with pm.tuned(reb_compact_min_n=1):
        yield


def t32(torch_mod, x):
    return torch_mod.from_numpy(np.ascontiguousarray(np.asarray(x, np.int32))).cuda()


def host(x):
    return x.cpu().numpy()


CASES = [("grid64", (2, 2, 4), (1, 10, 100)),
         ("rgg14", (4, 8, 8), (1, 10, 100)),
         ("rmat14", (4, 16, 8), (1, 10, 100)),
         ("rgg14", (4, 8, 3), (1, 10, 100)),
         ("rmat14", (3, 5, 2), (2, 7, 50))]


@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("start", ["balanced", "skewed"])
@pytest.mark.parametrize("jrb", [False, True])
def test_refine_with_compacted_rebalancing(pm, pmo, name, a, d, start, jrb):
    import torch
    g = gen.get(name).graph()
    k = int(np.prod(a))
    if start == "balanced":
        part = gen.random_balanced_mapping(g.n, k, 21)
    else:
        part = gen.random_mapping(g.n, k, 21)
        part[: g.n // 5] = 0
    say("refine compacted rebalancing", name, a, start, jrb)
    var = pmo.variants(j_rebalance=True) if jrb else None
    opts = pm.options(j_rebalance=True) if jrb else None
    rc_h, part_h, st_h = pmo.refine(g, a, d, 0.03, 9, part, level=3, var=var)
    part_d = t32(torch, part)
    rc_d, st_d = pm.pm_refine(pm.DeviceGraph.from_host(g), a, d, 0.03, 9, part_d, level=3,
                              opts=opts)
    assert rc_d == rc_h
    assert np.array_equal(host(part_d), part_h)
    for f in ["j_final", "maxw_final", "iterations", "weak_iterations", "strong_iterations"]:
        assert getattr(st_d, f) == getattr(st_h, f), f


@pytest.mark.parametrize("name", ["rgg14", "rmat14", "del16"])
def test_map_with_compacted_rebalancing(pm, pmo, name):
    w = gen.get(name)
    g = w.graph()
    say("map compacted rebalancing", name)
    rc_h, part_h, st_h = pmo.map_graph(g, w.a, w.d, w.eps, 2)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), w.a, w.d, w.eps, 2)
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert np.array_equal(host(part_d), part_h)
