"""Refinement variants (Section 4.2): Jet's relaxed first filter and
rebalancing by the J gain, on the GPU against the oracle, exactly."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

CASES = [("rgg14", (4, 8, 8), (1, 10, 100)),
         ("rmat14", (4, 16, 8), (1, 10, 100)),
         ("rgg14", (4, 8, 3), (1, 10, 100)),
         ("rmat14", (3, 5, 2), (2, 7, 50))]
JETS = [(1, 4), (1, 1), (3, 2)]


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


def test_jet_filter_hand_example_on_gpu(pm, torch_mod):
    g = gen.from_edges(4, [0, 0], [1, 2], [3, 2], [1, 1, 1, 1])
    nin = np.iinfo(np.int64).min
    dg = pm.DeviceGraph.from_host(g)
    for c, gains, targets in (((1, 1), [-1, nin, 2, nin], [1, 0, 0, 1]),
                              ((1, 2), [nin, nin, 2, nin], [0, 0, 0, 1])):
        say("jet hand example", c)
        part = t32(torch_mod, [0, 0, 1, 1])
        lock = torch_mod.zeros(4, dtype=torch_mod.uint8, device="cuda")
        tgt, gain, mv = pm.pm_lp_round(dg, (2,), (1,), part, lock, pm.options(jet_c=c))
        assert host(gain).tolist() == gains
        assert host(tgt).tolist() == targets
        assert host(mv).tolist() == [0, 0, 1, 0]
        assert host(part).tolist() == [0, 0, 0, 1]


@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("jet", JETS)
def test_lp_rounds_jet_parity(pm, pmo, torch_mod, name, a, d, jet):
    g = gen.get(name).graph()
    k = int(np.prod(a))
    part_h = gen.random_balanced_mapping(g.n, k, 5)
    lock_h = np.zeros(g.n, np.uint8)
    dg = pm.DeviceGraph.from_host(g)
    part_d = t32(torch_mod, part_h)
    lock_d = torch_mod.zeros(g.n, dtype=torch_mod.uint8, device="cuda")
    var, opt = pmo.variants(jet_c=jet), pm.options(jet_c=jet)
    for rnd in range(3):
        say("lp_round jet", jet, name, a, "round", rnd)
        part_h, lock_h, tgt_h, gain_h, mv_h = pmo.lp_round(g, a, d, part_h, lock_h, var)
        tgt_d, gain_d, mv_d = pm.pm_lp_round(dg, a, d, part_d, lock_d, opt)
        assert np.array_equal(host(gain_d), gain_h)
        assert np.array_equal(host(tgt_d), tgt_h)
        assert np.array_equal(host(mv_d), mv_h)
        assert np.array_equal(host(part_d), part_h)


@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("strong", [False, True])
def test_rebalance_j_objective_parity(pm, pmo, torch_mod, name, a, d, strong):
    g = gen.get(name).graph()
    k = int(np.prod(a))
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_mapping(g.n, k, 11)
    part[np.random.Generator(np.random.PCG64(2)).choice(g.n, g.n // 10, replace=False)] = 1
    dg = pm.DeviceGraph.from_host(g)
    var, opt = pmo.variants(j_rebalance=True), pm.options(j_rebalance=True)
    for it in range(1, 4):
        say("rebalance J", name, a, "strong" if strong else "weak", "iter", it)
        exp_part, exp_moved = pmo.rebalance(g, k, part, strong, lm, sg, 77, 2, it, a=a, d=d,
                                            var=var)
        part_d = t32(torch_mod, part)
        mv = pm.pm_rebalance(dg, a, d, part_d, strong, lm, sg, 77, 2, it, opt)
        assert np.array_equal(host(mv), exp_moved)
        assert np.array_equal(host(part_d), exp_part)
        part = exp_part


@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("which", ["jet", "jrb", "both"])
def test_refine_and_map_variant_parity(pm, pmo, torch_mod, name, a, d, which):
    jet = (1, 4) if which in ("jet", "both") else None
    jrb = which in ("jrb", "both")
    var, opt = pmo.variants(jet_c=jet, j_rebalance=jrb), pm.options(jet_c=jet, j_rebalance=jrb)
    g = gen.get(name).graph()
    k = int(np.prod(a))
    part = gen.random_mapping(g.n, k, 21)
    part[: g.n // 5] = 0
    say("refine", which, name, a)
    rc_h, part_h, st_h = pmo.refine(g, a, d, 0.03, 9, part, level=3, var=var)
    part_d = t32(torch_mod, part)
    rc_d, st_d = pm.pm_refine(pm.DeviceGraph.from_host(g), a, d, 0.03, 9, part_d, level=3,
                              opts=opt)
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert st_d.iterations == st_h.iterations
    assert np.array_equal(host(part_d), part_h)
    say("map", which, name, a)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 1, var)
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 1, opts=opt)
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert np.array_equal(host(part_d), part_h)


def test_invalid_options_are_rejected(pm, torch_mod):
    g = gen.get("grid64").graph()
    dg = pm.DeviceGraph.from_host(g)
    for bad in (pm.options(jet_c=(0, 1)), pm.options(jet_c=(1, 0)), pm.PmOptions(variants=8)):
        with pytest.raises(pm.PmError) as e:
            pm.pm_map(dg, (2, 2, 4), (1, 10, 100), 0.03, 1, opts=bad)
        assert e.value.code == pm.PM_EINVAL


@pytest.mark.parametrize("name,a,d", CASES + [("grid64", (2, 2, 4), (1, 10, 100))])
@pytest.mark.parametrize("repeats", [2, 5])
def test_map_ultra_parity(pm, pmo, torch_mod, name, a, d, repeats):
    """The "ultra" repetition (Algorithm 6 run `repeats` times per level) on
    the GPU against the oracle: mapping, J and the loop bodies per level."""
    g = gen.get(name).graph()
    say("map ultra", repeats, name, a)
    rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, 3, pmo.variants(repeats=repeats))
    rc_d, part_d, st_d = pm.pm_map(pm.DeviceGraph.from_host(g), a, d, 0.03, 3,
                                   opts=pm.options(repeats=repeats))
    assert rc_d == rc_h and st_d.j_final == st_h.j_final
    assert list(st_d.level_iterations[:st_d.levels]) == list(st_h.level_iterations[:st_h.levels])
    assert np.array_equal(host(part_d), part_h)


@pytest.mark.parametrize("name,a", [("rgg14", (4, 8, 8)), ("rmat14", (4, 16, 8))])
def test_hm_ultra_parity(pm, pmo, name, a):
    """GPU-HM-ultra: every partitioning call refines 18 times per level."""
    g = gen.get(name).graph()
    say("hm ultra", name, a)
    rc_o, part_o = pmo.hm(g, a, 0.03, 2, pmo.variants(repeats=18))
    rc, part, j, calls = pm.pm_map_hm(pm.DeviceGraph.from_host(g), a, (1, 10, 100), 0.03, 2,
                                      opts=pm.options(repeats=18))
    assert rc == rc_o and np.array_equal(host(part), part_o)


def test_invalid_repeats_are_rejected(pm):
    g = gen.get("grid64").graph()
    dg = pm.DeviceGraph.from_host(g)
    for r in (-1, 65):
        with pytest.raises(pm.PmError) as e:
            pm.pm_map(dg, (2, 2, 4), (1, 10, 100), 0.03, 1, opts=pm.options(repeats=r))
        assert e.value.code == pm.PM_EINVAL
