"""Parity of the gfx950 library with the CPU oracle, element by element.

Every comparison is exact (integer results, tolerance 0).  Inputs are seeded
synthetic graphs from gen/; each case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

import gen
from conftest import golden, graph_from_fixture, ip_fixture_graph

pytestmark = pytest.mark.gpu

NIN = np.iinfo(np.int64).min


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2510_12196_amd as pm
    pm.lib()
    return pm


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def dev(pm, g):
    return pm.DeviceGraph.from_host(g)


def t32(torch_mod, x):
    return torch_mod.from_numpy(np.ascontiguousarray(np.asarray(x, np.int32))).cuda()


def host(x):
    return x.cpu().numpy()


CASES = [("grid64", (2, 2, 4), (1, 10, 100)),
         ("rgg14", (4, 8, 8), (1, 10, 100)),
         ("rmat14", (4, 16, 8), (1, 10, 100)),
         ("rgg14", (4, 8, 3), (1, 10, 100)),       # non power of two
         ("rmat14", (3, 5, 2), (2, 7, 50))]         # no power of two at all


def k_of(a):
    return int(np.prod(a))


# ---------------------------------------------------------------------------
# J
# ---------------------------------------------------------------------------

def test_comm_cost_grid_tiling(pm, torch_mod):
    say("comm_cost grid64 tiling")
    fx = golden("grid64_tiling.json")
    g = gen.grid2d(64, 64)
    i, j = np.arange(4096) // 64, np.arange(4096) % 64
    r, c = i // 16, j // 16
    pe = ((c & 1) + 2 * (r & 1) + 4 * (c >> 1) + 8 * (r >> 1)).astype(np.int32)
    assert pm.pm_comm_cost(dev(pm, g), (2, 2, 4), (1, 10, 100), t32(torch_mod, pe),
                           validate=True) == fx["J_ordered"]


@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("seed", [1, 2])
def test_comm_cost_parity(pm, pmo, torch_mod, name, a, d, seed):
    say("comm_cost", name, a, seed)
    g = gen.get(name).graph()
    part = gen.random_mapping(g.n, k_of(a), seed)
    assert pm.pm_comm_cost(dev(pm, g), a, d, t32(torch_mod, part)) == pmo.comm_cost(g, part, a, d)


def test_block_weights_parity(pm, pmo, torch_mod):
    for name, a, d in CASES:
        say("block_weights", name, a)
        g = gen.get(name).graph()
        part = gen.random_mapping(g.n, k_of(a), 3)
        w = host(pm.pm_block_weights(dev(pm, g), a, d, t32(torch_mod, part)))
        assert np.array_equal(w, pmo.block_weights(g, part, k_of(a)))


# ---------------------------------------------------------------------------
# label propagation rounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("fixture", ["lp_round_p7.json", "lp_round_earlier_member.json"])
def test_lp_round_hand_examples_on_gpu(pm, torch_mod, fixture):
    say("lp_round fixture", fixture)
    fx = golden(fixture)
    g = graph_from_fixture(fx)
    part = t32(torch_mod, fx["part_in"])
    lock = torch_mod.zeros(g.n, dtype=torch_mod.uint8, device="cuda")
    target, gain, moved = pm.pm_lp_round(dev(pm, g), fx["a"], fx["d"], part, lock)
    assert [None if x == NIN else int(x) for x in host(gain)] == fx["gain"]
    assert host(target).tolist() == fx["target"]
    assert host(moved).tolist() == fx["moved"]
    assert host(part).tolist() == fx["part_out"]


@pytest.mark.parametrize("name,a,d", CASES)
def test_lp_rounds_parity(pm, pmo, torch_mod, name, a, d):
    g = gen.get(name).graph()
    k = k_of(a)
    part_h = gen.random_balanced_mapping(g.n, k, 5)
    lock_h = np.zeros(g.n, np.uint8)
    dg = dev(pm, g)
    part_d = t32(torch_mod, part_h)
    lock_d = torch_mod.zeros(g.n, dtype=torch_mod.uint8, device="cuda")
    for rnd in range(4):
        say("lp_round", name, a, "round", rnd)
        part_h, lock_h, tgt_h, gain_h, mv_h = pmo.lp_round(g, a, d, part_h, lock_h)
        tgt_d, gain_d, mv_d = pm.pm_lp_round(dg, a, d, part_d, lock_d)
        assert np.array_equal(host(gain_d), gain_h)
        assert np.array_equal(host(tgt_d), tgt_h)
        assert np.array_equal(host(mv_d), mv_h)
        assert np.array_equal(host(part_d), part_h)
        assert np.array_equal(host(lock_d), lock_h)


# ---------------------------------------------------------------------------
# rebalancing rounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("strong", [False, True])
def test_rebalance_parity(pm, pmo, torch_mod, name, a, d, strong):
    g = gen.get(name).graph()
    k = k_of(a)
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    sg = pmo.sigma(lm, total, k)
    part = gen.random_mapping(g.n, k, 11)
    part[: g.n // 10] = 1            # one heavily overloaded block
    dg = dev(pm, g)
    for it in range(1, 4):
        say("rebalance", name, a, "strong" if strong else "weak", "iter", it)
        exp_part, exp_moved = pmo.rebalance(g, k, part, strong, lm, sg, 77, 2, it)
        part_d = t32(torch_mod, part)
        mv = pm.pm_rebalance(dg, a, d, part_d, strong, lm, sg, 77, 2, it)
        assert np.array_equal(host(mv), exp_moved)
        assert np.array_equal(host(part_d), exp_part)
        part = exp_part


def test_weak_rebalance_hand_example_on_gpu(pm, torch_mod):
    say("rebalance fixture")
    fx = golden("weak_rebalance_buckets.json")
    g = graph_from_fixture(fx)
    part = t32(torch_mod, fx["part_in"])
    mv = pm.pm_rebalance(dev(pm, g), fx["a"], fx["d"], part, False, 3, 3, 1, 0, 1)
    assert host(mv).tolist() == fx["moved"]
    assert host(part).tolist() == fx["part_out"]


def test_strong_rebalance_hand_example_on_gpu(pm, torch_mod):
    say("strong rebalance fixture")
    fx = golden("strong_rebalance_weighted.json")
    g = graph_from_fixture(fx)
    part = t32(torch_mod, fx["part_in"])
    lm = fx["lmax"]
    mv = pm.pm_rebalance(dev(pm, g), fx["a"], fx["d"], part, True, lm, lm, 1, 0, 1)
    assert host(mv).tolist() == fx["moved"]
    assert host(part).tolist() == fx["part_out"]


@pytest.mark.parametrize("strong", [False, True])
def test_heavy_vertex_boundary_on_gpu(pm, pmo, torch_mod, strong):
    say("heavy vertex fixture", "strong" if strong else "weak")
    fx = golden("heavy_vertex_boundary.json")
    g = graph_from_fixture(fx)
    k = k_of(fx["a"])
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, fx["eps"])
    sg = pmo.sigma(lm, total, k)
    part = t32(torch_mod, fx["part_in"])
    mv = pm.pm_rebalance(dev(pm, g), fx["a"], fx["d"], part, strong, lm, sg, 1, 0, 1)
    tag = "strong" if strong else "weak"
    assert host(mv).tolist() == fx[tag + "_moved"]
    assert host(part).tolist() == fx[tag + "_part_out"]


def _reweighted(g, seed, wlog):
    """g with vertex weights floor(2^U(0, wlog)): refused movers of a strong
    round then fall into many weight classes."""
    rng = np.random.default_rng(seed)
    vw = np.floor(2.0 ** rng.uniform(0, wlog, g.n)).astype(np.int32)
    src = np.repeat(np.arange(g.n), np.diff(g.xadj))
    m = src < g.adjncy
    return gen.from_edges(g.n, src[m], g.adjncy[m], g.adjwgt[m], vw)


@pytest.mark.parametrize("name,a,frac,wlog", [("rmat14", (4, 16, 8), 0.1, 12),
                                              ("rmat17", (4, 16, 8), 0.1, 12),
                                              ("rmat17", (4, 16, 8), 0.2, 4),
                                              ("rmat17", (16, 16, 16), 0.1, 12),
                                              ("rgg17", (4, 8, 8), 0.3, 8),
                                              ("rgg14", (4, 8, 3), 0.3, 10)])
def test_strong_rebalance_weight_classes(pm, pmo, torch_mod, name, a, frac, wlog):
    """Strong rounds whose refused movers span up to 13 weight classes,
    with up to 10 000 refused movers and with 4096 codes (residuals and
    position starts outside LDS); the result equals the oracle and no block
    at or below L_max before the round ends above it."""
    g = _reweighted(gen.get(name).graph(), 5, wlog)
    k = k_of(a)
    d = (1, 10, 100)
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    part = gen.random_mapping(g.n, k, 11)
    part[: int(g.n * frac)] = 1
    say("strong classes", name, a, frac, wlog)
    exp_part, exp_moved = pmo.rebalance(g, k, part, True, lm, lm, 77, 2, 1)
    part_d = t32(torch_mod, part)
    mv = pm.pm_rebalance(dev(pm, g), a, d, part_d, True, lm, lm, 77, 2, 1)
    assert np.array_equal(host(mv), exp_moved)
    assert np.array_equal(host(part_d), exp_part)
    w0 = np.bincount(part, weights=g.vwgt, minlength=k)
    w1 = np.bincount(exp_part, weights=g.vwgt, minlength=k)
    assert not np.any((w0 <= lm) & (w1 > lm))


@pytest.fixture(scope="module")
def rmat19():
    return gen.rmat(19, 1 << 22, 0xC3, name="rmat19")


@pytest.mark.parametrize("a,frac", [((4, 16, 8), 0.5), ((16, 16, 16), 0.3)])
def test_strong_rebalance_many_refused(pm, pmo, torch_mod, rmat19, a, frac):
    """Strong rounds with about 15 000 and 30 000 refused movers (more than
    one 16 384-entry chunk of the placement), equal to the oracle."""
    g = rmat19
    k = k_of(a)
    total = int(g.vwgt.sum())
    lm = pmo.lmax(total, k, 0.03)
    part = gen.random_mapping(g.n, k, 11)
    part[: int(g.n * frac)] = 1
    say("strong many refused", a, frac)
    exp_part, exp_moved = pmo.rebalance(g, k, part, True, lm, lm, 77, 2, 1)
    part_d = t32(torch_mod, part)
    mv = pm.pm_rebalance(dev(pm, g), a, (1, 10, 100), part_d, True, lm, lm, 77, 2, 1)
    assert np.array_equal(host(mv), exp_moved)
    assert np.array_equal(host(part_d), exp_part)


# ---------------------------------------------------------------------------
# refinement (Algorithm 6)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,a,d", CASES)
@pytest.mark.parametrize("start", ["balanced", "skewed"])
def test_refine_parity(pm, pmo, torch_mod, name, a, d, start):
    say("refine", name, a, start)
    g = gen.get(name).graph()
    k = k_of(a)
    if start == "balanced":
        part = gen.random_balanced_mapping(g.n, k, 21)
    else:
        part = gen.random_mapping(g.n, k, 21)
        part[: g.n // 5] = 0
    rc_h, part_h, st_h = pmo.refine(g, a, d, 0.03, 9, part, level=3)
    part_d = t32(torch_mod, part)
    rc_d, st_d = pm.pm_refine(dev(pm, g), a, d, 0.03, 9, part_d, level=3)
    assert rc_d == rc_h
    assert np.array_equal(host(part_d), part_h)
    for f in ["j_initial", "j_final", "maxw_initial", "maxw_final", "iterations",
              "lp_iterations", "weak_iterations", "strong_iterations", "feasible"]:
        assert getattr(st_d, f) == getattr(st_h, f), f


# ---------------------------------------------------------------------------
# coarsening
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["grid64", "rgg14", "rmat14"])
def test_hem_and_contract_parity(pm, pmo, name):
    say("hem+contract", name)
    w = gen.get(name)
    g = w.graph()
    lm = pmo.lmax(int(g.vwgt.sum()), w.k, w.eps)
    rounds_h, match_h = pmo.hem(g, lm, 5, level=1)
    dg = dev(pm, g)
    match_d, rounds_d = pm.pm_hem(dg, lm, 5, level=1)
    assert rounds_d == rounds_h
    assert np.array_equal(host(match_d), match_h)
    nc_h, cmap_h = pmo.coarse_map(match_h)
    cx_h, ca_h, cw_h, cv_h = pmo.contract(g, cmap_h, nc_h)
    cmap_d, cg = pm.pm_contract(dg, match_d)
    assert np.array_equal(host(cmap_d), cmap_h)
    assert np.array_equal(host(cg.xadj), cx_h)
    assert np.array_equal(host(cg.adjncy), ca_h)
    assert np.array_equal(host(cg.adjwgt), cw_h)
    assert np.array_equal(host(cg.vwgt), cv_h)


@pytest.mark.parametrize("name,a,d", CASES)
def test_initial_partition_parity(pm, pmo, name, a, d):
    say("initial_partition", name, a)
    g = gen.get(name).graph()
    assert np.array_equal(host(pm.pm_initial_partition(dev(pm, g), a, d)),
                          pmo.initial_partition(g, a))


@pytest.mark.parametrize("fixture", ["ip_path16.json", "ip_star16.json", "ip_two_paths16.json"])
def test_initial_partition_closed_forms(pm, fixture):
    # the hand-derived partitions of tests/golden (path, star, two
    # interleaved components), on the library's own initial partitioner
    fx = golden(fixture)
    g = ip_fixture_graph(fx)
    say("initial_partition closed form", fixture)
    assert host(pm.pm_initial_partition(dev(pm, g), fx["a"], fx["d"])).tolist() == fx["part"]


# ---------------------------------------------------------------------------
# the whole multilevel map
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,a,d", CASES)
def test_map_parity(pm, pmo, name, a, d):
    for seed in (1, 2):
        say("map", name, a, "seed", seed)
        g = gen.get(name).graph()
        rc_h, part_h, st_h = pmo.map_graph(g, a, d, 0.03, seed)
        rc_d, part_d, st_d = pm.pm_map(dev(pm, g), a, d, 0.03, seed, validate=True)
        assert rc_d == rc_h
        assert st_d.levels == st_h.levels
        assert list(st_d.level_n[: st_d.levels]) == list(st_h.level_n[: st_h.levels])
        assert list(st_d.level_iterations[: st_d.levels]) == list(st_h.level_iterations[: st_h.levels])
        assert st_d.j_final == st_h.j_final
        assert np.array_equal(host(part_d), part_h)


@pytest.mark.parametrize("name", ["rgg16p", "del16"])
def test_map_parity_paper_shapes(pm, pmo, name):
    """The paper's rgg and Delaunay instance shapes at 2^16, hierarchy 4:8:6."""
    w = gen.get(name)
    g = w.graph()
    say("map", name, w.a, "seed 1")
    rc_h, part_h, st_h = pmo.map_graph(g, w.a, w.d, w.eps, 1)
    rc_d, part_d, st_d = pm.pm_map(dev(pm, g), w.a, w.d, w.eps, 1)
    assert rc_d == rc_h
    assert st_d.j_final == st_h.j_final
    assert np.array_equal(host(part_d), part_h)


def test_map_grid_all_paper_seeds(pm, pmo):
    w = gen.get("grid64")
    g = w.graph()
    for seed in range(1, 6):
        say("map grid64 seed", seed)
        rc_h, part_h, st_h = pmo.map_graph(g, w.a, w.d, w.eps, seed)
        rc_d, part_d, st_d = pm.pm_map(dev(pm, g), w.a, w.d, w.eps, seed)
        assert rc_d == rc_h == 0
        assert np.array_equal(host(part_d), part_h)


@pytest.mark.parametrize("name", ["grid64", "rmat14"])
def test_row_order_invariance_on_gpu(pm, name):
    say("row order invariance", name)
    w = gen.get(name)
    g = w.graph()
    gs = gen.shuffle_rows(g, 7)
    _, p1, s1 = pm.pm_map(dev(pm, g), w.a, w.d, w.eps, 4)
    _, p2, s2 = pm.pm_map(dev(pm, gs), w.a, w.d, w.eps, 4)
    assert np.array_equal(host(p1), host(p2)) and s1.j_final == s2.j_final


def test_repeat_runs_identical(pm):
    say("repeat runs rgg14")
    w = gen.get("rgg14")
    g = dev(pm, w.graph())
    outs = [host(pm.pm_map(g, w.a, w.d, w.eps, 3)[1]) for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
