"""Launch parameters (pm_tuning) and the autotuner: no setting changes a
result, invalid settings are refused and leave the old ones in place."""
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


def host(x, n):
    return x[:n].cpu().numpy()


def test_invalid_tuning_is_refused(pm):
    before = pm.get_tuning()
    for bad in ({"group_v": 3}, {"wave_min_count": 0}, {"hem_compact_min_n": -1},
                {"reb_compact_min_n": 0}, {"contract_rows_min_nnz": 0},
                {"contract_rows_long_pct": -1}, {"contract_rows_long_pct": 101},
                {"lp_cache": 2}, {"graph_bodies": 2}):
        with pytest.raises(pm.PmError) as e:
            pm.set_tuning(**bad)
        assert e.value.code == pm.PM_EINVAL
        assert pm.get_tuning() == before


@pytest.mark.parametrize("name", ["rgg14", "rmat14", "del16"])
def test_results_do_not_depend_on_tuning(pm, name):
    from paper_2510_12196_amd.autotune import candidates
    w = gen.get(name)
    dg = pm.DeviceGraph.from_host(w.graph())
    rc0, part0, st0 = pm.pm_map(dg, w.a, w.d, w.eps, 3)
    ref = host(part0, dg.n).copy()
    for c in candidates() + [{"wave_min_count": 1, "hem_compact_min_n": 1,
                              "reb_compact_min_n": 1, "contract_rows_min_nnz": 1,
                              "contract_rows_long_pct": 100}, {"lp_cache": 0},
                             {"graph_bodies": 1}]:
        say("tuning", name, c)
        with pm.tuned(**c):
            rc, part, st = pm.pm_map(dg, w.a, w.d, w.eps, 3)
        assert rc == rc0 and st.j_final == st0.j_final
        assert np.array_equal(host(part, dg.n), ref)


def test_autotune_batch_keeps_results(pm):
    import torch
    from paper_2510_12196_amd.autotune import autotune_batch
    members = gen.batch_members(24, log2_lo=10.0, log2_hi=12.0)
    inst = [(pm.DeviceGraph.from_host(m.graph), m.a, m.d, m.eps, m.seed) for m in members]
    plain = [pm.pm_map(*x) for x in inst]
    before = pm.get_tuning()
    say("autotune")
    best, workers, table = autotune_batch(inst, sample=8, workers=(2, 4),
                                          sync=torch.cuda.synchronize)
    try:
        assert pm.get_tuning() == best and workers in (2, 4)
        assert len(table) == 2 * len(__import__("paper_2510_12196_amd.autotune",
                                               fromlist=["candidates"]).candidates())
        res = pm.pm_map_batch(inst, workers=workers)
        for m, (rc, part, job), (rc_p, part_p, st_p) in zip(members, res, plain):
            assert rc == rc_p and job.j_final == st_p.j_final
            assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n))
    finally:
        pm.set_tuning(**before)


def test_batch_with_every_path_forced_equals_plain(pm):
    """Concurrent jobs with the W class, both compactions and the row-local
    contraction forced on: every
    batched result equals the plain run under the same launch parameters."""
    members = gen.batch_members(32, log2_lo=10.0, log2_hi=13.0)
    inst = [(pm.DeviceGraph.from_host(m.graph), m.a, m.d, m.eps, m.seed) for m in members]
    say("batch with forced paths")
    with pm.tuned(wave_min_count=1, hem_compact_min_n=1, reb_compact_min_n=1, group_v=2,
                  contract_rows_min_nnz=1, contract_rows_long_pct=100):
        plain = [pm.pm_map(*x) for x in inst]
        for rep in range(2):
            res = pm.pm_map_batch(inst, workers=8)
            for m, (rc, part, job), (rc_p, part_p, st_p) in zip(members, res, plain):
                assert rc == rc_p and job.j_final == st_p.j_final, rep
                assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n)), rep
    # and the same mappings as with the defaults
    for m, x, (rc_p, part_p, st_p) in zip(members, inst, plain):
        rc, part, st = pm.pm_map(*x)
        assert rc == rc_p and st.j_final == st_p.j_final
        assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n))


def test_result_caching_is_exact_on_hubs(pm):
    """Label propagation's result caching on a graph with many workgroup-sized
    (BIG) vertices: three maps with caching and one without give the same
    mapping (a vertex's cached result must be read by every wave of its
    workgroup before it is marked evaluated)."""
    g = gen.rmat(18, 1 << 21, 0xC3, name="rmat18")
    dg = pm.DeviceGraph.from_host(g)
    a, d = (4, 16, 8), (1, 10, 100)
    say("cache off")
    with pm.tuned(lp_cache=0):
        rc0, part0, st0 = pm.pm_map(dg, a, d, 0.03, 1)
    ref = host(part0, dg.n).copy()
    for rep in range(3):
        say("cache on", rep)
        with pm.tuned(lp_cache=1):
            rc, part, st = pm.pm_map(dg, a, d, 0.03, 1)
        assert rc == rc0 and st.j_final == st0.j_final, rep
        assert np.array_equal(host(part, dg.n), ref), rep


@pytest.mark.parametrize("name", ["grid64", "rgg14", "rmat14", "rgg16p", "del16"])
def test_graph_bodies_equal_the_oracle(pm, pmo, name):
    """Loop bodies replayed from captured HIP graphs (graph_bodies=1): every
    level replays its label-propagation and weak-rebalancing graphs many
    times, with launched strong rounds and mapping copies between the
    replays; the maps (two seeds, twice each) equal the oracle's."""
    import torch
    w = gen.get(name)
    g = w.graph()
    dg = pm.DeviceGraph.from_host(g)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()  # (the null stream cannot be captured)
    for seed in (1, 2):
        rc_h, part_h, st_h = pmo.map_graph(g, w.a, w.d, w.eps, seed)
        for rep in range(2):
            say("graph bodies", name, seed, rep)
            with pm.tuned(graph_bodies=1), torch.cuda.stream(stream):
                rc, part, st = pm.pm_map(dg, w.a, w.d, w.eps, seed)
            stream.synchronize()
            assert rc == rc_h and st.j_final == st_h.j_final, (seed, rep)
            assert list(st.level_iterations[:st.levels]) == \
                list(st_h.level_iterations[:st_h.levels])
            assert np.array_equal(host(part, dg.n), part_h), (seed, rep)


def test_graph_bodies_in_a_batch(pm):
    """Concurrent jobs, each capturing and replaying its own bodies on its
    worker's stream, equal the plain runs without graphs."""
    members = gen.batch_members(32, log2_lo=10.0, log2_hi=14.0)
    inst = [(pm.DeviceGraph.from_host(m.graph), m.a, m.d, m.eps, m.seed) for m in members]
    plain = [pm.pm_map(*x) for x in inst]
    say("batch with graph bodies")
    with pm.tuned(graph_bodies=1):
        for rep in range(2):
            res = pm.pm_map_batch(inst, workers=8)
            for m, (rc, part, job), (rc_p, part_p, st_p) in zip(members, res, plain):
                assert rc == rc_p and job.j_final == st_p.j_final, rep
                assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n)), rep
