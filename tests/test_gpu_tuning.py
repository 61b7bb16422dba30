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
                {"contract_rows_long_pct": -1}, {"contract_rows_long_pct": 101}):
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
                              "contract_rows_long_pct": 100}]:
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
