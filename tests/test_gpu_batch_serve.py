"""Batched and served mapping: every instance must come out exactly as the
plain per-instance pm_map (and, where the oracle is fast enough, as the
oracle), alone and in the mix."""
import sys
import time

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


@pytest.fixture(scope="module")
def members():
    say("building batch members")
    # the batched workload's distributions, at the low end of the size range
    return gen.batch_members(96, log2_lo=10.0, log2_hi=13.0)


def host(x, n):
    return x[:n].cpu().numpy()


def test_batch_equals_plain_and_oracle(pm, pmo, members):
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in members]
    say("batched", len(members))
    res = pm.pm_map_batch([(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, members)],
                          workers=8)
    for i, (m, dg, (rc, part, job)) in enumerate(zip(members, dgs, res)):
        rc_p, part_p, st_p = pm.pm_map(dg, m.a, m.d, m.eps, m.seed)
        assert rc == rc_p and job.j_final == st_p.j_final and job.levels == st_p.levels, i
        assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n)), i
        if i % 4 == 0:
            say("oracle", i, m.name, m.a)
            rc_h, part_h, st_h = pmo.map_graph(m.graph, m.a, m.d, m.eps, m.seed)
            assert rc == rc_h and np.array_equal(host(part, m.graph.n), part_h), i


def test_batch_repeated_equals_plain(pm, members):
    """Two more batched runs of every member: concurrent jobs change the
    timing of every kernel, so a result that depends on the order of device
    work shows up as a mismatch with the plain run."""
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in members]
    inst = [(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, members)]
    plain = [pm.pm_map(*x) for x in inst]
    for rep in range(2):
        say("batch repeat", rep)
        res = pm.pm_map_batch(inst, workers=8)
        for i, (m, (rc, part, job), (rc_p, part_p, st_p)) in enumerate(zip(members, res, plain)):
            assert rc == rc_p and job.j_final == st_p.j_final, (rep, i)
            assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n)), (rep, i)


def test_batch_worker_count_does_not_change_results(pm, members):
    sub = members[:24]
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in sub]
    inst = [(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, sub)]
    say("batch workers 1 vs 5")
    r1 = pm.pm_map_batch(inst, workers=1)
    r5 = pm.pm_map_batch(inst, workers=5)
    for m, a, b in zip(sub, r1, r5):
        assert a[0] == b[0] and a[2].j_final == b[2].j_final
        assert np.array_equal(host(a[1], m.graph.n), host(b[1], m.graph.n))


def test_batch_reports_bad_instances(pm, members):
    say("batch with an invalid hierarchy")
    m = members[0]
    dg = pm.DeviceGraph.from_host(m.graph)
    res = pm.pm_map_batch([(dg, m.a, m.d, m.eps, 1), (dg, (1 << 14,), (1,), 0.03, 1)], workers=2)
    assert res[0][0] >= 0 and res[1][0] == pm.PM_EOVERFLOW


def test_server_alone_equals_in_mix(pm, members):
    sub = members[:40]
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in sub]
    # budget for about three of the larger jobs at once: admission must queue
    fps = [pm.pm_job_footprint(dg, m.a, m.d) for dg, m in zip(dgs, sub)]
    budget = 3 * max(fps)
    say("server mix", len(sub), "budget", budget)
    alone = [pm.pm_map(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, sub)]
    with pm.PmServer(budget, workers=6) as srv:
        tickets = []
        for dg, m in zip(dgs, sub):
            tickets.append(srv.submit(dg, m.a, m.d, m.eps, m.seed))
            time.sleep(0.001)
        for t, m, (rc_a, part_a, st_a) in zip(tickets, sub, alone):
            rc, part, job, lat = srv.wait(t)
            assert rc == rc_a and job.j_final == st_a.j_final
            assert np.array_equal(host(part, m.graph.n), host(part_a, m.graph.n))
            assert lat > 0.0


def test_server_rejects_jobs_above_budget(pm, members):
    m = members[0]
    dg = pm.DeviceGraph.from_host(m.graph)
    fp = pm.pm_job_footprint(dg, m.a, m.d)
    with pm.PmServer(fp - 1, workers=1) as srv:
        with pytest.raises(pm.PmError) as e:
            srv.submit(dg, m.a, m.d, m.eps, 1)
        assert e.value.code == pm.PM_ENOMEM
    with pm.PmServer(fp, workers=2) as srv:
        t = srv.submit(dg, m.a, m.d, m.eps, 1)
        rc, part, job, lat = srv.wait(t)
        assert rc >= 0
        # wait() released the ticket
        with pytest.raises(pm.PmError):
            srv.poll(t)
