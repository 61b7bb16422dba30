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


def _full_range_sample():
    """Every 16th member of the 512-member batched workload and its largest
    member: n spans 2^10..2^16, all three kinds and hierarchies."""
    idx = list(range(0, 512, 16))
    big = max(range(512), key=lambda i: gen.batch_spec(i)[1])
    return idx + ([big] if big not in idx else [])


def test_batch_full_size_range_equals_plain_and_oracle(pm, pmo):
    idx = _full_range_sample()
    say("building batch sample over 2^10..2^16:", len(idx))
    members = [gen.batch_member(i) for i in idx]
    ns = [m.graph.n for m in members]
    assert min(ns) < 2 ** 11 and max(ns) > 2 ** 15.9
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in members]
    inst = [(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, members)]
    say("batched", len(inst))
    res = pm.pm_map_batch(inst, workers=8)
    for i, m, x, (rc, part, job) in zip(idx, members, inst, res):
        rc_p, part_p, st_p = pm.pm_map(*x)
        assert rc == rc_p and job.j_final == st_p.j_final and job.levels == st_p.levels, i
        assert np.array_equal(host(part, m.graph.n), host(part_p, m.graph.n)), i
        # the oracle on every grid and rgg member and on the smaller R-MAT
        # members (its R-MAT maps cost about 15 s at 2^16), and on one R-MAT
        # member above 2^15
        kind = gen.batch_spec(i)[0]
        if kind != "rmat" or m.graph.n <= 25000 or i == 112:
            say("oracle", i, m.name, m.a)
            rc_h, part_h, st_h = pmo.map_graph(m.graph, m.a, m.d, m.eps, m.seed)
            assert rc == rc_h and st_h.j_final == job.j_final, i
            assert np.array_equal(host(part, m.graph.n), part_h), i


def test_server_full_size_range_alone_equals_in_mix(pm, pmo):
    """Requests of the served workload over pool graphs up to 2^20 vertices
    (its two largest, its largest R-MAT graph and seven more), with a budget of about three of the
    largest jobs at once, against the plain path alone; the oracle on the
    requests whose graph it maps in seconds."""
    spec = gen.serve_pool_spec(128)
    order = sorted(range(128), key=lambda i: -spec[i][1])
    big_rmat = next(i for i in order if spec[i][0] == "rmat")
    pick = order[:2] + [big_rmat] + [i for i in order[20::13] if i != big_rmat][:7]
    say("building pool graphs", [spec[i][1] for i in pick])
    graphs = {i: gen.instance(spec[i][0], spec[i][1], (2,), spec[i][2], spec[i][3]).graph
              for i in pick}
    assert max(g.n for g in graphs.values()) > 2 ** 19.5
    dgs = {i: pm.DeviceGraph.from_host(g) for i, g in graphs.items()}
    reqs = [(pick[r % len(pick)], a, seed)
            for r, (_, a, seed) in enumerate(gen.serve_requests(24, 128))]
    jobs = [(dgs[gi], a, (1, 10, 100), 0.03, seed) for gi, a, seed in reqs]
    alone = [pm.pm_map(*j) for j in jobs]
    budget = 3 * max(pm.pm_job_footprint(dgs[gi], a, (1, 10, 100)) for gi, a, _ in reqs)
    say("server mix", len(jobs), "budget", budget)
    with pm.PmServer(budget, workers=6) as srv:
        tickets = []
        for j in jobs:
            tickets.append(srv.submit(*j))
            time.sleep(0.002)
        for r, (t, (gi, a, seed), (rc_a, part_a, st_a)) in enumerate(zip(tickets, reqs, alone)):
            rc, part, job, lat = srv.wait(t)
            n = graphs[gi].n
            assert rc == rc_a and job.j_final == st_a.j_final, r
            assert np.array_equal(host(part, n), host(part_a, n)), r
            g = graphs[gi]
            if n <= (2 ** 16 if spec[gi][0] == "rgg" else 2 ** 15):
                say("oracle", r, spec[gi][3], a)
                rc_h, part_h, st_h = pmo.map_graph(g, a, (1, 10, 100), 0.03, seed)
                assert rc == rc_h and np.array_equal(host(part, n), part_h), r
