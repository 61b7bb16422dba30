"""The recipes of the batched and served workloads (no graph is built here):
every member derives from (base seed, index) alone, sizes and choices stay
in the stated ranges and sets, and the arrival process has the requested
rate."""
import math

import numpy as np

import gen
from gen import workloads as wl


def test_batch_spec_is_a_function_of_seed_and_index():
    a = [gen.batch_spec(i) for i in range(64)]
    b = [gen.batch_spec(i) for i in reversed(range(64))][::-1]
    assert a == b
    assert gen.batch_spec(3, base_seed=0xC4) != gen.batch_spec(3, base_seed=0xC5)


def test_batch512_spans_the_stated_sizes_kinds_and_hierarchies():
    specs = [gen.batch_spec(i) for i in range(512)]
    ns = np.array([n for _, n, _, _, _ in specs])
    assert ns.min() >= 2 ** 10 and ns.max() < 2 ** 16
    # log2 n is uniform on [10, 16): every unit interval is populated
    assert set(np.floor(np.log2(ns)).astype(int)) == set(range(10, 16))
    kinds = [k for k, _, _, _, _ in specs]
    for k in ("grid", "rgg", "rmat"):
        assert 512 / 3 * 0.75 < kinds.count(k) < 512 / 3 * 1.25
    assert {tuple(a) for _, _, a, _, _ in specs} == set(map(tuple, wl.BATCH_HIERARCHIES))
    assert {s for _, _, _, _, s in specs} == {1, 2, 3, 4, 5}


def test_serve_pool_and_requests():
    pool = gen.serve_pool_spec(128)
    assert len(pool) == 128 and pool == gen.serve_pool_spec(128)
    ns = np.array([n for _, n, _, _ in pool])
    assert ns.min() >= 2 ** 12 and ns.max() < 2 ** 20
    assert {k for k, _, _, _ in pool} == {"rgg", "rmat"}
    assert all(name == f"{k}{n}" for k, n, _, name in pool)
    reqs = gen.serve_requests(1000, 128)
    assert reqs == gen.serve_requests(1000, 128)
    assert all(0 <= g < 128 for g, _, _ in reqs)
    assert {a for _, a, _ in reqs} == set(wl.SERVE_HIERARCHIES)
    assert {s for _, _, s in reqs} == {1, 2, 3, 4, 5}
    # the requests cover most of the pool
    assert len({g for g, _, _ in reqs}) > 120


def test_serve_arrivals_have_the_requested_rate():
    qps = 50.0
    t = np.array(wl.serve_arrivals(2000, qps))
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert (gaps > 0).all()
    # exponential gaps: mean 1/qps, standard error 1/(qps sqrt(n))
    assert abs(gaps.mean() - 1 / qps) < 4 / (qps * math.sqrt(len(gaps)))
    # the same arrivals at another rate are a rescaling of these
    t2 = np.array(wl.serve_arrivals(2000, 2 * qps))
    assert np.allclose(t2, t / 2)
