import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size workloads")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def graph_from_fixture(fx):
    import gen

    n = fx["n"]
    e = np.array(fx["edges"], dtype=np.int64)
    vw = fx.get("vwgt", [1] * n)
    return gen.from_edges(n, e[:, 0], e[:, 1], e[:, 2], vw)


def ip_fixture_graph(fx):
    """Graph of an initial-partitioning fixture: a path, a star (centre 0) or
    two interleaved paths (evens and odds), unit weights."""
    import gen

    n = fx["n"]
    if "star" in fx["what"]:
        u = np.zeros(n - 1, np.int64)
        v = np.arange(1, n)
    elif "interleaved" in fx["what"]:
        u = np.concatenate([np.arange(0, n - 2, 2), np.arange(1, n - 2, 2)])
        v = u + 2
    else:
        return gen.path_graph(n)
    return gen.from_edges(n, u, v, np.ones(len(u), np.int32), np.ones(n, np.int32))


@pytest.fixture(scope="session")
def pmo():
    import oracle

    if not os.path.exists(os.path.join(ROOT, "oracle", "libpmo.so")):
        oracle.build()
    return oracle
