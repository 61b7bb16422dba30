"""Launch-parameter autotuner.

Times candidate launch parameters (pm_tuning: lane-group tile depth, the
size from which a level uses the one-wave-per-vertex class, the level sizes
from which matching and rebalancing tile only their active vertices) and the
batch worker count on a sample of instances, and keeps the fastest.  None of
these parameters changes a result, so the tuner only trades time.
"""
import itertools
import time

from . import get_tuning, pm_map_batch, set_tuning


def candidates():
    """The searched settings: the library defaults first."""
    out = []
    for v, wmin, (hmin, rmin) in itertools.product(
            (1, 2), (8192, 1024), ((1 << 18, 1 << 19), (1 << 13, 1 << 13))):
        out.append({"group_v": v, "wave_min_count": wmin,
                    "hem_compact_min_n": hmin, "reb_compact_min_n": rmin})
    return out


def sample_of(instances, count):
    """Every len/count-th instance after sorting by size: the sample spans the
    size range of the batch."""
    order = sorted(range(len(instances)), key=lambda i: instances[i][0].nnz + instances[i][0].n)
    if count >= len(order):
        return [instances[i] for i in order]
    step = len(order) / count
    return [instances[order[int(j * step)]] for j in range(count)]


def autotune_batch(instances, sample=64, workers=(4, 8, 16), cands=None, sync=None):
    """instances: list of (DeviceGraph, a, d, eps, seed).  Times pm_map_batch
    on a sample for every (tuning, workers) pair, sets the fastest tuning and
    returns (tuning, workers, table): every launch parameter now in effect,
    the worker count, and every timing."""
    cands = cands or candidates()
    sub = sample_of(instances, sample)
    old = get_tuning()
    table = []
    best = None
    try:
        for c in cands:
            set_tuning(**c)
            pm_map_batch(sub[: min(8, len(sub))], workers=max(workers))  # warm-up
            for w in workers:
                if sync:
                    sync()
                t0 = time.perf_counter()
                pm_map_batch(sub, workers=w)
                if sync:
                    sync()
                dt = time.perf_counter() - t0
                table.append({**c, "workers": w, "s": round(dt, 4)})
                if best is None or dt < best[0]:
                    best = (dt, c, w)
    finally:
        set_tuning(**old)
    set_tuning(**best[1])
    return get_tuning(), best[2], table
