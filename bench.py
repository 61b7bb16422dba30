#!/usr/bin/env python3
"""Benchmark of the multilevel process-mapping hot path on one MI355X.

One step = one pm_map call (coarsening, contraction, initial partitioning,
projection and refinement at every level) on a synthetic task graph that is
already resident in HBM.  Reported value: refinement GTEPS = logical arcs
processed by refinement (iterations x arcs, summed over levels) / device
time of refinement.  The line also carries the end-to-end map time, the
roofline of the dominant kernel (label propagation phase 1, timed per launch
with start/stop events) and the CPU oracle timed on this host.

    python bench.py [--steps K] [--warmup W] [--workload rgg20]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "refinement GTEPS + end-to-end map time; batched/served vs plain at equal J"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rgg20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the mapping of one task graph runs on a single "
              "device; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2510_12196_amd as pm

    assert torch.cuda.is_available(), "bench.py needs a ROCm device"
    pm.lib()
    w = gen.get(args.workload)
    t = time.perf_counter()
    g = w.graph()
    log(f"workload {w.name}: n={g.n} arcs={g.nnz} k={w.k} built in {time.perf_counter() - t:.1f}s")
    dg = pm.DeviceGraph.from_host(g)
    torch.cuda.synchronize()

    def step(i, kernel_times):
        return pm.pm_map(dg, w.a, w.d, w.eps, 1 + i % 5, kernel_times=kernel_times)

    for i in range(args.warmup):
        rc, part, st = step(i, True)
        log(f"warmup {i}: rc={rc} J={st.j_final} levels={st.levels} total {st.total_ms:.2f} ms")
    torch.cuda.synchronize()

    stats = []
    first_part = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        rc, part, st = step(i, True)
        if i == 0:
            first_part = part
        stats.append((rc, st))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f}s")

    refine_arcs = sum(s.refine_arcs for _, s in stats)
    refine_ms = sum(s.refine_ms for _, s in stats)
    gteps = refine_arcs / (refine_ms * 1e-3) / 1e9 if refine_ms > 0 else 0.0
    map_ms = [s.total_ms for _, s in stats]
    kl = [sum(s.kernel_launches[j] for _, s in stats) for j in range(4)]
    kms = [sum(s.kernel_ms[j] for _, s in stats) for j in range(4)]
    kbytes = sum(s.kernel_bytes[0] for _, s in stats)
    achieved = kbytes / (kms[0] * 1e-3) / 1e9 if kms[0] > 0 else 0.0

    def avg(f):
        return statistics.fmean(getattr(s, f) for _, s in stats)

    s0 = stats[0][1]
    line = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {**w.describe(), "n": g.n, "arcs": g.nnz, "seeds": "1..5 cyclic"},
        "map_ms_median": round(statistics.median(map_ms), 3),
        "refine_ms_per_map": round(refine_ms / args.steps, 3),
        "phase_ms": {f: round(avg(f), 3) for f in
                     ["coarsen_ms", "contract_ms", "initial_ms", "uncoarsen_ms", "refine_ms",
                      "total_ms"]},
        "levels": s0.levels,
        "level_n": list(s0.level_n[: s0.levels]),
        "level_iterations": list(s0.level_iterations[: s0.levels]),
        "J_seed1": s0.j_final,
        "status": sorted({rc for rc, _ in stats}),
        "kernels": {name: {"launches": kl[j], "avg_us": round(kms[j] * 1e3 / kl[j], 3) if kl[j] else None}
                    for j, name in enumerate(pm.TIMED_KERNELS)},
        "roofline": {
            "kernel": "k_lp_phase1",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": round(kbytes / kl[0], 1) if kl[0] else None,
            "avg_launch_us": round(kms[0] * 1e3 / kl[0], 3) if kl[0] else None,
        },
    }

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        log("cpu baseline: oracle pm_map, seed 1, single thread")
        t = time.perf_counter()
        orc, opart, ost = oracle.map_graph(g, w.a, w.d, w.eps, 1)
        ocpu = time.perf_counter() - t
        arcs = sum(ost.level_iterations[i] * ost.level_nnz[i] for i in range(ost.levels))
        parity = bool(np.array_equal(first_part.cpu().numpy(), opart)) and orc == stats[0][0]
        line["cpu_baseline"] = {
            "value": round(arcs / ost.refine_seconds / 1e9, 5) if ost.refine_seconds > 0 else None,
            "unit": "GTEPS",
            "cores": 1,
            "kind": "oracle",
            "sample": f"one full map of {w.name} (seed 1); refinement {ost.refine_seconds:.2f}s "
                      f"of {ocpu:.2f}s total",
            "map_ms": round(ocpu * 1e3, 1),
        }
        line["parity_seed1"] = parity
        log(f"oracle: {ocpu:.2f}s, parity {parity}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
