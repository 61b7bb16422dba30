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
COPY_BYTES = 512 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lp_phase1_rgg20_traffic.txt")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2510_12196_amd", "csrc", f)
                   for f in ("refine.hip", "device_util.h", "pm_internal.h")]


def source_digest():
    """Digest of the sources that define the label-propagation phase-1 kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload):
    """Measured HBM bytes per launch of k_lp_phase1 from the committed counter
    summary, if it was taken on this workload and on the current sources."""
    try:
        kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE) if ":" in line)
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("workload") != workload or kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def summarize_pmc(d):
    """Reduce rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE, KiB per dispatch)
    for k_lp_phase1 and the calibration copy kernel to bytes per launch."""
    import csv
    import glob
    sums = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r.get("Kernel_Name", "")
            ctr = r.get("Counter_Name", "")
            val = float(r.get("Counter_Value", "0") or 0)
            disp = r.get("Dispatch_Id", "")
            kind = "lp1" if "k_lp_phase1" in name else ("copy" if "copyBuffer" in name else None)
            if kind is None:
                continue
            key = (kind, ctr)
            sums.setdefault(key, {})
            sums[key][disp] = sums[key].get(disp, 0.0) + val
    out = {}
    for (kind, ctr), per in sums.items():
        if kind == "copy":  # the 512 MiB calibration copy is the largest copy dispatch
            out[(kind, ctr)] = (max(per.values()), 1)
        else:
            out[(kind, ctr)] = (sum(per.values()), len(per))
    for k, v in sorted(out.items()):
        print(k, v)
    copy_mib = COPY_BYTES / 1024.0
    res = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        if ("copy", ctr) in out and ("lp1", ctr) in out:
            ctot, cn = out[("copy", ctr)]
            ltot, ln = out[("lp1", ctr)]
            scale = copy_mib / (ctot / cn) if ctot else float("nan")
            res[ctr] = (ltot / ln) * scale * 1024.0
            print(f"{ctr}: copy reads {ctot / cn:.0f} KiB for {copy_mib:.0f} KiB -> scale "
                  f"{scale:.4f}; k_lp_phase1 {ltot / ln:.1f} KiB/launch -> {res[ctr]:.0f} B")
    if len(res) == 2:
        print(f"hbm_bytes_per_launch: {res['FETCH_SIZE'] + res['WRITE_SIZE']:.0f}")
    print(f"source_digest: {source_digest()}")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rgg20")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device-to-device copy of 512 MiB (known traffic) for "
                         "scaling hardware byte counters")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="summarise rocprofv3 --pmc counter CSVs under DIR and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
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

    if args.copy_calibration:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {COPY_BYTES} bytes read, {COPY_BYTES} bytes written")
        del src, dst

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
            "traffic": read_traffic(w.name),
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
