#!/usr/bin/env python3
"""Benchmark of the multilevel process-mapping hot path on one MI355X.

One step = one pm_map call (coarsening, contraction, initial partitioning,
projection and refinement at every level) on a synthetic task graph that is
already resident in HBM.  Reported value: refinement GTEPS = logical arcs
processed by refinement (iterations x arcs, summed over levels) / device
time of refinement.  The line also carries the end-to-end map time, per
timed kernel its launches, device time (start/stop events of every launch
inside the timed region) and algorithmic bytes (counted in a second,
untimed pass over the same seeds), the roofline of the kernel with the
largest device time, the refinement kernels' aggregate, and the CPU oracle
timed on this host.

    python bench.py [--steps K] [--warmup W] [--workload rmat22]
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
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2510_12196_amd", "csrc", f)
                   for f in ("refine.hip", "coarsen.hip", "device_util.h", "pm_internal.h",
                             "kernels.h")]
# timed kernels of the library (pm_map_stats order) and their rocprof names
KERNEL_NAMES = {"lp_phase1": "k_lp_phase1", "lp_phase2": "k_lp_phase2",
                "apply_moves": "k_apply", "hem_prefer": "k_hem_prefer",
                "reb_select": "k_reb_select"}
REFINEMENT = ("lp_phase1", "lp_phase2", "apply_moves", "reb_select")


def source_digest():
    """Digest of the sources that define the timed kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel, workload):
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")


def read_traffic(kernel, workload):
    """Measured HBM bytes per launch of a kernel from the committed counter
    summary, if it was taken on this workload and on the current sources."""
    try:
        kv = dict(line.split(":", 1) for line in open(traffic_file(kernel, workload))
                  if ":" in line)
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("workload") != workload or kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def summarize_pmc(d, kernel):
    """Reduce rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE, KiB per dispatch)
    for `kernel` and the calibration copy kernel to bytes per launch; SQ_*
    counters of `kernel` are reported per launch, with the wave-cycle shares
    of waiting and of VALU and LDS issue."""
    import csv
    import glob
    import re
    sums = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r.get("Kernel_Name", "")
            ctr = r.get("Counter_Name", "")
            val = float(r.get("Counter_Value", "0") or 0)
            disp = r.get("Dispatch_Id", "")
            kind = ("k" if re.search(r"pm::%s(<|\()" % kernel, name) else
                    ("copy" if "neg_kernel" in name else None))
            if kind is None:
                continue
            key = (kind, ctr)
            sums.setdefault(key, {})
            sums[key][disp] = sums[key].get(disp, 0.0) + val
    out = {}
    for (kind, ctr), per in sums.items():
        if kind == "copy":  # the 512 MiB calibration pass is the largest such dispatch
            out[(kind, ctr)] = (max(per.values()), 1)
        else:
            out[(kind, ctr)] = (sum(per.values()), len(per))
    copy_mib = COPY_BYTES / 1024.0
    res = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        if ("copy", ctr) in out and ("k", ctr) in out:
            ctot, cn = out[("copy", ctr)]
            ltot, ln = out[("k", ctr)]
            scale = copy_mib / (ctot / cn) if ctot else float("nan")
            res[ctr] = (ltot / ln) * scale * 1024.0
            print(f"{ctr}: copy reads {ctot / cn:.0f} KiB for {copy_mib:.0f} KiB -> scale "
                  f"{scale:.4f}; {kernel} {ltot / ln:.1f} KiB/launch over {ln} launches -> "
                  f"{res[ctr]:.0f} B")
    if len(res) == 2:
        print(f"hbm_bytes_per_launch: {res['FETCH_SIZE'] + res['WRITE_SIZE']:.0f}")
    # shader-sequencer counters (summed over the SEs): where the waves' time goes
    sq = {ctr: out[("k", ctr)] for (kind, ctr) in out if kind == "k" and ctr.startswith("SQ_")}
    for ctr in sorted(sq):
        tot, n = sq[ctr]
        print(f"{ctr}: {tot / n:.4g} per launch over {n} launches")
    if "SQ_WAVE_CYCLES" in sq and sq["SQ_WAVE_CYCLES"][0] > 0:
        wc = sq["SQ_WAVE_CYCLES"][0]
        for ctr in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
                    "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_MISC"):
            if ctr in sq:
                print(f"{ctr} / SQ_WAVE_CYCLES: {sq[ctr][0] / wc:.3f}")
    print(f"source_digest: {source_digest()}")


def _phase_share(stats):
    tot = sum(s.total_ms for _, s in stats)
    if tot <= 0:
        return None
    out = {}
    for f, name in (("coarsen_ms", "coarsening"), ("contract_ms", "contraction"),
                    ("initial_ms", "initial_partitioning"), ("uncoarsen_ms", "uncontraction"),
                    ("refine_ms", "refine_and_rebalance")):
        out[name] = round(100.0 * sum(getattr(s, f) for _, s in stats) / tot, 2)
    out["misc"] = round(100.0 - sum(out.values()), 2)
    return out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-times", choices=("pass", "inline"), default="pass",
                    help="time the kernels' launches in a pass after the timed steps (pass) or "
                         "inside them (inline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise pass over 512 MiB (known traffic: 512 MiB "
                         "read, 512 MiB written) for scaling hardware byte counters")
    ap.add_argument("--serve-pool", type=int, default=128,
                    help="resident graphs of the served workload (serveN)")
    ap.add_argument("--hm", action="store_true",
                    help="time hierarchical multisection (GPU-HM) on the workload beside the "
                         "multilevel mapping")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="summarise rocprofv3 --pmc counter CSVs under DIR and exit")
    ap.add_argument("--pmc-kernel", default="k_lp_phase1",
                    help="kernel whose counters --summarize-pmc reduces")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.pmc_kernel)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the mapping of one task graph runs on a single "
              "device; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the served workload's graphs are built in worker processes, before
    # this process touches the GPU
    pool_graphs = None
    if args.workload.startswith("serve"):
        pool_graphs = build_serve_pool(int(args.workload[5:] or 64), args.serve_pool)

    import numpy as np
    import torch

    import gen
    import paper_2510_12196_amd as pm

    assert torch.cuda.is_available(), "bench.py needs a ROCm device"
    pm.lib()
    if args.workload.startswith("batch"):
        return bench_batch(args, int(args.workload[5:] or 512))
    if args.workload.startswith("serve"):
        return bench_serve(args, int(args.workload[5:] or 64), pool_graphs)
    w = gen.get(args.workload)
    t = time.perf_counter()
    g = w.graph()
    log(f"workload {w.name}: n={g.n} arcs={g.nnz} k={w.k} built in {time.perf_counter() - t:.1f}s")
    dg = pm.DeviceGraph.from_host(g)
    torch.cuda.synchronize()
    if args.hm:
        return bench_hm(args, w, g, dg)

    def step(i, kernel_times, kernel_counts=False):
        return pm.pm_map(dg, w.a, w.d, w.eps, 1 + i % 5, kernel_times=kernel_times,
                         kernel_counts=kernel_counts)

    if args.copy_calibration:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # an elementwise kernel: reads and writes COPY_BYTES once
        torch.cuda.synchronize()
        log(f"copy calibration: {COPY_BYTES} bytes read, {COPY_BYTES} bytes written")
        del src, dst

    inline = args.kernel_times == "inline"
    for i in range(args.warmup):
        rc, part, st = step(i, inline)
        log(f"warmup {i}: rc={rc} J={st.j_final} levels={st.levels} total {st.total_ms:.2f} ms")
    torch.cuda.synchronize()

    stats = []
    first_part = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        rc, part, st = step(i, inline)
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
    nk = len(pm.TIMED_KERNELS)
    # Device time of every launch of the timed kernels (start/stop events on
    # the launch's stream): inside the timed steps (--kernel-times inline), or
    # in a pass over the same seeds right after them (pass; the default,
    # since recording events around every launch adds host work that slows
    # the latency-bound small levels of the map being timed).
    timed = stats if inline else [(None, step(i, True)[2]) for i in range(args.steps)]
    assert [s.j_final for _, s in timed] == [s.j_final for _, s in stats]
    kl = [sum(s.kernel_launches[j] for _, s in timed) for j in range(nk)]
    kms = [sum(s.kernel_ms[j] for _, s in timed) for j in range(nk)]

    # Units of work of the same launches: the timed steps again (same seeds,
    # hence the same launches), outside the timed region, with the library's
    # counting launches beside the timed kernels.
    counted = [step(i, False, True)[2] for i in range(args.steps)]
    assert [s.j_final for s in counted] == [s.j_final for _, s in stats]
    kbytes = [sum(s.kernel_bytes[j] for s in counted) for j in range(nk)]
    kunits = [[sum(s.kernel_units[j][u] for s in counted) for u in range(3)] for j in range(nk)]

    def avg(f):
        return statistics.fmean(getattr(s, f) for _, s in stats)

    kernels = {}
    for j, name in enumerate(pm.TIMED_KERNELS):
        if not kl[j]:
            continue
        gbs = kbytes[j] / (kms[j] * 1e-3) / 1e9 if kms[j] > 0 else 0.0
        kernels[name] = {"kernel": KERNEL_NAMES[name], "launches": kl[j],
                         "total_ms": round(kms[j], 3), "avg_us": round(kms[j] * 1e3 / kl[j], 3),
                         "bytes_per_launch": round(kbytes[j] / kl[j], 1),
                         "units_per_launch": [round(x / kl[j], 1) for x in kunits[j]],
                         "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": read_traffic(KERNEL_NAMES[name], w.name)}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    kd = kernels[dom]
    rb = sum(kbytes[j] for j, n in enumerate(pm.TIMED_KERNELS) if n in REFINEMENT)
    rt = sum(kms[j] for j, n in enumerate(pm.TIMED_KERNELS) if n in REFINEMENT)
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
        # shares of the map time per phase, as in the paper's Table 2
        # (misc: everything outside the five phases)
        "phase_share": _phase_share(stats),
        "levels": s0.levels,
        "level_n": list(s0.level_n[: s0.levels]),
        "level_iterations": list(s0.level_iterations[: s0.levels]),
        "J_seed1": s0.j_final,
        "status": sorted({rc for rc, _ in stats}),
        "kernels": kernels,
        "kernel_times": args.kernel_times,
        # the timed kernel with the largest device time over the timed steps
        "roofline": {
            "kernel": kd["kernel"],
            "bound": "hbm",
            "achieved": kd["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": kd["frac"],
            "traffic": read_traffic(kd["kernel"], w.name),
            "bytes_per_launch": kd["bytes_per_launch"],
            "avg_launch_us": kd["avg_us"],
        },
        # the refinement kernels together: algorithmic bytes over their time
        "refinement_roofline": {
            "kernels": [KERNEL_NAMES[n] for n in REFINEMENT],
            "achieved": round(rb / (rt * 1e-3) / 1e9, 1) if rt > 0 else None,
            "frac": round(rb / (rt * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if rt > 0 else None,
            "kernel_ms_per_map": round(rt / args.steps, 3),
        },
    }

    if not args.no_cpu_baseline:
        if w.name == "rmat22":
            line["cpu_baseline"] = cpu_baseline_rounds(w, g, dg)
        else:
            import oracle
            oracle.build(force=False)
            log("cpu baseline: oracle pm_map, seed 1, one pinned thread")
            with pinned_to_one_cpu() as cpu:
                t = time.perf_counter()
                orc, opart, ost = oracle.map_graph(g, w.a, w.d, w.eps, 1)
                ocpu = time.perf_counter() - t
            arcs = sum(ost.level_iterations[i] * ost.level_nnz[i] for i in range(ost.levels))
            parity = bool(np.array_equal(first_part.cpu().numpy(), opart)) and orc == stats[0][0]
            line["cpu_baseline"] = {
                "value": round(arcs / ost.refine_seconds / 1e9, 5) if ost.refine_seconds > 0
                else None,
                "unit": "GTEPS",
                "cores": 1,
                "kind": "oracle",
                "sample": f"one full map of {w.name} (seed 1); refinement "
                          f"{ost.refine_seconds:.2f}s of {ocpu:.2f}s total",
                "map_ms": round(ocpu * 1e3, 1),
                "parity_with_gpu": parity,
                **host_info(cpu),
            }
            log(f"oracle: {ocpu:.2f}s, parity {parity}")
    print(json.dumps(line), flush=True)


def host_info(cpu):
    """The host the CPU baseline ran on: the core it was pinned to, the
    logical CPU count and the CPU model."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"pinned_cpu": cpu, "nproc": os.cpu_count(), "cpu_model": model}


class pinned_to_one_cpu:
    """Runs the block with the calling thread bound to one CPU of the
    process's affinity set (the oracle is single-threaded C called through
    ctypes, so it runs on this thread); restores the affinity afterwards."""

    def __enter__(self):
        self.old = os.sched_getaffinity(0)
        cpu = sorted(self.old)[0]
        os.sched_setaffinity(0, {cpu})
        return cpu

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.old)
        return False


def cpu_baseline_rounds(w, g, dg, reps=3):
    """Oracle baseline on a bounded sample of the R-MAT workload: `reps` weak
    and `reps` strong rebalancing rounds (Algorithm 5) over the whole
    level-0 graph, each from a mapping where one block holds a tenth of the
    vertices, on one pinned core.  Every round is also run on the GPU and
    compared element by element.  (The oracle's label-propagation round
    evaluates equation (1) for every pair of neighbour blocks of a vertex and
    takes minutes on this graph from a random mapping, so it is left out.)"""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_2510_12196_amd as pm
    oracle.build(force=False)
    total = int(g.vwgt.sum())
    lm = oracle.lmax(total, w.k, w.eps)
    sg = oracle.sigma(lm, total, w.k)
    secs = 0.0
    rounds = 0
    equal = True
    with pinned_to_one_cpu() as cpu:
        for r in range(reps):
            part = gen.random_mapping(g.n, w.k, 0xB0 + r)
            part[: g.n // 10] = 1 + r
            for strong in (False, True):
                log(f"cpu baseline: oracle {'strong' if strong else 'weak'} round {r}")
                t = time.perf_counter()
                exp_part, exp_moved = oracle.rebalance(g, w.k, part, strong, lm, sg, 7, 0, 1 + r)
                secs += time.perf_counter() - t
                rounds += 1
                pd = torch.from_numpy(part.copy()).cuda()
                mv = pm.pm_rebalance(dg, w.a, w.d, pd, strong, lm, sg, 7, 0, 1 + r)
                equal &= bool(np.array_equal(mv.cpu().numpy(), exp_moved) and
                              np.array_equal(pd.cpu().numpy(), exp_part))
    log(f"oracle: {rounds} rounds in {secs:.2f}s, equal to the GPU: {equal}")
    return {
        "value": round(rounds * g.nnz / secs / 1e9, 5),
        "unit": "GTEPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{reps} weak + {reps} strong rebalancing rounds over the whole level-0 graph "
                  f"of {w.name} ({g.nnz} arcs each) in {secs:.2f}s; the oracle's "
                  "label-propagation round is left out (minutes on this graph)",
        "parity_with_gpu": equal,
        **host_info(cpu),
    }


def bench_hm(args, w, g, dg):
    """Hierarchical multisection (Section 4.1, the GPU-HM variant): every
    level's subgraphs partitioned by the multilevel mapper with (a_i), d = 1
    and the adaptive imbalance of equation (2).  Timed beside the multilevel
    mapping of the same graph and seeds; J of both under the full hierarchy."""
    import statistics as stt

    import numpy as np
    import torch

    import paper_2510_12196_amd as pm
    for i in range(args.warmup):
        rc, part, j, calls = pm.pm_map_hm(dg, w.a, w.d, w.eps, 1 + i % 5)
        log(f"warmup {i}: rc={rc} J={j} calls={calls}")
    torch.cuda.synchronize()
    hm_ms, hm_j, im_ms, im_j, rcs = [], [], [], [], set()
    first = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        t = time.perf_counter()
        rc, part, j, calls = pm.pm_map_hm(dg, w.a, w.d, w.eps, 1 + i % 5)
        torch.cuda.synchronize()
        hm_ms.append((time.perf_counter() - t) * 1e3)
        hm_j.append(j)
        rcs.add(rc)
        if i == 0:
            first = (rc, part.cpu().numpy())
    wall = time.perf_counter() - t0
    for i in range(args.steps):
        t = time.perf_counter()
        rc, part, st = pm.pm_map(dg, w.a, w.d, w.eps, 1 + i % 5)
        torch.cuda.synchronize()
        im_ms.append((time.perf_counter() - t) * 1e3)
        im_j.append(st.j_final)
    log(f"hm {stt.median(hm_ms):.2f} ms, multilevel {stt.median(im_ms):.2f} ms")
    line = {
        "metric": "hierarchical multisection time", "value": round(stt.median(hm_ms), 3),
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {**w.describe(), "n": g.n, "arcs": g.nnz, "seeds": "1..5 cyclic",
                   "partitioner": "multilevel mapper, (a_i), d=1"},
        "hm_partitioning_calls": calls,
        "hm_J_mean": round(stt.fmean(hm_j), 1), "multilevel_J_mean": round(stt.fmean(im_j), 1),
        "J_ratio_hm_over_multilevel": round(stt.fmean(hm_j) / stt.fmean(im_j), 4),
        "multilevel_ms_median": round(stt.median(im_ms), 3),
        "status": sorted(rcs),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        log("cpu baseline: oracle hm, seed 1, one pinned thread")
        with pinned_to_one_cpu() as cpu:
            t = time.perf_counter()
            orc, opart = oracle.hm(g, w.a, w.eps, 1)
            ocpu = time.perf_counter() - t
        line["cpu_baseline"] = {"value": round(ocpu * 1e3, 1), "unit": "ms", "cores": 1,
                                "kind": "oracle", "sample": f"one hm of {w.name} (seed 1)",
                                **host_info(cpu)}
        line["parity_seed1"] = bool(orc == first[0] and np.array_equal(first[1], opart))
        log(f"oracle: {ocpu:.2f}s, parity {line['parity_seed1']}")
    print(json.dumps(line), flush=True)


def _hash_part(part, n):
    import hashlib
    return hashlib.sha256(part[:n].cpu().numpy().tobytes()).hexdigest()[:16]


def bench_batch(args, count):
    """Batched workload: `count` instances (grid / rgg / rmat, n = 2^U(10,16),
    hierarchy 2:2:4 / 4:4:8 / 4:8:8).  Plain = one pm_map after the other on
    one stream; batched = pm_map_batch.  Both must give the same mapping."""
    import torch

    import gen
    import paper_2510_12196_amd as pm
    t = time.perf_counter()
    members = gen.batch_members(count)
    dgs = [pm.DeviceGraph.from_host(m.graph) for m in members]
    torch.cuda.synchronize()
    n_tot = sum(m.graph.n for m in members)
    arcs = sum(m.graph.nnz for m in members)
    log(f"{count} instances, {n_tot} vertices, {arcs} arcs, built in {time.perf_counter() - t:.1f}s")
    inst = [(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, members)]
    pm.pm_map_batch(inst[: min(16, count)], workers=8)  # warm-up
    torch.cuda.synchronize()
    # launch parameters and worker count picked on a sample (not timed)
    from paper_2510_12196_amd.autotune import autotune_batch
    t0 = time.perf_counter()
    tuning, best, table = autotune_batch(inst, sample=min(64, count), workers=(4, 8, 16),
                                         sync=torch.cuda.synchronize)
    t_tune = time.perf_counter() - t0
    log(f"autotune: {tuning}, {best} workers ({t_tune:.1f}s, {len(table)} timings)")
    t0 = time.perf_counter()
    plain = [pm.pm_map(dg, m.a, m.d, m.eps, m.seed) for dg, m in zip(dgs, members)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    res = {}
    for workers in sorted({4, 8, 16, best}):
        t0 = time.perf_counter()
        out = pm.pm_map_batch(inst, workers=workers)
        torch.cuda.synchronize()
        res[workers] = (time.perf_counter() - t0, out)
        log(f"batched, {workers} workers: {res[workers][0]:.3f}s")
    t_b, out = res[best]
    equal = all(o[0] == p[0] and o[2].j_final == p[2].j_final and
                _hash_part(o[1], m.graph.n) == _hash_part(p[1], m.graph.n)
                for o, p, m in zip(out, plain, members))
    line = {
        "metric": METRIC, "value": round(count / t_b, 2), "unit": "maps/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(t_b * 1e3, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch{count}", "instances": count, "vertices": n_tot,
                   "arcs": arcs, "hierarchies": "2:2:4|4:4:8|4:8:8", "distance": "1:10:100",
                   "eps": 0.03, "workers": best},
        "plain_maps_per_s": round(count / t_plain, 2), "plain_s": round(t_plain, 3),
        "batched_s": {str(k): round(v[0], 3) for k, v in res.items()},
        "speedup_vs_plain": round(t_plain / t_b, 2), "identical_to_plain": bool(equal),
        "tuning": tuning, "autotune_s": round(t_tune, 2),
        "autotune_sample": min(64, count), "autotune_table": table,
    }
    print(json.dumps(line), flush=True)


def _pool_graph(spec):
    import gen
    kind, n, gseed, name = spec
    return gen.instance(kind, n, (2,), gseed, name).graph


def build_serve_pool(count, pool):
    """The resident graphs of the served workload, built in worker processes
    (before anything touches the GPU)."""
    import concurrent.futures
    import multiprocessing

    import gen
    spec = gen.serve_pool_spec(min(count, pool))
    t = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1, len(spec)))
    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        graphs = list(ex.map(_pool_graph, spec, chunksize=1))
    log(f"{len(graphs)} pool graphs ({sum(g.n for g in graphs)} vertices, "
        f"{sum(g.nnz for g in graphs)} arcs) built in {time.perf_counter() - t:.1f}s "
        f"with {workers} processes")
    return graphs


def bench_serve(args, count, graphs):
    """Served workload: a Poisson stream of `count` requests over a pool of
    resident graphs (rgg / rmat, n = 2^U(12,20)); each request maps one pool
    graph, drawn uniformly, onto hierarchy 4:8:8 or 4:16:8 with its own seed.
    The stream is submitted at 0.5x and 0.9x of the plain path's capacity;
    latency = submission to completion.  The plain comparison is the same
    stream through a single-worker server (FIFO, one request on the device at
    a time)."""
    import threading

    import numpy as np
    import torch

    import gen
    import paper_2510_12196_amd as pm
    reqs = gen.serve_requests(count, len(graphs))
    dgs = [pm.DeviceGraph.from_host(g) for g in graphs]
    torch.cuda.synchronize()
    eps = 0.03
    jobs = [(dgs[gi], a, gen.workloads.D3, eps, seed) for gi, a, seed in reqs]
    nv = [graphs[gi].n for gi, _, _ in reqs]
    # plain capacity: one request after the other
    for j in jobs[:4]:
        pm.pm_map(*j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [pm.pm_map(*j) for j in jobs]
    torch.cuda.synchronize()
    cap = count / (time.perf_counter() - t0)
    log(f"plain: {count} requests at {cap:.1f} maps/s")
    budget = 64 << 30

    def run(qps, workers):
        arrivals = gen.serve_arrivals(count, qps)
        lat = [0.0] * count
        outs = [None] * count
        with pm.PmServer(budget, workers=workers) as srv:
            tickets = [None] * count
            t_start = time.perf_counter()

            def submitter():
                for i, j in enumerate(jobs):
                    delay = t_start + arrivals[i] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                    tickets[i] = srv.submit(*j)
            th = threading.Thread(target=submitter)
            th.start()
            th.join()
            for i in range(count):
                rc, part, job, l_ms = srv.wait(tickets[i])
                lat[i] = l_ms
                outs[i] = (rc, job.j_final, _hash_part(part, nv[i]))
            t_end = time.perf_counter()
        return {"qps": round(qps, 3), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "throughput_maps_s": round(count / (t_end - t_start), 3)}, outs

    ref = [(p[0], p[2].j_final, _hash_part(p[1], n)) for p, n in zip(plain, nv)]
    results = {}
    identical = True
    for frac in (0.5, 0.9):
        served, o1 = run(frac * cap, 8)
        log(f"load {frac}: served {served}")
        fifo, o2 = run(frac * cap, 1)
        identical &= (o1 == ref) and (o2 == ref)
        results[str(frac)] = {"served": served, "plain_fifo": fifo}
        log(f"load {frac}: plain {fifo}")
    s09 = results["0.9"]["served"]
    line = {
        "metric": METRIC, "value": s09["p99_ms"], "unit": "ms p99 latency at 0.9x plain capacity",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": s09["p50_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"serve{count}", "requests": count, "pool_graphs": len(graphs),
                   "pool_vertices": sum(g.n for g in graphs),
                   "sizes": "n = 2^U(12,20)", "kinds": "rgg|rmat", "hierarchies": "4:8:8|4:16:8",
                   "eps": eps, "workers": 8, "hbm_budget_bytes": budget},
        "plain_capacity_maps_s": round(cap, 3), "loads": results,
        "identical_to_plain": bool(identical),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
