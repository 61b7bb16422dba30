"""Writes the expected results of full-size mappings, computed by the CPU
oracle only (no GPU code is imported).

    python tests/golden/make_fullsize_golden.py rmat22 1

writes tests/golden/<workload>_seed<seed>.json: the input's identity (sizes
and SHA-256 of its CSR arrays), the oracle's status, J, L_max, the graph
sizes, refinement loop bodies and matching rounds of every level, the SHA-256
of the final mapping (int32, little endian), its block weights and every
4096th entry of it.  The oracle is single-threaded: rmat22 takes tens of
minutes.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_identity(g) -> dict:
    return {"n": int(g.n), "nnz": int(g.nnz), "xadj": sha(g.xadj.astype("<i8")),
            "adjncy": sha(g.adjncy.astype("<i4")), "adjwgt": sha(g.adjwgt.astype("<i4")),
            "vwgt": sha(g.vwgt.astype("<i4"))}


def main(name: str, seed: int) -> None:
    w = gen.get(name)
    t0 = time.time()
    g = w.graph()
    print(f"{name}: n={g.n} nnz={g.nnz} built in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    rc, part, st = oracle.map_graph(g, w.a, w.d, w.eps, seed)
    secs = time.time() - t0
    L = st.levels
    k = int(np.prod(w.a))
    out = {
        "what": f"Oracle result of the full multilevel map of {name} (hierarchy "
                f"{':'.join(map(str, w.a))}, d = {':'.join(map(str, w.d))}, eps = {w.eps}), "
                f"method seed {seed}; written by tests/golden/make_fullsize_golden.py, which "
                "calls only oracle/.",
        "workload": name, "seed": seed, "a": list(w.a), "d": list(w.d), "eps": w.eps,
        "graph": graph_identity(g),
        "status": rc, "j_final": int(st.j_final), "lmax": int(st.lmax),
        "feasible": int(st.feasible), "levels": L,
        "level_n": [int(x) for x in st.level_n[:L]],
        "level_nnz": [int(x) for x in st.level_nnz[:L]],
        "level_iterations": [int(x) for x in st.level_iterations[:L]],
        "level_hem_rounds": [int(x) for x in st.level_hem_rounds[:L]],
        "part_sha256": sha(part.astype("<i4")),
        "block_weights": [int(x) for x in np.bincount(part, weights=g.vwgt, minlength=k)
                          .astype(np.int64)],
        "part_every_4096": [int(x) for x in part[::4096]],
        "oracle_seconds": round(secs, 1),
    }
    path = os.path.join(HERE, f"{name}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {path}: J={out['j_final']} levels={L} in {secs:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 1)
