"""Code generation of the gfx950 kernels: no kernel of the library may keep
values in private (scratch) memory or address global memory through flat
instructions.  Both are silent performance cliffs that parity tests do not
see: a by-value kernel argument written in the kernel, or a kernel grown
past the point where the compiler keeps its argument block in registers,
moves the arguments to scratch and turns every access into a flat one (the
rebalancing selection once ran 5x slower that way).  The one exception is
k_place_rejects, whose residual tables sit in LDS or in global memory behind
one pointer on purpose."""
import concurrent.futures
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_12196_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f != "prim.hip")
FLAT_ALLOWED = ("k_place_rejects",)


def _assemble(src, out):
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _per_kernel(asm):
    flat, scratch, names, cur = {}, {}, set(), None
    for line in open(asm):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            cur = m.group(1)
            names.add(cur)
            continue
        op = line.strip().split(";")[0].split()
        if not cur or not op:
            continue
        if op[0].startswith("flat_"):
            flat[cur] = flat.get(cur, 0) + 1
        elif op[0].startswith("scratch_"):
            scratch[cur] = scratch.get(cur, 0) + 1
    return flat, scratch, names


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="no hipcc")
def test_no_scratch_and_no_flat_access_in_kernels():
    with tempfile.TemporaryDirectory() as tmp:
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
            outs = list(ex.map(lambda s: _assemble(s, os.path.join(tmp, s + ".s")), SOURCES))
        bad, seen = [], set()
        for src, asm in zip(SOURCES, outs):
            flat, scratch, names = _per_kernel(asm)
            seen |= names
            for k, c in scratch.items():
                bad.append(f"{src}: {k} has {c} scratch instructions")
            for k, c in flat.items():
                if not any(a in k for a in FLAT_ALLOWED):
                    bad.append(f"{src}: {k} has {c} flat instructions")
        assert not bad, "\n".join(bad)
        # the scan saw the hot kernels
        for k in ("k_apply", "k_reb_select", "k_lp_phase1", "k_lp_phase2", "k_hem_prefer"):
            assert any(k in n for n in seen), k
