"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/pm.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pm.h")
LIB = os.path.join(ROOT, "paper_2510_12196_amd", "libpm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_entry_points():
    names = declared_functions()
    for required in ["pm_comm_cost", "pm_refine", "pm_map", "pm_lp_round", "pm_rebalance",
                     "pm_hem", "pm_contract", "pm_initial_partition", "pm_block_weights",
                     "pm_strerror", "pm_version", "pm_release", "pm_map_batch",
                     "pm_job_footprint", "pm_server_create", "pm_server_submit",
                     "pm_server_poll", "pm_server_wait", "pm_server_destroy"]:
        assert required in names


@pytest.fixture(scope="module")
def libpm():
    if not os.path.exists(LIB):
        import paper_2510_12196_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(libpm):
    missing = [n for n in declared_functions() if not hasattr(libpm, n)]
    assert not missing, missing


def test_strerror_and_version_need_no_device(libpm):
    libpm.pm_strerror.restype = ctypes.c_char_p
    libpm.pm_version.restype = ctypes.c_char_p
    assert libpm.pm_strerror(0) == b"ok"
    assert b"invalid" in libpm.pm_strerror(-1)
    assert libpm.pm_strerror(12345) == b"unknown error"
    assert b"gfx950" in libpm.pm_version()


def test_struct_layouts_match_header():
    import paper_2510_12196_amd as pm
    # pm_graph: int32 n (padded), int64 nnz, four pointers
    assert ctypes.sizeof(pm.PmGraph) == 8 + 8 + 4 * 8
    assert ctypes.sizeof(pm.PmHierarchy) == 4 + 8 * 4 + 8 * 4
    assert ctypes.sizeof(pm.PmRefineStats) == 4 * 8 + 6 * 4 + 8 + 8
    assert pm.PmMapStats.kernel_units.offset == ctypes.sizeof(pm.PmMapStats) - 5 * 3 * 8
    assert pm.PmMapStats.kernel_bytes.offset == pm.PmMapStats.kernel_units.offset - 5 * 8
    assert pm.PmMapStats.refine_arcs.offset + 8 == pm.PmMapStats.kernel_launches.offset
    # pm_map_job: graph 48, hierarchy 68 (+4 padding), eps, seed, part, 2 x int32, j, ms
    assert ctypes.sizeof(pm.PmMapJob) == 168 and pm.PmMapJob.eps.offset == 120
    assert ctypes.sizeof(pm.PmOptions) == 16


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2510_12196_amd as pm
    monkeypatch.setattr(pm, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(pm, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pm.lib()


def test_tuning_struct_layout():
    import paper_2510_12196_amd as pm
    assert ctypes.sizeof(pm.PmTuning) == 32


def test_tuning_host_logic_without_gpu():
    """Launch parameters are host state: defaults, refusal of out-of-range
    values (nothing changed), and a round trip, all without a device."""
    import paper_2510_12196_amd as pm
    pm.lib()
    before = pm.get_tuning()
    try:
        for bad in ({"group_v": 0}, {"wave_min_count": 0}, {"contract_rows_min_nnz": 0},
                    {"contract_rows_long_pct": -1}, {"contract_rows_long_pct": 101},
                    {"lp_cache": 2}, {"lp_cache": -1}, {"graph_bodies": 2}):
            with pytest.raises(pm.PmError) as e:
                pm.set_tuning(**bad)
            assert e.value.code == pm.PM_EINVAL and pm.get_tuning() == before
        pm.set_tuning(contract_rows_long_pct=0, contract_rows_min_nnz=5)
        t = pm.get_tuning()
        assert t["contract_rows_long_pct"] == 0 and t["contract_rows_min_nnz"] == 5
    finally:
        pm.set_tuning(**before)


@pytest.mark.parametrize("env,expect", [({}, 100), ({"PM_CONTRACT_ROWS_LONG_PCT": "0"}, 0),
                                        ({"PM_CONTRACT_ROWS_LONG_PCT": "37"}, 37),
                                        ({"PM_CONTRACT_ROWS_LONG_PCT": "101"}, 100),
                                        ({"PM_CONTRACT_ROWS_LONG_PCT": "12x"}, 100)])
def test_tuning_environment(env, expect):
    """Initial values come from the environment; malformed or out-of-range
    values leave the default (a fresh process per case)."""
    import os
    import subprocess
    import sys
    code = ("import paper_2510_12196_amd as pm; pm.lib(); "
            "t = pm.get_tuning(); print(t['contract_rows_long_pct'], t['contract_rows_min_nnz'])")
    e = {k: v for k, v in os.environ.items() if not k.startswith("PM_")}
    e.update(env)
    out = subprocess.run([sys.executable, "-c", code], env=e, cwd=ROOT, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    pct, nnz = map(int, out.stdout.split())
    assert pct == expect and nnz == 1 << 20
