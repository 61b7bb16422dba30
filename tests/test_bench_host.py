"""Host logic of bench.py that needs no GPU: the reduction of rocprofv3
counter runs (copy-kernel calibration of FETCH_SIZE / WRITE_SIZE, shares of
the shader-sequencer counters) and the source-digest check that decides
whether a committed traffic summary still describes the current kernels."""
import csv
import os

import pytest

import bench


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_pmc_calibrates_and_reports_shares(tmp_path, capsys):
    d = tmp_path / "pmc"
    d.mkdir()
    copy = "void at::native::neg_kernel(...)"
    kern = "void pm::k_reb_select<1>(pm::RebArgs)"
    other = "void pm::k_reb_select_other(pm::RebArgs)"  # a different kernel name
    rows = [
        # the calibration copy reads half of what it moves: FETCH scale 2
        {"Dispatch_Id": 1, "Kernel_Name": copy, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 262144},
        {"Dispatch_Id": 1, "Kernel_Name": copy, "Counter_Name": "WRITE_SIZE",
         "Counter_Value": 524288},
        # two launches of the kernel, the first counted over two channels
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 600},
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 400},
        {"Dispatch_Id": 3, "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 3000},
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE",
         "Counter_Value": 400},
        {"Dispatch_Id": 3, "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE",
         "Counter_Value": 600},
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "SQ_WAVE_CYCLES",
         "Counter_Value": 1000},
        {"Dispatch_Id": 3, "Kernel_Name": kern, "Counter_Name": "SQ_WAVE_CYCLES",
         "Counter_Value": 3000},
        {"Dispatch_Id": 2, "Kernel_Name": kern, "Counter_Name": "SQ_WAIT_ANY",
         "Counter_Value": 700},
        {"Dispatch_Id": 3, "Kernel_Name": kern, "Counter_Name": "SQ_WAIT_ANY",
         "Counter_Value": 2300},
        {"Dispatch_Id": 4, "Kernel_Name": other, "Counter_Name": "FETCH_SIZE",
         "Counter_Value": 10 ** 9},
    ]
    _write_counters(d / "x_counter_collection.csv", rows)
    bench.summarize_pmc(str(d), "k_reb_select")
    out = capsys.readouterr().out
    kv = {}
    for line in out.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    # FETCH: (1000 + 3000) / 2 launches = 2000 KiB, scale 2 -> 4 096 000 B
    # WRITE: 500 KiB per launch, scale 1 -> 512 000 B
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(4096000 + 512000)
    assert "over 2 launches" in kv["FETCH_SIZE"]
    # waiting share over all waves of all launches: 3000 / 4000
    assert float(kv["SQ_WAIT_ANY / SQ_WAVE_CYCLES"]) == pytest.approx(0.75)
    assert kv["SQ_WAVE_CYCLES"].startswith("2000 per launch")
    assert kv["source_digest"] == bench.source_digest()


def test_read_traffic_requires_workload_and_current_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.txt"
    monkeypatch.setattr(bench, "traffic_file", lambda kernel, workload: str(f))
    assert bench.read_traffic("k_apply", "rmat22") is None  # no file
    f.write_text(f"workload: rmat22\nsource_digest: {bench.source_digest()}\n"
                 "hbm_bytes_per_launch: 1234\n")
    assert bench.read_traffic("k_apply", "rmat22") == 1234.0
    assert bench.read_traffic("k_apply", "rgg20") is None  # another workload
    f.write_text("workload: rmat22\nsource_digest: 0000000000000000\n"
                 "hbm_bytes_per_launch: 1234\n")
    assert bench.read_traffic("k_apply", "rmat22") is None  # stale sources


def test_committed_traffic_summaries_name_their_workload():
    for kern in bench.KERNEL_NAMES.values():
        path = bench.traffic_file(kern, "rmat22")
        if not os.path.exists(path):
            continue
        text = open(path).read()
        assert "workload: rmat22" in text
        assert "source_digest:" in text and "hbm_bytes_per_launch:" in text
