"""Host-side measurement tools on the CPU: the iteration kernel's
algorithmic byte count, the counter-calibrated HBM traffic summary, its
staleness guard, the kernel-time table, and bench.py's single-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2511_14419_amd import profiling as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_one_pair():
    alg = pr._iter_algorithmic(3, 2048, 4)
    assert [l for l, _ in alg] == [2, 2, 2, 1, 1, 1, 0, 0, 0]
    px2, px1, px0 = 512 ** 2, 1024 ** 2, 2048 ** 2
    # both frames' 5 FP32 planes + flow out, then the prior: none at the
    # coarsest level's first update, the coarser flow (a quarter of the
    # pixels) at a finer level's first, the previous iterate otherwise; the
    # last launch also writes the 1-byte pre-mask
    assert alg[0][1] == px2 * 48
    assert alg[1][1] == px2 * 56
    assert alg[3][1] == px1 * 48 + px1 // 4 * 8
    assert alg[8][1] == px0 * 56 + px0
    assert round(sum(b for _, b in alg) / 9) == 99498212


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": 256, "Counter_Name": counter,
                        "Counter_Value": v})


def test_traffic_calibrates_with_the_copy(tmp_path):
    alg = pr._iter_algorithmic(3, 2048, 4)
    copy = "__amd_rocclr_copyBuffer"
    # the copy reads back half its bytes in FETCH_SIZE (KiB) and all in WRITE_SIZE
    fetch = [(copy, pr.COPY_BYTES / 2048.0)]
    write = [(copy, pr.COPY_BYTES / 1024.0)]
    for _ in range(2):  # two pairs
        for l, b in alg:
            fetch.append(("void flowroi::k_iter<float, 7, 1>", 0.75 * b / 2048.0))  # 0.75 b read
            write.append(("void flowroi::k_iter<float, 7, 1>", 0.5 * b / 1024.0))   # 0.5 b written
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    t = pr.traffic(str(tmp_path / "f"), str(tmp_path / "w"))
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert t["launches"] == 18
    assert t["hbm_over_algorithmic"] == 1.25
    assert t["algorithmic_bytes_per_launch"] == 99498212
    assert all(v["ratio"] == 1.25 for v in t["per_level"].values())
    assert t["kernel_source_sha256"] == pr.kernel_source_sha()


def test_traffic_rejects_a_partial_pair(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    rows = [(copy, 1.0)] + [("k_iter<float, 7, 1>", 1.0)] * 8
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", rows)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", rows)
    with pytest.raises(ValueError):
        pr.traffic(str(tmp_path / "f"), str(tmp_path / "w"))


def test_traffic_summary_is_dropped_when_sources_change(tmp_path):
    good = {"kernel": "k_iter", "kernel_source_sha256": pr.kernel_source_sha(), "hbm_bytes_per_launch": 1}
    p = tmp_path / "t.txt"
    p.write_text("header text\n\n" + json.dumps(good, indent=1) + "\n")
    assert pr.load_traffic(str(p))["hbm_bytes_per_launch"] == 1
    p.write_text(json.dumps(dict(good, kernel_source_sha256="0" * 64)))
    assert pr.load_traffic(str(p)) is None
    assert pr.load_traffic(str(tmp_path / "missing.txt")) is None


def test_kernel_sha_covers_only_the_iteration_kernel_and_above():
    src = open(pr.KERNEL_SOURCES[0]).read()
    assert src.count(pr.ITER_SECTION[0]) == 1 and src.count(pr.ITER_SECTION[1]) == 1
    assert src.index(pr.ITER_SECTION[0]) < src.index(pr.ITER_SECTION[1])


def test_stats_table(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": "k_a", "Calls": 4, "TotalDurationNs": 2000000, "AverageNs": 500000.0, "Percentage": 80})
    lines = pr.stats(str(p)).splitlines()
    assert lines[0].startswith("| kernel |") and lines[2] == "| k_a | 4 | 2.00 | 500.00 | 80 |"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
