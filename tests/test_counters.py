"""The rocprofv3 counter summaries (paper_2607_05302_amd.counters) on synthetic
counter files: the byte scale comes from the copy kernel of known size, the
round kernel's bytes follow, and the source hash names the round kernel's code."""
import csv
import json

import pytest

from paper_2607_05302_amd import counters

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]
ROUND = "void rs::k_round<4, 4, false, 8, 256, rs::RoundShape<8, 16, false, true, 4>, 1, false>(x)"
COPY = "rs::k_stream_copy(a, b)"


def write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for d, name, counter, value in rows:
            r = dict.fromkeys(FIELDS, 0)
            r.update(Dispatch_Id=d, Kernel_Name=name, Counter_Name=counter, Counter_Value=value)
            w.writerow(r)


def test_traffic_scales_by_the_copy(tmp_path):
    n, eb = 1 << 20, 8
    copy_bytes = n * eb
    # a FETCH_SIZE unit of 2048 B and a WRITE_SIZE unit of 1024 B, as on MI355X
    fr = [(1, COPY, "FETCH_SIZE", copy_bytes / 2048), (2, ROUND, "FETCH_SIZE", 1.1 * copy_bytes / 2048),
          (3, ROUND, "FETCH_SIZE", 1.3 * copy_bytes / 2048), (4, "other", "FETCH_SIZE", 1e9)]
    wr = [(1, COPY, "WRITE_SIZE", copy_bytes / 1024), (2, ROUND, "WRITE_SIZE", 1.2 * copy_bytes / 1024),
          (3, ROUND, "WRITE_SIZE", 1.2 * copy_bytes / 1024)]
    write(tmp_path / "f.csv", fr)
    write(tmp_path / "w.csv", wr)
    r = counters.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), n, eb, 2048)
    assert r["fetch_bytes_per_unit"] == pytest.approx(2048)
    assert r["write_bytes_per_unit"] == pytest.approx(1024)
    assert r["read_bytes_per_launch"] == pytest.approx(1.2 * copy_bytes, abs=1)
    assert r["write_bytes_per_launch"] == pytest.approx(1.2 * copy_bytes, abs=1)
    assert r["over_algorithmic"] == pytest.approx(1.2)
    assert r["kernel_sha"] == counters.kernel_sha()
    json.dumps(r)  # the record is written as JSON


def test_traffic_needs_both_kernels(tmp_path):
    write(tmp_path / "f.csv", [(1, ROUND, "FETCH_SIZE", 10)])
    write(tmp_path / "w.csv", [(1, ROUND, "WRITE_SIZE", 10)])
    with pytest.raises(SystemExit):
        counters.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 1, 8, 64)


def test_sq_ratios(tmp_path):
    rows = [(1, ROUND, "SQ_WAVE_CYCLES", 400), (1, ROUND, "SQ_BUSY_CYCLES", 100),
            (1, ROUND, "SQ_WAIT_ANY", 200), (2, ROUND, "SQ_WAVE_CYCLES", 800),
            (2, ROUND, "SQ_BUSY_CYCLES", 100), (2, ROUND, "SQ_WAIT_ANY", 400),
            (3, COPY, "SQ_WAVE_CYCLES", 1e9)]
    write(tmp_path / "s.csv", rows)
    r = counters.sq_table([str(tmp_path / "s.csv")], "k_round<")
    assert r["means"]["SQ_WAVE_CYCLES"] == (600, 2)
    ratios = r["ratios"]
    assert ratios["waves resident per busy cycle (SQ_WAVE_CYCLES / SQ_BUSY_CYCLES)"] == 6
    assert ratios["wave-cycles waiting for anything"] == 0.5


def test_committed_traffic_record_matches_the_source():
    """bench.py reports the committed HBM bytes only while the round kernel's source
    is the one they were measured on; the record in profiles/ is current."""
    import os
    rec = json.load(open(os.path.join(counters.ROOT, "profiles", "k_round_traffic.json")))
    assert rec["kernel_sha"] == counters.kernel_sha()
    assert 1.0 < rec["bytes_per_launch"] / rec["alg_bytes_per_launch"] < 1.5
