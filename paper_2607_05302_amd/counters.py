"""Summaries of rocprofv3 counter runs of the benchmark (profiling aids; the
library does not use them).

HBM traffic of the Radsort round kernel: FETCH_SIZE and WRITE_SIZE per dispatch
(each from a run of its own), scaled to bytes by the same counters of the
library's streaming copy in the same run (k_stream_copy: n (s_k + s_v) bytes
read and as many written per launch), written to a JSON file that bench.py
reports as roofline.traffic while the kernel source is unchanged:

    python -m paper_2607_05302_amd.counters traffic FETCH.csv WRITE.csv \\
        --n 268435456 --elem-bytes 8 --block 2048 --out profiles/k_round_traffic.json

SQ counters of one kernel (any number of counter runs), as a table of means per
dispatch and a few ratios:

    python -m paper_2607_05302_amd.counters sq RUN1.csv RUN2.csv ... --kernel k_round<

The CSV files are rocprofv3's counter_collection.csv (--output-format csv).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources of the round kernel and of the host code that picks its shape:
# counters taken on other text are stale
KERNEL_SOURCES = ["paper_2607_05302_amd/csrc/kernel_round.hpp",
                  "paper_2607_05302_amd/csrc/common.hpp",
                  "paper_2607_05302_amd/csrc/radsort.hip"]
ROUND_KERNEL = "k_round<"
COPY_KERNEL = "k_stream_copy"


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def read_counters(path: str) -> list:
    """Rows of (dispatch id, kernel name, counter, value) of a counter CSV."""
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"],
                        float(r["Counter_Value"])))
    return out


def per_dispatch(rows, counter, name_part):
    """{dispatch: value} of one counter for the kernels whose name contains
    name_part (values of one dispatch summed: rocprofv3 may split a counter)."""
    vals = {}
    for d, name, c, v in rows:
        if c == counter and name_part in name:
            vals[d] = vals.get(d, 0.0) + v
    return [vals[d] for d in sorted(vals)]


def kernel_names(rows, name_part):
    return sorted({name for _, name, _, _ in rows if name_part in name})


def traffic(fetch_csv, write_csv, n, elem_bytes, block):
    fr, wr = read_counters(fetch_csv), read_counters(write_csv)
    f_round = per_dispatch(fr, "FETCH_SIZE", ROUND_KERNEL)
    w_round = per_dispatch(wr, "WRITE_SIZE", ROUND_KERNEL)
    f_copy = per_dispatch(fr, "FETCH_SIZE", COPY_KERNEL)
    w_copy = per_dispatch(wr, "WRITE_SIZE", COPY_KERNEL)
    if not (f_round and w_round and f_copy and w_copy):
        raise SystemExit("traffic: the runs hold no round or copy dispatches")
    copy_bytes = n * elem_bytes  # read and written per copy launch
    f_scale = copy_bytes / statistics.median(f_copy)
    w_scale = copy_bytes / statistics.median(w_copy)
    rb = statistics.mean(f_round) * f_scale
    wb = statistics.mean(w_round) * w_scale
    alg = 2 * n * elem_bytes
    return {
        "kernel": kernel_names(fr, ROUND_KERNEL),
        "kernel_sha": kernel_sha(),
        "n": n, "elem_bytes": elem_bytes, "block_elems": block,
        "fetch_size_raw_per_launch": f_round,
        "write_size_raw_per_launch": w_round,
        "copy_fetch_size_raw": f_copy,
        "copy_write_size_raw": w_copy,
        "copy_bytes_each_way": copy_bytes,
        "fetch_bytes_per_unit": f_scale,
        "write_bytes_per_unit": w_scale,
        "read_bytes_per_launch": round(rb),
        "write_bytes_per_launch": round(wb),
        "bytes_per_launch": round(rb + wb),
        "alg_bytes_per_launch": alg,
        "over_algorithmic": (rb + wb) / alg,
    }


def sq_table(paths, name_part):
    rows = []
    for p in paths:
        rows += read_counters(p)
    counters = sorted({c for _, name, c, _ in rows if name_part in name})
    means = {}
    for c in counters:
        v = per_dispatch(rows, c, name_part)
        if v:
            means[c] = (statistics.mean(v), len(v))
    ratios = {}

    def ratio(label, a, b):
        if a in means and b in means and means[b][0]:
            ratios[label] = means[a][0] / means[b][0]

    ratio("waves resident per busy cycle (SQ_WAVE_CYCLES / SQ_BUSY_CYCLES)",
          "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES")
    ratio("wave-cycles waiting for anything", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES")
    ratio("wave-cycles waiting at s_waitcnt", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")
    ratio("wave-cycles issuing any instruction", "SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES")
    ratio("LDS bank-conflict cycles per LDS-active cycle", "SQ_LDS_BANK_CONFLICT",
          "SQ_ACTIVE_INST_LDS")
    ratio("LDS instructions per VALU instruction", "SQ_INSTS_LDS", "SQ_INSTS_VALU")
    return {"kernel": kernel_names(rows, name_part), "means": means, "ratios": ratios}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--n", type=int, required=True)
    t.add_argument("--elem-bytes", type=int, required=True)
    t.add_argument("--block", type=int, required=True)
    t.add_argument("--out")
    s = sub.add_parser("sq")
    s.add_argument("csv", nargs="+")
    s.add_argument("--kernel", default=ROUND_KERNEL)
    a = ap.parse_args(argv)
    if a.cmd == "traffic":
        r = traffic(a.fetch_csv, a.write_csv, a.n, a.elem_bytes, a.block)
        text = json.dumps(r, indent=1)
        if a.out:
            open(a.out, "w").write(text + "\n")
        print(text)
    else:
        r = sq_table(a.csv, a.kernel)
        print("kernel:", "; ".join(r["kernel"]))
        print(f"{'counter':28s} {'mean per dispatch':>20s} {'dispatches':>10s}")
        for c, (m, k) in r["means"].items():
            print(f"{c:28s} {m:20.0f} {k:10d}")
        for label, v in r["ratios"].items():
            print(f"{label}: {v:.3f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
