#!/usr/bin/env python3
"""Radsort on one MI355X against the out-of-place LSD baseline of Alg. 1.

Workload: n = 2^28 uint32 keys, uniform over [0, 2^32) (splitmix64, seed
0x5EED0002), uint32 payload = original index, 8-bit digits (sigma = 256, n_t = 4),
block size b = 2048 (the fastest b whose workspace stays under 1% of the input;
--block picks another).  One step is one complete Radsort of that array on the
GPU: digit histograms, setup, four sort rounds (each a super-tile counting pass
and the round kernel) with their fixups, and finalize.  The input is restored
from a pristine device copy before every step; the restore lies outside the HIP
events that time the step.

Printed: one JSON line with keys/s (value), the per-round roofline of the
sort-round kernel (algorithmic bytes 2 n (s_k + s_v) per launch over its event
time), peak extra device bytes of Radsort and of the baseline, the baseline's
throughput on the same input, and the CPU oracle timed on a sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
from paper_2607_05302_amd.counters import kernel_sha  # noqa: E402  (source hash)

METRIC = "keys/s & HBM GB/s, uint32 n=2^28, vs out-of-place LSD; peak extra bytes"
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_round_traffic.json")



def carries_keys(keys0, v, k, n):
    """True when every index in v lies in [0, n) and keys0 at it (as unsigned 32-bit)
    equals k; indices are checked before any gather with them."""
    import torch
    if not bool(((v >= 0) & (v < n)).all()):
        return False
    return bool(((keys0.to(torch.int64) & 0xFFFFFFFF)[v] == k).all())

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(n, elem_bytes, b):
    """HBM bytes per sort-round launch from the committed counter runs, if they
    were taken on the current kernel source and workload; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if (t.get("kernel_sha") != kernel_sha() or t.get("n") != n
            or t.get("elem_bytes") != elem_bytes or t.get("block_elems") != b):
        return None
    return t.get("bytes_per_launch")


def host_cpu() -> dict:
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def library_stable_sort(keys_np, target_s):
    """numpy's stable argsort (one host thread) on the first keys of the same input,
    with the payload gathered by the permutation: the library sort beside the
    oracle, on a sample sized for about target_s seconds."""
    import numpy as np

    m = 1 << 20
    t = time.perf_counter()
    np.argsort(keys_np[:m], kind="stable")
    per_key = (time.perf_counter() - t) / m
    m = int(min(len(keys_np), max(1 << 20, target_s / per_key)))
    m = 1 << (m.bit_length() - 1)
    k = keys_np[:m]
    t = time.perf_counter()
    o = np.argsort(k, kind="stable")
    ks, vs = k[o], o.astype(np.uint32)
    dt = time.perf_counter() - t
    del ks, vs
    return {"value": m / dt, "unit": "keys/s", "cores": 1,
            "kind": "numpy.argsort(kind='stable') + gather",
            "sample": f"first {m} keys of the same input (2^{m.bit_length() - 1}), {dt:.2f} s"}


def cpu_baseline(keys_np, target_s, b):
    """The sequential C oracle on a prefix of the same input (1 host thread)."""
    import numpy as np

    import oracle

    oracle.load()
    m = 1 << 20
    t = time.perf_counter()
    oracle.radsort(keys_np[:m], np.arange(m, dtype=np.uint32), 256, 4, b)
    per_key = (time.perf_counter() - t) / m
    m = int(min(len(keys_np), max(1 << 20, target_s / per_key)))
    m = 1 << (m.bit_length() - 1)  # a power of two
    vals = np.arange(m, dtype=np.uint32)
    t = time.perf_counter()
    oracle.radsort(keys_np[:m], vals, 256, 4, b)
    dt = time.perf_counter() - t
    return {"value": m / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} of the {len(keys_np)} keys (2^{m.bit_length() - 1}), "
                      f"uint32 keys + uint32 index payload, b={b}, 8-bit digits, sequential "
                      f"C oracle (Alg. 2-7), {dt:.1f} s",
            "host": host_cpu(),
            "library_stable_sort": library_stable_sort(keys_np, min(6.0, target_s / 2))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--block", type=int, default=None,
                    help="block size b (default 2048; 4096 for the structured inputs)")
    ap.add_argument("--no-oop", action="store_true", help="skip the out-of-place baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", choices=["single", "segments", "serving", "resort",
                                           "structured", "msd"],
                    default="single",
                    help="segments: 4096 uint32 arrays of log-uniform sizes in one call; "
                         "serving: a stream of sort requests admitted by memory footprint; "
                         "resort: new keys written in place and sorted again from the same "
                         "state, without finalize; structured: 2^30 uint64 keys, four "
                         "skewed and structured inputs; msd: the MSD-first split beside "
                         "the LSD sort at 2^28 uint32 pairs")
    ap.add_argument("--requests", type=int, default=400, help="serving: requests in the trace")
    ap.add_argument("--rate", type=float, default=800.0, help="serving: offered requests/s")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: device memory budget")
    ap.add_argument("--slots", type=int, default=8, help="serving: requests on the GPU at once")
    ap.add_argument("--min-log2", type=float, default=12, help="serving: smallest size, log2")
    ap.add_argument("--max-log2", type=float, default=28, help="serving: largest size, log2")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scales HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the sort runs on a single MI355X.", flush=True)
        sys.exit(1)

    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    if args.workload == "segments":
        return bench_segments(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "resort":
        return bench_resort(args)
    if args.workload == "structured":
        return bench_structured(args)
    if args.workload == "msd":
        return bench_msd(args)
    n = 1 << args.log2n
    b, bits, kb, vb = args.block or 2048, 8, 4, 4
    seed = workloads.SEED_SMALL if args.log2n == 20 else workloads.SEED_LARGE
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: generating n=2^{args.log2n} uniform uint32 keys")
    keys_np = workloads.uniform(seed, n, 4)
    keys0 = torch.from_numpy(keys_np.view(np.int32)).to(dev)
    vals0 = torch.arange(n, dtype=torch.int32, device=dev)
    keys = torch.empty_like(keys0)
    vals = torch.empty_like(vals0)
    ws_bytes = radsort.workspace_bytes(n, kb, vb, bits, b)
    oop_bytes = radsort.oop_workspace_bytes(n, kb, vb, bits, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def run(fn, wsbuf, steps, warmup, label):
        for _ in range(warmup):
            keys.copy_(keys0)
            vals.copy_(vals0)
            fn(keys, vals, digit_bits=bits, block_elems=b, workspace=wsbuf, check=True)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        times, stats = [], []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(steps):
            keys.copy_(keys0)
            vals.copy_(vals0)
            ev0.record(stream)
            fn(keys, vals, digit_bits=bits, block_elems=b, workspace=wsbuf, timing=True)
            ev1.record(stream)
            st = radsort.last_stats()  # waits for the sort's own last event
            ev1.synchronize()
            times.append(ev0.elapsed_time(ev1))
            stats.append(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        log(f"bench: {label}: mean {np.mean(times):.3f} ms, min {np.min(times):.3f} ms")
        return times, stats, wall

    log("bench: Radsort")
    times, stats, wall = run(radsort.sort_, ws, args.steps, args.warmup, "radsort")
    # check the last result: sorted, stable, and a permutation carrying its keys
    k = keys.to(torch.int64) & 0xFFFFFFFF
    v = vals.to(torch.int64)
    ok = bool((k[1:] >= k[:-1]).all())
    eq = k[1:] == k[:-1]
    ok &= bool((v[1:][eq] > v[:-1][eq]).all())
    ok &= carries_keys(keys0, v, k, n)
    ok &= bool((torch.bincount(v, minlength=n) == 1).all())
    del k, v, eq
    if not ok:
        log("bench: Radsort output failed the sortedness/stability/permutation check")

    oop = None
    if not args.no_oop:
        log("bench: out-of-place baseline")
        del ws
        torch.cuda.empty_cache()
        ows = torch.empty(oop_bytes, dtype=torch.uint8, device=dev)
        otimes, ostats, _ = run(radsort.oop_sort_, ows, args.steps, args.warmup, "oop")
        del ows
        torch.cuda.empty_cache()
        oop = {
            "value": n / (np.mean(otimes) / 1e3), "unit": "keys/s",
            "ms_per_step": float(np.mean(otimes)), "min_ms": float(np.min(otimes)),
            "round_ms_mean": float(np.mean([np.mean(s["round_ms"]) for s in ostats])),
            "count_ms_mean": float(np.mean([np.mean(s["count_ms"]) for s in ostats])),
            "peak_extra_bytes": oop_bytes,
            "peak_extra_frac_of_input": oop_bytes / (n * (kb + vb)),
        }

    # the practical HBM ceiling: the library's streaming copy of the same bytes
    # (keys and payload: one read and one write of n (s_k + s_v) bytes)
    csrc = torch.empty(n * (kb + vb) // 4, dtype=torch.int32, device=dev)
    cdst = torch.empty_like(csrc)
    for _ in range(3):
        radsort.copy_(cdst, csrc)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        radsort.copy_(cdst, csrc)
    c1.record(stream)
    c1.synchronize()
    copy_ms = c0.elapsed_time(c1) / 10
    copy_gbps = 2 * n * (kb + vb) / (copy_ms / 1e3) / 1e9
    del csrc, cdst
    log(f"bench: streaming copy of {n * (kb + vb)} bytes: {copy_ms:.3f} ms, {copy_gbps:.0f} GB/s")

    if args.copy_calibration:
        # a plain copy of known size: the HBM counters of this kernel give the scale
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration: 1 GiB read + 1 GiB write per copy, 3 copies")
        del src, dst

    mean_ms = float(np.mean(times))
    round_ms = [float(np.mean([s["round_ms"][r] for s in stats])) for r in range(4)]
    per_round = float(np.mean(round_ms))
    alg_bytes = 2 * n * (kb + vb)  # n reads + n writes of (key, payload) per round
    achieved = alg_bytes / (per_round / 1e3) / 1e9
    traffic = measured_traffic(n, kb + vb, b)
    out = {
        "metric": METRIC,
        "value": n / (mean_ms / 1e3),
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mean_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"radsort n=2^{args.log2n} uint32 keys uniform (splitmix64 seed "
                        f"{seed:#x}) + uint32 index payload, 8-bit digits, b={b}",
            "n": n, "key_bytes": kb, "payload_bytes": vb, "digit_bits": bits,
            "block_elems": b,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_round (one sort round, Alg. 5)",
            "alg_bytes_per_launch": alg_bytes, "launch_ms": per_round,
        },
        "hbm_gbps_whole_sort": 4 * alg_bytes / (mean_ms / 1e3) / 1e9,
        "copy_ceiling": {"gbps": copy_gbps, "ms": copy_ms,
                         "kernel": "k_stream_copy (radsort_copy), 16-byte words",
                         "round_frac_of_copy": achieved / copy_gbps},
        "phases_ms": {
            "setup": float(np.mean([s["setup_ms"] for s in stats])),
            "rounds": round_ms,
            "supertile_counts": [float(np.mean([s["count_ms"][r] for s in stats])) for r in range(4)],
            "fixup_total": float(np.mean([s["fixup_ms"] for s in stats])),
            "finalize": float(np.mean([s["finalize_ms"] for s in stats])),
        },
        "min_ms": float(np.min(times)),
        "runs_ms": [round(t, 4) for t in times],
        "wall_ms_per_step_incl_restore": wall / args.steps * 1e3,
        "peak_extra_bytes": ws_bytes,
        "peak_extra_frac_of_input": ws_bytes / (n * (kb + vb)),
        "oop": oop,
        "verified": ok,
    }
    if oop:
        out["speed_vs_oop"] = oop["ms_per_step"] / mean_ms
        out["extra_bytes_vs_oop"] = ws_bytes / oop_bytes
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(keys_np, args.cpu_seconds, b)
    print(json.dumps(out), flush=True)


SEG_SEED = 0x5EED0004
SEG_METRIC = "keys/s, batched segmented sort: 4096 uint32 arrays + uint32 index, " \
             "sizes log-uniform in [2^10, 2^22], one call"


def bench_segments(args):
    """The batched workload: 4096 independent arrays sorted by one call
    (radsort_sort_segments), eagerly and as a replayed graph."""
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads
    from paper_2607_05302_amd.tune import load_table

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sizes = workloads.log_uniform_sizes(SEG_SEED, 4096, 10, 22)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(offsets[-1])
    log(f"bench: {len(sizes)} arrays, {total} elements")
    off_dev = torch.from_numpy(offsets.view(np.int64)).to(dev)
    keys0 = workloads.uniform_t(SEG_SEED, total, 4, dev)
    vals0 = torch.arange(total, dtype=torch.int32, device=dev)
    keys, vals = torch.empty_like(keys0), torch.empty_like(vals0)
    tuning = "auto"
    ws_bytes = radsort.segments_workspace_bytes(offsets, 4, 4, tuning)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def restore():
        keys.copy_(keys0)
        vals.copy_(vals0)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            restore()
            fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            restore()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return times

    def call():
        radsort.sort_segments_(keys, vals, offsets, tuning=tuning, workspace=ws,
                               offsets_dev=off_dev)

    restore()
    radsort.sort_segments_(keys, vals, offsets, tuning=tuning, workspace=ws,
                           offsets_dev=off_dev, check=True)
    # check: every array ascending, stable, and a permutation of its own elements
    k = keys.to(torch.int64) & 0xFFFFFFFF
    v = vals.to(torch.int64)
    starts = torch.zeros(total, dtype=torch.bool, device=dev)
    starts[off_dev[:-1][torch.from_numpy(sizes > 0).to(dev)]] = True
    inner = ~starts[1:]
    ok = bool(((k[1:] >= k[:-1]) | ~inner).all())
    ok &= bool(((v[1:] > v[:-1]) | ~(inner & (k[1:] == k[:-1]))).all())
    seg = torch.repeat_interleave(torch.arange(len(sizes), device=dev),
                                  torch.from_numpy(sizes).to(dev))
    ok &= bool((torch.searchsorted(off_dev[1:], v, right=True) == seg).all())
    in_range = carries_keys(keys0, v, k, total)
    ok &= in_range
    if in_range:
        seen = torch.zeros(total, dtype=torch.bool, device=dev)
        seen[v] = True
        ok &= bool(seen.all())
        del seen
    del k, v, starts, inner, seg
    log(f"bench: verified {ok}")

    times = timed(call, args.steps, args.warmup)
    g = torch.cuda.CUDAGraph()
    restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        call()
    gtimes = timed(g.replay, args.steps, 1)
    mean_ms = float(np.mean(times))
    out = {
        "metric": SEG_METRIC,
        "value": total / (mean_ms / 1e3),
        "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mean_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"4096 arrays, sizes log-uniform in [2^10, 2^22] (splitmix64 seed "
                               f"{SEG_SEED:#x}), {total} uint32 keys uniform + uint32 index",
                   "arrays": int(len(sizes)), "elements": total,
                   "tuning": load_table(4, 4)},
        "graph_ms_per_step": float(np.mean(gtimes)),
        "graph_value": total / (float(np.mean(gtimes)) / 1e3),
        "min_ms": float(np.min(times)),
        "runs_ms": [round(t, 3) for t in times],
        "read_write_once_gbps": 2 * total * 8 / (mean_ms / 1e3) / 1e9,
        "peak_extra_bytes": ws_bytes,
        "peak_extra_frac_of_input": ws_bytes / (total * 8),
        "verified": ok,
    }
    print(json.dumps(out), flush=True)


SERVE_SEED = 0x5EED0005


def bench_serving(args):
    """Poisson arrivals of sort requests (sizes log-uniform in [2^12, 2^28], uint32 or
    uint64 keys with a uint32 index payload), served under a device memory budget
    by Radsort and, on the same trace, by the out-of-place baseline."""
    import torch

    from paper_2607_05302_amd import serve

    torch.cuda.set_device(0)
    trace = serve.make_trace(SERVE_SEED, args.requests, args.rate, args.min_log2, args.max_log2)
    res = {}
    for method in ("radsort", "oop"):
        srv = serve.Server(method, budget=args.budget_gb * 1e9, slots=args.slots)
        srv.run(trace[: min(8, len(trace))])  # warm-up: kernels loaded, streams made
        torch.cuda.empty_cache()
        log(f"bench: serving {len(trace)} requests with {method}")
        out = srv.run(trace)
        res[method] = serve.summarize(trace, out)
        # the same trace again, every result checked completely on the device when it
        # completes (the checks share the GPU, so this run is not the timed one)
        log(f"bench: serving the trace again with every result checked ({method})")
        chk = srv.run(trace, verify=True)
        res[method]["wrong_results"] = len(chk["bad"])
        res[method]["device_errors"] = len(chk["device_errors"])
        log(f"bench: {method}: {res[method]}")
        del srv
        torch.cuda.empty_cache()
    r = res["radsort"]
    out = {
        "metric": "sort serving: keys/s and p50/p99 latency, Poisson arrivals, sizes log-uniform "
                  f"in [2^{args.min_log2:g}, 2^{args.max_log2:g}], 50/50 uint32/uint64 keys, "
                  f"{args.budget_gb:g} GB budget, Radsort vs out-of-place",
        "value": r["keys_per_s"], "unit": "keys/s", "n_gpus": 1, "steps": args.requests,
        "warmup": 8, "ms_per_step": r["span_ms"] / args.requests, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64", "data": "synthetic",
        "config": {"workload": f"{args.requests} requests at {args.rate:g}/s offered "
                               f"(arrivals and sizes: splitmix64 seed {SERVE_SEED:#x}; keys: torch's "
                               f"device generator seeded per request), budget {args.budget_gb:g} GB, "
                               f"{args.slots} slots", "offered_rps": serve.offered_load(trace)},
        "radsort": r, "oop": res["oop"],
        "p99_ratio_oop_over_radsort": res["oop"]["p99_ms"] / r["p99_ms"],
        "verified": all(x["wrong_results"] == 0 and x["device_errors"] == 0
                        for x in (r, res["oop"])),
    }
    print(json.dumps(out), flush=True)


RESORT_SEED = 0x5EED0006


def resort_multiplier(step: int) -> int:
    """The odd multiplier of step `step`: key = payload * m mod 2^32 (as int32)."""
    m = ((0x9E3779B1 + step * 0x632BE5A6) | 1) & 0xFFFFFFFF
    return m - (1 << 32) if m >= 1 << 31 else m


STRUCT_METRIC = "keys/s, uint64 keys only, n=2^30, 8-bit digits (8 rounds): " \
                "Zipf(1.1) over 2^16 values, all equal, sorted, low 20 bits random"


def bench_structured(args):
    """The four skewed and structured uint64 inputs at n = 2^30 (keys only), each
    sorted steps times after a warm-up; per-round roofline at 16 bytes per element
    (8-byte read + 8-byte write).  Each result is checked: keys ascending, and the
    same sum of keys as the input (modulo 2^64).  The full check of these inputs
    (stability and permutation through an index payload) is a GPU test."""
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log2n = 30 if args.log2n == 28 else args.log2n
    n, b, bits = 1 << log2n, args.block or 4096, 8
    ws = torch.empty(radsort.workspace_bytes(n, 8, 0, bits, b), dtype=torch.uint8, device=dev)
    keys = torch.empty(n, dtype=torch.int64, device=dev)
    steps = max(1, min(args.steps, 3))
    per, total_keys, total_ms = {}, 0, 0.0
    for dist in ["zipf", "equal", "sorted", "low20"]:
        log(f"bench: structured {dist} n=2^{log2n}")
        keys0 = workloads.make_t(dist, workloads.SEED_SKEWED, n, 8, dev)
        ksum = int(keys0.sum())  # modulo 2^64, like the result's
        keys.copy_(keys0)
        radsort.sort_(keys, None, digit_bits=bits, block_elems=b, workspace=ws, check=True)
        times, rounds = [], []
        for _ in range(steps):
            keys.copy_(keys0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            radsort.sort_(keys, None, digit_bits=bits, block_elems=b, workspace=ws, timing=True)
            e1.record()
            st = radsort.last_stats()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
            rounds.append(st["round_ms"])
        flip = keys ^ (-(1 << 63))
        ok = bool((flip[1:] >= flip[:-1]).all()) and int(keys.sum()) == ksum
        del flip, keys0
        torch.cuda.empty_cache()
        rms = np.mean(np.array(rounds), axis=0)
        achieved = 2 * n * 8 / (rms / 1e3) / 1e9
        per[dist] = {"ms_per_sort": float(np.mean(times)), "keys_per_s": n / (np.mean(times) / 1e3),
                     "round_ms": [float(x) for x in rms],
                     "round_gbps": [float(x) for x in achieved],
                     "round_frac": [float(x / HBM_PEAK_GBS) for x in achieved],
                     "finalize_ms": float(st["finalize_ms"]), "verified": ok}
        total_keys += n * len(times)
        total_ms += float(np.sum(times))
        log(f"bench: {dist}: {np.mean(times):.2f} ms per sort, verified {ok}")
    ws_bytes = ws.numel()
    mean_ms = total_ms / (total_keys / n)
    all_rounds = np.array([r for d in per.values() for r in d["round_ms"]])
    out = {
        "metric": STRUCT_METRIC, "value": total_keys / (total_ms / 1e3), "unit": "keys/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": mean_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"radsort n=2^{log2n} uint64 keys only, four inputs (seed "
                               f"0x5EED0003), 8-bit digits, b={b}",
                   "n": n, "key_bytes": 8, "payload_bytes": 0, "digit_bits": bits,
                   "block_elems": b},
        "roofline": {"bound": "hbm", "achieved": float(2 * n * 8 / (all_rounds.mean() / 1e3) / 1e9),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": float(2 * n * 8 / (all_rounds.mean() / 1e3) / 1e9 / HBM_PEAK_GBS),
                     "traffic": None, "kernel": "k_round (one sort round, Alg. 5)",
                     "alg_bytes_per_launch": 2 * n * 8, "launch_ms": float(all_rounds.mean())},
        "inputs": per,
        "peak_extra_bytes": ws_bytes, "peak_extra_frac_of_input": ws_bytes / (n * 8),
        "verified": all(d["verified"] for d in per.values()),
    }
    print(json.dumps(out), flush=True)


MSD_METRIC = "keys/s, MSD-first split (top-digit round + batched per-group sort), " \
             "uint32 n=2^28 + uint32 index, beside the LSD Radsort"


def bench_msd(args):
    """The MSD-first split (radsort_msd_sort_pairs) and the LSD Radsort on the same
    2^28 uint32 pairs; both results are checked."""
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, b, bits = 1 << args.log2n, args.block or 2048, 8
    keys0 = workloads.uniform_t(workloads.SEED_LARGE, n, 4, dev)
    vals0 = torch.arange(n, dtype=torch.int32, device=dev)
    keys, vals = torch.empty_like(keys0), torch.empty_like(vals0)
    res = {}
    for name, fn in [("msd", radsort.msd_sort_), ("lsd", radsort.sort_)]:
        log(f"bench: {name}")
        keys.copy_(keys0)
        vals.copy_(vals0)
        fn(keys, vals, digit_bits=bits, block_elems=b, check=True)
        times = []
        for _ in range(max(1, args.steps)):
            keys.copy_(keys0)
            vals.copy_(vals0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(keys, vals, digit_bits=bits, block_elems=b)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        extra = radsort.last_stats()["workspace_bytes"]
        k = keys.to(torch.int64) & 0xFFFFFFFF
        v = vals.to(torch.int64)
        ok = bool((k[1:] >= k[:-1]).all())
        eq = k[1:] == k[:-1]
        ok &= bool((v[1:][eq] > v[:-1][eq]).all())
        ok &= carries_keys(keys0, v, k, n)
        del k, v, eq
        res[name] = {"ms_per_sort": float(np.mean(times)), "min_ms": float(np.min(times)),
                     "keys_per_s": n / (np.mean(times) / 1e3), "peak_extra_bytes": int(extra),
                     "peak_extra_frac_of_input": extra / (n * 8), "verified": ok}
        log(f"bench: {name}: {np.mean(times):.2f} ms, extra {extra} bytes, verified {ok}")
    out = {
        "metric": MSD_METRIC, "value": res["msd"]["keys_per_s"], "unit": "keys/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": res["msd"]["ms_per_sort"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"MSD-first split, n=2^{args.log2n} uint32 keys uniform (seed "
                               f"0x5EED0002) + uint32 index, 8-bit digits, b={b} (host wall "
                               f"clock: the call waits once between its phases)",
                   "n": n, "key_bytes": 4, "payload_bytes": 4, "digit_bits": bits,
                   "block_elems": b},
        "msd": res["msd"], "lsd": res["lsd"],
        "verified": res["msd"]["verified"] and res["lsd"]["verified"],
    }
    print(json.dumps(out), flush=True)


def bench_resort(args):
    """Sorting the same data again by new keys without finalize (Sec. 4.1).  n uint32
    keys with a uint32 index payload are sorted once; then each step gives every
    element the key payload * m_step mod 2^32, written in place in the permuted
    representation (one elementwise pass over the key and payload planes of A and
    T: every element sits at the same slot in both), and sorts the same state
    again (restart: histograms read through the block table, the plan; then n_t
    rounds), with no finalize and no setup.  Beside it, the usual way: the same
    new keys in plain arrays, then a full sort (setup, rounds, finalize).  Also
    timed once: truncate (Alg. 8) after the last round, truncate between rounds
    (with the new plan of the rounds left), and finalize of a truncated state."""
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    b, bits, kb, vb = args.block or 2048, 8, 4, 4
    nt = 4
    keys = workloads.uniform_t(RESORT_SEED, n, 4, dev)
    vals = torch.arange(n, dtype=torch.int32, device=dev)
    ws_bytes = radsort.workspace_bytes(n, kb, vb, bits, b)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st = radsort.State(keys, vals, digit_bits=bits, block_elems=b, workspace=ws)
    tk, tv, bb = st.planes()
    tbytes = 2 * st.sigma * bb * 4
    t_keys = ws[tk - ws.data_ptr():tk - ws.data_ptr() + tbytes].view(torch.int32)
    t_vals = ws[tv - ws.data_ptr():tv - ws.data_ptr() + tbytes].view(torch.int32)
    st.setup()
    for _ in range(nt):
        st.round()

    def rekey(k, v, step):
        torch.mul(v, resort_multiplier(step), out=k)

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    log(f"bench: resort n=2^{args.log2n}, b={b}")
    phases = {"rekey": [], "restart": [], "rounds": []}
    times = []
    step = 0
    for it in range(args.warmup + args.steps):
        step += 1
        e0 = ev()
        rekey(keys, vals, step)
        rekey(t_keys, t_vals, step)
        e1 = ev()
        st.restart()
        e2 = ev()
        for _ in range(nt):
            st.round()
        e3 = ev()
        e3.synchronize()
        if it >= args.warmup:
            times.append(e0.elapsed_time(e3))
            phases["rekey"].append(e0.elapsed_time(e1))
            phases["restart"].append(e1.elapsed_time(e2))
            phases["rounds"].append(e2.elapsed_time(e3))
    st.read()  # device-side error word
    # check: the dataset in logical order is sorted by its new keys, which are
    # payload * m mod 2^32, and the payloads are a permutation of 0 .. n-1
    lk, lv = st.logical()
    k = lk.to(torch.int64) & 0xFFFFFFFF
    v = lv.to(torch.int64)
    m = resort_multiplier(step) & 0xFFFFFFFF
    ok = bool((k[1:] > k[:-1]).all())
    ok &= bool(((v * m) & 0xFFFFFFFF == k).all())
    ok &= bool((torch.bincount(v, minlength=n) == 1).all())
    del k, v, lk, lv

    # truncate after the last round, truncate between rounds, finalize truncated
    e0 = ev()
    st.truncate(n - n // 4)
    e1 = ev()
    rekey(keys, vals, step + 1)
    rekey(t_keys, t_vals, step + 1)
    st.restart()
    st.round()
    st.round()
    e2 = ev()
    st.truncate(n // 2)
    e3 = ev()
    st.round()
    st.round()
    e4 = ev()
    st.finalize()
    e5 = ev()
    e5.synchronize()
    st.read()
    c = n // 2
    k = keys[:c].to(torch.int64) & 0xFFFFFFFF
    v = vals[:c].to(torch.int64)
    m = resort_multiplier(step + 1) & 0xFFFFFFFF
    ok &= bool(((k[1:] >> 16) >= (k[:-1] >> 16)).all())
    ok &= bool(((v * m) & 0xFFFFFFFF == k).all())
    del k, v
    trunc = {"truncate_after_last_round_ms": e0.elapsed_time(e1),
             "truncate_between_rounds_ms": e2.elapsed_time(e3),
             "finalize_truncated_ms": e4.elapsed_time(e5)}
    st.close()

    # the usual way: new keys in the plain arrays, then a full sort
    keys.copy_(workloads.uniform_t(RESORT_SEED, n, 4, dev))
    vals.copy_(torch.arange(n, dtype=torch.int32, device=dev))
    radsort.sort_(keys, vals, digit_bits=bits, block_elems=b, workspace=ws)
    ftimes = []
    for it in range(args.warmup + args.steps):
        e0 = ev()
        rekey(keys, vals, it + 1)
        radsort.sort_(keys, vals, digit_bits=bits, block_elems=b, workspace=ws)
        e1 = ev()
        e1.synchronize()
        if it >= args.warmup:
            ftimes.append(e0.elapsed_time(e1))
    mean_ms = float(np.mean(times))
    full_ms = float(np.mean(ftimes))
    out = {
        "metric": "keys/s, sorting again without finalize (Sec. 4.1): 2^28 uint32 keys "
                  "rewritten in place from their uint32 payload, restart + 4 rounds",
        "value": n / (mean_ms / 1e3), "unit": "keys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mean_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"resort n=2^{args.log2n}: uint32 keys uniform (splitmix64 seed "
                               f"{RESORT_SEED:#x}) sorted once, then per step key = payload * "
                               f"m_step mod 2^32 in place and a new sort of the same state; "
                               f"8-bit digits, b={b}", "n": n, "block_elems": b},
        "phases_ms": {k: float(np.mean(x)) for k, x in phases.items()},
        "full_sort_ms_per_step": full_ms,
        "speedup_vs_full_sort": full_ms / mean_ms,
        "truncate": trunc,
        "runs_ms": [round(t, 4) for t in times],
        "peak_extra_bytes": ws_bytes,
        "verified": ok,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
