"""Autotuner of the batched segmented sort: per size class, the block size b and
the digit width with the shortest measured time on this GPU.

The table serves the arrays that run the Radsort steps on streams: those above
the one-workgroup path (more than 4 423 680 elements); smaller arrays are sorted
by the LDS sort or by one workgroup each and do not use it.  For each class
(arrays of 2^k elements, k = lo .. hi) it sorts a batch of such arrays (seeded
uniform keys, index payload) with every candidate (b, digit bits), b in
{256 .. 8192} and digit bits in {4, 8, 11}, and keeps the fastest; the last class
also covers every larger array.  The result is a JSON table that sort_segments_
loads by default:

    python -m paper_2607_05302_amd.tune --key-bytes 4 --payload-bytes 4
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
BLOCKS = [256, 512, 1024, 2048, 4096, 8192]
DIGITS = [4, 8, 11]


def table_path(key_bytes: int, payload_bytes: int) -> str:
    return os.path.join(HERE, "tuning", f"segments_k{key_bytes}_v{payload_bytes}.json")


def load_table(key_bytes: int, payload_bytes: int):
    """[(max_log2n, b, digit_bits), ...] from the tuning file, or None."""
    try:
        t = json.load(open(table_path(key_bytes, payload_bytes)))
    except (OSError, ValueError):
        return None
    return [tuple(c) for c in t["classes"]]


def tune(key_bytes=4, payload_bytes=4, lo=23, hi=26, elems=1 << 27, reps=3, seed=0x7E57,
         log=print):
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    dev = torch.device("cuda:0")
    classes, measured = [], {}
    for k in range(lo, hi + 1):
        n = 1 << k
        count = max(4, elems // n)
        offsets = np.arange(count + 1, dtype=np.uint64) * np.uint64(n)
        off_dev = torch.from_numpy(offsets.view(np.int64)).to(dev)
        keys0 = workloads.uniform_t(seed + k, count * n, key_bytes, dev)
        vals0 = (torch.arange(count * n, dtype=torch.int64, device=dev)
                 .to({4: torch.int32, 8: torch.int64}[payload_bytes]) if payload_bytes else None)
        keys = torch.empty_like(keys0)
        vals = torch.empty_like(vals0) if payload_bytes else None
        best = None
        for b in BLOCKS:
            if b > n:
                continue
            for bits in DIGITS:
                table = [(k, b, bits)]
                ws = torch.empty(radsort.segments_workspace_bytes(offsets, key_bytes,
                                                                  payload_bytes, table),
                                 dtype=torch.uint8, device=dev)
                times = []
                for r in range(reps + 1):
                    keys.copy_(keys0)
                    if payload_bytes:
                        vals.copy_(vals0)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    radsort.sort_segments_(keys, vals, offsets, tuning=table, workspace=ws,
                                           offsets_dev=off_dev, check=(r == 0))
                    e1.record()
                    e1.synchronize()
                    if r:
                        times.append(e0.elapsed_time(e1))
                ms = float(np.median(times))
                measured[f"{k}/{b}/{bits}"] = ms
                if best is None or ms < best[0]:
                    best = (ms, b, bits)
                del ws
        log(f"tune: 2^{k}: b={best[1]} digits={best[2]} bits, {best[0]:.3f} ms for {count} arrays "
            f"({count * n / best[0] / 1e6:.2f} G keys/s)")
        classes.append((k, best[1], best[2]))
        del keys0, keys, vals0, vals
    classes[-1] = (32, classes[-1][1], classes[-1][2])  # the last class covers larger arrays
    return classes, measured


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--key-bytes", type=int, default=4)
    ap.add_argument("--payload-bytes", type=int, default=4)
    ap.add_argument("--lo", type=int, default=23)
    ap.add_argument("--hi", type=int, default=26)
    ap.add_argument("--elems", type=int, default=1 << 27, help="elements per timed batch")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    classes, measured = tune(args.key_bytes, args.payload_bytes, args.lo, args.hi, args.elems)
    out = args.out or table_path(args.key_bytes, args.payload_bytes)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    json.dump({"key_bytes": args.key_bytes, "payload_bytes": args.payload_bytes,
               "classes": classes, "measured_ms": measured}, open(out, "w"), indent=1)
    print(out)


if __name__ == "__main__":
    main()
