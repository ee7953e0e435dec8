"""Autotuner of the batched segmented sort: per size class, the path, block size b
and digit width with the shortest measured time on this GPU.

Arrays of up to 8192 elements (4096 for records of 12 bytes or more) are sorted
whole in LDS and take no tuning.  For each larger class (arrays of up to 2^k
elements, k = lo .. hi) the tuner times a batch with every candidate for that
class and keeps the fastest: the one-workgroup path (one workgroup per array,
5-bit digits, b = 1024; written as b = 0) for classes it can take (up to 4 423 680
elements), and the Radsort steps on the multi-workgroup lanes with b in
{256 .. 8192} and digit bits in {4, 8, 11}.  The earlier classes keep their
choices.  Classes the one-workgroup path can take are timed in a mixed batch of
4096 arrays with sizes log-uniform in [2^10, 2^k], because the two paths share
the GPU when both are used (each class timed alone chose the lanes for 2^22, which
in the mixed batch was slower); larger classes in a batch of arrays of 2^k
elements (at least 2^27 elements, at most 2^30).  Keys are seeded uniform with an
index payload.  The last class also covers every larger array.  The result is a JSON table that sort_segments_ loads by default:

    python -m paper_2607_05302_amd.tune --key-bytes 4 --payload-bytes 4
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
BLOCKS = [256, 512, 1024, 2048, 4096, 8192]
DIGITS = [4, 8, 11]
WG_MAX_ELEMS = (4352 - 32) * 1024  # the one-workgroup path's largest array
WG_MARGIN = 0.02  # how much faster the lanes must be to replace it


def table_path(key_bytes: int, payload_bytes: int) -> str:
    return os.path.join(HERE, "tuning", f"segments_k{key_bytes}_v{payload_bytes}.json")


def load_table(key_bytes: int, payload_bytes: int):
    """[(max_log2n, b, digit_bits), ...] from the tuning file, or None."""
    try:
        t = json.load(open(table_path(key_bytes, payload_bytes)))
    except (OSError, ValueError):
        return None
    return [tuple(c) for c in t["classes"]]


def tune(key_bytes=4, payload_bytes=4, lo=14, hi=26, reps=2, seed=0x7E57, log=print):
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    dev = torch.device("cuda:0")
    classes, measured = [], {}
    prev = []  # the classes chosen so far: earlier classes keep their choice
    for k in range(lo, hi + 1):
        n = 1 << k
        if n <= WG_MAX_ELEMS:  # a mixed batch, as the paths meet in real batches
            sizes = workloads.log_uniform_sizes(seed + k, 4096, 10, k)
            offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        else:
            elems = min(1 << 30, max(1 << 27, 256 * n))
            count = max(4, elems // n)
            offsets = np.arange(count + 1, dtype=np.uint64) * np.uint64(n)
        count, total = len(offsets) - 1, int(offsets[-1])
        off_dev = torch.from_numpy(offsets.view(np.int64)).to(dev)
        keys0 = workloads.uniform_t(seed + k, total, key_bytes, dev)
        vals0 = (torch.arange(total, dtype=torch.int64, device=dev)
                 .to({4: torch.int32, 8: torch.int64}[payload_bytes]) if payload_bytes else None)
        keys = torch.empty_like(keys0)
        vals = torch.empty_like(vals0) if payload_bytes else None
        cands = [(0, 4)] if n <= WG_MAX_ELEMS else []
        cands += [(b, bits) for b in BLOCKS if b <= n for bits in DIGITS]
        best = None
        for b, bits in cands:
            # this class as the candidate, every larger array on the lanes
            table = prev + [(k, b, bits), (64, max(b, 1024), 8)]
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
            # the lanes must beat the one-workgroup path by more than the noise of
            # the timing (it needs less workspace and no lane launches)
            if best is None or ms < best[0] * (1.0 - (WG_MARGIN if best[1] == 0 else 0.0)):
                best = (ms, b, bits)
            del ws
        path = "one workgroup" if best[1] == 0 else f"lanes, b={best[1]}, {best[2]}-bit digits"
        log(f"tune: 2^{k}: {path}: {best[0]:.3f} ms for {count} arrays of {total} elements "
            f"({total / best[0] / 1e6:.2f} G keys/s)", flush=True)
        classes.append((k, best[1], best[2]))
        prev = list(classes)
        del keys0, keys, vals0, vals
        torch.cuda.empty_cache()
    classes[-1] = (32, classes[-1][1], classes[-1][2])  # the last class covers larger arrays
    return classes, measured


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--key-bytes", type=int, default=4)
    ap.add_argument("--payload-bytes", type=int, default=4)
    ap.add_argument("--lo", type=int, default=14)
    ap.add_argument("--hi", type=int, default=26)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    classes, measured = tune(args.key_bytes, args.payload_bytes, args.lo, args.hi)
    out = args.out or table_path(args.key_bytes, args.payload_bytes)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    json.dump({"key_bytes": args.key_bytes, "payload_bytes": args.payload_bytes,
               "classes": classes, "measured_ms": measured}, open(out, "w"), indent=1)
    print(out)


if __name__ == "__main__":
    main()
