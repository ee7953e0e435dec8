"""Per-tile timeline of the Radsort round kernel (a profiling build).

Builds the library with RS_TIMELINE defined into ``_lib_timeline/``; in that
build thread 0 of every workgroup of the round kernel records the GPU's 100 MHz
real-time counter at the boundaries of each tile's steps.  One sort is run, and
the stamps of its last round are summarised per step (mean and median over the
tiles, in microseconds).  Steps (stamp pairs):

    start      workgroup launch -> tile claimed and its block table read
    load+rank  the tile's loads issued, stable ranks within waves, loads waited for
    counts     tile counts published, digit scan, wave offsets
    stage      records staged in LDS in (digit, slot) order
    lookback   digit starts from the super-tile start and earlier tiles' counts
    (the default draw order stages the tile after publishing its draws)
    d:count    blocks drawn and written per digit, F, their scans
    d:pool+wait  pool entries read, waits for the tiles that read those blocks
    d:publish  the tile's draws published in pi'
    d:first    each digit's first block (drawn by an earlier tile) waited for
    ptrs       the table of block addresses
    keys       keys written out
    stage_v    payload staged in LDS
    vals       payload written out (stores waited for)

    python -m paper_2607_05302_amd.timeline [--log2n 28] [--block 2048] [--seq-draws]

The timeline build is a separate library; the product library records nothing.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import subprocess

from . import build as hipbuild

HERE = os.path.dirname(os.path.abspath(__file__))
TL_DIR = os.path.join(HERE, "_lib_timeline")
TL_LIB = os.path.join(TL_DIR, "libradsort.so")
STAMPS = 16
# a step is named by the stamp that ends it and runs from the stamp before it in
# time (the order of the steps differs between draw orders)
STEP_END = {0: "start", 1: "load+rank", 2: "counts", 13: "(to stage)", 3: "stage",
            4: "lookback", 10: "d:count", 11: "d:pool+wait", 12: "d:publish", 5: "d:first",
            6: "ptrs", 7: "keys", 8: "stage_v", 9: "vals"}


def build_timeline() -> str:
    os.makedirs(TL_DIR, exist_ok=True)
    subprocess.run(hipbuild._command(TL_LIB, ("RS_TIMELINE",)), check=True)
    return TL_LIB


def run(log2n: int, block: int, seq_draws: bool, rebuild: bool = True) -> dict:
    import numpy as np
    import torch

    import paper_2607_05302_amd as radsort
    import workloads

    if rebuild or not os.path.exists(TL_LIB):
        build_timeline()
    radsort.LIB_PATH = TL_LIB
    lib = radsort.load()
    fn = lib.radsort_timeline_buffer
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    dev = torch.device("cuda:0")
    n = 1 << log2n
    keys = workloads.make_t("uniform", workloads.SEED_LARGE, n, 4, dev)
    vals = torch.arange(n, dtype=torch.int32, device=dev)
    tiles_cap = (n >> 10) + 1024  # more than the tiles of any round here
    buf = torch.zeros(tiles_cap * STAMPS, dtype=torch.int64, device=dev)
    fn(ctypes.c_void_p(buf.data_ptr()), tiles_cap)
    radsort.sort_(keys.clone(), vals.clone(), block_elems=block, seq_draws=seq_draws)
    torch.cuda.synchronize()
    buf.zero_()
    radsort.sort_(keys, vals, block_elems=block, seq_draws=seq_draws, check=True)
    torch.cuda.synchronize()
    fn(None, 0)
    st = buf.cpu().numpy().reshape(tiles_cap, STAMPS)
    used = st[:, 9] != 0
    st = st[used]
    out = {"tiles": int(used.sum()), "steps_us": {}}
    order = [15] + sorted(STEP_END, key=lambda k: np.median(st[:, k] - st[:, 15]))
    for prev, k in zip(order, order[1:]):
        d = (st[:, k] - st[:, prev]) / 100.0  # 100 MHz ticks -> us
        out["steps_us"][STEP_END[k]] = (float(d.mean()), float(np.median(d)))
    whole = (st[:, 9] - st[:, 15]) / 100.0
    span = (st[:, 9].max() - st[:, 15].min()) / 100.0
    out["tile_us"] = (float(whole.mean()), float(np.median(whole)))
    out["span_us"] = float(span)
    out["tiles_in_flight"] = float(whole.sum() / span)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--block", type=int, default=2048)
    ap.add_argument("--seq-draws", action="store_true")
    ap.add_argument("--no-build", action="store_true", help="use the timeline library built before")
    args = ap.parse_args()
    r = run(args.log2n, args.block, args.seq_draws, rebuild=not args.no_build)
    print(f"last round of a sort of 2^{args.log2n} uint32 keys + uint32 index, b = {args.block}: "
          f"{r['tiles']} tiles, span {r['span_us']:.0f} us, "
          f"{r['tiles_in_flight']:.0f} tiles in flight on average")
    print(f"{'step':12s} {'mean us':>9s} {'median us':>10s}")
    for name, (m, md) in r["steps_us"].items():
        print(f"{name:12s} {m:9.2f} {md:10.2f}")
    m, md = r["tile_us"]
    print(f"{'whole tile':12s} {m:9.2f} {md:10.2f}")


if __name__ == "__main__":
    main()
