"""A serving loop for sort requests: continuous batching by device-memory footprint.

Requests arrive over time (Poisson arrivals, log-uniform sizes, uint32 or uint64
keys with a uint32 index payload).  A request is admitted as soon as a slot (a
stream) is free and its footprint fits in the memory budget still unused;
admitted requests run at the same time on their own streams, and their memory is
returned when they finish.  The footprint is what the method needs on the device:
the keys and payload plus Radsort's O(sqrt n) workspace, or plus a second copy of
the arrays for the out-of-place baseline (Alg. 1), so under the same budget
Radsort admits about twice as much work.

The sorts run with RADSORT_F_SHARED: their kernels need no co-resident grid, so
several can share the GPU.  Inputs are drawn on the device when a request is
admitted, on the request's stream (`draw_input`: torch's device generator seeded
with the request's seed, one pass over the keys).

Device memory: one buffer of the budget's size, allocated when the server starts,
carved first-fit into one region per admitted request (keys, payload, workspace)
by `Arena`.  A request is admitted when a free range holds its region, so the
budget is a hard limit, and the loop makes no device allocation of that size
while it runs (allocating and freeing arrays of ever different sizes through
torch's caching allocator grew its reserve to the whole device, and the frees that
followed stalled every stream for up to seconds).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the trace
    n: int
    key_bytes: int
    seed: int


def make_trace(seed: int, count: int, rate: float, lo_log2: float = 12, hi_log2: float = 28):
    """``count`` requests: exponential gaps of mean 1/rate, sizes log-uniform in
    [2^lo_log2, 2^hi_log2], keys of 4 or 8 bytes with probability 1/2 each."""
    import workloads
    w = workloads.words(seed, 2 * count)
    u = (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    gaps = -np.log1p(-u[:count]) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = workloads.log_uniform_sizes(seed ^ 0x51235, count, lo_log2, hi_log2)
    widths = np.where(u[count:] < 0.5, 4, 8)
    return [Request(i, float(arrivals[i]), int(max(1, sizes[i])), int(widths[i]),
                    seed * 1000003 + i) for i in range(count)]


ALIGN = 256  # bytes; every array of a region starts on this boundary


def _align(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


def region(req: Request, method: str, block: int = 1024):
    """Byte offsets of the keys, the payload and the workspace within a request's
    region, and the region's size."""
    import paper_2607_05302_amd as radsort
    if method == "radsort":  # its sorts run with shared=True
        wsb = radsort.workspace_bytes(req.n, req.key_bytes, 4, 8, block, shared=True)
    else:
        wsb = radsort.oop_workspace_bytes(req.n, req.key_bytes, 4, 8, block)
    o_v = _align(req.n * req.key_bytes)
    o_w = o_v + _align(req.n * 4)
    return 0, o_v, o_w, o_w + _align(wsb)


def footprint(req: Request, method: str, block: int = 1024) -> int:
    """Device bytes a request holds while it runs: keys and payload plus Radsort's
    workspace, or plus the baseline's second arrays (each array 256-byte aligned)."""
    return region(req, method, block)[3]


DRAW_CHUNK = 1 << 24  # keys per piece when drawing and checking inputs


def draw_input(req: Request, keys, vals):
    """Fills ``keys`` (int32 or int64, read as unsigned) with the request's input,
    uniform over all bit patterns, and ``vals`` with 0 .. n-1, on the current
    stream: torch's device generator seeded with the request's seed, drawn in
    pieces of DRAW_CHUNK keys, so that the same request always gets the same keys
    and a draw costs one pass over them."""
    import torch
    g = torch.Generator(device=keys.device)
    g.manual_seed(req.seed & 0x7FFFFFFFFFFFFFFF)
    lo_hi = (-(1 << 31), 1 << 31) if req.key_bytes == 4 else (-(1 << 63), (1 << 63) - 1)
    for lo in range(0, req.n, DRAW_CHUNK):
        hi = min(req.n, lo + DRAW_CHUNK)
        torch.randint(*lo_hi, (hi - lo,), generator=g, dtype=keys.dtype, device=keys.device,
                      out=keys[lo:hi])
        torch.arange(lo, hi, dtype=torch.int32, device=vals.device, out=vals[lo:hi])


class Arena:
    """First-fit allocation of byte ranges in [0, size): `alloc` returns the lowest
    offset of a free range that holds ``nbytes`` (rounded up to ALIGN), or None;
    `release` returns a range and merges it with free neighbours."""

    def __init__(self, size: int):
        self.size = size // ALIGN * ALIGN
        self.free = [(0, self.size)] if self.size else []  # (offset, length), by offset

    def alloc(self, nbytes: int):
        need = _align(max(nbytes, 1))
        for i, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, ln - need)
                return off
        return None

    def release(self, off: int, nbytes: int):
        ln = _align(max(nbytes, 1))
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] > off:
            raise ValueError("range released twice or overlaps a free range")
        if i < len(self.free) and off + ln > self.free[i][0]:
            raise ValueError("range released twice or overlaps a free range")
        self.free.insert(i, (off, ln))
        if i + 1 < len(self.free) and off + ln == self.free[i + 1][0]:
            self.free[i] = (off, ln + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def free_bytes(self) -> int:
        return sum(ln for _, ln in self.free)


class Server:
    def __init__(self, method: str = "radsort", budget: float = 64e9, slots: int = 16,
                 block: int = 1024, device: str = "cuda:0"):
        import torch
        if method not in ("radsort", "oop"):
            raise ValueError(method)
        self.method, self.budget, self.block = method, float(budget), block
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.arena = Arena(int(budget))
        self.buf = torch.empty(self.arena.size, dtype=torch.uint8, device=self.device)

    def _start(self, req: Request, stream, base: int):
        """Draws the request's input into its region at byte offset ``base`` of the
        arena and sorts it, all on ``stream``."""
        import torch

        import paper_2607_05302_amd as radsort
        o_k, o_v, o_w, end = region(req, self.method, self.block)
        kdt = torch.int32 if req.key_bytes == 4 else torch.int64
        keys = self.buf[base + o_k: base + o_k + req.n * req.key_bytes].view(kdt)
        vals = self.buf[base + o_v: base + o_v + req.n * 4].view(torch.int32)
        ws = self.buf[base + o_w: base + end]
        with torch.cuda.stream(stream):
            draw_input(req, keys, vals)
            sort = radsort.sort_ if self.method == "radsort" else radsort.oop_sort_
            sort(keys, vals, block_elems=self.block, stream=stream, workspace=ws, shared=True)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        return keys, vals, ws, done

    def _check(self, req: Request, keys, vals, k_in, seen) -> bool:
        """On the device, after the request's sort, the complete check of a stable
        sort with an index payload: keys ascending (unsigned), equal keys in
        ascending index, the payload a permutation of 0 .. n-1, and every key equal
        to the input key at its index (the input drawn again from the request's
        seed into ``k_in``; ``seen`` holds at least n flags)."""
        import torch
        n = req.n
        g = torch.Generator(device=keys.device)
        g.manual_seed(req.seed & 0x7FFFFFFFFFFFFFFF)
        lo_hi = (-(1 << 31), 1 << 31) if req.key_bytes == 4 else (-(1 << 63), (1 << 63) - 1)
        kin = k_in[:n * req.key_bytes // k_in.element_size()].view(keys.dtype)
        for lo in range(0, n, DRAW_CHUNK):  # as draw_input draws it
            hi = min(n, lo + DRAW_CHUNK)
            torch.randint(*lo_hi, (hi - lo,), generator=g, dtype=keys.dtype, device=keys.device,
                          out=kin[lo:hi])
        flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=keys.device)
        bad = torch.zeros((), dtype=torch.int64, device=keys.device)
        seen_n = seen[:n]
        seen_n.zero_()
        for lo in range(0, n, DRAW_CHUNK):  # neighbouring pieces overlap by one record
            hi = min(n, lo + DRAW_CHUNK)
            a = max(lo - 1, 0)
            k = keys[a:hi]
            u = (k.to(torch.int64) & 0xFFFFFFFF) if req.key_bytes == 4 else k ^ flip
            v = vals[a:hi].to(torch.int64)
            bad += (u[1:] < u[:-1]).sum()                                   # ascending
            bad += ((u[1:] == u[:-1]) & (v[1:] <= v[:-1])).sum()            # stable
            vv = vals[lo:hi].to(torch.int64)
            bad += ((vv < 0) | (vv >= n)).sum()
            vc = vv.clamp(0, n - 1)
            seen_n[vc] = True                                               # permutation
            bad += (kin[vc] != keys[lo:hi]).sum()                           # its own key
        bad += (~seen_n).sum()
        return int(bad.item()) == 0

    def run(self, trace, keep=(), verify=False):
        """Serves the trace in real time.  Returns per-request latencies (ms, from
        arrival to the end of its sort on the GPU), the makespan, the sorted arrays
        of the requests whose ids are in ``keep`` (on the host), the number of
        requests that waited for memory while a slot was free, and with verify the
        ids of the requests whose result failed `_check` (checked when each
        request completes, on its stream, which adds device work to the run)."""
        import torch

        import paper_2607_05302_amd as radsort
        keep = set(keep)
        k_in = seen = None
        if verify:  # scratch of the complete check, sized for the largest request
            big = max((r.n for r in trace), default=1)
            k_in = torch.empty(big * 8, dtype=torch.uint8, device=self.device)
            seen = torch.empty(big, dtype=torch.bool, device=self.device)
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        queue = collections.deque()
        free = list(range(len(self.streams)))
        active = {}
        used, peak_used, peak_active = 0, 0, 0
        waited = set()  # requests that found a free slot but not enough free memory
        out = {"latency_ms": {}, "kept": {}, "admit_wait_ms": {}, "bad": [], "device_errors": [],
               "memory_waits": 0}
        torch.cuda.synchronize(self.device)
        t0_ev = torch.cuda.Event(enable_timing=True)
        t0_ev.record(torch.cuda.current_stream(self.device))
        t0_ev.synchronize()
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
                progressed = True
            for slot in list(active):
                req, keys, vals, ws, done, fp, base = active[slot]
                if done.query():
                    out["latency_ms"][req.rid] = t0_ev.elapsed_time(done) - req.arrival * 1e3
                    if req.rid in keep:
                        out["kept"][req.rid] = (keys.cpu().numpy(), vals.cpu().numpy())
                    if verify:
                        with torch.cuda.stream(self.streams[slot]):
                            if not self._check(req, keys, vals, k_in, seen):
                                out["bad"].append(req.rid)
                        if radsort.workspace_error(keys, vals, block_elems=self.block,
                                                   stream=self.streams[slot], workspace=ws,
                                                   out_of_place=self.method == "oop"):
                            out["device_errors"].append(req.rid)
                    del active[slot], keys, vals, ws
                    self.arena.release(base, fp)
                    free.append(slot)
                    used -= fp
                    progressed = True
            while queue and free:
                fp = footprint(queue[0], self.method, self.block)
                if fp > self.arena.size:
                    raise ValueError(f"request {queue[0].rid} needs {fp} bytes, more than the budget")
                base = self.arena.alloc(fp)
                if base is None:
                    # first come, first served: a slot is free, the memory is not
                    if queue[0].rid not in waited:
                        waited.add(queue[0].rid)
                        out["memory_waits"] += 1
                    break
                req = queue.popleft()
                slot = free.pop()
                out["admit_wait_ms"][req.rid] = (time.perf_counter() - t0 - req.arrival) * 1e3
                keys, vals, ws, done = self._start(req, self.streams[slot], base)
                active[slot] = (req, keys, vals, ws, done, fp, base)
                used += fp
                peak_used = max(peak_used, used)
                peak_active = max(peak_active, len(active))
                progressed = True
            if not progressed:
                time.sleep(20e-6)
        torch.cuda.synchronize(self.device)
        out["makespan_ms"] = (time.perf_counter() - t0) * 1e3
        out["peak_footprint_bytes"] = peak_used
        out["peak_active"] = peak_active
        return out


def summarize(trace, out) -> dict:
    lat = np.array([out["latency_ms"][r.rid] for r in trace])
    keys = sum(r.n for r in trace)
    span = max(out["latency_ms"][r.rid] + r.arrival * 1e3 for r in trace)
    return {
        "requests": len(trace),
        "keys": keys,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "keys_per_s": keys / (span / 1e3),
        "span_ms": float(span),
        "peak_footprint_bytes": int(out["peak_footprint_bytes"]),
        "peak_active": int(out["peak_active"]),
        # requests on the GPU at once, averaged over the span: each is active from
        # its admission to the end of its sort
        "mean_active": float(sum(out["latency_ms"][r.rid] - out["admit_wait_ms"][r.rid]
                                 for r in trace) / span),
        "mean_admit_wait_ms": float(np.mean(list(out["admit_wait_ms"].values()))),
        "memory_waits": int(out.get("memory_waits", 0)),
        "wrong_results": len(out.get("bad", [])),
        "device_errors": len(out.get("device_errors", [])),
    }


def offered_load(trace) -> float:
    """Requests per second of the trace."""
    if len(trace) < 2:
        return math.inf
    return (len(trace) - 1) / (trace[-1].arrival - trace[0].arrival)
