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
admitted (the seeded streams of `workloads`), on the request's stream.
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


def footprint(req: Request, method: str, block: int = 1024) -> int:
    import paper_2607_05302_amd as radsort
    data = req.n * (req.key_bytes + 4)
    if method == "radsort":
        return data + radsort.workspace_bytes(req.n, req.key_bytes, 4, 8, block)
    return data + radsort.oop_workspace_bytes(req.n, req.key_bytes, 4, 8, block)


class Server:
    def __init__(self, method: str = "radsort", budget: float = 64e9, slots: int = 16,
                 block: int = 1024, device: str = "cuda:0"):
        import torch
        if method not in ("radsort", "oop"):
            raise ValueError(method)
        self.method, self.budget, self.block = method, float(budget), block
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]

    def _start(self, req: Request, stream):
        import torch

        import paper_2607_05302_amd as radsort
        import workloads
        with torch.cuda.stream(stream):
            keys = workloads.uniform_t(req.seed, req.n, req.key_bytes, self.device)
            vals = torch.arange(req.n, dtype=torch.int32, device=self.device)
            if self.method == "radsort":
                ws = torch.empty(radsort.workspace_bytes(req.n, req.key_bytes, 4, 8, self.block),
                                 dtype=torch.uint8, device=self.device)
                radsort.sort_(keys, vals, block_elems=self.block, stream=stream, workspace=ws,
                              shared=True)
            else:
                ws = torch.empty(radsort.oop_workspace_bytes(req.n, req.key_bytes, 4, 8,
                                                             self.block),
                                 dtype=torch.uint8, device=self.device)
                radsort.oop_sort_(keys, vals, block_elems=self.block, stream=stream,
                                  workspace=ws, shared=True)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        return keys, vals, ws, done

    def _check(self, req: Request, keys, vals) -> bool:
        """On the device, after the request's sort: keys ascending (unsigned), the
        same multiset sums as the input keys drawn again from the request's seed,
        and the index payload summing to n (n - 1) / 2.  A check, not a proof: it
        catches lost, duplicated and misplaced records."""
        import torch
        import workloads
        if req.key_bytes == 4:
            k = keys.to(torch.int64) & 0xFFFFFFFF
        else:
            k = keys ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=keys.device)
        ok = req.n < 2 or bool((k[1:] >= k[:-1]).all())
        k0 = workloads.uniform_t(req.seed, req.n, req.key_bytes, self.device)
        ok = ok and bool((k0.to(torch.int64).sum() == keys.to(torch.int64).sum()).item())
        return ok and int(vals.to(torch.int64).sum().item()) == req.n * (req.n - 1) // 2

    def run(self, trace, keep=(), verify=False):
        """Serves the trace in real time.  Returns per-request latencies (ms, from
        arrival to the end of its sort on the GPU), the makespan, the sorted arrays
        of the requests whose ids are in ``keep`` (on the host), and with verify the
        ids of the requests whose result failed `_check` (checked when each
        request completes, on its stream, which adds device work to the run)."""
        import torch

        import paper_2607_05302_amd as radsort
        keep = set(keep)
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        queue = collections.deque()
        free = list(range(len(self.streams)))
        active = {}
        used, peak_used, peak_active = 0, 0, 0
        out = {"latency_ms": {}, "kept": {}, "admit_wait_ms": {}, "bad": [], "device_errors": []}
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
                req, keys, vals, ws, done, fp = active[slot]
                if done.query():
                    out["latency_ms"][req.rid] = t0_ev.elapsed_time(done) - req.arrival * 1e3
                    if req.rid in keep:
                        out["kept"][req.rid] = (keys.cpu().numpy(), vals.cpu().numpy())
                    if verify:
                        with torch.cuda.stream(self.streams[slot]):
                            if not self._check(req, keys, vals):
                                out["bad"].append(req.rid)
                        if radsort.workspace_error(keys, vals, block_elems=self.block,
                                                   stream=self.streams[slot], workspace=ws,
                                                   out_of_place=self.method == "oop"):
                            out["device_errors"].append(req.rid)
                    del active[slot]
                    free.append(slot)
                    used -= fp
                    progressed = True
            while queue and free:
                fp = footprint(queue[0], self.method, self.block)
                if fp > self.budget:
                    raise ValueError(f"request {queue[0].rid} needs {fp} bytes, more than the budget")
                if used + fp > self.budget:
                    break  # first come, first served: wait for memory
                req = queue.popleft()
                slot = free.pop()
                out["admit_wait_ms"][req.rid] = (time.perf_counter() - t0 - req.arrival) * 1e3
                keys, vals, ws, done = self._start(req, self.streams[slot])
                active[slot] = (req, keys, vals, ws, done, fp)
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
        "mean_admit_wait_ms": float(np.mean(list(out["admit_wait_ms"].values()))),
        "wrong_results": len(out.get("bad", [])),
        "device_errors": len(out.get("device_errors", [])),
    }


def offered_load(trace) -> float:
    """Requests per second of the trace."""
    if len(trace) < 2:
        return math.inf
    return (len(trace) - 1) / (trace[-1].arrival - trace[0].arrival)
