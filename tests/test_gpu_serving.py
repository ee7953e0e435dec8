"""The serving loop: each request's result is the same when it runs alone (with
the same method) and when it runs in the mix (admitted by footprint under a
budget that makes requests wait for memory, sharing the GPU with others), for
Radsort and for the out-of-place baseline; small ones also match the oracle."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402
from paper_2607_05302_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def drawn(req):
    """The request's input as the server draws it."""
    keys = torch.empty(req.n, dtype=torch.int32 if req.key_bytes == 4 else torch.int64, device=DEV)
    vals = torch.empty(req.n, dtype=torch.int32, device=DEV)
    serve.draw_input(req, keys, vals)
    return keys, vals


def alone(req, method="radsort"):
    keys, vals = drawn(req)
    sort = radsort.sort_ if method == "radsort" else radsort.oop_sort_
    sort(keys, vals, check=True)
    return keys.cpu().numpy(), vals.cpu().numpy()


@pytest.mark.parametrize("method", ["radsort", "oop"])
def test_results_alone_and_in_the_mix(method):
    trace = serve.make_trace(0x5E4, 14, rate=2e4, lo_log2=10, hi_log2=21)
    # one large request among the small ones, and a mid-size one right after it
    trace[5] = serve.Request(5, trace[5].arrival, (1 << 24) + 3, 8, trace[5].seed)
    trace[6] = serve.Request(6, trace[6].arrival, 1 << 21, 8, trace[6].seed)
    # the largest footprint and 5 % more: while the large request runs, the next
    # one cannot fit although slots are free, so it waits for memory
    big = max(serve.footprint(r, method) for r in trace)
    budget = big + big // 20
    assert serve.footprint(trace[6], method) > big // 20
    srv = serve.Server(method, budget=budget, slots=6)
    out = srv.run(trace, keep=[r.rid for r in trace])
    assert len(out["latency_ms"]) == len(trace)
    assert out["peak_footprint_bytes"] <= budget
    assert out["memory_waits"] > 0, "no request waited for memory while a slot was free"
    for r in trace:
        mk, mv = out["kept"][r.rid]
        ak, av = alone(r, method)
        assert np.array_equal(mk, ak), f"keys of request {r.rid} differ"
        assert np.array_equal(mv, av), f"payload of request {r.rid} differs"
        if r.n <= 1 << 16:
            src = drawn(r)[0].cpu().numpy()
            src = src.view(np.uint32 if r.key_bytes == 4 else np.uint64)
            ok, ov = oracle.radsort(src, np.arange(r.n, dtype=np.uint32), 256,
                                    r.key_bytes, 1024)
            assert np.array_equal(mk.view(src.dtype).astype(np.uint64), ok)
            assert np.array_equal(mv.view(np.uint32).astype(np.uint64), ov)


@pytest.mark.parametrize("method", ["radsort", "oop"])
@pytest.mark.parametrize("n,kb", [(3_000_001, 8), (5_000_000, 4)])
def test_workspace_error_reads_clear_after_shared_sorts(method, n, kb):
    req = serve.Request(0, 0.0, n, kb, 0x77 + n)
    keys, vals = drawn(req)
    if method == "radsort":  # sized for a call with shared=True
        wsb = radsort.workspace_bytes(n, kb, 4, 8, 1024, shared=True)
    else:
        wsb = radsort.oop_workspace_bytes(n, kb, 4, 8, 1024)
    ws = torch.full((wsb,), 0xFF, dtype=torch.uint8, device=DEV)
    sort = radsort.sort_ if method == "radsort" else radsort.oop_sort_
    sort(keys, vals, workspace=ws, shared=True)
    assert radsort.workspace_error(keys, vals, workspace=ws,
                                   out_of_place=method == "oop") == 0
    ak, av = alone(req)
    assert np.array_equal(keys.cpu().numpy(), ak)
    assert np.array_equal(vals.cpu().numpy(), av)


def test_concurrent_shared_sorts_are_right():
    """Eight slots of large uint64 and uint32 sorts at a high arrival rate: every
    result checked completely on the device (ascending, stable, the payload a
    permutation, every key the input key at its index) and every sort's error
    word clear.  Tiles of a sort that shares the GPU can run far apart in
    time, which is when a block drawn by one tile and continued by later tiles must
    not be written before its old contents have been loaded."""
    trace = serve.make_trace(0x5E5, 48, rate=2e3, lo_log2=20, hi_log2=25)
    srv = serve.Server("radsort", budget=16e9, slots=8)
    out = srv.run(trace, verify=True)
    assert len(out["latency_ms"]) == len(trace)
    assert out["bad"] == [] and out["device_errors"] == []
