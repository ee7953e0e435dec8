"""The serving loop: each request's result is the same when it runs alone and
when it runs in the mix (admitted by footprint, sharing the GPU with others),
for Radsort and for the out-of-place baseline; small ones also match the oracle."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402
from paper_2607_05302_amd import serve  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def alone(req):
    keys = workloads.uniform_t(req.seed, req.n, req.key_bytes, DEV)
    vals = torch.arange(req.n, dtype=torch.int32, device=DEV)
    radsort.sort_(keys, vals, check=True)
    return keys.cpu().numpy(), vals.cpu().numpy()


@pytest.mark.parametrize("method", ["radsort", "oop"])
def test_results_alone_and_in_the_mix(method):
    trace = serve.make_trace(0x5E4, 14, rate=2e4, lo_log2=10, hi_log2=21)
    budget = 6 * max(serve.footprint(r, method) for r in trace)  # forces waits for memory
    srv = serve.Server(method, budget=budget, slots=6)
    out = srv.run(trace, keep=[r.rid for r in trace])
    assert len(out["latency_ms"]) == len(trace)
    assert out["peak_footprint_bytes"] <= budget
    for r in trace:
        mk, mv = out["kept"][r.rid]
        ak, av = alone(r)
        assert np.array_equal(mk, ak), f"keys of request {r.rid} differ"
        assert np.array_equal(mv, av), f"payload of request {r.rid} differs"
        if r.n <= 1 << 16:
            src = workloads.uniform_t(r.seed, r.n, r.key_bytes, "cpu").numpy()
            src = src.view(np.uint32 if r.key_bytes == 4 else np.uint64)
            ok, ov = oracle.radsort(src, np.arange(r.n, dtype=np.uint32), 256,
                                    r.key_bytes, 1024)
            assert np.array_equal(mk.view(src.dtype).astype(np.uint64), ok)
            assert np.array_equal(mv.view(np.uint32).astype(np.uint64), ov)
