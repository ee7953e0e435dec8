"""The largest array the boundary takes: n = 2^32 - 1 uint32 keys + uint32 index
(32 GiB of records), 8-bit digits, b = 2048 and b = 512.

Logical slot indices of a round run to (floor(n/b) + sigma)·b, past 2^32, so this
covers the 64-bit slot and position arithmetic of every step (setup, counting
pass, rounds, finalize).  The oracle does not run at this size: the result is
checked chunk by chunk by the properties that fix a stable sort's result (keys
ascending, indices ascending within equal keys, the indices a permutation, every
key equal to the input key at its index).  At these sizes the block permutation
of finalize has more nodes than one cooperative launch of F1 held in jobs of 1024
nodes (n_pi > 2^20), which once left blocks unmoved; b = 512 (n_pi > 2^23) takes
the two-kernel form of F1.
"""
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
M32 = 0xFFFFFFFF
CHUNK = 1 << 27


@pytest.mark.parametrize("b", [2048, 512])
def test_max_n_u32_pairs(b):
    n = (1 << 32) - 1
    print(f"max-size sort: n = {n} uint32 keys + uint32 index, b = {b}", flush=True)
    keys = torch.empty(n, dtype=torch.int32, device=DEV)
    vals = torch.empty(n, dtype=torch.int32, device=DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        keys[lo:hi] = workloads.uniform_t(workloads.SEED_LARGE, hi - lo, 4, DEV, start=lo)
        vals[lo:hi] = torch.arange(lo, hi, dtype=torch.int64, device=DEV).to(torch.int32)
    orig = keys.clone()
    radsort.sort_(keys, vals, block_elems=b, check=True)
    torch.cuda.synchronize()
    seen = torch.zeros(n, dtype=torch.bool, device=DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        lo0 = max(lo - 1, 0)  # one element of overlap joins the chunks
        k = keys[lo0:hi].long() & M32
        v = vals[lo0:hi].long() & M32
        assert bool((k[1:] >= k[:-1]).all()), f"keys not ascending in [{lo0}, {hi})"
        eq = k[1:] == k[:-1]
        assert bool((v[1:][eq] > v[:-1][eq]).all()), f"not stable in [{lo0}, {hi})"
        idx = vals[lo:hi].long() & M32
        seen[idx] = True
        assert bool((orig[idx] == keys[lo:hi]).all()), f"key not the input's in [{lo}, {hi})"
        del k, v, eq, idx
    assert bool(seen.all()), "the indices are not a permutation"
    del keys, vals, orig, seen
    torch.cuda.empty_cache()
