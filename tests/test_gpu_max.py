"""The largest arrays the boundary takes: n = 2^32 - 1 records (uint32 or uint64 keys +
uint32 index, 32 or 48 GiB), 8-bit digits.

Logical slot indices of a round run to (floor(n/b) + sigma)·b, past 2^32, so this
covers the 64-bit slot and position arithmetic of every step (setup, counting
pass, rounds, finalize) for Radsort, the out-of-place baseline and the MSD split.
The oracle does not run at this size: the result is checked chunk by chunk by the
properties that fix a stable sort's result (keys ascending, indices ascending
within equal keys, the indices a permutation, every key equal to the input key at
its index).  At these sizes the block permutation of finalize has more nodes than
one cooperative launch of F1 held in jobs of 1024 nodes (n_pi > 2^20), which once
left blocks unmoved; b = 512 (n_pi > 2^23) takes the two-kernel form of F1.
"""
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
M32 = 0xFFFFFFFF
CHUNK = 1 << 27
SORTS = {"radsort": radsort.sort_, "oop": radsort.oop_sort_, "msd": radsort.msd_sort_}


def unsigned_order(k, kb):
    """Keys as int64 whose signed order is the keys' unsigned order."""
    return (k.long() & M32) if kb == 4 else (k ^ (-(1 << 63)))


@pytest.mark.parametrize("method,kb,b", [("radsort", 4, 2048), ("radsort", 4, 512),
                                         ("radsort", 8, 2048), ("oop", 4, 2048),
                                         ("msd", 4, 2048)])
def test_max_n_pairs(method, kb, b):
    n = (1 << 32) - 1
    print(f"max-size sort: {method}, n = {n} uint{8 * kb} keys + uint32 index, b = {b}",
          flush=True)
    tk = torch.int32 if kb == 4 else torch.int64
    keys = torch.empty(n, dtype=tk, device=DEV)
    vals = torch.empty(n, dtype=torch.int32, device=DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        keys[lo:hi] = workloads.uniform_t(workloads.SEED_LARGE, hi - lo, kb, DEV, start=lo)
        vals[lo:hi] = torch.arange(lo, hi, dtype=torch.int64, device=DEV).to(torch.int32)
    orig = keys.clone()
    SORTS[method](keys, vals, block_elems=b, check=True)
    torch.cuda.synchronize()
    seen = torch.zeros(n, dtype=torch.bool, device=DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        lo0 = max(lo - 1, 0)  # one element of overlap joins the chunks
        k = unsigned_order(keys[lo0:hi], kb)
        v = vals[lo0:hi].long() & M32
        assert bool((k[1:] >= k[:-1]).all()), f"keys not ascending in [{lo0}, {hi})"
        eq = k[1:] == k[:-1]
        assert bool((v[1:][eq] > v[:-1][eq]).all()), f"not stable in [{lo0}, {hi})"
        idx = vals[lo:hi].long() & M32
        assert bool((idx < n).all()), f"index past the array in [{lo}, {hi})"
        seen[idx] = True
        assert bool((orig[idx] == keys[lo:hi]).all()), f"key not the input's in [{lo}, {hi})"
        del k, v, eq, idx
    assert bool(seen.all()), "the indices are not a permutation"
    del keys, vals, orig, seen
    torch.cuda.empty_cache()


def test_max_segments_past_2e32():
    """A batch of more than 2^32 elements: one array of 2^32 - 1 (the Radsort steps
    on a lane) followed by arrays of the small-array and one-workgroup paths whose
    offsets all lie past 2^32."""
    import numpy as np
    rng = np.random.default_rng(0x5EED0007)
    sizes = [(1 << 32) - 1] + rng.integers(1, 8192, 300).tolist() \
        + rng.integers(8193, 4 << 20, 6).tolist()
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offsets[-1])
    print(f"max-size batch: {len(sizes)} arrays, {n} uint32 keys + uint32 index", flush=True)
    keys = torch.empty(n, dtype=torch.int32, device=DEV)
    vals = torch.empty(n, dtype=torch.int32, device=DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        keys[lo:hi] = workloads.uniform_t(workloads.SEED_LARGE, hi - lo, 4, DEV, start=lo)
    for i, s in enumerate(sizes):  # payload: the index within the array
        o = int(offsets[i])
        for lo in range(0, s, CHUNK):
            hi = min(s, lo + CHUNK)
            vals[o + lo:o + hi] = torch.arange(lo, hi, dtype=torch.int64,
                                               device=DEV).to(torch.int32)
    orig = keys.clone()
    radsort.sort_segments_(keys, vals, offsets, check=True)
    torch.cuda.synchronize()
    seen = torch.zeros(n, dtype=torch.bool, device=DEV)
    starts = torch.from_numpy(offsets.astype(np.int64)).to(DEV)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        lo0 = max(lo - 1, 0)
        pos = torch.arange(lo0, hi, dtype=torch.int64, device=DEV)
        seg = torch.searchsorted(starts, pos, right=True) - 1  # array of each position
        k = keys[lo0:hi].long() & M32
        v = vals[lo0:hi].long() & M32
        same = seg[1:] == seg[:-1]
        assert bool((~same | (k[1:] >= k[:-1])).all()), f"keys not ascending in [{lo0}, {hi})"
        eq = same & (k[1:] == k[:-1])
        assert bool((v[1:][eq] > v[:-1][eq]).all()), f"not stable in [{lo0}, {hi})"
        src = starts[seg] + v  # where the element came from
        assert bool((src < starts[seg + 1]).all()), f"index past its array in [{lo0}, {hi})"
        take = slice(lo - lo0, None)
        seen[src[take]] = True
        assert bool((orig[src[take]] == keys[lo:hi]).all()), f"key not the input's in [{lo}, {hi})"
        del pos, seg, k, v, same, eq, src
    assert bool(seen.all()), "the indices are not a permutation of each array"
    del keys, vals, orig, seen
    torch.cuda.empty_cache()
