"""GPU parity of the batched segmented sort (many independent arrays in one call),
through the C ABI, against the oracle applied to every array; and the same call
captured into a graph and replayed."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NP = {4: np.uint32, 8: np.uint64}
TV = {4: torch.int32, 8: torch.int64}


def say(msg):
    print(msg, flush=True)


def batch(seed, sizes, kb):
    """Concatenated arrays: seeded uniform keys, payload = index within the array."""
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = workloads.uniform(seed, int(offsets[-1]), kb)
    vals = np.concatenate([np.arange(s, dtype=np.uint32) for s in sizes]) if len(sizes) else \
        np.zeros(0, np.uint32)
    return offsets, keys, vals


def to_dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view({4: np.int32, 8: np.int64}[a.dtype.itemsize])).to(DEV)


def expected(offsets, keys, vals, kb):
    ek = np.empty(len(keys), np.uint64)
    ev = np.empty(len(vals), np.uint64)
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        if b > a:
            k, v = oracle.radsort(keys[a:b], vals[a:b], 256, kb, 1024)
            ek[a:b], ev[a:b] = k, v
    return ek, ev


EDGE = [0, 1, 2, 3, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 20000, 70000]
# the one-workgroup path takes arrays of 8193 .. WG_MAX elements (4096 + 1 .. for
# records of 12 bytes or more: n_pi = n / 1024 + 32 <= 4352); larger ones run the
# Radsort steps on the lanes
WG_MAX = (4352 - 32) * 1024


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("tuned", [False, True])
def test_segments_match_oracle(kb, tuned):
    say(f"segments kb={kb} tuned={tuned}")
    sizes = list(workloads.log_uniform_sizes(0x5E6, 200, 0, 19)) + EDGE
    if tuned:  # one array past the one-workgroup path: the table's last class takes it
        sizes.append(WG_MAX + 1000)
    offsets, keys, vals = batch(0x5E7 + kb, sizes, kb)
    tuning = [(13, 128, 4), (16, 512, 8), (32, 1024, 11)] if tuned else None
    dk, dv = to_dev(keys), to_dev(vals)
    radsort.sort_segments_(dk, dv, offsets, tuning=tuning, check=True)
    ek, ev = expected(offsets, keys, vals, kb)
    assert np.array_equal(dk.cpu().numpy().view(NP[kb]).astype(np.uint64), ek)
    assert np.array_equal(dv.cpu().numpy().view(np.uint32).astype(np.uint64), ev)


@pytest.mark.parametrize("kb", [4, 8])
def test_segments_mixed_paths_match_oracle(kb):
    """A table that keeps arrays up to 2^15 on the one-workgroup path and sends the
    larger ones to the lanes (two classes there); the lanes run beside the batched
    kernels."""
    say(f"segments mixed paths kb={kb}")
    sizes = list(workloads.log_uniform_sizes(0x5E8, 120, 10, 20)) + EDGE
    offsets, keys, vals = batch(0x5E9 + kb, sizes, kb)
    tuning = [(15, 0, 4), (18, 512, 8), (32, 2048, 11)]
    dk, dv = to_dev(keys), to_dev(vals)
    radsort.sort_segments_(dk, dv, offsets, tuning=tuning, check=True)
    ek, ev = expected(offsets, keys, vals, kb)
    assert np.array_equal(dk.cpu().numpy().view(NP[kb]).astype(np.uint64), ek)
    assert np.array_equal(dv.cpu().numpy().view(np.uint32).astype(np.uint64), ev)


def test_segments_keys_only_and_empty():
    sizes = [0, 5, 0, 9000, 1, 0]
    offsets, keys, _ = batch(11, sizes, 4)
    dk = to_dev(keys)
    radsort.sort_segments_(dk, None, offsets, check=True)
    got = dk.cpu().numpy().view(np.uint32)
    for i in range(len(sizes)):
        a, b = int(offsets[i]), int(offsets[i + 1])
        assert np.array_equal(got[a:b], np.sort(keys[a:b]))
    radsort.sort_segments_(dk, None, np.zeros(1, np.uint64), check=True)  # no arrays


def test_segments_graph_replay():
    """The call, with a caller workspace, captured once and replayed three times;
    between replays the input is restored and other work runs eagerly, and every
    replay must give the eager result."""
    sizes = list(workloads.log_uniform_sizes(0x5E8, 64, 6, 18))
    offsets, keys, vals = batch(0x5E9, sizes, 4)
    k0, v0 = to_dev(keys), to_dev(vals)
    dk, dv = k0.clone(), v0.clone()
    off_dev = torch.from_numpy(offsets.view(np.int64)).to(DEV)
    ws = torch.empty(radsort.segments_workspace_bytes(offsets, 4, 4), dtype=torch.uint8,
                     device=DEV)
    radsort.sort_segments_(dk, dv, offsets, workspace=ws, offsets_dev=off_dev, check=True)
    ek, ev = dk.clone(), dv.clone()
    dk.copy_(k0)
    dv.copy_(v0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        radsort.sort_segments_(dk, dv, offsets, workspace=ws, offsets_dev=off_dev)
    for rep in range(3):
        dk.copy_(k0)
        dv.copy_(v0)
        junk = torch.arange(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(junk) == (1 << 20) * ((1 << 20) - 1) // 2
        assert torch.equal(dk, ek), f"keys differ on replay {rep}"
        assert torch.equal(dv, ev), f"payload differs on replay {rep}"




@pytest.mark.parametrize("kb,vb", [(4, 0), (4, 4), (4, 8), (8, 0), (8, 4), (8, 8)])
def test_segments_one_workgroup_path(kb, vb):
    """Every key and payload width through the one-workgroup path, at the sizes
    that bound it (a block, a tile, several thousand blocks, its largest array)
    and the first size past it (the lanes)."""
    sizes = [0, 5, 4096, 4097, 8192, 8193, 9000, 1 << 13 | 1 << 10, (1 << 16) + 3, 70000,
             (1 << 18) + 11, 1 << 20, 3 * (1 << 20) + 5, WG_MAX, WG_MAX + 1]
    say(f"one-workgroup path kb={kb} vb={vb}")
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = workloads.uniform(0x5EA + kb + vb, int(offsets[-1]), kb)
    vals = (np.concatenate([np.arange(s, dtype=NP[vb]) for s in sizes]) if vb else None)
    dk = to_dev(keys)
    dv = to_dev(vals) if vb else None
    radsort.sort_segments_(dk, dv, offsets, check=True)
    got_k = dk.cpu().numpy().view(NP[kb])
    got_v = dv.cpu().numpy().view(NP[vb]) if vb else None
    for i in range(len(sizes)):
        a, b = int(offsets[i]), int(offsets[i + 1])
        if b - a < 2:
            continue
        k, v = oracle.radsort(keys[a:b], vals[a:b] if vb else None, 256, kb, 1024)
        assert np.array_equal(got_k[a:b].astype(np.uint64), k), (i, sizes[i])
        if vb:
            assert np.array_equal(got_v[a:b].astype(np.uint64), v), (i, sizes[i])


@pytest.mark.parametrize("dist", ["equal", "sorted", "zipf", "few", "low20"])
def test_segments_one_workgroup_path_structured(dist):
    """Structured keys through the one-workgroup path: one bucket takes every
    element (all equal), runs already in order (sorted), heavy skew (Zipf), three
    values, and rounds whose digits are all zero (low 20 bits)."""
    kb = 8
    sizes = [9000, 70000, (1 << 20) + 333, WG_MAX]
    say(f"one-workgroup path structured {dist}")
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([workloads.make(dist, 0x5EB + i, s, kb) for i, s in enumerate(sizes)])
    vals = np.concatenate([np.arange(s, dtype=np.uint32) for s in sizes])
    dk, dv = to_dev(keys), to_dev(vals)
    radsort.sort_segments_(dk, dv, offsets, check=True)
    got_k = dk.cpu().numpy().view(np.uint64)
    got_v = dv.cpu().numpy().view(np.uint32)
    for i in range(len(sizes)):
        a, b = int(offsets[i]), int(offsets[i + 1])
        k, v = oracle.radsort(keys[a:b], vals[a:b], 256, kb, 1024)
        assert np.array_equal(got_k[a:b], k), (dist, sizes[i])
        assert np.array_equal(got_v[a:b].astype(np.uint64), v), (dist, sizes[i])


def test_segments_one_workgroup_path_repeated():
    """The same batch sorted ten times in a row, each time from fresh copies: a
    3 M-element array of 12-byte records (one workgroup for a long time) beside
    its neighbours in the batch.  A hazard that shows only now and then (a wrong
    histogram, a block written before it was read) fails one of the calls."""
    kb, vb = 4, 8
    sizes = [9000, (1 << 20), 3 * (1 << 20) + 5, 70000]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = workloads.uniform(0x5EC, int(offsets[-1]), kb)
    vals = np.concatenate([np.arange(s, dtype=np.uint64) for s in sizes])
    want = []
    for i in range(len(sizes)):
        a, b = int(offsets[i]), int(offsets[i + 1])
        want.append(oracle.radsort(keys[a:b], vals[a:b], 256, kb, 1024))
    for rep in range(10):
        say(f"one-workgroup path repeated call {rep}")
        dk, dv = to_dev(keys), to_dev(vals)
        radsort.sort_segments_(dk, dv, offsets, check=True)
        got_k = dk.cpu().numpy().view(np.uint32)
        got_v = dv.cpu().numpy().view(np.uint64)
        for i, (k, v) in enumerate(want):
            a, b = int(offsets[i]), int(offsets[i + 1])
            assert np.array_equal(got_k[a:b].astype(np.uint64), k), (rep, sizes[i])
            assert np.array_equal(got_v[a:b], v), (rep, sizes[i])


@pytest.mark.parametrize("kb", [4, 8])
def test_segments_lanes_run_concurrently(kb):
    """Eight arrays past the one-workgroup path: the lanes sort them on four
    streams at once in the dynamic launch form (the form whose tiles can run far
    apart in time), each array against the oracle."""
    sizes = [WG_MAX + 1 + i * 1_300_021 for i in range(8)]
    say(f"segments lanes kb={kb} total={sum(sizes)}")
    offsets, keys, vals = batch(0x5EA + kb, sizes, kb)
    dk, dv = to_dev(keys), to_dev(vals)
    radsort.sort_segments_(dk, dv, offsets, check=True)
    ek, ev = expected(offsets, keys, vals, kb)
    assert np.array_equal(dk.cpu().numpy().view(NP[kb]).astype(np.uint64), ek)
    assert np.array_equal(dv.cpu().numpy().view(np.uint32).astype(np.uint64), ev)
