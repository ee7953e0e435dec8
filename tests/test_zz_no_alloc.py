"""The allocation-free entry point (radsort_sort_pairs_noalloc) against the
existing one (radsort_sort_pairs), through the C ABI: two calls in a row on the
same stream, the second smaller, each compared element by element; then a sort
whose workspace exceeds the static scratch is refused before anything runs."""
import ctypes

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _pair(n, seed, kb):
    keys = workloads.uniform(seed, n, kb)
    view = {4: np.int32, 8: np.int64}[kb]
    k = torch.from_numpy(keys.view(view)).to(DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV)
    return k, v


@pytest.mark.parametrize("kb,b,seq", [(4, 2048, False), (8, 1024, True)])
def test_noalloc_matches_sort_pairs_on_two_calls(kb, b, seq):
    for n, seed in [((1 << 22) + 12345, 0xA110C), ((1 << 16) + 77, 0xA110D)]:
        print(f"noalloc kb={kb} b={b} seq_draws={seq} n={n}", flush=True)
        k1, v1 = _pair(n, seed, kb)
        k2, v2 = k1.clone(), v1.clone()
        radsort.sort_(k1, v1, block_elems=b, seq_draws=seq, check=True)
        radsort.sort_noalloc_(k2, v2, block_elems=b, seq_draws=seq, check=True)
        torch.cuda.synchronize()
        assert torch.equal(k1, k2), n
        assert torch.equal(v1, v2), n


def test_noalloc_keys_only_then_wide_payload():
    """Keys only (8-byte keys), then 4-byte keys with an 8-byte payload, on the
    same scratch: the second call is smaller and its record size differs."""
    n1, n2 = 3_000_017, 100_003
    print(f"noalloc keys only kb=8 n={n1}", flush=True)
    k1 = torch.from_numpy(workloads.uniform(0xA110E, n1, 8).view(np.int64)).to(DEV)
    k2 = k1.clone()
    radsort.sort_(k1, None, block_elems=1024, check=True)
    radsort.sort_noalloc_(k2, None, block_elems=1024, check=True)
    torch.cuda.synchronize()
    assert torch.equal(k1, k2)
    print(f"noalloc kb=4 vb=8 n={n2}", flush=True)
    k1 = torch.from_numpy(workloads.uniform(0xA110F, n2, 4).view(np.int32)).to(DEV)
    v1 = torch.arange(n2, dtype=torch.int64, device=DEV) * 3
    k2, v2 = k1.clone(), v1.clone()
    radsort.sort_(k1, v1, block_elems=512, check=True)
    radsort.sort_noalloc_(k2, v2, block_elems=512, check=True)
    torch.cuda.synchronize()
    assert torch.equal(k1, k2)
    assert torch.equal(v1, v2)


def test_noalloc_refuses_a_workspace_past_the_scratch():
    lib = radsort.load()
    k, v = _pair(1024, 1, 4)
    n = 1 << 30  # its workspace exceeds the static array; refused before any launch
    need = radsort.workspace_bytes(n, 4, 4, 8, 1024)
    assert need > radsort.NOALLOC_SCRATCH_BYTES
    rc = lib.radsort_sort_pairs_noalloc(ctypes.c_void_p(k.data_ptr()),
                                        ctypes.c_void_p(v.data_ptr()), n, 4, 4, 8, 1024, 0,
                                        None)
    assert rc == radsort.E_NOMEM
    # timing events would be created (allocated): refused
    rc = lib.radsort_sort_pairs_noalloc(ctypes.c_void_p(k.data_ptr()),
                                        ctypes.c_void_p(v.data_ptr()), 1024, 4, 4, 8, 1024,
                                        radsort.F_TIMING, None)
    assert rc == radsort.E_INVALID
    # the small sort still runs afterwards and is right
    radsort.sort_noalloc_(k, v, check=True)
    ku = k.cpu().numpy().view(np.uint32)
    assert (ku[1:] >= ku[:-1]).all()
