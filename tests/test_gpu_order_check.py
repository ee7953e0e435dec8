"""The ordering check of the Radsort round (the library built with RS_DEBUG_ORDER,
flag RADSORT_F_DEBUG_ORDER): every input block is marked once the loads of the
tile that reads it have returned, and every draw of a block that holds input of
the round checks the mark before the draw is published (Lemma 1 on the GPU: a
block is reused only after its old contents were read).  Run under the launch
forms for a GPU shared with other work (RADSORT_F_SHARED), where tiles run in the
most varied order, and under the default forms; with both draw orders.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2607_05302_amd as radsort
from paper_2607_05302_amd import build as hipbuild
import workloads

pytestmark = pytest.mark.gpu


def debug_lib():
    # built by __graft_entry__.build() beside the product library; no fallback
    return radsort.load(hipbuild.DEBUG_ORDER_LIB)


def run(lib, keys, vals, bits, b, flags):
    o = radsort.Opts()
    o.block_elems, o.flags = b, flags | radsort.F_CHECK
    kb = keys.element_size()
    vb = vals.element_size() if vals is not None else 0
    rc = lib.radsort_sort_pairs(ctypes.c_void_p(keys.data_ptr()),
                                ctypes.c_void_p(vals.data_ptr()) if vals is not None else None,
                                keys.numel(), kb, vb, bits, ctypes.byref(o),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    st = radsort.Stats()
    lib.radsort_last_stats(ctypes.byref(st))
    return rc, st.error_bits


def expect_sorted(k0, keys, vals):
    kn = k0.cpu().numpy()
    if kn.dtype == np.int32:
        kn = kn.view(np.uint32)
    else:
        kn = kn.view(np.uint64)
    order = np.argsort(kn, kind="stable")
    gk = keys.cpu().numpy().view(kn.dtype)
    assert np.array_equal(gk, kn[order])
    if vals is not None:
        assert np.array_equal(vals.cpu().numpy().astype(np.int64), order.astype(np.int64))


CASES = [
    # (log2 n or n, key bytes, payload, digit bits, b, flags)
    (1 << 24, 4, True, 8, 1024, radsort.F_SHARED),
    (1 << 24, 4, True, 8, 2048, radsort.F_SHARED),
    (1 << 24, 4, True, 8, 2048, radsort.F_SHARED | radsort.F_SEQ_DRAWS),
    (1 << 24, 4, True, 8, 2048, 0),
    ((1 << 22) + 12345, 8, True, 8, 512, radsort.F_SHARED),
    ((1 << 22) + 777, 4, False, 11, 1024, radsort.F_SHARED),
]


@pytest.mark.parametrize("n,kb,pay,bits,b,flags", CASES)
def test_no_block_drawn_before_its_loads(n, kb, pay, bits, b, flags):
    lib = debug_lib()
    dev = torch.device("cuda:0")
    print(f"ordering check: n={n} key_bytes={kb} payload={pay} bits={bits} b={b} "
          f"flags={flags}", flush=True)
    k0 = workloads.uniform_t(0x0D0E + n + b, n, kb, dev)
    keys = k0.clone()
    vals = (torch.arange(n, dtype=torch.int32 if kb == 4 else torch.int64, device=dev)
            if pay else None)
    rc, bits_set = run(lib, keys, vals, bits, b, flags | radsort.F_DEBUG_ORDER)
    assert rc == radsort.OK and bits_set == 0, (radsort.strerror(rc), bits_set)
    expect_sorted(k0, keys, vals)


def test_check_reports_wrong_marks():
    """With the planted tag every checked draw fails the check: the check can
    report (forced from the host: the kernels run as usual and end normally)."""
    lib = debug_lib()
    dev = torch.device("cuda:0")
    n = 1 << 22
    print(f"ordering check, planted tag: n={n}", flush=True)
    keys = workloads.uniform_t(0x0D0F, n, 4, dev)
    vals = torch.arange(n, dtype=torch.int32, device=dev)
    rc, bits_set = run(lib, keys, vals, 8, 1024,
                       radsort.F_SHARED | radsort.F_DEBUG_ORDER | radsort.F_DEBUG_PLANT)
    assert rc == radsort.E_ORDER
    assert bits_set & 4
