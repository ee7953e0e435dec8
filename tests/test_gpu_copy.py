"""The streaming copy (radsort_copy) that gives the practical HBM ceiling: every
byte copied, for sizes with and without a tail of fewer than 16 bytes and for
sizes that end the unrolled loop at every remainder."""
import ctypes

import pytest
import torch

import paper_2607_05302_amd as radsort

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 17, 31, 4096 * 16 + 15, 4 * 256 * 16 * 3 + 48,
                                    (1 << 24) + 7, (1 << 28) + 16 * 257 + 9])
def test_copy_is_exact(nbytes):
    print(f"copy {nbytes} bytes", flush=True)
    gen = torch.Generator(device="cuda:0").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda:0", generator=gen)
    dst = torch.zeros_like(src)
    lib = radsort.load()
    rc = lib.radsort_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                          None)
    assert rc == radsort.OK
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert not dst[nbytes:].any(), "bytes past the end were written"


def test_copy_binding():
    a = torch.arange(1 << 20, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    radsort.copy_(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
