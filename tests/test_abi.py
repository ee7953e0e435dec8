"""The C ABI without a GPU: the library loads, exports every function that
include/radsort.h declares, sizes its workspace, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_2607_05302_amd as radsort

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radsort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(radsort_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(radsort.ABI)


def test_library_exports_every_declared_symbol():
    lib = radsort.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_formula_and_one_percent_budget():
    # n = 2^28 uint32 keys + uint32 payload, b = 1024, 8-bit digits
    n = 1 << 28
    ws = radsort.workspace_bytes(n, 4, 4, 8, 1024)
    sigma, b = 256, 1024
    t_bytes = 2 * sigma * b * 8
    npi = n // b + 2 * sigma
    assert ws >= t_bytes + 2 * 4 * npi
    assert ws <= 0.01 * n * 8, ws / (n * 8)
    # the out-of-place baseline needs a second array
    assert radsort.oop_workspace_bytes(n, 4, 4, 8, 1024) >= n * 8


def test_workspace_is_order_sqrt_n():
    ratios = []
    for lg in range(16, 31, 2):
        n = 1 << lg
        b = max(64, 1 << ((lg + 1) // 2))
        ratios.append(radsort.workspace_bytes(n, 4, 4, 8, b) / (n ** 0.5))
    assert max(ratios) / min(ratios) < 8


@pytest.mark.parametrize("args,code", [
    ((1000, 3, 0, 8), radsort.E_INVALID),      # key width
    ((1000, 4, 2, 8), radsort.E_INVALID),      # payload width
    ((1000, 4, 0, 0), radsort.E_INVALID),      # digit width
    ((1000, 4, 0, 12), radsort.E_UNSUPPORTED),
    ((1 << 32, 4, 0, 8), radsort.E_UNSUPPORTED),
])
def test_argument_errors(args, code):
    lib = radsort.load()
    n, kb, vb, bits = args
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation comes first
    rc = lib.radsort_sort_pairs(fake, fake if vb else None, n, kb, vb, bits, None, None)
    assert rc == code
    assert radsort.workspace_bytes(n, kb, vb, bits) == 0


@pytest.mark.parametrize("bits", range(12, 17))
@pytest.mark.parametrize("kb,vb", [(4, 0), (4, 4), (8, 8)])
def test_wide_digits_are_unsupported(bits, kb, vb):
    """digit_bits 12 .. 16 is a valid argument that every call refuses (the state's
    2 sigma head blocks, the per-wave LDS counts and sub-line digit runs rule it
    out); 17 is invalid."""
    lib = radsort.load()
    fake = ctypes.c_void_p(0x1000)
    n = 1 << 20
    pv = fake if vb else None
    assert lib.radsort_sort_pairs(fake, pv, n, kb, vb, bits, None, None) == radsort.E_UNSUPPORTED
    assert lib.radsort_oop_sort_pairs(fake, pv, n, kb, vb, bits, None, None) == radsort.E_UNSUPPORTED
    assert lib.radsort_msd_sort_pairs(fake, pv, n, kb, vb, bits, None, None) == radsort.E_UNSUPPORTED
    assert lib.radsort_sort_pairs_noalloc(fake, pv, n, kb, vb, bits, 1024, 0,
                                          None) == radsort.E_UNSUPPORTED
    st = ctypes.c_void_p()
    assert lib.radsort_state_create(ctypes.byref(st), fake, pv, n, kb, vb, bits,
                                    None) == radsort.E_UNSUPPORTED
    assert not st.value
    assert lib.radsort_histograms(fake, n, kb, bits, fake, None) == radsort.E_UNSUPPORTED
    assert radsort.workspace_bytes(n, kb, vb, bits) == 0
    assert lib.radsort_sort_pairs(fake, pv, n, kb, vb, 17, None, None) == radsort.E_INVALID


@pytest.mark.parametrize("b", [32, 100, 1 << 17])
def test_block_size_validation(b):
    lib = radsort.load()
    o = radsort.Opts()
    o.block_elems = b
    fake = ctypes.c_void_p(0x1000)
    rc = lib.radsort_sort_pairs(fake, None, 1000, 4, 0, 8, ctypes.byref(o), None)
    assert rc == radsort.E_INVALID
    assert radsort.workspace_bytes(1000, 4, 0, 8, b) == 0


def test_workspace_too_small_is_rejected():
    lib = radsort.load()
    o = radsort.Opts()
    o.block_elems = 1024
    o.workspace = 0x2000
    o.workspace_bytes = 16
    fake = ctypes.c_void_p(0x1000)
    assert lib.radsort_sort_pairs(fake, None, 100000, 4, 0, 8, ctypes.byref(o), None) == \
        radsort.E_NOMEM
    assert lib.radsort_oop_sort_pairs(fake, None, 100000, 4, 0, 8, ctypes.byref(o), None) == \
        radsort.E_NOMEM


def test_null_pointers_rejected():
    lib = radsort.load()
    assert lib.radsort_sort_pairs(None, None, 10, 4, 0, 8, None, None) == radsort.E_INVALID
    fake = ctypes.c_void_p(0x1000)
    assert lib.radsort_sort_pairs(fake, None, 10, 4, 4, 8, None, None) == radsort.E_INVALID
    assert lib.radsort_sort_pairs(fake, fake, 10, 4, 0, 8, None, None) == radsort.E_INVALID
    assert lib.radsort_state_create(None, fake, None, 10, 4, 0, 8, None) == radsort.E_INVALID
    assert lib.radsort_histograms(fake, 10, 4, 8, None, None) == radsort.E_INVALID


def test_workspace_error_argument_checks():
    lib = radsort.load()
    fake = ctypes.c_void_p(0x1000)
    bits = ctypes.c_uint32(7)
    assert lib.radsort_workspace_error(None, 1000, 4, 4, 8, None, 0, ctypes.byref(bits),
                                       None) == radsort.E_INVALID
    assert bits.value == 0
    o = radsort.Opts()
    o.block_elems, o.workspace, o.workspace_bytes = 1024, fake, 16
    for oop in (0, 1):
        assert lib.radsort_workspace_error(fake, 100000, 4, 4, 8, ctypes.byref(o), oop, None,
                                           None) == radsort.E_NOMEM
    o.workspace_bytes = 1 << 40
    assert lib.radsort_workspace_error(fake, 1, 4, 4, 8, ctypes.byref(o), 0, None,
                                       None) == radsort.OK
    assert lib.radsort_workspace_error(fake, 1000, 3, 4, 8, ctypes.byref(o), 0, None,
                                       None) == radsort.E_INVALID


def test_trivial_sizes_are_no_ops():
    lib = radsort.load()
    # n <= 1 returns before anything is enqueued, so no device is needed
    assert lib.radsort_sort_pairs(None, None, 0, 4, 0, 8, None, None) == radsort.OK
    fake = ctypes.c_void_p(0x1000)
    assert lib.radsort_sort_pairs(fake, None, 1, 8, 0, 8, None, None) == radsort.OK
    assert lib.radsort_oop_sort_pairs(fake, fake, 1, 8, 8, 8, None, None) == radsort.OK


def test_strerror_texts():
    for code in (radsort.OK, radsort.E_INVALID, radsort.E_NOMEM, radsort.E_UNSUPPORTED,
                 radsort.E_TIMEOUT, radsort.E_ORDER):
        assert radsort.strerror(code)
    assert radsort.strerror(radsort.E_ORDER) != radsort.strerror(radsort.E_TIMEOUT)


def test_ordering_check_only_in_its_build():
    """RADSORT_F_DEBUG_ORDER is refused by the product library; the ordering-check
    build exports the same symbols and refuses blocks larger than the tile."""
    from paper_2607_05302_amd import build as hipbuild
    fake = ctypes.c_void_p(0x1000)
    o = radsort.Opts()
    o.block_elems, o.flags = 1024, radsort.F_DEBUG_ORDER
    lib = radsort.load()
    assert lib.radsort_sort_pairs(fake, fake, 1 << 20, 4, 4, 8, ctypes.byref(o),
                                  None) == radsort.E_UNSUPPORTED
    dbg = radsort.load(hipbuild.DEBUG_ORDER_LIB)
    for name in declared_functions():
        assert hasattr(dbg, name), name
    o.block_elems = 16384  # the tile of 4-byte keys and payload holds 8192 elements
    assert dbg.radsort_sort_pairs(fake, fake, 1 << 20, 4, 4, 8, ctypes.byref(o),
                                  None) == radsort.E_UNSUPPORTED
    # without the flag the ordering-check build takes what the product build takes
    assert dbg.radsort_workspace_bytes(1 << 20, 4, 4, 8, None) > 0


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError):
        radsort.load(str(tmp_path / "missing.so"))


def test_noalloc_refusals_need_no_device():
    """radsort_sort_pairs_noalloc refuses a workspace past its static scratch, and
    the timing flag, before touching the device."""
    lib = radsort.load()
    fake = ctypes.c_void_p(0x1000)
    text = open(HEADER).read()
    m = re.search(r"#define RADSORT_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == radsort.NOALLOC_SCRATCH_BYTES
    n = 1 << 30
    assert radsort.workspace_bytes(n, 4, 4, 8, 1024) > radsort.NOALLOC_SCRATCH_BYTES
    assert lib.radsort_sort_pairs_noalloc(fake, fake, n, 4, 4, 8, 1024, 0, None) == \
        radsort.E_NOMEM
    assert lib.radsort_sort_pairs_noalloc(fake, fake, 1000, 4, 4, 8, 1024, radsort.F_TIMING,
                                          None) == radsort.E_INVALID
    assert lib.radsort_sort_pairs_noalloc(fake, fake, 1000, 3, 4, 8, 1024, 0, None) == \
        radsort.E_INVALID
    assert lib.radsort_sort_pairs_noalloc(None, None, 0, 4, 0, 8, 0, 0, None) == radsort.OK


def test_copy_argument_errors():
    """radsort_copy refuses null and unaligned pointers before anything is enqueued,
    and a copy of 0 bytes is a no-op that needs no device."""
    lib = radsort.load()
    fake = ctypes.c_void_p(0x1000)
    assert lib.radsort_copy(None, fake, 16, None) == radsort.E_INVALID
    assert lib.radsort_copy(fake, None, 16, None) == radsort.E_INVALID
    assert lib.radsort_copy(ctypes.c_void_p(0x1004), fake, 16, None) == radsort.E_INVALID
    assert lib.radsort_copy(fake, ctypes.c_void_p(0x1008), 16, None) == radsort.E_INVALID
    assert lib.radsort_copy(None, None, 0, None) == radsort.OK


def test_shared_calls_need_their_own_workspace_size():
    """The workspace depends on RADSORT_F_SHARED: a shared call's finalize takes the
    two-kernel form of its block permutation, whose temporary blocks the workspace
    must hold (they share memory with the look-back ring, so small states need no
    more).  Each call refuses a workspace one byte smaller than its own size, before
    any launch."""
    lib = radsort.load()
    fake = ctypes.c_void_p(0x1000)
    for n, b in ((1 << 28, 1024), (1 << 28, 2048), (1 << 24, 1024)):
        plain = radsort.workspace_bytes(n, 4, 4, 8, b)
        shared = radsort.workspace_bytes(n, 4, 4, 8, b, shared=True)
        assert shared >= plain > 0
        if n == 1 << 28:
            assert shared > plain
        for flags, size in ((radsort.F_SHARED, shared), (0, plain)):
            o = radsort.Opts()
            o.block_elems = b
            o.workspace = 0x1000  # never dereferenced: the size check comes first
            o.workspace_bytes = size - 1
            o.flags = flags
            assert lib.radsort_sort_pairs(fake, fake, n, 4, 4, 8, ctypes.byref(o), None) == \
                radsort.E_NOMEM
