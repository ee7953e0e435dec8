"""Trace generation and footprints of the serving loop (no GPU needed)."""
import numpy as np
import pytest

from paper_2607_05302_amd import serve


def test_trace_is_seeded_and_shaped():
    a = serve.make_trace(7, 500, rate=100.0)
    b = serve.make_trace(7, 500, rate=100.0)
    assert [(r.arrival, r.n, r.key_bytes) for r in a] == [(r.arrival, r.n, r.key_bytes) for r in b]
    assert all(a[i].arrival <= a[i + 1].arrival for i in range(len(a) - 1))
    sizes = np.array([r.n for r in a])
    assert sizes.min() >= 1 << 12 and sizes.max() <= 1 << 28
    assert 0.35 < np.mean([r.key_bytes == 8 for r in a]) < 0.65
    assert 50 < serve.offered_load(a) < 200


def test_radsort_footprint_is_about_half_of_the_baseline():
    r = serve.Request(0, 0.0, 1 << 26, 4, 1)
    rad, oop = serve.footprint(r, "radsort"), serve.footprint(r, "oop")
    data = r.n * 8
    assert rad < 1.02 * data
    assert oop > 1.95 * data


def test_region_layout_is_aligned_and_covers_the_arrays():
    for n, kb in [(1, 4), (4097, 8), (1 << 20, 4), (3_000_001, 8)]:
        for method in ("radsort", "oop"):
            r = serve.Request(0, 0.0, n, kb, 1)
            o_k, o_v, o_w, end = serve.region(r, method)
            assert o_k == 0 and o_v >= n * kb and o_w >= o_v + n * 4
            assert o_v % serve.ALIGN == 0 and o_w % serve.ALIGN == 0 and end % serve.ALIGN == 0
            assert end == serve.footprint(r, method)


def test_arena_first_fit_and_merging():
    a = serve.Arena(10 * serve.ALIGN + 7)  # the odd tail is unusable
    assert a.size == 10 * serve.ALIGN and a.free_bytes() == a.size
    x = a.alloc(1)             # one unit
    y = a.alloc(3 * 256)       # three
    z = a.alloc(2 * 256 + 1)   # three (rounded up)
    assert (x, y, z) == (0, 256, 4 * 256)
    assert a.alloc(4 * 256) is None  # 3 units left
    a.release(y, 3 * 256)
    assert a.alloc(2 * 256) == 256  # first fit: the hole left by y
    a.release(x, 1)
    a.release(256, 2 * 256)
    assert a.free == [(0, 4 * 256), (7 * 256, 3 * 256)]  # x, the two units and the rest of y's hole
    a.release(z, 2 * 256 + 1)
    assert a.free == [(0, a.size)]  # everything merged back
    with pytest.raises(ValueError):
        a.release(0, 256)  # already free


def test_arena_random_against_a_byte_map():
    rng = np.random.default_rng(5)
    a = serve.Arena(64 * serve.ALIGN)
    owned = np.zeros(64, dtype=bool)
    held = []
    for _ in range(2000):
        if held and (rng.random() < 0.5 or len(held) > 20):
            off, nb = held.pop(rng.integers(len(held)))
            a.release(off, nb)
            owned[off // 256: (off + nb + 255) // 256] = False
        else:
            nb = int(rng.integers(1, 6 * 256))
            off = a.alloc(nb)
            units = (nb + 255) // 256
            free_runs = [i for i in range(64 - units + 1) if not owned[i:i + units].any()]
            if off is None:
                assert free_runs == []
            else:
                assert off // 256 == free_runs[0]  # the lowest range that fits
                owned[off // 256: off // 256 + units] = True
                held.append((off, nb))
        assert a.free_bytes() == (64 - owned.sum()) * 256


def test_draw_input_is_seeded_and_covers_the_key_range():
    import torch
    for kb, dt in [(4, torch.int32), (8, torch.int64)]:
        n = serve.DRAW_CHUNK + 1000  # two pieces
        r = serve.Request(0, 0.0, n, kb, 12345)
        a, av = torch.empty(n, dtype=dt), torch.empty(n, dtype=torch.int32)
        b, bv = torch.empty(n, dtype=dt), torch.empty(n, dtype=torch.int32)
        serve.draw_input(r, a, av)
        serve.draw_input(r, b, bv)
        assert torch.equal(a, b) and torch.equal(av, torch.arange(n, dtype=torch.int32))
        c, cv = torch.empty(n, dtype=dt), torch.empty(n, dtype=torch.int32)
        serve.draw_input(serve.Request(0, 0.0, n, kb, 12346), c, cv)
        assert not torch.equal(a, c)
        assert (a < 0).any() and (a > 0).any()  # both halves of the unsigned range
        assert a.unique().numel() > 0.99 * n
