"""Trace generation and footprints of the serving loop (no GPU needed)."""
import numpy as np

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
