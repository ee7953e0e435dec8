"""The device-side input generators draw the same bytes as the host ones."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal", "low20", "sorted"])
@pytest.mark.parametrize("kb", [4, 8])
def test_device_generators_match_host(dist, kb):
    n = 100003
    host = workloads.make(dist, 0x5EED0003, n, kb)
    dev = workloads.make_t(dist, 0x5EED0003, n, kb, "cpu").numpy().view(host.dtype)
    assert np.array_equal(host, dev)


def test_words_at_an_offset():
    a = workloads.words(7, 1000, start=123456)
    b = workloads.words_t(7, 1000, "cpu", start=123456).numpy().view(np.uint64)
    assert np.array_equal(a, b)
