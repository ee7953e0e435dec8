"""Host-side planning of the segmented sort (no GPU needed)."""
import numpy as np

import paper_2607_05302_amd as radsort


# the one-workgroup path: arrays of 8193 .. (4384 - 64) * 1024 elements (5-bit
# digits, b = 1024); each of its workgroups owns T = 2 * 32 * 1024 elements (keys
# and payload)
WG_MAX = (4384 - 64) * 1024
WG_SLOT = 2 * 32 * 1024 * (4 + 4)


def test_workspace_covers_only_the_large_arrays():
    small = np.cumsum([0] + [8192] * 100).astype(np.uint64)
    assert radsort.segments_workspace_bytes(small, 4, 4, None) <= 4096  # error words only
    # mid-size arrays: one T per workgroup of the one-workgroup path, at most 256
    mid = np.cumsum([0] + [1 << 20] * 4).astype(np.uint64)
    ws = radsort.segments_workspace_bytes(mid, 4, 4, None)
    assert 4 * WG_SLOT <= ws <= 4 * WG_SLOT + 8192
    many = np.cumsum([0] + [9000] * 1000).astype(np.uint64)
    ws = radsort.segments_workspace_bytes(many, 4, 4, None)
    assert 256 * WG_SLOT <= ws <= 256 * WG_SLOT + 4 * 1000 + 8192
    # larger arrays run the Radsort steps on the lanes, each lane its own workspace
    n = WG_MAX + 1
    big = np.array([0, n, n + 5], dtype=np.uint64)
    one = radsort.workspace_bytes(n, 4, 4, 8, 2048, shared=True)  # the lanes run shared
    assert radsort.segments_workspace_bytes(big, 4, 4, None) >= one
    four = np.cumsum([0] + [n] * 4).astype(np.uint64)
    assert radsort.segments_workspace_bytes(four, 4, 4, None) >= 4 * one


def test_bad_offsets_rejected():
    assert radsort.segments_workspace_bytes(np.array([0, 10, 5], np.uint64), 4, 4) == 0
    assert radsort.segments_workspace_bytes(np.array([0, 10], np.uint64), 3, 4) == 0
