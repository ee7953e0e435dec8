"""Host-side planning of the segmented sort (no GPU needed)."""
import numpy as np

import paper_2607_05302_amd as radsort


def test_workspace_covers_only_the_large_arrays():
    small = np.cumsum([0] + [8192] * 100).astype(np.uint64)
    assert radsort.segments_workspace_bytes(small, 4, 4, None) <= 4096  # error words only
    big = np.array([0, 1 << 20, (1 << 20) + 5], dtype=np.uint64)
    one = radsort.workspace_bytes(1 << 20, 4, 4, 8, 1024)
    assert radsort.segments_workspace_bytes(big, 4, 4, None) >= one
    # four arrays of the same size go to four lanes
    four = np.cumsum([0] + [1 << 20] * 4).astype(np.uint64)
    assert radsort.segments_workspace_bytes(four, 4, 4, None) >= 4 * one


def test_bad_offsets_rejected():
    assert radsort.segments_workspace_bytes(np.array([0, 10, 5], np.uint64), 4, 4) == 0
    assert radsort.segments_workspace_bytes(np.array([0, 10], np.uint64), 3, 4) == 0
