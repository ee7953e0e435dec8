"""The MSD-first split (Sec. 4.3): a Radsort round on the top digit, finalize, then
every top-digit group sorted by the remaining digits as one batch.  Compared
element by element with the oracle's Radsort (whose result, with an index payload,
is the unique stable order), through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NP = {4: np.uint32, 8: np.uint64}

CASES = [
    # (dist, n, key bytes, payload bytes, digit bits, b)
    ("uniform", (1 << 20) + 123, 4, 4, 8, 1024),   # groups of ~4 K: whole in LDS
    ("uniform", 1 << 26, 4, 4, 8, 2048),           # groups of 2^18: one workgroup each
    ("zipf", 1 << 22, 8, 4, 8, 1024),              # one group of ~14 %, many tiny ones
    ("equal", 1 << 21, 8, 4, 8, 1024),             # a single group holding everything
    ("low20", (1 << 23) + 5, 8, 0, 8, 1024),       # top digit constant: one group of 2^23
    ("uniform", 300000, 4, 8, 4, 512),             # 4-bit digits: 16 groups
    ("uniform", 5000, 4, 4, 11, 1024),             # 11-bit digits (top digit of 10 bits)
    ("uniform", 2, 4, 4, 8, 64),
]


def to_dev(a):
    view = {4: np.int32, 8: np.int64}[a.dtype.itemsize]
    return torch.from_numpy(np.ascontiguousarray(a).view(view)).to(DEV)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_msd_split_matches_oracle(case):
    dist, n, kb, vb, bits, b = case
    print(f"msd split {case}", flush=True)
    keys = workloads.make(dist, 0x35D + n, n, kb)
    vals = np.arange(n, dtype=NP[vb]) if vb else None
    sigma, nt = oracle.digit_params(kb, bits)
    dk = to_dev(keys)
    dv = to_dev(vals) if vb else None
    radsort.msd_sort_(dk, dv, digit_bits=bits, block_elems=b, check=True)
    ok, ov = oracle.radsort(keys, vals, sigma, nt, b)
    assert np.array_equal(dk.cpu().numpy().view(NP[kb]).astype(np.uint64), ok)
    if vb:
        assert np.array_equal(dv.cpu().numpy().view(NP[vb]).astype(np.uint64), ov)
    s = radsort.last_stats()
    assert s["error_bits"] == 0 and s["workspace_bytes"] > 0
