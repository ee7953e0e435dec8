"""Pins of the oracle's truncate (Alg. 8) and of its use of the permuted
representation without finalize (Sec. 4.1).

The pins, none of which compare the oracle with itself:
  - truncating keeps exactly a prefix of the logical sequence, and that
    sequence is fixed independently: after r rounds it is the input stably
    sorted by its low r digits (numpy's stable argsort);
  - the remaining rounds then sort the prefix stably by the remaining digits,
    which together are key >> (bits * r) (numpy again);
  - finalize after truncate leaves that sequence at the front of A, with every
    assertion counter of the oracle at zero;
  - keys rewritten through the permuted representation and sorted again from
    the same state give numpy's stable sort of the rewritten sequence;
  - the data invariant (Sec. 2.2) holds after every step.
"""
import numpy as np
import pytest

import oracle
import workloads

SIGMA, NT = oracle.digit_params(4, 8)


def low_sorted(keys, vals, r, bits=8):
    """The input stably sorted by its low r digits (the sequence after r rounds)."""
    if r == 0:
        return keys, vals
    o = np.argsort(keys & np.uint64((1 << (bits * r)) - 1), kind="stable")
    return keys[o], vals[o]


def high_sorted(keys, vals, r, bits=8):
    """Stable sort by the digits that rounds r .. n_t - 1 sort."""
    o = np.argsort(keys >> np.uint64(bits * r), kind="stable")
    return keys[o], vals[o]


def counts_for(n, b, seed):
    rng = np.random.default_rng(seed)
    cs = {0, 1, n // 2, max(n - 1, 0), n, (n // b) * b, max((n // b) * b - 1, 0)}
    cs.update(int(x) for x in rng.integers(0, n + 1, size=3))
    return sorted(c for c in cs if 0 <= c <= n)


def run_truncated(keys, vals, b, r, count):
    R = oracle.Radsort(keys, vals, SIGMA, NT, b)
    R.setup()
    for q in range(r):
        R.round(NT - 1 - q)
    R.truncate_count(count)
    return R


@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal", "sorted"])
@pytest.mark.parametrize("b", [1, 3, 64])
def test_truncate_keeps_a_prefix(dist, b):
    for n in [1, 300, 2500]:
        keys = workloads.make(dist, 808 + n, n, 4).astype(np.uint64)
        vals = np.arange(n, dtype=np.uint64)
        for r in range(NT + 1):
            ek, ev = low_sorted(keys, vals, r)
            for c in counts_for(n, b, n + r):
                R = run_truncated(keys, vals, b, r, c)
                assert R.n == c
                assert R.invariant() == 0, (dist, b, n, r, c)
                lk, lv, cnt = R.logical()
                assert cnt == c
                assert np.array_equal(lk, ek[:c]) and np.array_equal(lv, ev[:c]), (n, r, c)
                # the final block holds the last datum (or block sigma is empty)
                idx, ln = R.P()
                last = [int(ln[e]) for e in range(SIGMA) if int(idx[e]) == R.f - 1]
                assert len(last) == 1
                assert (last[0] >= 1) if c else (R.f == SIGMA + 1 and last[0] == 0)


def test_truncate_leaves_pi_alone_and_rejects_bad_counts():
    n, b = 1000, 16
    keys = workloads.uniform(5, n, 4).astype(np.uint64)
    R = oracle.Radsort(keys, np.arange(n), SIGMA, NT, b)
    R.setup()
    R.round(NT - 1)
    pi = R.pi().copy()
    with pytest.raises(ValueError):
        R.truncate_count(n + 1)
    with pytest.raises(ValueError):
        R.truncate(SIGMA - 1, 0)          # the head start is not part of the dataset
    with pytest.raises(ValueError):
        R.truncate(R.f, 0)                # past the final block
    R.truncate_count(n - 100)
    assert np.array_equal(R.pi(), pi)    # Alg. 8 touches only f and P
    assert R.n == n - 100 and R.invariant() == 0


@pytest.mark.parametrize("dist", ["uniform", "zipf", "few"])
@pytest.mark.parametrize("b", [1, 4, 64, 256])
def test_rounds_and_finalize_after_truncate(dist, b):
    for n in [7, 700, 3000]:
        keys = workloads.make(dist, 909 + n, n, 4).astype(np.uint64)
        vals = np.arange(n, dtype=np.uint64)
        for r in range(NT + 1):
            lk0, lv0 = low_sorted(keys, vals, r)
            for c in counts_for(n, b, 7 * n + r):
                R = run_truncated(keys, vals, b, r, c)
                for q in range(r, NT):
                    R.round(NT - 1 - q)
                    assert R.invariant() == 0, (dist, b, n, r, c, q)
                ek, ev = high_sorted(lk0[:c], lv0[:c], r)
                lk, lv, _ = R.logical()
                assert np.array_equal(lk, ek) and np.array_equal(lv, ev), (n, r, c)
                R.finalize()
                fk, fv = R.result()
                assert np.array_equal(fk, ek) and np.array_equal(fv, ev), (dist, b, n, r, c)
                cs = R.counters()
                bad = {k: v for k, v in cs.items()
                       if k not in ("rounds", "lemma1_equal", "finalize_copies") and v}
                assert not bad, (dist, b, n, r, c, bad)


def test_repeated_truncation_between_rounds():
    n, b = 5000, 32
    keys = workloads.uniform(11, n, 4).astype(np.uint64)
    vals = np.arange(n, dtype=np.uint64)
    R = oracle.Radsort(keys, vals, SIGMA, NT, b)
    R.setup()
    k, v = keys, vals
    for r, c in enumerate([4700, 3000, 2999, 1024]):
        R.truncate_count(c)
        k, v = k[:c], v[:c]
        R.round(NT - 1 - r)
        o = np.argsort((k >> np.uint64(8 * r)) & np.uint64(255), kind="stable")
        k, v = k[o], v[o]
        lk, lv, _ = R.logical()
        assert np.array_equal(lk, k) and np.array_equal(lv, v)
        assert R.invariant() == 0
    R.truncate_count(1000)
    R.finalize()
    fk, fv = R.result()
    assert np.array_equal(fk, k[:1000]) and np.array_equal(fv, v[:1000])


@pytest.mark.parametrize("b", [1, 16, 256])
def test_sort_again_by_new_keys_without_finalize(b):
    """Sort, rewrite the keys through the permuted representation, truncate and
    sort again from the same state (the use of Sec. 4.1), then finalize."""
    n = 4000
    keys = workloads.uniform(21, n, 4).astype(np.uint64)
    vals = np.arange(n, dtype=np.uint64)
    R = oracle.Radsort(keys, vals, SIGMA, NT, b)
    R.setup()
    for q in range(NT):
        R.round(NT - 1 - q)
    k, v = high_sorted(keys, vals, 0)
    lk, lv, _ = R.logical()
    assert np.array_equal(lk, k) and np.array_equal(lv, v)
    for step in range(3):
        newk = workloads.mix64(v * np.uint64(2654435761) + np.uint64(step)) & np.uint64(0xFFFFFFFF)
        R.set_logical(newk)
        c = R.n - 333 * (step + 1)
        R.truncate_count(c)
        k, v = newk[:c], v[:c]
        for q in range(NT):
            R.round(NT - 1 - q)
            assert R.invariant() == 0
        k, v = high_sorted(k, v, 0)
        lk, lv, cnt = R.logical()
        assert cnt == c
        assert np.array_equal(lk, k) and np.array_equal(lv, v), (b, step)
    R.finalize()
    fk, fv = R.result()
    assert np.array_equal(fk, k) and np.array_equal(fv, v)


def test_truncate_to_empty_then_finalize():
    for b in [1, 8, 64]:
        n = 1000
        keys = workloads.uniform(3, n, 4).astype(np.uint64)
        R = oracle.Radsort(keys, np.arange(n), SIGMA, NT, b)
        R.setup()
        R.round(NT - 1)
        R.truncate_count(0)
        assert R.f == SIGMA + 1 and R.n == 0 and R.invariant() == 0
        for q in range(1, NT):
            R.round(NT - 1 - q)
            assert R.invariant() == 0
        R.finalize()
        fk, _ = R.result()
        assert len(fk) == 0


def test_finalize_after_truncate_small_alphabet():
    """sigma = 4: few buckets, so truncated states often end in empty partial
    blocks and the A block after the homes often holds a block of the tail that
    the tail copies of finalize reach (reading G14)."""
    rng = np.random.default_rng(0x7A11)
    sigma, nt, bits = 4, 3, 2
    for _ in range(3000):
        n = int(rng.integers(1, 200))
        b = int(rng.choice([1, 2, 3, 4, 5, 8, 16]))
        scale = np.uint64(int(rng.choice([1, 4, 16])))
        keys = (rng.integers(0, int(rng.integers(1, 5)), size=n).astype(np.uint64) * scale) & np.uint64(63)
        vals = np.arange(n, dtype=np.uint64)
        r, c = int(rng.integers(0, nt + 1)), int(rng.integers(0, n + 1))
        R = oracle.Radsort(keys, vals, sigma, nt, b)
        R.setup()
        for q in range(r):
            R.round(nt - 1 - q)
        R.truncate_count(c)
        for q in range(r, nt):
            R.round(nt - 1 - q)
        lk, lv = low_sorted(keys, vals, r, bits)
        ek, ev = high_sorted(lk[:c], lv[:c], r, bits)
        R.finalize()
        fk, fv = R.result()
        assert np.array_equal(fk, ek) and np.array_equal(fv, ev), (n, b, r, c)
        assert R.counters()["finalize_tail_overwritten"] == 0, (n, b, r, c)
