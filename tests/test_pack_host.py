"""Host model of the packed last round and its finalize (CPU only).

The index arithmetic of plan_round (packed), k_round's pool of draws, k_pack_fixup,
k_pack_table, k_pack_homes and k_pack_merge is restated here in Python and run on
random and adversarial bucket counts:
  - every draw of a tile takes an extra block or an input block that a tile at or
    before it has read (the GPU form of Lemma 1 with the packed offsets);
  - pi after the packed fixup is a permutation of the n_pi + sigma physical blocks;
  - the homes form a permutation, each block of A is the home of exactly one block;
  - moving the blocks to their homes and merging the spare blocks' slots puts
    every element at its final position.
"""
import numpy as np
import pytest

GARBAGE = 1 << 31


def plan(counts, b):
    """plan_round, packed: est, offsets, blocks per bucket, S, f."""
    sigma = len(counts)
    est = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    o = est % b
    C = 1 + (counts + o) // b
    S = sigma + np.concatenate([[0], np.cumsum(C)[:-1]])
    f = sigma + int(C.sum())
    return est, o, C, S, f


def spare_id(k, sigma, npi):
    return k if k < 2 * sigma else npi + (k - 2 * sigma)


def pack_table(est, counts, n, b):
    sigma = len(counts)
    nA = n // b
    spare = np.zeros(sigma, bool)
    empty = np.zeros(sigma, bool)
    for d in range(sigma):
        c, e0 = int(counts[d]), int(est[d])
        o = e0 % b
        if c:
            ql = (o + c - 1) // b
            gl = e0 // b + ql
            hl = o + c - ql * b
            spare[d] = gl >= nA or hl < b
        empty[d] = c == 0 or (o + c) % b == 0
    srank = np.where(spare, np.cumsum(spare) - spare, -1)
    erank = np.where(empty, np.cumsum(empty) - empty, -1)
    return srank, erank, int(spare.sum()), int(empty.sum())


def homes_of(counts, n, b, npi):
    """k_pack_homes: (home, has data) per logical block 0 .. npi + sigma - 1."""
    sigma = len(counts)
    est, o, C, S, f = plan(counts, b)
    srank, erank, ns, ne = pack_table(est, counts, n, b)
    nA = n // b
    out = []
    for L in range(npi + sigma):
        if L < sigma:
            out.append((spare_id(ns + L, sigma, npi), False, None))
        elif L >= f:
            out.append((spare_id(ns + sigma + ne + (L - f), sigma, npi), False, None))
        else:
            d = int(np.searchsorted(S, L, side="right")) - 1
            q = L - int(S[d])
            c, e0 = int(counts[d]), int(est[d])
            od = e0 % b
            start, g = q * b, e0 // b + q
            lo = od if q == 0 else 0
            hi = min(b, od + c - start) if od + c > start else 0
            if hi <= lo:
                assert erank[d] >= 0
                out.append((spare_id(ns + sigma + erank[d], sigma, npi), False, None))
            elif g < nA and hi == b:
                out.append((2 * sigma + g, True, (g, lo, hi)))
            else:
                assert srank[d] >= 0
                out.append((spare_id(srank[d], sigma, npi), True, (g, lo, hi)))
    return out, (est, o, C, S, f)


def draws_are_behind_reads(counts_per_tile, b, E):
    """k_round's draws in the packed round: tile k's draw indices [F_k, F_k + nfills_k)
    name extra blocks (< sigma) or input block index - sigma, which must lie in the
    slots of tiles 0 .. k (every tile holds E slots, input blocks full)."""
    tiles, sigma = counts_per_tile.shape
    totals = counts_per_tile.sum(axis=0)
    est = np.concatenate([[0], np.cumsum(totals)[:-1]])
    o = est % b
    before = np.zeros(sigma, np.int64)
    for k in range(tiles):
        base = before + o                     # ranks as the blocks see them
        F = int((base // b).sum())
        after = base + counts_per_tile[k]
        nfills = int((after // b).sum()) - F
        if nfills:
            last = F + nfills - 1
            if last >= sigma:
                assert (last - sigma) * b < (k + 1) * E, (k, last)
        before += counts_per_tile[k]


@pytest.mark.parametrize("seed", range(40))
def test_pack_permutations_and_final_positions(seed):
    rng = np.random.default_rng(seed)
    sigma = int(rng.choice([2, 4, 16, 64]))
    b = int(rng.choice([4, 8, 64]))
    n = int(rng.integers(1, 40 * b))
    kind = seed % 4
    if kind == 0:
        digits = rng.integers(0, sigma, n)
    elif kind == 1:
        digits = np.minimum(rng.geometric(0.3, n) - 1, sigma - 1)
    elif kind == 2:
        digits = np.full(n, sigma - 1)
    else:
        digits = rng.integers(0, max(1, sigma // 4), n) * 4 % sigma
    counts = np.bincount(digits, minlength=sigma).astype(np.int64)
    nA = n // b
    npi = nA + 2 * sigma
    est, o, C, S, f = plan(counts, b)
    assert f <= npi + sigma
    drawn = f - 2 * sigma
    # physical blocks of the round's input state: a random permutation pi_old of
    # 0 .. npi - 1; heads pi_old[0 .. sigma); pool entry k: extra block npi + k for
    # k < sigma, then pi_old[k]
    pi_old = rng.permutation(npi)
    pool = [npi + k if k < sigma else int(pi_old[k]) for k in range(npi)]
    pi_new = np.full(npi + sigma, -1, np.int64)
    # the round: bucket d's blocks q >= 1 get the drawn entries, in some order
    order = rng.permutation(drawn)
    it = iter(order)
    for d in range(sigma):
        for q in range(1, int(C[d])):
            pi_new[int(S[d]) + q] = pool[next(it)]
    # k_pack_fixup
    for j in range(npi + sigma):
        if j < sigma:
            pi_new[int(S[j])] = pi_old[j]
            k = drawn + j
            pi_new[j] = npi + k if k < sigma else pi_old[k]
        elif j >= f:
            pi_new[j] = pi_old[j - sigma]
    assert sorted(pi_new.tolist()) == list(range(npi + sigma))
    # homes
    hl, _ = homes_of(counts, n, b, npi)
    homes = [h for h, _, _ in hl]
    assert sorted(homes) == list(range(npi + sigma))
    prim = [info[0] for h, data, info in hl if data and h >= 2 * sigma and h < npi]
    assert sorted(prim) == list(range(nA))
    # data: logical block L of bucket d, slot s holds final position g b + s
    store = {p: [None] * b for p in range(npi + sigma)}
    for L in range(npi + sigma):
        h, data, info = hl[L]
        if data:
            g, lo, hi = info
            for slot in range(lo, hi):
                store[int(pi_new[L])][slot] = g * b + slot
    # F1: every block with data to its home (garbage elsewhere is not copied)
    moved = {p: [None] * b for p in range(npi + sigma)}
    for L in range(npi + sigma):
        h, data, info = hl[L]
        if data:
            moved[h] = list(store[int(pi_new[L])])
    A = [None] * n
    for g in range(nA):
        for slot in range(b):
            A[g * b + slot] = moved[2 * sigma + g][slot]
    # merge: the spare blocks' slots into A
    for L in range(npi + sigma):
        h, data, info = hl[L]
        if data and not (2 * sigma <= h < npi):
            g, lo, hi = info
            for slot in range(lo, hi):
                A[g * b + slot] = moved[h][slot]
    assert A == list(range(n))


@pytest.mark.parametrize("seed", range(30))
def test_packed_draws_stay_behind_reads(seed):
    rng = np.random.default_rng(1000 + seed)
    sigma = int(rng.choice([4, 16, 64, 256]))
    b = int(rng.choice([8, 64, 256]))
    E = b * int(rng.choice([1, 2, 4]))
    tiles = int(rng.integers(1, 60))
    kind = seed % 3
    counts = np.zeros((tiles, sigma), np.int64)
    for k in range(tiles):
        if kind == 0:
            dg = rng.integers(0, sigma, E)
        elif kind == 1:  # every bucket crosses a block boundary early
            dg = np.repeat(np.arange(sigma), E // sigma + 1)[:E]
        else:
            dg = np.minimum(rng.geometric(0.05, E) - 1, sigma - 1)
        counts[k] = np.bincount(dg, minlength=sigma)
    draws_are_behind_reads(counts, b, E)
