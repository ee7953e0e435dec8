"""Host model of finalize's cycle finding (CPU only).

k_fin_init and k_fin_jump4 restated in Python: pointer jumping two doubling steps
per launch leaves, for every node p of a permutation, the smallest node of p's
cycle and the distance from p to it, which k_fin_rank turns into ranks and cycle
lengths.  Checked against walking each cycle, on random permutations and on a few
of fixed shape (one cycle, all fixed points, pairs).
"""
import numpy as np
import pytest


def jump4(nxt):
    n = len(nxt)
    J, V, O = nxt.copy(), np.arange(n), np.zeros(n, np.int64)
    w = 1
    while w < n:
        Jn, Vn, On = np.empty_like(J), np.empty_like(V), np.empty_like(O)
        for p in range(n):
            v, o, q = V[p], O[p], p
            for k in range(1, 4):
                q = J[q]
                if V[q] < v:
                    v, o = V[q], O[q] + k * w
            Jn[p], Vn[p], On[p] = J[q], v, o
        J, V, O = Jn, Vn, On
        w *= 4
    return V, O


def ranks(nxt, V, O):
    """k_fin_rank: rank of p in its cycle (0 at its smallest node) and the cycle length."""
    n = len(nxt)
    rank, clen = np.zeros(n, np.int64), np.zeros(n, np.int64)
    for p in range(n):
        leader = V[p]
        ln = nxt[leader]
        length = 1 if ln == leader else O[ln] + 1
        rank[p] = 0 if p == leader else length - O[p]
        clen[p] = length
    return rank, clen


def cases():
    rng = np.random.default_rng(11)
    out = [rng.permutation(n) for n in (1, 2, 3, 5, 17, 64, 65, 257, 1000, 4099)]
    out.append(np.roll(np.arange(300), 1))      # one cycle
    out.append(np.arange(77))                    # fixed points only
    out.append(np.arange(100) ^ 1)               # pairs
    return out


@pytest.mark.parametrize("nxt", cases(), ids=lambda a: f"n{len(a)}")
def test_jump4_finds_leaders_distances_ranks(nxt):
    V, O = jump4(nxt)
    rank, clen = ranks(nxt, V, O)
    for p in range(len(nxt)):
        cyc = [p]
        x = nxt[p]
        while x != p:
            cyc.append(x)
            x = nxt[x]
        m = min(cyc)
        assert V[p] == m and O[p] == cyc.index(m)
        assert clen[p] == len(cyc)
        # walking from the leader, p is reached after rank[p] steps
        y, steps = m, 0
        while y != p:
            y, steps = nxt[y], steps + 1
        assert rank[p] == steps
