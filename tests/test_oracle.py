"""Pins of the Radsort oracle against facts the paper and the mathematics fix.

None of these tests compare the oracle with itself.  The pins are:
  - a hand-worked trace of Alg. 3-7 (tests/golden);
  - library stable sorts (numpy's stable argsort) for the final output;
  - exhaustive brute force on tiny inputs against a by-hand lexicographic
    stable insertion sort;
  - Alg. 1 (a stable counting sort) round by round, itself pinned by numpy;
  - closed forms of C, S, P, f derived from the histogram (Alg. 5-6);
  - the data invariant (Sec. 2.2), Lemma 1 (tight) and Lemma 2;
  - the finalize copy bound and the space formula (Sec. 3, Sec. 4);
  - the layout of Fig. 1 after setup.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def stable_ref(keys):
    order = np.argsort(np.asarray(keys), kind="stable")
    return np.asarray(keys)[order], order


# ---------------------------------------------------------------- hand trace

def test_hand_trace_matches_golden():
    g = json.load(open(os.path.join(GOLDEN, "hand_trace_n5_b2_sigma2.json")))
    p = g["params"]
    R = oracle.Radsort(np.array(g["keys"]), np.array(g["vals"]), p["sigma"], p["nt"], p["b"])
    R.setup()
    s = g["after_setup"]
    assert R.pi().tolist() == s["pi"]
    assert R.f == s["f"]
    idx, ln = R.P()
    assert idx.tolist() == s["P_idx"] and ln.tolist() == s["P_len"]
    k, v, cnt = R.logical()
    assert cnt == 5 and k.tolist() == s["logical_keys"] and v.tolist() == s["logical_vals"]
    R.sort_phase(0)
    r = g["after_round_t0"]
    assert R.C().tolist() == r["C"] and R.i_out == r["i_out"]
    R.fixup_phase()
    assert R.pi().tolist() == r["pi"] and R.f == r["f"]
    idx, ln = R.P()
    assert idx.tolist() == r["P_idx"] and ln.tolist() == r["P_len"]
    k, v, _ = R.logical()
    assert k.tolist() == r["logical_keys"] and v.tolist() == r["logical_vals"]
    R.finalize()
    k, v = R.result()
    assert k.tolist() == g["final"]["keys"] and v.tolist() == g["final"]["vals"]
    c = R.counters()
    assert all(c[name] == 0 for name in oracle.COUNTER_NAMES[oracle.C_FIRST_ERROR:])


# ---------------------------------------------------------------- final output

SIZES = [0, 1, 2, 3, 63, 64, 65, 511, 512, 513, 1000, 4096, 3 * 1024 + 7, 20000]


@pytest.mark.parametrize("b", [1, 2, 3, 4, 8, 64, 512, 1024])
@pytest.mark.parametrize("dist", ["uniform", "equal", "sorted", "reverse", "few", "zipf"])
def test_final_equals_library_stable_sort(b, dist):
    for n in SIZES:
        if b == 1 and n > 5000:
            continue
        keys = workloads.make(dist, 1000 + n, n, 4)
        sigma, nt = oracle.digit_params(4, 8)
        k, v = oracle.radsort(keys, np.arange(n), sigma, nt, b)
        rk, ro = stable_ref(keys)
        assert np.array_equal(k, rk.astype(np.uint64)), (n, b, dist)
        assert np.array_equal(v, ro.astype(np.uint64)), (n, b, dist)


@pytest.mark.parametrize("key_bytes,bits", [(4, 4), (4, 11), (8, 8), (8, 11), (4, 1), (4, 16)])
def test_digit_widths(key_bytes, bits):
    sigma, nt = oracle.digit_params(key_bytes, bits)
    for n in [0, 5, 700, 5000]:
        keys = workloads.uniform(77 + n, n, key_bytes)
        for b in [1, 64, 256]:
            k, v = oracle.radsort(keys, np.arange(n), sigma, nt, b)
            rk, ro = stable_ref(keys)
            assert np.array_equal(k, rk.astype(np.uint64)) and np.array_equal(v, ro)


def test_general_alphabet_strings():
    """sigma = 3 tuple keys of length n_t = 4, n = 26, b = 4 (the parameters of Fig. 2)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        tuples = rng.integers(0, 3, size=(26, 4))
        keys = tuples[:, 0] * 27 + tuples[:, 1] * 9 + tuples[:, 2] * 3 + tuples[:, 3]
        k, v = oracle.radsort(keys, np.arange(26), 3, 4, 4)
        ref = sorted(range(26), key=lambda i: tuple(tuples[i]))
        assert v.tolist() == ref


# ---------------------------------------------------------------- brute force

def _digits(x, sigma, nt):
    out = []
    for _ in range(nt):
        out.append(x % sigma)
        x //= sigma
    return tuple(reversed(out))


def _insertion_sort_lex(seq, sigma, nt):
    """By-hand stable sort: insert each element after every element whose digit
    tuple is lexicographically <= its own."""
    out = []
    for i, x in enumerate(seq):
        dx = _digits(x, sigma, nt)
        pos = len(out)
        while pos > 0:
            dy = _digits(out[pos - 1][0], sigma, nt)
            greater = False
            for a, c in zip(dy, dx):
                if a != c:
                    greater = a > c
                    break
            if not greater:
                break
            pos -= 1
        out.insert(pos, (x, i))
    return out


@pytest.mark.parametrize("sigma,nt,nmax", [(2, 1, 6), (2, 2, 5), (2, 3, 4), (3, 1, 6),
                                             (3, 2, 4), (3, 3, 3)])
def test_bruteforce_all_tiny_inputs(sigma, nt, nmax):
    lib = oracle.load()
    universe = range(sigma ** nt)
    for n in range(0, nmax + 1):
        for seq in itertools.product(universe, repeat=n):
            ref = _insertion_sort_lex(seq, sigma, nt)
            for b in (1, 2, 3):
                k, v = oracle.radsort(np.array(seq, np.uint64), np.arange(n), sigma, nt, b,
                                      lib=lib)
                assert [(int(a), int(c)) for a, c in zip(k, v)] == ref, (seq, b)


# ---------------------------------------------------------------- per round

def _run_rounds(keys, vals, sigma, nt, b):
    """Yields the oracle state after setup and after each round."""
    R = oracle.Radsort(keys, vals, sigma, nt, b)
    R.setup()
    yield -1, R
    for r in range(nt):
        R.round(nt - 1 - r)
        yield r, R


@pytest.mark.parametrize("dist", ["uniform", "equal", "sorted", "zipf", "low20"])
@pytest.mark.parametrize("b", [1, 4, 64])
def test_rounds_follow_alg1_and_closed_forms(dist, b):
    sigma, nt = oracle.digit_params(4, 8)
    for n in [0, 1, 300, 2500]:
        keys = workloads.make(dist, 4242 + n, n, 4).astype(np.uint64)
        vals = np.arange(n, dtype=np.uint64)
        for r, R in _run_rounds(keys, vals, sigma, nt, b):
            assert R.invariant() == 0, (r, n)
            lk, lv, cnt = R.logical()
            assert cnt == n
            if r < 0:
                assert np.array_equal(lk, keys) and np.array_equal(lv, vals)
                continue
            # logical sequence = Alg. 1 applied r+1 times
            ok, ov = oracle.oop_lsd(keys, vals, sigma, nt, rounds=r + 1)
            assert np.array_equal(lk, ok) and np.array_equal(lv, ov)
            # closed forms from the histogram of this round's key position
            t = nt - 1 - r
            shift = 8 * (nt - 1 - t)
            cnt_d = np.bincount(((keys >> np.uint64(shift)) & np.uint64(255)).astype(np.int64),
                                minlength=sigma)
            C = 1 + cnt_d // b
            S = sigma + np.concatenate([[0], np.cumsum(C)[:-1]])
            assert np.array_equal(R.C(), C)
            assert R.f == sigma + C.sum()
            idx, ln = R.P()
            assert np.array_equal(idx, S + C - 1)
            assert np.array_equal(ln, cnt_d % b)
        c = R.counters()
        assert c["lemma1_violation"] == 0 and c["lemma2_violation"] == 0
        assert c["pool_overrun"] == 0


def test_alg1_round_is_a_stable_counting_sort():
    """Pins the oracle's Alg. 1 by numpy's stable argsort on the digit of each round."""
    sigma, nt = oracle.digit_params(4, 8)
    keys = workloads.uniform(99, 5000, 4).astype(np.uint64)
    vals = np.arange(5000, dtype=np.uint64)
    k, v = keys.copy(), vals.copy()
    for r in range(nt):
        shift = np.uint64(8 * r)
        o = np.argsort((k >> shift) & np.uint64(255), kind="stable")
        k, v = k[o], v[o]
        ok, ov = oracle.oop_lsd(keys, vals, sigma, nt, rounds=r + 1)
        assert np.array_equal(ok, k) and np.array_equal(ov, v)


def test_histograms_match_bincount():
    sigma, nt = oracle.digit_params(8, 8)
    keys = workloads.uniform(5, 10000, 8)
    h = oracle.histograms(keys, sigma, nt)
    for t in range(nt):
        shift = np.uint64(8 * (nt - 1 - t))
        ref = np.bincount(((keys >> shift) & np.uint64(255)).astype(np.int64), minlength=256)
        assert np.array_equal(h[t], ref)


# ---------------------------------------------------------------- lemmas, bounds

def test_lemma1_equality_case_occurs_and_is_safe():
    """All-equal keys make bucket 0 draw block i_in right after its last element."""
    keys = np.full(4096, 7, np.uint64)
    R = oracle.Radsort(keys, np.arange(4096), 256, 4, 64)
    R.setup()
    R.round(3)
    c = R.counters()
    assert c["lemma1_equal"] > 0 and c["lemma1_violation"] == 0


@pytest.mark.parametrize("dist", ["uniform", "equal", "sorted", "zipf"])
def test_finalize_copy_bound(dist):
    """finalize copies at most 2 floor(n/b) blocks plus the remaining <= sigma (Sec. 3)."""
    sigma, nt = oracle.digit_params(4, 8)
    for n, b in [(5000, 64), (70000, 256), (3000, 1)]:
        keys = workloads.make(dist, 11 + n, n, 4)
        R = oracle.Radsort(keys, np.arange(n), sigma, nt, b)
        R.setup()
        for t in range(nt - 1, -1, -1):
            R.round(t)
        R.finalize()
        c = R.counters()
        assert c["finalize_copies"] <= 2 * (n // b) + sigma
        assert c["finalize_tail_overwritten"] == 0 and c["finalize_count_mismatch"] == 0
        assert c["finalize_home_taken"] == 0
        k, v = R.result()
        assert np.array_equal(v, np.argsort(keys, kind="stable"))


def test_setup_layout_matches_fig1():
    """Fig. 1: head start -> T[0..sigma), data -> the A blocks in order, the
    remaining logical indices -> T[sigma..2 sigma)."""
    sigma, b, n = 256, 64, 10000
    R = oracle.Radsort(workloads.uniform(1, n, 4), None, sigma, 4, b)
    R.setup()
    pi = R.pi()
    nb = n // b
    assert (pi[:sigma] < sigma).all()
    assert np.array_equal(pi[sigma:sigma + nb], 2 * sigma + np.arange(nb))
    assert np.array_equal(np.sort(pi[sigma + nb:]), sigma + np.arange(sigma))
    assert R.f == sigma + nb + 1


def test_space_matches_worked_numbers():
    """Sec. 4: b = 512, 8-byte elements, sigma = 256 gives T = 2 MiB, B, C, P, S =
    8 KiB and 9 bytes per block (0.22 % of the input)."""
    n = 512 * 1000
    total = oracle.extra_bytes(n, 256, 512, 8, ptr_bytes=8, int_bytes=4)
    t_bytes = 2 * 256 * 512 * 8
    assert t_bytes == 2 * 2 ** 20
    npi = n // 512 + 512
    assert total - t_bytes - 9 * npi == 8 * 1024
    assert abs(9 / (512 * 8) - 0.0022) < 0.0001


def test_space_is_order_sqrt_n():
    """Sec. 3: with b ~ sqrt(n) the extra space is O(sqrt n)."""
    ratios = []
    for lg in range(10, 31, 2):
        n = 1 << lg
        b = 1 << ((lg + 1) // 2)
        ratios.append(oracle.extra_bytes(n, 256, b, 8) / np.sqrt(n))
    assert max(ratios) < 2 * 256 * 8 * 2 + 64


# ---------------------------------------------------------------- key function

def test_key_positions_by_hand():
    assert oracle.key(0x12345678, 3, 256, 4) == 0x78
    assert oracle.key(0x12345678, 0, 256, 4) == 0x12
    assert oracle.key(0xFFFFFFFF, 0, 2048, 3) == 0x3FF      # top digit has 10 bits
    assert oracle.key(0xFFFFFFFF, 2, 2048, 3) == 0x7FF
    assert oracle.key(2 * 9 + 1 * 3 + 2, 0, 3, 3) == 2      # base-3 tuple (2, 1, 2)
    assert oracle.key(2 * 9 + 1 * 3 + 2, 1, 3, 3) == 1
    assert oracle.key(2 * 9 + 1 * 3 + 2, 2, 3, 3) == 2


# ---------------------------------------------------------------- the invariant checker

def _state_after_one_round(b=64, n=20000, lib=None):
    keys = workloads.uniform(0xC0DE, n, 4)
    R = oracle.Radsort(keys, np.arange(n), 256, 4, b, lib=lib)
    R.setup()
    R.round(3)
    assert R.invariant() == 0
    return R


def _plant(R, case):
    """Plants one broken clause of the data invariant (Sec. 2.2) into a valid state."""
    sigma, npi, f = R.sigma, R.npi, R.f
    pi = R.pi()
    idx, ln = R.P()
    if case == "pi_duplicate":            # clause 1: pi is a permutation
        R.plant_pi(sigma + 1, int(pi[sigma + 2]))
    elif case == "pi_out_of_range":
        R.plant_pi(5, npi)
    elif case == "P_not_ascending":       # clause 2: P ascending, partial lengths < b
        R.plant_P(3, int(idx[4]), int(ln[4]))
        R.plant_P(4, int(idx[3]), int(ln[3]))
    elif case == "P_in_head_start":
        R.plant_P(0, sigma - 1, int(ln[0]))
    elif case == "partial_block_full":
        k = int(np.flatnonzero(idx != f - 1)[0])
        R.plant_P(k, int(idx[k]), R.b)
    elif case == "last_block_not_partial":  # clause 3: block f-1 is partial
        assert f + 1 <= npi
        R.plant_f(f + 1)
    elif case == "f_past_npi":            # clause 4: the allocated range ends inside n_pi
        R.plant_P(sigma - 1, npi, 0)
        R.plant_f(npi + 1)
    elif case == "lengths_miss_n":        # the used lengths add up to n
        k = int(np.flatnonzero(ln > 0)[0])
        R.plant_P(k, int(idx[k]), int(ln[k]) - 1)
    else:
        raise ValueError(case)


BROKEN = {"pi_duplicate": 1, "pi_out_of_range": 1, "P_not_ascending": 2, "P_in_head_start": 2,
          "partial_block_full": 2, "last_block_not_partial": 3, "f_past_npi": 4,
          "lengths_miss_n": 5}


@pytest.mark.parametrize("case", sorted(BROKEN))
def test_invariant_checker_names_the_broken_clause(case):
    """A checker that always answers 'fine' (or checks the wrong clause) fails here:
    each planted state breaks exactly one clause of the invariant of Sec. 2.2."""
    R = _state_after_one_round()
    _plant(R, case)
    assert R.invariant() == BROKEN[case], case
