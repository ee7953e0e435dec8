"""Planted mistakes in the oracle must fail at least one pin.

Each case copies the oracle's C source, plants one plausible mistake with a
textual substitution, builds the copy, and runs pins that need no GPU against it
in a child process: the hand trace, library stable sorts, the per-round logical
sequence against Alg. 1, the closed forms of C, S, P and f, the data invariant
after every round, and the invariant checker on planted broken states.  The two
literal readings of the garbled lines of the paper (Alg. 3 and Alg. 7) are among
the mutants: the pins reject them, which is why the oracle takes readings G1 and
G2.  Mistakes in truncate (Alg. 8) and in finalize after truncate (reading G14)
are caught by sorting truncated prefixes over a four-letter alphabet.

A second group plants mistakes that the oracle's own run-time checks must
report: each must make its counter (Lemma 1, Lemma 2, pool overrun) fire on a
given input, so a counter that never fires cannot pass.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "radsort_oracle.c")

MUTANTS = {
    "alg3_literal_pi_compare": ("st->Pi[*iP] == i)", "st->Pi[*iP] == st->pi[i])"),
    "alg7_literal_home_minus_sigma": ("const uint64_t home = L + sigma, from",
                                      "const uint64_t home = L - sigma, from"),
    "block_full_off_by_one": ("if (st->cur_fill[c] < b) continue;",
                              "if (st->cur_fill[c] < b - 1) continue;"),
    "msd_first_round_order": ("for (uint64_t t = nt; t-- > 0;) orc_round(st, t);",
                              "for (uint64_t t = 0; t < nt; t++) orc_round(st, t);"),
    "head_start_from_front": ("st->pi2[k] = st->pi[taken + k];", "st->pi2[k] = st->pi[k];"),
    "partial_length_from_end": ("st->Pl[c] = st->cur_fill[c];",
                                "st->Pl[c] = st->b - 1 - st->cur_fill[c];"),
    "partial_index_first_block": ("st->Pi[c] = st->start[c] + st->blocks_of[c] - 1;",
                                  "st->Pi[c] = st->start[c];"),
    "bucket_start_without_head": ("uint64_t next_free = sigma;", "uint64_t next_free = 0;"),
    "bucket_blocks_reversed": ("for (uint64_t h = 0; h < taken; h++) {",
                               "for (uint64_t h = taken; h-- > 0;) {"),
    "unallocated_shifted": ("st->pi2[L] = st->pi[L]; /* unallocated */",
                            "st->pi2[L] = st->pi[L - 1]; /* unallocated */"),
    "setup_tail_wrong_offset": ("memcpy(blockat(st, sigma), st->A + b * (n / b),",
                                "memcpy(blockat(st, sigma), st->A + b * (n / b) - 1,"),
    "no_push_before_pull": ("if (bound_there > L && bound_there < st->f) bound_there =",
                            "if (0 && bound_there > L) bound_there ="),
    "free_slot_not_updated": ("spare.logical = bound_there;\n            spare.phys = from;",
                              "(void)0;"),
    "digit_from_low_end": ("uint64_t below = nt - 1 - t;", "uint64_t below = t;"),
    "truncate_keeps_f": ("st->f = i + 1;                                  /* block i is",
                         "(void)0;                                        /* block i is"),
    "truncate_length_off_by_one": ("st->Pl[e] = (uint64_t)(j + 1);",
                                   "st->Pl[e] = (uint64_t)(j + 2);"),
    "truncate_entry_after_block": ("if (i <= st->Pi[e]) {", "if (i < st->Pi[e]) {"),
    "finalize_no_tail_relocation": ("    clear_behind_homes(st, homes);\n",
                                    "    (void)clear_behind_homes;\n"),
    # the invariant checker itself
    "checker_always_fine": ("int orc_check_invariant(orc_state *st)\n{",
                            "int orc_check_invariant(orc_state *st)\n{\n    return 0;"),
    "checker_clause3_never": ("if (!found) return 3;", "if (0) return 3;"),
    "checker_lengths_never": ("if (k != st->n) return 5;", "if (0) return 5;"),
}

CHECK = r'''
import json, os, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
sys.path.insert(0, os.path.join(sys.argv[2], "tests"))
import oracle, workloads
from test_oracle import BROKEN, _plant, _state_after_one_round
lib = oracle.load(sys.argv[1])
fails = []
def stable(keys):
    o = np.argsort(keys, kind="stable"); return keys[o].astype(np.uint64), o.astype(np.uint64)
for dist in ["uniform", "equal", "sorted", "zipf", "few"]:
    for n in [5, 70, 300, 1000, 2500]:
        for b in [1, 3, 64]:
            keys = workloads.make(dist, n + b, n, 4)
            try:
                k, v = oracle.radsort(keys, np.arange(n), 256, 4, b, lib=lib)
            except RuntimeError:
                fails.append(("assert", dist, n, b)); continue
            rk, ro = stable(keys)
            if not (np.array_equal(k, rk) and np.array_equal(v, ro)):
                fails.append(("final", dist, n, b))
# every round: logical sequence = Alg. 1 (numpy), closed forms of C, S, P, f, invariant
for dist in ["uniform", "equal", "zipf"]:
    for n, b in [(3000, 16), (700, 3)]:
        keys = workloads.make(dist, 77 + n, n, 4).astype(np.uint64)
        vals = np.arange(n, dtype=np.uint64)
        R = oracle.Radsort(keys, vals, 256, 4, b, lib=lib)
        R.setup()
        k, v = keys, vals
        for r in range(4):
            R.round(3 - r)
            o = np.argsort((k >> np.uint64(8 * r)) & np.uint64(255), kind="stable")
            k, v = k[o], v[o]
            lk, lv, _ = R.logical()
            if not (np.array_equal(lk, k) and np.array_equal(lv, v)):
                fails.append(("round", dist, n, b, r)); break
            cnt = np.bincount(((keys >> np.uint64(8 * r)) & np.uint64(255)).astype(np.int64),
                              minlength=256)
            C = 1 + cnt // b
            S = 256 + np.concatenate([[0], np.cumsum(C)[:-1]])
            idx, ln = R.P()
            if not (np.array_equal(R.C(), C) and R.f == 256 + C.sum()
                    and np.array_equal(idx, S + C - 1) and np.array_equal(ln, cnt % b)):
                fails.append(("closed_forms", dist, n, b, r)); break
            if R.invariant() != 0:
                fails.append(("invariant", dist, n, b, r)); break
# the checker names the clause each planted state breaks
for case, clause in sorted(BROKEN.items()):
    try:
        R = _state_after_one_round(lib=lib)
        _plant(R, case)
        if R.invariant() != clause:
            fails.append(("checker", case))
    except AssertionError:
        fails.append(("checker_setup", case))
# truncate (Alg. 8), more rounds and finalize, against numpy on the prefix
rng = np.random.default_rng(0x7A11)
for trial in range(1500):
    n = int(rng.integers(1, 200)); b = int(rng.choice([1, 2, 3, 4, 5, 8, 16]))
    scale = np.uint64(int(rng.choice([1, 4, 16])))
    keys = (rng.integers(0, int(rng.integers(1, 5)), size=n).astype(np.uint64) * scale) & np.uint64(63)
    vals = np.arange(n, dtype=np.uint64)
    r, c = int(rng.integers(0, 4)), int(rng.integers(0, n + 1))
    R = oracle.Radsort(keys, vals, 4, 3, b, lib=lib)
    R.setup()
    for q in range(r): R.round(2 - q)
    R.truncate_count(c)
    for q in range(r, 3): R.round(2 - q)
    o = np.argsort(keys & np.uint64((1 << (2 * r)) - 1), kind="stable")
    pk, pv = keys[o][:c], vals[o][:c]
    o = np.argsort(pk >> np.uint64(2 * r), kind="stable")
    R.finalize()
    fk, fv = R.result()
    if not (np.array_equal(fk, pk[o]) and np.array_equal(fv, pv[o])):
        fails.append(("truncate", n, b, r, c)); break
    if any(v for k, v in R.counters().items() if k not in ("rounds", "lemma1_equal", "finalize_copies")):
        fails.append(("truncate_counters", n, b, r, c)); break
g = json.load(open(os.path.join(sys.argv[2], "tests", "golden", "hand_trace_n5_b2_sigma2.json")))
try:
    k, v = oracle.radsort(np.array(g["keys"]), np.array(g["vals"]), 2, 1, 2, lib=lib)
    if k.tolist() != g["final"]["keys"] or v.tolist() != g["final"]["vals"]:
        fails.append(("hand_trace",))
except RuntimeError:
    fails.append(("hand_trace_assert",))
print(json.dumps(fails[:5]))
sys.exit(1 if fails else 0)
'''

# mistakes the oracle's run-time checks must report: (site, replacement, counter,
# input distribution, n, b).  The run is setup and one round (8-bit digits of
# uint32 keys), after which the counter must be non-zero.
COUNTER_MUTANTS = {
    # the pool hands out one entry too many before the scan: a bucket's next block
    # can be the input block being read (Lemma 1)
    "pool_skips_one_entry": ("    st->taken = 0;\n", "    st->taken = 1;\n",
                             "lemma1_violation", "equal", 4096, 64),
    # T of sigma + 1 blocks instead of 2 sigma: too few unallocated blocks remain
    # for the next head start (Lemma 2)
    "T_of_sigma_plus_one_blocks": ("st->npi = n / b + 2 * sigma;",
                                   "st->npi = n / b + sigma + 1;",
                                   "lemma2_violation", "uniform", 200000, 64),
    # a bucket takes a new block after b/2 elements: the pool runs out
    "bucket_takes_block_at_half": ("if (st->cur_fill[c] < b) continue;",
                                   "if (st->cur_fill[c] < b / 2) continue;",
                                   "pool_overrun", "uniform", 200000, 64),
}

COUNTER_CHECK = r'''
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle, workloads
lib = oracle.load(sys.argv[1])
dist, n, b = sys.argv[3], int(sys.argv[4]), int(sys.argv[5])
keys = workloads.make(dist, 0xBAD, n, 4)
R = oracle.Radsort(keys, np.arange(n), 256, 4, b, lib=lib)
R.setup()
R.round(3)
print(json.dumps(R.counters()))
'''


def _build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mutated = tmp_path / "radsort_oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "radsort_oracle.h").write_text(
        open(os.path.join(ROOT, "oracle", "radsort_oracle.h")).read())
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", lib, str(mutated)],
                   check=True)
    return lib


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, old, new)
    script = tmp_path / "check.py"
    script.write_text(CHECK)
    proc = subprocess.run([sys.executable, str(script), lib, ROOT], capture_output=True,
                          text=True, timeout=300)
    # exit 0 means every pin passed: the planted mistake survived
    assert proc.returncode != 0, f"mutant {name} passed every pin: {proc.stdout}"


@pytest.mark.parametrize("name", sorted(COUNTER_MUTANTS))
def test_counter_reports_planted_mistake(name, tmp_path):
    import json
    old, new, counter, dist, n, b = COUNTER_MUTANTS[name]
    lib = _build_mutant(tmp_path, old, new)
    script = tmp_path / "counters.py"
    script.write_text(COUNTER_CHECK)
    proc = subprocess.run([sys.executable, str(script), lib, ROOT, dist, str(n), str(b)],
                          capture_output=True, text=True, timeout=300)
    assert proc.returncode == 0, proc.stderr[-2000:]
    counters = json.loads(proc.stdout.strip().splitlines()[-1])
    assert counters[counter] > 0, f"{name}: {counter} did not fire: {counters}"


@pytest.mark.parametrize("name", sorted(COUNTER_MUTANTS))
def test_counter_stays_zero_without_the_mistake(name):
    """The same inputs on the oracle as written: every error counter stays zero."""
    import numpy as np

    import oracle
    import workloads
    _, _, counter, dist, n, b = COUNTER_MUTANTS[name]
    keys = workloads.make(dist, 0xBAD, n, 4)
    R = oracle.Radsort(keys, np.arange(n), 256, 4, b)
    R.setup()
    R.round(3)
    assert R.counters()[counter] == 0
