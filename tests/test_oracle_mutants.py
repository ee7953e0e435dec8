"""Planted mistakes in the oracle must fail at least one pin.

Each case copies the oracle's C source, plants one plausible mistake with a
textual substitution, builds the copy, and runs the pins of test_oracle.py that
need no GPU (hand trace, library stable sort, closed forms, invariant) against
it in a child process.  The two literal readings of the garbled lines of the
paper (Alg. 3 and Alg. 7) are among the mutants: the pins reject them, which is
why the oracle takes readings G1 and G2.  Mistakes in truncate (Alg. 8) and in
finalize after truncate (reading G14) are caught by sorting truncated prefixes
over a four-letter alphabet.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "radsort_oracle.c")

MUTANTS = {
    "alg3_literal_pi_compare": ("st->Pi[*iP] == i)", "st->Pi[*iP] == st->pi[i])"),
    "alg7_literal_home_minus_sigma": ("uint64_t j_out = i_in + sigma;",
                                      "uint64_t j_out = i_in - sigma;"),
    "block_full_off_by_one": ("if (p_next + 1 == st->Bend[c]) {",
                              "if (p_next + 2 == st->Bend[c]) {"),
    "msd_first_round_order": ("for (uint64_t t = nt; t-- > 0;) orc_round(st, t);",
                              "for (uint64_t t = 0; t < nt; t++) orc_round(st, t);"),
    "head_start_from_front": ("st->pi2[i] = st->pi[i_out + i];",
                              "st->pi2[i] = st->pi[i];"),
    "partial_length_from_end": ("st->Pl[c] = (uint64_t)(st->Bnext[c] - base);",
                                "st->Pl[c] = (uint64_t)(st->Bend[c] - base) - 1;"),
    "bucket_start_without_head": ("st->S[0] = sigma;", "st->S[0] = 0;"),
    "setup_tail_wrong_offset": ("memcpy(blockat(st, sigma), st->A + b * (n / b),",
                                "memcpy(blockat(st, sigma), st->A + b * (n / b) - 1,"),
    "no_push_before_pull": ("if (i_in < i_out && i_out < st->f) {",
                            "if (0 && i_in < i_out && i_out < st->f) {"),
    "free_slot_not_updated": ("i_free = i_out;\n            j_free = j_in;",
                              "(void)0;"),
    "digit_from_low_end": ("uint64_t below = nt - 1 - t;", "uint64_t below = t;"),
    "truncate_keeps_f": ("st->f = i + 1;                                  /* block i is",
                         "(void)0;                                        /* block i is"),
    "truncate_length_off_by_one": ("st->Pl[e] = (uint64_t)(j + 1);",
                                   "st->Pl[e] = (uint64_t)(j + 2);"),
    "truncate_entry_after_block": ("if (i <= st->Pi[e]) {", "if (i < st->Pi[e]) {"),
    "finalize_no_tail_relocation": ("if (2 * sigma + nb < st->npi) {",
                                    "if (0 && 2 * sigma + nb < st->npi) {"),
}

CHECK = r'''
import json, os, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle, workloads
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
k, v = oracle.radsort(np.array(g["keys"]), np.array(g["vals"]), 2, 1, 2, lib=lib)
if k.tolist() != g["final"]["keys"] or v.tolist() != g["final"]["vals"]:
    fails.append(("hand_trace",))
print(json.dumps(fails[:5]))
sys.exit(1 if fails else 0)
'''


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique for {name}"
    mutated = tmp_path / "radsort_oracle.c"
    mutated.write_text(src.replace(old, new))
    (tmp_path / "radsort_oracle.h").write_text(
        open(os.path.join(ROOT, "oracle", "radsort_oracle.h")).read())
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", lib, str(mutated)],
                   check=True)
    script = tmp_path / "check.py"
    script.write_text(CHECK)
    proc = subprocess.run([sys.executable, str(script), lib, ROOT], capture_output=True,
                          text=True, timeout=300)
    # exit 0 means every pin passed: the planted mistake survived
    assert proc.returncode != 0, f"mutant {name} passed every pin: {proc.stdout}"
