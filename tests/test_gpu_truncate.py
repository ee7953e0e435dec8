"""GPU parity of the step interface used without finalize (Sec. 4.1): truncate
(Alg. 8) between rounds, the block table of the permuted representation, keys
rewritten in place through it, and a new sort of the same state.

The oracle runs the same steps (truncate_count, set_logical, more rounds), and the
GPU draws blocks in the sequential order (RADSORT_F_SEQ_DRAWS).  After
every step pi, P and f must equal the oracle's bit for bit, and so must the
dataset read in logical order and, after finalize, the front of the arrays.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
import paper_2607_05302_amd as radsort  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NP = {4: np.uint32, 8: np.uint64}


def to_dev(a):
    a = np.ascontiguousarray(a)
    view = {4: np.int32, 8: np.int64}[a.dtype.itemsize]
    return torch.from_numpy(a.view(view)).to(DEV)


def from_dev(t, width):
    return t.cpu().numpy().view(NP[width])


def say(*a):
    print(*a, flush=True)


def same_state(st, R, what):
    pi, pidx, plen, f = st.read()
    assert f == R.f, (what, f, R.f)
    assert np.array_equal(pi.astype(np.uint64), R.pi()), f"pi differs {what}"
    oidx, olen = R.P()
    assert np.array_equal(pidx.astype(np.uint64), oidx), f"P idx differs {what}"
    assert np.array_equal(plen.astype(np.uint64), olen), f"P len differs {what}"
    assert st.count == R.n, what
    lk, lv = st.logical()
    ok, ov, cnt = R.logical()
    assert cnt == R.n
    assert np.array_equal(from_dev(lk, st.kb).astype(np.uint64), ok), f"logical keys {what}"
    if st.vb:
        assert np.array_equal(from_dev(lv, st.vb).astype(np.uint64), ov), f"logical payload {what}"


CASES = [
    # (dist, n, key bytes, payload bytes, digit bits, b)
    ("uniform", 5000, 4, 4, 8, 64),
    ("uniform", (1 << 16) + 777, 4, 4, 8, 1024),
    ("zipf", 300000, 8, 4, 8, 1024),
    ("few", 123457, 4, 4, 8, 64),
    ("uniform", 70000, 8, 8, 11, 1024),
    ("uniform", 70000, 4, 0, 8, 16384),
]


def counts(n, b, seed):
    rng = np.random.default_rng(seed)
    cs = [n - 1, (n // b) * b, n // 3, 1, int(rng.integers(0, n + 1))]
    return [c for c in cs if 0 <= c <= n]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("at", [0, 1, "last"])
def test_truncate_between_rounds_matches_oracle(case, at):
    dist, n, kb, vb, bits, b = case
    sigma, nt = oracle.digit_params(kb, bits)
    r_at = nt if at == "last" else at
    for c in counts(n, b, n + r_at)[:3]:
        say(f"truncate {case} after round {r_at} to {c}")
        keys = workloads.make(dist, 31 * n + c, n, kb)
        vals = np.arange(n, dtype=NP[vb]) if vb else None
        dk = to_dev(keys)
        dv = to_dev(vals) if vb else None
        st = radsort.State(dk, dv, digit_bits=bits, block_elems=b, seq_draws=True)
        R = oracle.Radsort(keys, vals, sigma, nt, b)
        st.setup()
        R.setup()
        for r in range(r_at):
            st.round()
            R.round(nt - 1 - r)
        st.truncate(c)
        R.truncate_count(c)
        same_state(st, R, f"after truncate at {r_at}")
        for r in range(r_at, nt):
            st.round()
            R.round(nt - 1 - r)
            same_state(st, R, f"round {r} after truncate at {r_at}")
        st.finalize()
        st.read()  # waits and reports device-side errors
        R.finalize()
        ok, ov = R.result()
        assert np.array_equal(from_dev(dk, kb)[:c].astype(np.uint64), ok), (case, r_at, c)
        if vb:
            assert np.array_equal(from_dev(dv, vb)[:c].astype(np.uint64), ov), (case, r_at, c)
        st.close()


def write_logical(st, ws, keys_dev, new_keys):
    """Writes new_keys (logical order, numpy) into the permuted representation
    through the block table, as a user of the library would."""
    phys, ln = st.blocks()
    phys = phys.cpu().numpy().view(np.uint32).astype(np.int64)
    ln = ln.cpu().numpy().view(np.uint32).astype(np.int64)
    tk, _, b = st.planes()
    two_sigma = 2 * st.sigma
    sel = ln > 0
    phys, ln = phys[sel], ln[sel]
    assert ln.sum() == len(new_keys)
    starts = np.repeat(phys * b, ln) + (np.arange(ln.sum()) - np.repeat(np.cumsum(ln) - ln, ln))
    in_t = np.repeat(phys < two_sigma, ln)
    a_pos = starts - two_sigma * b
    width = st.kb
    tdt = {4: torch.int32, 8: torch.int64}[width]
    off = tk - ws.data_ptr()
    assert off % width == 0
    t_plane = ws[off:off + two_sigma * b * width].view(tdt)
    # every index in range before the device writes
    assert np.all(starts[in_t] >= 0) and np.all(starts[in_t] < two_sigma * b)
    assert np.all(a_pos[~in_t] >= 0) and np.all(a_pos[~in_t] < keys_dev.numel())
    assert off >= 0 and off + two_sigma * b * width <= ws.numel()
    nk = to_dev(new_keys.astype(NP[width]))
    ti = torch.from_numpy(starts[in_t]).to(DEV)
    ai = torch.from_numpy(a_pos[~in_t]).to(DEV)
    t_plane[ti] = nk[torch.from_numpy(np.nonzero(in_t)[0]).to(DEV)]
    keys_dev[ai] = nk[torch.from_numpy(np.nonzero(~in_t)[0]).to(DEV)]
    torch.cuda.synchronize()


@pytest.mark.parametrize("kb,vb,b", [(4, 4, 256), (8, 4, 1024), (4, 8, 64)])
def test_sort_again_without_finalize(kb, vb, b):
    """Sort; rewrite the keys in place through the block table; truncate; sort the
    same state again (restart); twice; then finalize."""
    n = 200000 + 13
    bits = 8
    sigma, nt = oracle.digit_params(kb, bits)
    keys = workloads.make("uniform", 77, n, kb)
    vals = np.arange(n, dtype=NP[vb])
    dk, dv = to_dev(keys), to_dev(vals)
    ws = torch.empty(radsort.workspace_bytes(n, kb, vb, bits, b), dtype=torch.uint8, device=DEV)
    st = radsort.State(dk, dv, digit_bits=bits, block_elems=b, workspace=ws,
                       seq_draws=True)
    R = oracle.Radsort(keys, vals, sigma, nt, b)
    st.setup()
    R.setup()
    for r in range(nt):
        st.round()
        R.round(nt - 1 - r)
    same_state(st, R, "first sort")
    for step in range(2):
        say(f"sort again kb={kb} vb={vb} b={b} step {step}")
        _, ov, _ = R.logical()
        newk = workloads.mix64(ov * np.uint64(0x9E3779B97F4A7C15 & 0xFFFFFFFF) + np.uint64(step))
        if kb == 4:
            newk = newk & np.uint64(0xFFFFFFFF)
        write_logical(st, ws, dk, newk)
        R.set_logical(newk)
        same_state(st, R, f"rewritten {step}")
        c = st.count - 4321 * (step + 1)
        st.truncate(c)
        R.truncate_count(c)
        st.restart()
        for r in range(nt):
            st.round()
            R.round(nt - 1 - r)
            same_state(st, R, f"step {step} round {r}")
    st.finalize()
    st.read()
    R.finalize()
    ok, ov = R.result()
    c = R.n
    assert np.array_equal(from_dev(dk, kb)[:c].astype(np.uint64), ok)
    assert np.array_equal(from_dev(dv, vb)[:c].astype(np.uint64), ov)
    st.close()


def test_block_table_matches_oracle_state():
    n, kb, vb, bits, b = 100003, 4, 4, 8, 512
    sigma, nt = oracle.digit_params(kb, bits)
    keys = workloads.make("zipf", 5, n, kb)
    vals = np.arange(n, dtype=np.uint32)
    st = radsort.State(to_dev(keys), to_dev(vals), digit_bits=bits, block_elems=b,
                       seq_draws=True)
    R = oracle.Radsort(keys, vals, sigma, nt, b)
    st.setup()
    R.setup()
    for r in range(2):
        st.round()
        R.round(nt - 1 - r)
    st.truncate(60000)
    R.truncate_count(60000)
    phys, ln = st.blocks()
    phys = phys.cpu().numpy().view(np.uint32).astype(np.uint64)
    ln = ln.cpu().numpy().view(np.uint32).astype(np.uint64)
    f = R.f
    assert np.array_equal(phys[:f - sigma], R.pi()[sigma:f])
    assert np.all(phys[f - sigma:] == 0xFFFFFFFF) and np.all(ln[f - sigma:] == 0)
    assert int(ln.sum()) == R.n == 60000
    # lengths: b except the partial blocks of P (Alg. 3)
    idx, plen = R.P()
    want = np.full(f - sigma, b, np.uint64)
    for e in range(sigma):
        if idx[e] < f:
            want[idx[e] - sigma] = plen[e]
    assert np.array_equal(ln[:f - sigma], want)
    st.close()


def test_truncate_edges():
    n, kb, vb, bits, b = 40000, 4, 4, 8, 256
    sigma, nt = oracle.digit_params(kb, bits)
    keys = workloads.make("uniform", 9, n, kb)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    st = radsort.State(dk, dv, digit_bits=bits, block_elems=b, seq_draws=True)
    R = oracle.Radsort(keys, vals, sigma, nt, b)
    st.setup()
    R.setup()
    st.round()
    R.round(nt - 1)
    with pytest.raises(radsort.RadsortError):
        st.truncate(n + 1)                 # past the data: rejected, state unchanged
    same_state(st, R, "after a rejected truncate")
    st.truncate(n)                         # the whole dataset: nothing is lost
    R.truncate_count(n)
    same_state(st, R, "truncate to n")
    st.truncate(0)                         # empty
    R.truncate_count(0)
    same_state(st, R, "truncate to 0")
    for r in range(1, nt):
        st.round()
        R.round(nt - 1 - r)
        same_state(st, R, f"empty, round {r}")
    with pytest.raises(radsort.RadsortError):
        st.finalize_sequential()           # the sequential form has no truncated case
    st.finalize()
    st.read()
    assert st.count == 0
    with pytest.raises(radsort.RadsortError):
        st.truncate(0)                     # the state is used up
    with pytest.raises(radsort.RadsortError):
        st.restart()
    st.close()


@pytest.mark.parametrize("kb,b", [(4, 2048), (8, 1024)])
def test_truncate_at_scale(kb, b):
    """2^24 keys: many super-tiles; truncate after the second round, finish, finalize."""
    n, vb, bits = (1 << 24) + 1001, 4, 8
    sigma, nt = oracle.digit_params(kb, bits)
    say(f"truncate at scale kb={kb} b={b}")
    keys = workloads.make("uniform", 123, n, kb)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = to_dev(keys), to_dev(vals)
    st = radsort.State(dk, dv, digit_bits=bits, block_elems=b, seq_draws=True)
    R = oracle.Radsort(keys, vals, sigma, nt, b)
    st.setup()
    R.setup()
    for r in range(2):
        st.round()
        R.round(nt - 1 - r)
    c = n - 3 * n // 7
    st.truncate(c)
    R.truncate_count(c)
    for r in range(2, nt):
        st.round()
        R.round(nt - 1 - r)
    pi, pidx, plen, f = st.read()
    assert f == R.f and np.array_equal(pi.astype(np.uint64), R.pi())
    st.finalize()
    st.read()
    R.finalize()
    ok, ov = R.result()
    assert np.array_equal(from_dev(dk, kb)[:c].astype(np.uint64), ok)
    assert np.array_equal(from_dev(dv, vb)[:c].astype(np.uint64), ov)
    st.close()
