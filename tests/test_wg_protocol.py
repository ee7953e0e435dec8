"""A model of the one-workgroup batched sort (Radsort run by one workgroup on one
array, Sec. 2 with the work of each step split over the threads), run on the
CPU: it replays the kernel's global loads and stores, each with the thread that
makes it, between the kernel's synchronisation points, and checks that every
pair of accesses by different threads to the same address is ordered the way
the kernel's rules require.

Synchronisation points, as the kernel has them:
  B  a barrier (__syncthreads): orders LDS; it waits for neither the global
     loads nor the global stores still in flight in a thread (on gfx950 the
     compiler puts no vmcnt wait before s_barrier at workgroup scope);
  W  every thread waits for all its memory operations, then a barrier (F2);
  H  the full hand-off: fence, wait, barrier, fence (one round to the next,
     setup to the first round, F1 to F2, one array to the next).
Rules checked for two accesses to one address by different threads:
  store then load (the load must see the store) and store then store: an H
     between them (a store is visible to other threads only through a hand-off);
  load then store (the load must not see the store): the load's value was used
     by its thread before a barrier between them (so it has returned), or a W
     or an H lies between them;
  never both in one stretch between synchronisation points.
The model computes the sort, so a block written before it is read (Lemma 1 on
the GPU: every drawn pool block was loaded by the same or an earlier tile)
shows up as a wrong result too.  Threads, lanes, tile and block sizes are small
parameters; the kernel's thread of every access follows its index arithmetic:
tile slot s = wave * (E / waves) + j * lanes + lane, staged position p and block
column c handled by thread p mod NT and c mod NT.
"""
import random

import pytest


class Memory:
    """Global memory with an access log per address."""

    def __init__(self):
        self.seg = 0
        self.H = [0]
        self.W = [0]
        self.B = [0]
        self.val = {}
        self.last_store = {}   # addr -> (seg, thread)
        self.loads = {}        # addr -> [(seg, thread, consumed)]
        self.errors = []

    def sync(self, kind, site=""):
        self.seg += 1
        self.H.append(self.H[-1] + (kind == "H"))
        self.W.append(self.W[-1] + (kind in "HW"))
        self.B.append(self.B[-1] + 1)

    def _between(self, arr, a, b):
        return arr[b] - arr[a] > 0

    def consume(self, addr, th):
        """A load issued earlier (consumed=False) is waited for here: from now on
        it counts as returned before the next barrier."""
        for i, (s, t, c) in enumerate(self.loads.get(addr, ())):
            if t == th and not c:
                self.loads[addr][i] = (self.seg, t, True)
                return
        raise AssertionError("no pending load")

    def load(self, addr, th, consumed=True):
        st = self.last_store.get(addr)
        if st is not None and st[1] != th:
            if st[0] == self.seg:
                self.errors.append(("race store/load", addr, st, th))
            elif not self._between(self.H, st[0], self.seg):
                self.errors.append(("store->load without hand-off", addr, st, th))
        self.loads.setdefault(addr, []).append((self.seg, th, consumed))
        return self.val.get(addr)

    def store(self, addr, th, v):
        st = self.last_store.get(addr)
        if st is not None and st[1] != th:
            if st[0] == self.seg:
                self.errors.append(("race store/store", addr, st, th))
            elif not self._between(self.H, st[0], self.seg):
                self.errors.append(("store->store without hand-off", addr, st, th))
        for (s, t, consumed) in self.loads.get(addr, ()):
            if t == th:
                continue
            if s == self.seg:
                self.errors.append(("race load/store", addr, (s, t), th))
            elif not ((consumed and self._between(self.B, s, self.seg))
                      or self._between(self.W, s, self.seg)):
                self.errors.append(("load->store, load not waited for", addr, (s, t), th))
        self.loads[addr] = []
        self.last_store[addr] = (self.seg, th)
        self.val[addr] = v


def run_array(mem, keys, cfg, base_addr):
    """One array through the kernel's steps; keys are written at ('A', base + i)
    as (key, original index) pairs.  Returns nothing; the result is in mem."""
    sigma, b, bits, NT, LANES, ITEMS, DEPTH, kbits = (
        cfg["sigma"], cfg["b"], cfg["bits"], cfg["NT"], cfg["LANES"], cfg["ITEMS"],
        cfg["DEPTH"], cfg["kbits"])
    WAVES = NT // LANES
    E = NT * ITEMS
    SEG = E // WAVES
    NBLK = E // b
    nt = (kbits + bits - 1) // bits
    dmask = sigma - 1
    two_sigma = 2 * sigma
    n = len(keys)
    nb, tail = n // b, n % b
    npi = nb + two_sigma

    def A(i):
        return ("A", base_addr + i)

    def blockat(j, off):
        return ("T", j * b + off) if j < two_sigma else A((j - two_sigma) * b + off)

    def slot_thread(s):
        wave, within = divmod(s, SEG)
        return wave * LANES + within % LANES

    mem.sync("H", "top")  # loop top
    mem.sync("B")  # the claimed array index
    mem.sync("B")  # histogram rows cleared
    hist = [[0] * sigma for _ in range(nt)]
    for i in range(n):
        k, _ = mem.load(A(i), i % NT)
        for t in range(nt):
            hist[t][(k >> (bits * (nt - 1 - t))) & dmask] += 1
    # setup (Alg. 4): logical L -> physical; the tail of A goes to T block sigma
    f0 = sigma + nb + 1
    pit = [L if L < sigma else (L + sigma if L + 1 < f0 else sigma + (L - (f0 - 1)))
           for L in range(npi)]
    for i in range(tail):
        v = mem.load(A(nb * b + i), i % NT)
        mem.store(("T", sigma * b + i), i % NT, v)
    Pidx = [f0 - 1 if d == 0 else npi for d in range(sigma)]
    Plen = [tail if d == 0 else 0 for d in range(sigma)]
    f = f0
    mem.sync("H", "setup")
    for r in range(nt):
        shift = bits * r
        counts = hist[nt - 1 - r]
        S, Pnidx, Pnlen = [], [], []
        run = 0
        for d in range(sigma):
            c = 1 + counts[d] // b
            S.append(sigma + run)
            Pnidx.append(sigma + run + c - 1)
            Pnlen.append(counts[d] % b)
            run += c
        fout = sigma + run
        mem.sync("B")  # round start
        if any(c == n for c in counts):
            continue  # every element has the same digit here: the round is left out
        base = [0] * sigma
        F = 0
        pit2 = list(pit)  # pi'; entries not written this round are rewritten by fixup
        tiles = ((f - sigma) * b + E - 1) // E

        def issue(t):
            """The loads of tile t, issued early (during tile t - 1)."""
            out = []
            for k in range(NBLK):
                L = sigma + t * NBLK + k
                if t >= tiles or L >= f:
                    continue
                ln = b
                for e in range(sigma):
                    if Pidx[e] == L:
                        ln = Plen[e]
                for off in range(ln):
                    s = k * b + off
                    addr = blockat(pit[L], off)
                    out.append((s, addr, slot_thread(s),
                                mem.load(addr, slot_thread(s), consumed=False)))
            return out

        pending = issue(0)
        for tile in range(tiles):
            mem.sync("B")  # top of the tile: the previous tile is done with LDS
            elems = []  # (slot, key pair) in slot order
            for s, addr, th, kv in pending:
                mem.consume(addr, th)
                elems.append((s, kv))
            mem.sync("B")  # ranked
            mem.sync("B")  # tile counts
            cnt = [0] * sigma
            rank = []
            for s, kv in elems:
                d = (kv[0] >> shift) & dmask
                rank.append(base[d] + cnt[d])
                cnt[d] += 1
            mem.sync("B")  # fills per wave
            fill = 0
            for (s, kv), g in zip(elems, rank):
                if g % b == b - 1:
                    d = (kv[0] >> shift) & dmask
                    slot = S[d] + g // b + 1
                    pool = sigma + F + fill
                    assert slot < npi and pool < npi
                    pit2[slot] = pit[pool]
                    fill += 1
            tdo, run = [], 0
            for d in range(sigma):
                tdo.append(run)
                run += cnt[d]
            stage = [None] * len(elems)
            seen = [0] * sigma
            for s, kv in elems:
                d = (kv[0] >> shift) & dmask
                stage[tdo[d] + seen[d]] = kv
                seen[d] += 1
            pending = issue(tile + 1)
            mem.sync("B")  # staged, draws in pi'
            for p, kv in enumerate(stage):
                d = (kv[0] >> shift) & dmask
                g = base[d] + (p - tdo[d])
                q, off = divmod(g, b)
                phys = pit[d] if q == 0 else pit2[S[d] + q]
                mem.store(blockat(phys, off), p % NT, kv)
            mem.sync("B")  # end of the tile
            for d in range(sigma):
                base[d] += cnt[d]
            F += fill
        mem.sync("H", "round")  # the round's stores, for the next round
        # fixupPhase (Alg. 6) on the tables
        c = fout - sigma
        new = list(pit2)
        for j in range(npi):
            v = pit[j]
            if j < sigma:
                new[S[j]] = v
            elif c <= j < c + sigma:
                new[j - c] = v
            elif j >= c + sigma:
                new[j] = v
        pit = new
        Pidx, Plen = Pnidx, Pnlen
        f = fout
        mem.sync("B")
    # finalize F1: content(p) <- content(pred(p)) along the cycles
    inv = [0] * npi
    for L in range(npi):
        inv[pit[L]] = L
    mem.sync("B")
    COLS = b // NT

    def pred(p):
        return pit[p - sigma] if p >= sigma else pit[p + npi - sigma]

    def garbage(p):
        L = inv[p]
        return L < sigma or L >= f

    visited = [False] * npi
    for p0 in range(npi):
        if visited[p0] or pred(p0) == p0:
            continue
        for tid in range(NT):
            for cc in range(COLS):
                col = tid + cc * NT
                hg = garbage(p0)
                hk = None if hg else mem.load(blockat(p0, col), tid)
                cur = p0
                while True:
                    nodes = []
                    x = cur
                    while len(nodes) < DEPTH:
                        pr = pred(x)
                        if pr == p0:
                            break
                        nodes.append(pr)
                        x = pr
                    got = [None if garbage(nd) else mem.load(blockat(nd, col), tid)
                           for nd in nodes]
                    for u, nd in enumerate(nodes):
                        dst = cur if u == 0 else nodes[u - 1]
                        if got[u] is not None:
                            mem.store(blockat(dst, col), tid, got[u])
                    if nodes:
                        cur = nodes[-1]
                    if len(nodes) < DEPTH:
                        if not hg:
                            mem.store(blockat(cur, col), tid, hk)
                        break
        y = p0
        while True:
            visited[y] = True
            y = pred(y)
            if y == p0:
                break
        mem.sync("B")
    mem.sync("H", "f1")  # F1's stores, before F2 overwrites the unused tails
    # finalize F2: close the gaps; logical L sits at physical rot(L)
    k_out = 0
    for L0 in range(sigma, f, DEPTH):
        batch = []
        for L in range(L0, min(L0 + DEPTH, f)):
            ln = b
            for e in range(sigma):
                if Pidx[e] == L:
                    ln = Plen[e]
            phys = L + sigma if L + sigma < npi else L + sigma - npi
            vals = []
            for col in range(ln):
                vals.append(mem.load(blockat(phys, col), col % NT, consumed=False))
            batch.append((k_out, vals))
            k_out += ln
        mem.sync("W")
        for dst0, vals in batch:
            for col, v in enumerate(vals):
                mem.store(A(dst0 + col), col % NT, v)
        mem.sync("B")
    assert k_out == n


CFGS = [
    dict(sigma=4, bits=2, b=8, NT=8, LANES=2, ITEMS=4, DEPTH=2, kbits=8),
    dict(sigma=4, bits=2, b=16, NT=8, LANES=4, ITEMS=4, DEPTH=3, kbits=8),
    dict(sigma=16, bits=4, b=8, NT=4, LANES=2, ITEMS=4, DEPTH=2, kbits=8),
    dict(sigma=8, bits=3, b=8, NT=8, LANES=8, ITEMS=2, DEPTH=4, kbits=8),
]


def sort_batch(arrays, cfg):
    mem = Memory()
    base = 0
    spans = []
    for keys in arrays:
        for i, k in enumerate(keys):
            mem.val[("A", base + i)] = (k, i)
        spans.append((base, len(keys)))
        base += len(keys)
    for (b0, n), keys in zip(spans, arrays):  # one workgroup, arrays one after another
        run_array(mem, keys, cfg, b0)
    outs = [[mem.val[("A", b0 + i)] for i in range(n)] for b0, n in spans]
    return mem, outs


def gen(rng, n, kind, kbits):
    if kind == "uniform":
        return [rng.randrange(1 << kbits) for _ in range(n)]
    if kind == "equal":
        return [rng.randrange(1 << kbits)] * n
    if kind == "few":
        vals = [rng.randrange(1 << kbits) for _ in range(3)]
        return [rng.choice(vals) for _ in range(n)]
    if kind == "sorted":
        return sorted(rng.randrange(1 << kbits) for _ in range(n))
    return sorted((rng.randrange(1 << kbits) for _ in range(n)), reverse=True)


@pytest.mark.parametrize("ci", range(len(CFGS)))
@pytest.mark.parametrize("seed", range(6))
def test_accesses_ordered_and_result_sorted(ci, seed):
    cfg = CFGS[ci]
    rng = random.Random(seed * 31 + ci)
    b = cfg["b"]
    arrays = []
    for kind in ("uniform", "equal", "few", "sorted", "reversed"):
        n = rng.choice([0, 1, b - 1, b, 2 * b, 5 * b + 3, rng.randrange(3 * b, 40 * b)])
        arrays.append(gen(rng, n, kind, cfg["kbits"]))
    mem, outs = sort_batch(arrays, cfg)
    assert not mem.errors, mem.errors[:5]
    for keys, out in zip(arrays, outs):
        assert out == sorted(((k, i) for i, k in enumerate(keys)), key=lambda kv: kv[0])


def _first_error(cfg, arrays, mutate):
    mem = Memory()
    orig_sync = mem.sync
    mem.sync = lambda kind, site="": orig_sync(mutate(kind, site), site)
    base = 0
    for keys in arrays:
        for i, k in enumerate(keys):
            mem.val[("A", base + i)] = (k, i)
        run_array(mem, keys, cfg, base)
        base += len(keys)
    return mem.errors


def test_model_flags_a_missing_hand_off():
    """Each hand-off after setup, after a round and after F1 is needed: turning
    any one of them into a plain barrier makes the checker report an unordered
    pair (a pin of the checker itself).  By these rules the hand-off at the top
    of each array orders no global access: the previous array's last accesses to
    the workgroup's T are F1's stores (ordered by the hand-off after F1) and F2's
    loads (waited for in F2).  The kernel keeps it all the same: without it the
    GPU sorted an array of 3 145 733 pairs wrong, which these rules do not
    explain."""
    cfg = CFGS[0]
    rng = random.Random(5)
    arrays = [gen(rng, 37 * cfg["b"] + 5, "uniform", cfg["kbits"]) for _ in range(3)]
    sites = []
    assert not _first_error(cfg, arrays, lambda kind, site: sites.append(site) or kind)
    hs = [i for i, site in enumerate(sites) if site]
    assert {sites[i] for i in hs} == {"top", "setup", "round", "f1"}
    for victim in hs:
        errs = _first_error(cfg, arrays, lambda kind, site, c=iter(range(len(sites))):
                            "B" if next(c) == victim else kind)
        if sites[victim] == "top":
            assert not errs, errs[:3]
        else:
            assert errs, (victim, sites[victim])


def test_model_flags_f2_without_wait():
    """F2 must wait for its loads before the barrier: without the wait, a load
    still in flight could return a later store of another thread."""
    cfg = CFGS[1]
    rng = random.Random(9)
    arrays = [gen(rng, 23 * cfg["b"] + 7, "uniform", cfg["kbits"])]
    errs = _first_error(cfg, arrays, lambda kind, site: "B" if kind == "W" else kind)
    assert any(e[0] == "load->store, load not waited for" for e in errs)
