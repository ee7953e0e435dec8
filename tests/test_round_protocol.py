"""A model of the waits between the tiles of one round (Alg. 5 on the GPU), run
under random schedules on the CPU: every block a tile writes into must have been
loaded by the tile that reads its old contents first.

Per tile t the model has the steps of the round kernel, each allowed to run once
the waits the kernel makes before it are satisfied:
  load      its input blocks (no wait);
  publish   its digit counts: after its loads, and after the done words of the
            tiles whose ring slot it reuses (t - W .. end of that tile's super-tile);
  lookback  the counts of the earlier tiles of its super-tile;
  done      its done word, after the look-back;
  wait      the done words of the tiles before its super-tile whose input blocks
            it draws (pool entry sigma + m is input block m, read by tile m b / E);
  pi        its draws published in pi' (after `wait`; before it with the order the
            kernel had until the race was found: `pi_early`);
  first     the pi' entries of the blocks that earlier tiles drew and this tile
            continues (its first block of each digit);
  scatter   its writes, after `wait`, `first` and `pi`.
The draws themselves follow the sequential pool order (Sec. 2, eager allocation):
bucket d's block q >= 1 is drawn by the tile that writes rank q b - 1 of bucket d,
the tile's draws taking pool entries in the slot order of those elements.
"""
import random

import pytest

# the kernel's order of the steps within a tile, and the order it had before
STEPS = ("load", "publish", "lookback", "done", "wait", "pi", "first", "scatter")
STEPS_EARLY = ("load", "publish", "lookback", "done", "pi", "wait", "first", "scatter")


def plan(tiles_digits, sigma, b):
    """Per tile: F (draws of the earlier tiles), its draws {(d, q): m}, and the
    blocks (d, q) it writes."""
    base = [0] * sigma
    F = 0
    out = []
    for ds in tiles_digits:
        cnt = [0] * sigma
        fills = []
        for slot, d in enumerate(ds):
            r = base[d] + cnt[d]
            cnt[d] += 1
            if (r + 1) % b == 0:
                fills.append((slot, d, (r + 1) // b))
        fills.sort()
        draws = {(d, q): F + i for i, (_, d, q) in enumerate(fills)}
        writes = {(d, q) for d in range(sigma) if cnt[d]
                  for q in range(base[d] // b, (base[d] + cnt[d] - 1) // b + 1)}
        out.append((F, draws, writes))
        F += len(fills)
        for d in range(sigma):
            base[d] += cnt[d]
    return out


def dependencies(tiles_digits, sigma, b, E, W, ST, pi_early):
    """The steps of every tile in kernel order, the waits before each step, and
    the blocks each tile writes with the tile that reads their old contents."""
    P = plan(tiles_digits, sigma, b)
    n_t = len(P)
    drawer = {}
    for t, (_, draws, _) in enumerate(P):
        for blk, m in draws.items():
            drawer[blk] = (t, m)
    # Lemma 1 on the GPU: every drawn pool entry is an input block of a tile <= t
    for t, (F, draws, _) in enumerate(P):
        assert all(m * b // E <= t for m in draws.values())

    def deps(t, step):
        st0 = t - t % ST
        if step == "load":
            return []
        if step == "publish":
            d = [(t, "load")]
            if t >= W:
                j0 = t - W
                d += [(j, "done") for j in range(j0, min(j0 - j0 % ST + ST, n_t))]
            return d
        if step == "lookback":
            return [(t, "publish")] + [(j, "publish") for j in range(st0, t)]
        if step == "done":
            return [(t, "lookback")]
        if step == "wait":
            F, draws, _ = P[t]
            d = [(t, "lookback")]
            if draws:
                olo = F * b // E
                ohi = min(((F + len(draws)) * b - 1) // E + 1, st0)
                d += [(o, "done") for o in range(olo, ohi)]
            return d
        if step == "pi":
            return [(t, "lookback")] if pi_early else [(t, "wait")]
        if step == "first":
            return [(drawer[blk][0], "pi") for blk in P[t][2]
                    if blk[1] >= 1 and drawer[blk][0] != t]
        if step == "scatter":
            return [(t, "wait"), (t, "first"), (t, "pi")]
        raise ValueError(step)

    steps = STEPS_EARLY if pi_early else STEPS
    dep = {(t, s): deps(t, s) for t in range(n_t) for s in steps}
    writes = {t: [(blk, drawer[blk][1] * b // E) for blk in P[t][2] if blk[1] >= 1]
              for t in range(n_t)}
    return steps, dep, writes


def simulate(tiles_digits, sigma, b, E, W, ST, rng, pi_early, slow=0.15):
    """Runs one random schedule; returns the violations (tile, block, reader) and
    whether every step ran (no deadlock).  A random fraction ``slow`` of the tiles
    runs a step only when no other tile can: tiles far apart in time, as when
    other kernels hold compute units."""
    steps, dep, writes = dependencies(tiles_digits, sigma, b, E, W, ST, pi_early)
    n_t = len(tiles_digits)
    done = set()
    pos = {t: 0 for t in range(n_t)}  # next step of each tile, in kernel order
    violations = []
    lagging = {t for t in range(n_t) if rng.random() < slow}
    while len(done) < len(dep):
        ready = [t for t in range(n_t) if pos[t] < len(steps)
                 and all(x in done for x in dep[(t, steps[pos[t]])])]
        if not ready:
            return violations, False
        fast = [t for t in ready if t not in lagging]
        t = rng.choice(fast or ready)
        step = steps[pos[t]]
        if step == "scatter":
            violations += [(t, blk, r) for blk, r in writes[t] if (r, "load") not in done]
        done.add((t, step))
        pos[t] += 1
    return violations, True


def unordered_writes(tiles_digits, sigma, b, E, W, ST, pi_early):
    """The writes that some schedule can make before their reader's loads: those
    whose reader's `load` is not among the steps every schedule runs before the
    writer's `scatter` (its ancestors through the waits and the order of steps
    within a tile).  Empty means no schedule at all breaks the rule."""
    steps, dep, writes = dependencies(tiles_digits, sigma, b, E, W, ST, pi_early)
    n_t = len(tiles_digits)
    anc = {}
    for t in range(n_t):  # every wait points to an earlier tile or an earlier step
        for i, st in enumerate(steps):
            a = set()
            for x in dep[(t, st)] + ([(t, steps[i - 1])] if i else []):
                a.add(x)
                a |= anc[x]
            anc[(t, st)] = a
    return [(t, blk, r) for t in range(n_t) for blk, r in writes[t]
            if (r, "load") not in anc[(t, "scatter")]]


def workload(seed, n_t, sigma, E):
    rng = random.Random(seed)
    return [[rng.randrange(sigma) for _ in range(E)] for _ in range(n_t)]


# 4 digits, blocks of 32, tiles of 16: a bucket's block takes the elements of
# about 8 tiles, and its old contents are read about 4 tiles before the tile
# that draws it; a ring of 16 tiles (wider than that distance, as in the kernel),
# super-tiles of 2
GEO = dict(sigma=4, b=32, E=16, W=16, ST=2)


@pytest.mark.parametrize("seed", range(6))
def test_publishing_after_the_wait_never_writes_unread_blocks(seed):
    digits = workload(seed, 40, GEO["sigma"], GEO["E"])
    rng = random.Random(1000 + seed)
    for _ in range(60):
        violations, finished = simulate(digits, rng=rng, pi_early=False, **GEO)
        assert finished, "a schedule deadlocked"
        assert violations == []


def test_publishing_before_the_wait_can_write_unread_blocks():
    """The earlier order: the same model finds schedules in which a later tile
    writes into a drawn block whose reader has not loaded it."""
    digits = workload(7, 40, GEO["sigma"], GEO["E"])
    rng = random.Random(77)
    found = 0
    for _ in range(200):
        violations, finished = simulate(digits, rng=rng, pi_early=True, **GEO)
        assert finished
        found += bool(violations)
    assert found > 0


def test_plan_draws_match_the_closed_form():
    """F of each tile is the number of filled blocks of the earlier tiles,
    sum over d of floor(base[d] / b)."""
    sigma, b, E = GEO["sigma"], GEO["b"], GEO["E"]
    digits = workload(3, 30, sigma, E)
    P = plan(digits, sigma, b)
    base = [0] * sigma
    for t, (F, draws, _) in enumerate(P):
        assert F == sum(x // b for x in base)
        for d in digits[t]:
            base[d] += 1
        assert F + len(draws) == sum(x // b for x in base)


@pytest.mark.parametrize("geo", [GEO, dict(sigma=4, b=32, E=16, W=4, ST=2),
                                 dict(sigma=8, b=64, E=32, W=32, ST=4),
                                 dict(sigma=4, b=128, E=16, W=64, ST=8)])
@pytest.mark.parametrize("seed", range(3))
def test_no_schedule_writes_a_block_before_its_reader_loads_it(geo, seed):
    digits = workload(seed, 120, geo["sigma"], geo["E"])
    assert unordered_writes(digits, pi_early=False, **geo) == []


def test_the_earlier_order_leaves_writes_unordered():
    digits = workload(7, 120, GEO["sigma"], GEO["E"])
    assert unordered_writes(digits, pi_early=True, **GEO) != []
