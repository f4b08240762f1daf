"""Pins for the oracle's asynchronous schedule (Sec. 2 Methods: per-neighbour
immigration and emigration buffers, consumed and refilled at the start of each
pass of an island's update loop) in its reproducible interleavings: islands go
in consecutive groups, group c running generation t at step t + (c mod
(skew + 1)), each group reading its arrivals, updating, then publishing.

What fixes it independently of the oracle's own code: without skew it is the
synchronous schedule (pinned elsewhere); with migration off every interleaving
is; a brute-force model of one-agent islands, driven by Philox draws computed
here, gives every buffer, stamp and population value under skew (late and
overwritten genomes included); and each buffer holds the latest emission its
island's migration draws sent that way in a generation of its parity."""
import numpy as np
import pytest

import oracle

P10 = 429496729  # floor(0.1 * 2^32)


def cfg(**kw):
    base = dict(width=8, height=8, pop=32, sites=64, k=2, selection=1, p32=P10,
                migration=1, seed=1, run_id=0)
    base.update(kw)
    return base


def _neighbour(i, q, W, H):
    x, y = i % W, i // W
    if q == 0:
        y = (y - 1) % H
    elif q == 1:
        x = (x + 1) % W
    elif q == 2:
        y = (y + 1) % H
    else:
        x = (x - 1) % W
    return y * W + x


def _migration_draw(c, island, t):
    """The MIGRATE stream block of one island at generation t."""
    ctr = [0, island, t & 0xFFFFFFFF, ((t >> 32) << 2) | 1]
    return oracle.philox(ctr, [c["seed"], c["run_id"]])


def _same_population(a, b):
    fa, Ta, Da = a.population()
    fb, Tb, Db = b.population()
    return (np.array_equal(fa.view(np.uint32), fb.view(np.uint32)) and np.array_equal(Ta, Tb)
            and np.array_equal(Da, Db))


@pytest.mark.parametrize("kw", [
    dict(),
    dict(width=5, height=3, pop=8, sites=32, k=5),
    dict(width=1, height=6, pop=4, selection=0),
    dict(width=7, height=1, pop=16, law=1, p_ben32=12884902, p32=1417339207, k=5),
    dict(width=2, height=2, pop=64, sites=32, k=8),
])
@pytest.mark.parametrize("group", [1, 3, 64])
def test_unskewed_interleaving_is_the_synchronous_schedule(kw, group):
    # with neighbours never more than a generation apart, every genome sent in
    # t-1 is still in its parity buffer when the receiver runs t, and nothing
    # newer is eligible
    c = cfg(**kw)
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(c)
    a.step(37)
    b.step_async(20, group)
    b.step_async(17, group + 2)
    assert b.generation == 37
    assert _same_population(a, b)


@pytest.mark.parametrize("group,skew", [(1, 3), (3, 1), (7, 5), (64, 2)])
def test_without_migration_every_interleaving_is_synchronous(group, skew):
    c = cfg(migration=0, width=9, height=7, pop=16)
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(c)
    a.step(25)
    b.step_async(25, group, skew)
    assert _same_population(a, b)
    assert (b.mailboxes()["stamp"] == 0).all()


def test_skew_changes_the_result_when_migrating():
    c = cfg(width=6, height=6, pop=8)
    ref = oracle.OracleRun(c)
    ref.step(40)
    for group, skew in ((1, 1), (6, 3)):
        r = oracle.OracleRun(c)
        r.step_async(40, group, skew)
        assert not np.array_equal(r.population()[0], ref.population()[0])


@pytest.mark.parametrize("W,H,group,skew,n", [(4, 3, 1, 2, 15), (4, 3, 5, 1, 12), (1, 5, 2, 3, 20),
                                               (6, 1, 1, 4, 18), (2, 2, 3, 1, 9), (3, 3, 1, 0, 14),
                                               (5, 4, 2, 6, 25)])
def test_one_agent_islands_brute_force(W, H, group, skew, n):
    # One agent per island, no mutation: after a generation the agent is the
    # last arrival taken (directions in order N, E, S, W) or itself, so every
    # value, buffer and stamp follows from the migration draws alone.
    c = cfg(width=W, height=H, pop=1, p32=0, seed=4)
    I = W * H
    run = oracle.OracleRun(c)
    marks = np.arange(I, dtype=np.float32) * 2 + 1
    run.set_population(f=marks)
    value = marks.copy()
    deposits = np.zeros(I, dtype=np.uint32)       # T travels with the genome
    stamp = np.zeros((I, 4, 2), dtype=np.uint64)
    held = np.zeros((I, 4, 2), dtype=np.float32)
    held_T = np.zeros((I, 4, 2), dtype=np.uint32)
    seen = np.zeros((I, 4), dtype=np.uint64)
    late = lost = 0
    for step in range(n + skew):
        for grp, lo in enumerate(range(0, I, group)):
            t = step - grp % (skew + 1)
            if not 0 <= t < n:
                continue
            members = range(lo, min(lo + group, I))
            for i in members:
                for q in range(4):
                    j = _neighbour(i, q, W, H)
                    # sent before this generation and not taken yet; the newest
                    ok = [p for p in (0, 1) if seen[i, q] < stamp[j, q ^ 2, p] <= t]
                    if not ok:
                        continue
                    p = max(ok, key=lambda p: stamp[j, q ^ 2, p])
                    late += stamp[j, q ^ 2, p] < t
                    seen[i, q] = stamp[j, q ^ 2, p]
                    value[i] = held[j, q ^ 2, p]
                    deposits[i] = held_T[j, q ^ 2, p]
            sends = [(i, int(_migration_draw(c, i, t)[1] >> 30), value[i], deposits[i])
                     for i in members]
            for i in members:
                deposits[i] += 1
            for i, d, v, dT in sends:
                receiver, back = _neighbour(i, d, W, H), d ^ 2
                lost += stamp[i, d, t & 1] > seen[receiver, back]
                stamp[i, d, t & 1] = t + 1
                held[i, d, t & 1] = v
                held_T[i, d, t & 1] = dT
    run.step_async(n, group, skew)
    f, T, _ = run.population()
    assert np.array_equal(f, value)
    assert np.array_equal(T, deposits)
    mb = run.mailboxes()
    assert np.array_equal(mb["stamp"], stamp)
    assert np.array_equal(mb["seen"], seen)
    live = stamp > 0
    assert np.array_equal(mb["f"][live], held[live])
    assert np.array_equal(mb["T"][live], held_T[live])
    # every genome was taken at least one generation after it was sent
    assert (deposits <= n).all()
    if skew >= 2 and group < I:
        assert late > 0 and lost > 0          # the model exercised both


@pytest.mark.parametrize("group,skew", [(1, 0), (5, 2), (16, 1)])
def test_buffers_hold_the_latest_emission_of_each_parity(group, skew):
    c = cfg(width=8, height=5, pop=16, seed=9, run_id=3)
    I = c["width"] * c["height"]
    n = 23
    run = oracle.OracleRun(c)
    run.step_async(n, group, skew)
    dirs = np.array([[int(_migration_draw(c, i, t)[1] >> 30) for t in range(n)] for i in range(I)])
    mb = run.mailboxes()
    for i in range(I):
        for d in range(4):
            for p in range(2):
                gens = [t for t in range(n) if t % 2 == p and dirs[i, t] == d]
                assert mb["stamp"][i, d, p] == (gens[-1] + 1 if gens else 0)
    # a receiver takes nothing sent in or after its own last generation
    assert (mb["seen"] <= n - 1).all()


def test_clear_and_errors():
    c = cfg(width=4, height=4, pop=4)
    run = oracle.OracleRun(c)
    run.step_async(5, 3, 1)
    assert (run.mailboxes()["stamp"] > 0).any()
    run.clear_mailboxes()
    mb = run.mailboxes()
    assert (mb["stamp"] == 0).all() and (mb["seen"] == 0).all()
    with pytest.raises(RuntimeError):
        run.step_async(1, 0)
    lin = oracle.OracleRun(c, lineage=True)
    with pytest.raises(RuntimeError):
        lin.step_async(1, 4)
