"""Pins for the oracle's asynchronous schedule (Sec. 2 Methods: per-neighbour
immigration and emigration buffers, consumed and refilled at the start of each
pass of an island's update loop) in its sequential interleaving: islands go in
consecutive groups, each reading its arrivals, updating, then publishing.

What fixes it independently of the oracle's own code: a single group is the
synchronous schedule (pinned elsewhere); with migration off every group size
is; a brute-force model of one-agent islands, driven by Philox draws computed
here, gives every buffer, stamp and population value; and each buffer holds the
latest emission its island's migration draws sent that way."""
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
def test_single_group_is_the_synchronous_schedule(kw):
    c = cfg(**kw)
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(c)
    islands = c["width"] * c["height"]
    a.step(37)
    b.step_async(20, islands)
    b.step_async(17, islands + 5)
    assert b.generation == 37
    assert _same_population(a, b)


@pytest.mark.parametrize("group", [1, 3, 7, 64])
def test_without_migration_every_group_size_is_synchronous(group):
    c = cfg(migration=0, width=9, height=7, pop=16)
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(c)
    a.step(25)
    b.step_async(25, group)
    assert _same_population(a, b)
    assert (b.mailboxes()["stamp"] == 0).all()


def test_groups_change_the_result_when_migrating():
    c = cfg(width=6, height=6, pop=8)
    runs = {}
    for group in (1, 4, 36):
        r = oracle.OracleRun(c)
        r.step_async(40, group)
        runs[group] = r.population()[0]
    assert not np.array_equal(runs[1], runs[36])
    assert not np.array_equal(runs[4], runs[36])


@pytest.mark.parametrize("W,H,group", [(4, 3, 1), (4, 3, 5), (1, 5, 2), (6, 1, 4), (2, 2, 3),
                                       (3, 3, 9)])
def test_one_agent_islands_brute_force(W, H, group):
    # One agent per island, no mutation: the agent after a generation is the
    # last fresh arrival (directions in order N, E, S, W) or itself, so every
    # value, buffer and stamp follows from the migration draws alone.
    c = cfg(width=W, height=H, pop=1, p32=0, seed=4)
    I = W * H
    run = oracle.OracleRun(c)
    marks = np.arange(I, dtype=np.float32) * 2 + 1
    run.set_population(f=marks)
    value = marks.copy()
    deposits = np.zeros(I, dtype=np.uint32)       # T travels with the genome
    stamp = np.zeros((I, 4), dtype=np.uint64)
    held = np.zeros((I, 4), dtype=np.float32)
    held_T = np.zeros((I, 4), dtype=np.uint32)
    seen = np.zeros((I, 4), dtype=np.uint64)
    for t in range(15):
        for lo in range(0, I, group):
            members = range(lo, min(lo + group, I))
            for i in members:
                for q in range(4):
                    j = _neighbour(i, q, W, H)
                    if stamp[j, q ^ 2] > seen[i, q]:
                        seen[i, q] = stamp[j, q ^ 2]
                        value[i] = held[j, q ^ 2]
                        deposits[i] = held_T[j, q ^ 2]
            sends = [(i, int(_migration_draw(c, i, t)[1] >> 30), value[i], deposits[i])
                     for i in members]
            for i in members:
                deposits[i] += 1
            for i, d, v, dT in sends:
                stamp[i, d] = t + 1
                held[i, d] = v
                held_T[i, d] = dT
        run.step_async(1, group)
        f, T, _ = run.population()
        assert np.array_equal(f, value), t
        assert np.array_equal(T, deposits), t
        mb = run.mailboxes()
        assert np.array_equal(mb["stamp"], stamp), t
        assert np.array_equal(mb["seen"], seen), t
        live = stamp > 0
        assert np.array_equal(mb["f"][live], held[live]), t
        assert np.array_equal(mb["T"][live], held_T[live]), t
    # a group that reads a neighbour after it published sees a genome one
    # deposit younger than the synchronous schedule would deliver
    if group < I:
        assert len(np.unique(deposits)) > 1


@pytest.mark.parametrize("group", [1, 5, 16])
def test_buffers_hold_the_latest_emission_and_receivers_take_them_in_order(group):
    c = cfg(width=8, height=5, pop=16, seed=9, run_id=3)
    I = c["width"] * c["height"]
    n = 23
    run = oracle.OracleRun(c)
    run.step_async(n, group)
    dirs = np.array([[int(_migration_draw(c, i, t)[1] >> 30) for t in range(n)] for i in range(I)])
    mb = run.mailboxes()

    def latest(i, d, last_gen):
        gens = np.nonzero(dirs[i, :last_gen + 1] == d)[0]
        return int(gens[-1]) + 1 if gens.size else 0

    for i in range(I):
        for d in range(4):
            assert mb["stamp"][i, d] == latest(i, d, n - 1)
    # in the last generation, a receiver read a sender's buffer before or after
    # the sender published, as their groups are ordered
    for i in range(I):
        for q in range(4):
            j = _neighbour(i, q, c["width"], c["height"])
            before = j // group < i // group
            assert mb["seen"][i, q] == latest(j, q ^ 2, n - 1 if before else n - 2)


def test_clear_and_errors():
    c = cfg(width=4, height=4, pop=4)
    run = oracle.OracleRun(c)
    run.step_async(5, 3)
    assert (run.mailboxes()["stamp"] > 0).any()
    run.clear_mailboxes()
    mb = run.mailboxes()
    assert (mb["stamp"] == 0).all() and (mb["seen"] == 0).all()
    with pytest.raises(RuntimeError):
        run.step_async(1, 0)
    lin = oracle.OracleRun(c, lineage=True)
    with pytest.raises(RuntimeError):
        lin.step_async(1, 4)
