"""Pins for the oracle's genome models (Sec. 2 Methods: any fixed-length genome
through initialize, mutate and evaluate): OneMax and Trap-4 on a 64-bit string.

Independent facts: hand-worked values and the extreme points of the two
fitness functions (Trap-4 by its definition: all-ones blocks score 4, a block
with u < 4 ones scores 3 - u); founders equal to the sampling-stream draws
computed here; every child one bit flip (at the drawn index) or none away from
its recorded parent; the stored fitness always the function of the string,
migrants included; selection on OneMax climbing toward the optimum."""
import numpy as np
import pytest
from scipy import stats

import oracle

P10 = 429496729


def cfg(**kw):
    base = dict(width=8, height=8, pop=32, sites=64, k=2, selection=1, p32=P10,
                migration=1, seed=1, run_id=0, model=1)
    base.update(kw)
    return base


@pytest.mark.parametrize("p0,p1,onemax,trap", [
    (0, 0, 0, 48),                         # every block u = 0 scores 3
    (0xFFFFFFFF, 0xFFFFFFFF, 64, 64),      # every block u = 4 scores 4 (global optimum)
    (0x77777777, 0x77777777, 48, 0),       # every block u = 3 scores 0 (minimum)
    (0x11111111, 0x11111111, 16, 32),      # every block u = 1 scores 2
    (0x33333333, 0x00000000, 16, 32),      # 8 blocks u = 2 score 1, 8 blocks u = 0 score 3
    (0x0000000F, 0x00000000, 4, 49),       # one block u = 4, fifteen u = 0
    (0x00000001, 0x80000000, 2, 46),       # two blocks u = 1, fourteen u = 0
])
def test_model_functions_hand_worked(p0, p1, onemax, trap):
    assert oracle.evaluate(1, p0, p1) == onemax
    assert oracle.evaluate(2, p0, p1) == trap


def test_founders_are_sampling_draws_and_evaluated():
    c = cfg(width=5, height=3, pop=8, model=2)
    run = oracle.OracleRun(c)
    P = run.payload()
    f, T, D = run.population()
    for i in range(15):
        for s in range(8):
            w = oracle.philox([s, i, 0xFFFFFFFF, 0xFFFFFFFE], [c["seed"], c["run_id"]])
            assert P[i * 8 + s, 0] == w[0] and P[i * 8 + s, 1] == w[1]
    assert all(f[a] == oracle.evaluate(2, *P[a]) for a in range(P.shape[0]))
    assert (T == 0).all() and (D == 0).all()
    # founders' bits are fair coins
    big = oracle.OracleRun(cfg(width=32, height=32, pop=32))
    bits = np.unpackbits(big.payload().view(np.uint8))
    assert stats.binomtest(int(bits.sum()), bits.size, 0.5).pvalue > 1e-4


@pytest.mark.parametrize("model", [1, 2])
def test_children_are_one_flip_from_their_parent(model):
    c = cfg(width=6, height=5, pop=16, model=model, migration=0, p32=2 ** 31)
    run = oracle.OracleRun(c, lineage=True)
    before = run.payload()
    run.step(1)
    after = run.payload()
    f, _, _ = run.population()
    N = c["pop"]
    flips = 0
    for i in range(c["width"] * c["height"]):
        for s in range(N):
            child = i * N + s
            gens, isl, slot = run.ancestry(child)   # newest first: the child, then its parent
            assert gens[1] == 0
            par = int(isl[1]) * N + int(slot[1])
            w = oracle.philox([s, i, 0, 0], [c["seed"], c["run_id"]])
            diff = (int(after[child, 0]) ^ int(before[par, 0])) | \
                   ((int(after[child, 1]) ^ int(before[par, 1])) << 32)
            if w[2] < c["p32"]:
                assert diff == 1 << (int(w[3]) & 63)
                flips += 1
            else:
                assert diff == 0
            assert f[child] == oracle.evaluate(model, *after[child])
    assert 0.35 < flips / (c["width"] * c["height"] * N) < 0.65


@pytest.mark.parametrize("model", [1, 2])
def test_fitness_is_always_the_function_of_the_string(model):
    # with migration and selection: migrants carry their strings
    c = cfg(width=7, height=5, pop=8, model=model, k=5)
    run = oracle.OracleRun(c)
    for _ in range(4):
        run.step(25)
        f, _, _ = run.population()
        P = run.payload()
        assert all(f[a] == oracle.evaluate(model, *P[a]) for a in range(P.shape[0]))
    ob = run.outbox()
    assert ob["valid"].all()


def test_onemax_climbs_under_selection_and_drifts_without():
    sel = oracle.OracleRun(cfg(width=8, height=8, pop=32, k=4, p32=P10 // 4))
    neu = oracle.OracleRun(cfg(width=8, height=8, pop=32, selection=0, p32=P10 // 4))
    f0 = sel.population()[0].mean()
    sel.step(300)
    neu.step(300)
    assert 31 < f0 < 33                          # founders: fair coins
    assert sel.population()[0].mean() > 60       # near the optimum
    assert abs(neu.population()[0].mean() - 32) < 6


def test_model_zero_unchanged_and_validation():
    a = oracle.OracleRun(cfg(model=0))
    a.step(10)
    assert (a.payload() == 0).all()
    assert not oracle.validate(cfg(model=3))
    assert not oracle.validate(cfg(model=1, law=1, p_ben32=5))
    assert oracle.validate(cfg(model=2))


@pytest.mark.parametrize("model", [1, 2])
def test_async_unskewed_equals_synchronous_with_strings(model):
    c = cfg(width=6, height=4, pop=8, model=model)
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(c)
    a.step(30)
    b.step_async(30, 5)
    assert np.array_equal(a.payload(), b.payload())
    assert np.array_equal(a.population()[0], b.population()[0])
