"""Pins for wider differentia (2, 4 or 8 bits per stratum at the surface's
32- or 64-bit footprint, so S = 64/b or 32/b sites): each deposit writes, at
the policy's site, the top b bits of word 0 of its own Philox block, and
nothing else changes; the MRCA interval from two such surfaces never sits
below the true MRCA's counter at U and misses at L with rate at most
2^-(b kc); single-bit runs are unchanged (their pins live with the
dynamics tests)."""
import numpy as np
import pytest

import oracle

P10 = 429496729
SHAPES = [(32, 2), (16, 4), (8, 8), (16, 2), (8, 4), (4, 8)]   # (sites, bits)


def cfg(**kw):
    base = dict(width=6, height=5, pop=8, sites=16, dbits=4, k=2, selection=1, p32=P10,
                migration=1, seed=1, run_id=0)
    base.update(kw)
    return base


def _field(words, site, bits):
    pos = site * bits
    return (int(words[pos // 32]) >> (pos % 32)) & ((1 << bits) - 1)


@pytest.mark.parametrize("sites,bits", SHAPES)
def test_each_deposit_writes_its_drawn_field_only(sites, bits):
    # no migration: every child at generation t has T = t before its deposit,
    # and its parent is its island's tournament winner
    c = cfg(sites=sites, dbits=bits, migration=0, width=4, height=3, pop=8, seed=5)
    run = oracle.OracleRun(c, lineage=True)
    N, I = c["pop"], 12
    words = sites * bits // 32
    assert run.population()[2].shape == (run.agents, words)
    for t in range(3 * sites + 5):
        before = run.population()[2].copy()
        run.step(1)
        after = run.population()[2]
        site = oracle.site_of(t, sites)
        for i in range(I):
            for s in range(N):
                child = i * N + s
                _, isl, slot = run.ancestry(child)
                parent = int(isl[1]) * N + int(slot[1])
                want = before[parent].copy()
                if site != oracle.DISCARD:
                    d = oracle.philox([s + 256, i, t, 3], [c["seed"], c["run_id"]])
                    value = int(d[0]) >> (32 - bits)
                    pos = site * bits
                    w = pos // 32
                    mask = ((1 << bits) - 1) << (pos % 32)
                    want[w] = (int(want[w]) & ~mask & 0xFFFFFFFF) | (value << (pos % 32))
                    assert _field(after[child], site, bits) == value
                assert np.array_equal(after[child], want), (t, child)


@pytest.mark.parametrize("sites,bits,kc", [(16, 4, 2), (32, 2, 3), (8, 8, 1)])
def test_interval_brackets_true_mrca(sites, bits, kc):
    c = cfg(width=10, height=8, pop=16, sites=sites, dbits=bits, seed=43)
    run = oracle.OracleRun(c, lineage=True)
    run.step(900)
    _, T, D = run.population()
    rng = np.random.default_rng(5)
    sample = rng.choice(run.agents, size=150, replace=False)
    hi = lo = pairs = related = 0
    for x in range(len(sample)):
        for y in range(x + 1, len(sample)):
            a, b = int(sample[x]), int(sample[y])
            g = max(run.true_mrca(a, b), 0)
            L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], sites, kc, bits)
            pairs += 1
            hi += g > U
            lo += g < L
            related += g > 0
    assert hi == 0
    assert related > 1000
    bound = 2.0 ** -(bits * kc)
    assert lo <= 1.25 * bound * pairs + 4 * np.sqrt(bound * pairs) + 1


def test_interval_special_cases_and_matrix():
    sites, bits = 8, 8
    D = np.array([0x12345678, 0x9ABCDEF0], dtype=np.uint32)
    assert oracle.mrca_interval(1000, D, 900, D, sites, 3, bits)[1] == 900
    # a mismatch in the rank-0 field (site 0, bits 0..7)
    assert oracle.mrca_interval(1000, D, 1000, D ^ np.array([0x80, 0], np.uint32), sites, 3,
                                bits) == (0, 0)
    # with 3 deposits only fields 0..2 (bits 0..23) are retained: a mismatch in
    # field 5 (word 1, bits 8..15) changes nothing
    assert oracle.mrca_interval(3, D, 3, D ^ np.array([0, 0x100], np.uint32), sites, 3,
                                bits)[1] == 3
    assert oracle.mrca_interval(3, D, 3, D ^ np.array([0x10000, 0], np.uint32), sites, 3,
                                bits)[1] == 2
    rng = np.random.default_rng(2)
    T = rng.integers(0, 5000, 12).astype(np.uint32)
    DD = rng.integers(0, 2 ** 32, (12, 2), dtype=np.uint64).astype(np.uint32)
    L, U = oracle.mrca_interval_matrix(T, DD, sites, 3, bits)
    for x in range(12):
        for y in range(12):
            assert (L[x, y], U[x, y]) == oracle.mrca_interval(int(T[x]), DD[x], int(T[y]), DD[y],
                                                              sites, 3, bits)


def test_validation_and_single_bit_default():
    for sites, bits in SHAPES + [(32, 1), (64, 1)]:
        assert oracle.validate(cfg(sites=sites, dbits=bits))
    for sites, bits in [(32, 4), (64, 2), (16, 1), (2, 16), (12, 4), (16, 3), (4, 4)]:
        assert not oracle.validate(cfg(sites=sites, dbits=bits))
    # without the field, one bit per differentia
    c = cfg(sites=32)
    del c["dbits"]
    a = oracle.OracleRun(c)
    b = oracle.OracleRun(dict(c, dbits=1))
    a.step(40)
    b.step(40)
    assert np.array_equal(a.population()[2], b.population()[2])
