"""Pins for the oracle's surface policy (the site each stratum deposit writes).

The policy ("doubling steady") keeps, after n deposits on S sites, the ranks that
are multiples of 2^e(n) below n, with e(n) = max(0, ceil(log2 n) - log2 S); the
j-th rank written in epoch e reuses the site of the j-th smallest rank dropped
when that epoch began. The oracle computes sites by a closed-form recursion; the
test below simulates the retained set explicitly, with a queue of freed sites,
and checks the guarantees the policy must give:
  G1 retained ranks sit in distinct sites,
  G2 |R(n)| = ceil(n / 2^e) lies in (S/2, S] once n > S,
  G3 rank 0 is kept, kept ranks are 2^e apart with 2^e < 2n/S, and the newest
     kept rank is at least n - 2^e,
  G4 a deposit only overwrites a rank that has just left the retained set.
"""
import math

import numpy as np
import pytest

import oracle


def _ceil_log2(n):
    return 0 if n <= 1 else (n - 1).bit_length()


def _simulate(S, n_max):
    s = S.bit_length() - 1
    site_rank = [None] * S
    free = []
    cur_e = 0
    sites = []
    for r in range(n_max):
        n = r + 1
        e = max(0, _ceil_log2(n) - s)
        step = 1 << e
        if e != cur_e:
            assert e == cur_e + 1
            dropped = sorted((rk, st) for st, rk in enumerate(site_rank)
                             if rk is not None and rk % step != 0)
            assert len(dropped) == S // 2
            assert not free  # the previous epoch used every freed site
            free = [st for _, st in dropped]
            cur_e = e
        if r % step != 0:
            sites.append(oracle.DISCARD)
        else:
            st = r if r < S else free.pop(0)
            old = site_rank[st]
            assert old is None or old % step != 0  # G4
            site_rank[st] = r
            sites.append(st)
        # G1/G2/G3 on the retained set after this deposit
        retained = set(range(0, n, step))
        held = {rk for rk in site_rank if rk is not None and rk % step == 0 and rk < n}
        assert held == retained
        assert len(retained) == -(-n // step)
        if n > S:
            assert S // 2 < len(retained) <= S
            assert step < 2 * n / S
        assert 0 in retained
        assert max(retained) >= n - step
    return sites


@pytest.mark.parametrize("S", [2, 4, 8, 16, 32, 64])
def test_closed_form_matches_explicit_simulation(S):
    n_max = 1 << 13 if S <= 16 else 1 << 12
    expect = _simulate(S, n_max)
    got = oracle.site_of_range(0, n_max, S)
    assert [int(x) for x in got] == expect


def test_small_case_by_hand():
    # S = 4 worked by hand from the definition: ranks 0-3 fill sites 0-3; at
    # n = 5 the epoch becomes 1, ranks 1 and 3 drop, ranks 4 and 6 reuse their
    # sites (1, 3); at n = 9 the epoch becomes 2, ranks 2 and 6 drop (sites 2
    # and 3), ranks 8 and 12 reuse them.
    got = [int(x) for x in oracle.site_of_range(0, 16, 4)]
    D = oracle.DISCARD
    assert got == [0, 1, 2, 3, 1, D, 3, D, 2, D, D, D, 3, D, D, D]


@pytest.mark.parametrize("S", [32, 64])
def test_large_ranks_keep_distinct_sites(S):
    rng = np.random.default_rng(7)
    ns = np.concatenate([rng.integers(S + 1, 1 << 31, size=300),
                         [S + 1, 2 * S, 2 * S + 1, (1 << 20) + 1, (1 << 31)]])
    for n in ns:
        n = int(n)
        e = oracle.epoch(n, S)
        step = 1 << e
        assert e == max(0, _ceil_log2(n) - int(math.log2(S)))
        ranks = list(range(0, n, step))
        assert S // 2 < len(ranks) <= S
        sites = [oracle.site_of(r, S) for r in ranks]
        assert oracle.DISCARD not in sites
        assert len(set(sites)) == len(sites)
        assert all(0 <= x < S for x in sites)


def test_written_iff_multiple_of_epoch_step():
    S = 32
    r = np.arange(0, 1 << 16, dtype=np.uint64)
    got = oracle.site_of_range(0, len(r), S)
    for rank in range(0, 1 << 16, 97):
        e = max(0, _ceil_log2(rank + 1) - 5)
        written = rank % (1 << e) == 0
        assert (got[rank] != oracle.DISCARD) == written
