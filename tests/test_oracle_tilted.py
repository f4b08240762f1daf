"""Pins for the "tilted" (recency-proportional) surface policy and the general
retained-rank MRCA estimator.

Independent facts: hand-worked sites; the retained set derived in closed form
equal to a brute-force replay of every deposit's write (last writer per site);
the recency-proportional guarantee (at least k + 1 retained ranks among the
last 2^(k+1) deposits); the general estimator equal to the steady policy's
closed form on steady surfaces; intervals bracketing the true MRCA with the
lower-bound miss rate within 2^-kc; recent MRCAs resolved more tightly than
under the steady policy; and the hybrid policy's two halves replaying as a
steady and a tilted surface on the even and odd ranks."""
import numpy as np
import pytest

import oracle

P10 = 429496729


def cfg(**kw):
    base = dict(width=10, height=8, pop=16, sites=32, k=2, selection=1, p32=P10, migration=1,
                seed=1, run_id=0, policy=1)
    base.update(kw)
    return base


def test_sites_hand_worked():
    # S = 32: one slot per level; the level is the number of trailing zeros
    want32 = {0: 31, 1: 0, 2: 1, 3: 0, 4: 2, 6: 1, 8: 3, 12: 2, 40: 3, 2 ** 20: 20, 3 << 30: 30,
              2 ** 31: 31}
    for r, site in want32.items():
        assert oracle.site_of_tilted(r, 32) == site, r
    # S = 64: two slots per level, alternating between consecutive members
    want64 = {1: 0, 3: 1, 5: 0, 7: 1, 2: 2, 6: 3, 10: 2, 4: 4, 12: 5, 0: 62, 2 ** 31: 63}
    for r, site in want64.items():
        assert oracle.site_of_tilted(r, 64) == site, r


@pytest.mark.parametrize("sites,limit", [(32, 3000), (64, 2000)])
def test_retained_set_equals_replay(sites, limit):
    last = {}
    for n in range(1, limit + 1):
        last[oracle.site_of_tilted(n - 1, sites)] = n - 1        # deposit of rank n - 1
        want = np.array(sorted(last.values()), dtype=np.uint64)
        assert np.array_equal(oracle.retained(n, sites, 1), want), n


@pytest.mark.parametrize("sites", [32, 64])
def test_retained_set_at_large_counts(sites):
    m = sites // 32
    rng = np.random.default_rng(sites)
    for n in list(rng.integers(2 ** 20, 2 ** 32, 200)) + [2 ** 31, 2 ** 31 + 1, 2 ** 32 - 1]:
        n = int(n)
        R = oracle.retained(n, sites, 1)
        sites_of = [oracle.site_of_tilted(int(r), sites) for r in R]
        assert len(set(sites_of)) == len(R) <= sites and (R < n).all()
        for r in R:
            r = int(r)
            k = min((r & -r).bit_length() - 1, 31) if r else 31
            # the next rank to take the same slot comes too late
            nxt = r + (m << (k + 1)) if k < 31 else r + (m << 31)
            assert nxt >= n, (n, r)


@pytest.mark.parametrize("sites", [32, 64])
def test_recency_proportional_guarantee(sites):
    for n in range(2, 5000):
        R = oracle.retained(n, sites, 1)
        age = n - 1 - R.astype(np.int64)
        k = 0
        while 2 ** (k + 1) <= n and k < 31:
            assert (age < 2 ** (k + 1)).sum() >= k + 1, (n, k)
            k += 1


@pytest.mark.parametrize("sites,bits", [(32, 1), (64, 1), (32, 2), (16, 4), (8, 8)])
def test_general_estimator_equals_steady_closed_form(sites, bits):
    rng = np.random.default_rng(sites + bits)
    words = sites * bits // 32
    for _ in range(300):
        Ta, Tb = (int(x) for x in rng.integers(0, 2 ** 20, 2))
        Da = rng.integers(0, 2 ** 32, words, dtype=np.uint64).astype(np.uint32)
        Db = Da.copy()
        if rng.random() < 0.7:
            Db[rng.integers(words)] ^= np.uint32(1 << int(rng.integers(32)))
        for kc in (1, 3):
            assert oracle.mrca_interval(Ta, Da, Tb, Db, sites, kc, bits) == \
                oracle.mrca_interval(Ta, Da, Tb, Db, sites, kc, bits, general=True)


@pytest.mark.parametrize("sites,kc", [(32, 4), (64, 5)])
def test_tilted_interval_brackets_true_mrca(sites, kc):
    c = cfg(sites=sites, seed=47)
    run = oracle.OracleRun(c, lineage=True)
    run.step(1200)
    _, T, D = run.population()
    rng = np.random.default_rng(9)
    sample = rng.choice(run.agents, size=150, replace=False)
    hi = lo = pairs = 0
    for x in range(len(sample)):
        for y in range(x + 1, len(sample)):
            a, b = int(sample[x]), int(sample[y])
            g = max(run.true_mrca(a, b), 0)
            L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], sites, kc, 1, policy=1)
            pairs += 1
            hi += g > U
            lo += g < L
    assert hi == 0
    bound = 2.0 ** -kc
    assert lo <= 1.25 * bound * pairs + 4 * np.sqrt(bound * pairs) + 1


def test_tilted_resolves_recent_ancestry_more_tightly():
    # pairs within one island share a recent ancestor; after 4,000 generations
    # the steady surface keeps every 128th rank, the tilted one dense recent ranks
    widths = {}
    for policy in (0, 1):
        c = cfg(width=6, height=4, pop=32, policy=policy, seed=3)
        run = oracle.OracleRun(c)
        run.step(4000)
        _, T, D = run.population()
        w = []
        for i in range(24):
            for s in range(1, 32, 3):
                a, b = i * 32, i * 32 + s
                L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], 32, 3, 1,
                                            policy=policy)
                w.append(U - L)
        widths[policy] = np.mean(w)
    assert widths[1] < 0.5 * widths[0], widths


def test_validation():
    assert oracle.validate(cfg(sites=32)) and oracle.validate(cfg(sites=64))
    assert oracle.validate(cfg(sites=32, dbits=2))
    assert not oracle.validate(cfg(sites=16, dbits=4))
    assert not oracle.validate(cfg(policy=3))


# --------------------------------------------------------------------------
# hybrid policy (64 sites): even ranks to a steady half, odd ranks to a tilted
# half
# --------------------------------------------------------------------------
def test_hybrid_sites_hand_worked():
    want = {0: 0, 2: 1, 4: 2, 62: 31, 1: 32 + 31, 3: 32 + 0, 5: 32 + 1, 7: 32 + 0, 9: 32 + 2}
    for r, site in want.items():
        assert oracle.site_of_policy(r, 64, 2) == site, r
    # even ranks 2q follow the steady half's policy on rank q (64 = 2 * 32)
    assert oracle.site_of_policy(64, 64, 2) == oracle.site_of(32, 32)
    assert oracle.site_of_policy(66, 64, 2) == oracle.site_of(33, 32) == oracle.DISCARD


def test_hybrid_retained_set_matches_replay():
    # Every retained rank is still the last writer of its site. The tilted half
    # keeps exactly its odd ranks; the steady half keeps the multiples of its
    # epoch's step, while ranks between them may linger until their sites are
    # taken over (the estimator does not rely on those).
    last = {}
    for n in range(1, 3001):
        site = oracle.site_of_policy(n - 1, 64, 2)
        if site != oracle.DISCARD:
            last[site] = n - 1
        R = oracle.retained(n, 64, 2)
        for r in R:
            assert last[oracle.site_of_policy(int(r), 64, 2)] == r, (n, r)
        odd = sorted(r for r in last.values() if r % 2)
        assert np.array_equal(R[R % 2 == 1], np.array(odd, dtype=np.uint64)), n
        even = R[R % 2 == 0] // 2
        assert np.array_equal(even, oracle.retained((n + 1) // 2, 32, 0)), n


def test_hybrid_interval_brackets_true_mrca():
    c = cfg(sites=64, policy=2, seed=53)
    run = oracle.OracleRun(c, lineage=True)
    run.step(1200)
    _, T, D = run.population()
    rng = np.random.default_rng(11)
    sample = rng.choice(run.agents, size=140, replace=False)
    hi = lo = pairs = 0
    kc = 4
    for x in range(len(sample)):
        for y in range(x + 1, len(sample)):
            a, b = int(sample[x]), int(sample[y])
            g = max(run.true_mrca(a, b), 0)
            L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], 64, kc, 1, policy=2)
            pairs += 1
            hi += g > U
            lo += g < L
    assert hi == 0
    bound = 2.0 ** -kc
    assert lo <= 1.25 * bound * pairs + 4 * np.sqrt(bound * pairs) + 1


def test_hybrid_validation():
    assert oracle.validate(cfg(sites=64, policy=2))
    assert not oracle.validate(cfg(sites=32, policy=2))
    assert not oracle.validate(cfg(sites=32, dbits=2, policy=2))
