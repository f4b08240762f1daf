"""Pins for the oracle's generation step against what the paper and the
mathematics fix: tournament winner distribution (closed form), mutation law,
migration geometry and replacement (brute-force model for one agent per
island), lineage consistency, Wright-Fisher coalescence, MRCA-interval bounds,
determinism and resume."""
import numpy as np
import pytest
from scipy import stats

import oracle

P10 = 429496729  # floor(0.1 * 2^32)


def cfg(**kw):
    base = dict(width=8, height=8, pop=32, sites=64, k=2, selection=1, p32=P10,
                migration=1, seed=1, run_id=0)
    base.update(kw)
    return base


def _chi2_ok(observed, expected, alpha=1e-4):
    observed = np.asarray(observed, dtype=float)
    expected = np.asarray(expected, dtype=float)
    keep = expected > 0
    stat = ((observed[keep] - expected[keep]) ** 2 / expected[keep]).sum()
    dof = keep.sum() - 1
    return stats.chi2.sf(stat, dof) > alpha, stat


# --------------------------------------------------------------------------
# selection (Sec. 2: best of n randomly sampled individuals, ties random)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 5, 8])
def test_tournament_winner_rank_closed_form(k):
    N = 32
    c = cfg(width=64, height=64, pop=N, k=k, p32=0, migration=0, seed=11)
    run = oracle.OracleRun(c)
    rng = np.random.default_rng(k)
    perm = np.concatenate([rng.permutation(N) for _ in range(64 * 64)]).astype(np.float32)
    run.set_population(f=perm)
    run.step(1)
    f, _, _ = run.population()
    v = np.arange(N)
    # winner value v (0 worst .. N-1 best) has P = ((v+1)/N)^k - (v/N)^k
    p = ((v + 1) / N) ** k - (v / N) ** k
    counts = np.bincount(f.astype(int), minlength=N)
    ok, stat = _chi2_ok(counts, p * f.size)
    assert ok, stat


def test_neutral_is_uniform_and_k1_equals_neutral():
    N = 16
    a = oracle.OracleRun(cfg(pop=N, k=1, selection=1, seed=3))
    b = oracle.OracleRun(cfg(pop=N, k=6, selection=0, seed=3))
    a.step(40)
    b.step(40)
    for x, y in zip(a.population(), b.population()):
        assert np.array_equal(x, y)
    c = cfg(width=64, height=64, pop=N, selection=0, p32=0, migration=0, seed=5)
    run = oracle.OracleRun(c)
    vals = np.tile(np.arange(N, dtype=np.float32), 64 * 64)
    run.set_population(f=vals)
    run.step(1)
    counts = np.bincount(run.population()[0].astype(int), minlength=N)
    ok, stat = _chi2_ok(counts, np.full(N, vals.size / N))
    assert ok, stat


def test_ties_broken_uniformly():
    # Fitness 1 on half the slots, 0 on the rest: a tournament of k picks a
    # fit winner with P = 1 - 2^-k, and among fit slots every one equally often.
    N, k = 32, 3
    c = cfg(width=64, height=64, pop=N, k=k, p32=0, migration=0, seed=9)
    run = oracle.OracleRun(c, lineage=True)
    f0 = np.tile((np.arange(N) % 2).astype(np.float32), 64 * 64)
    run.set_population(f=f0)
    run.step(1)
    f, _, _ = run.population()
    n = f.size
    frac = f.mean()
    sd = np.sqrt((1 - 2.0 ** -k) * 2.0 ** -k / n)
    assert abs(frac - (1 - 2.0 ** -k)) < 5 * sd
    slots = []
    for a in range(0, n, 7):
        _, _, s = run.ancestry(a)
        if f[a] == 1.0:
            slots.append(int(s[1]))
    counts = np.bincount(slots, minlength=N)[1::2]
    ok, stat = _chi2_ok(counts, np.full(N // 2, len(slots) / (N // 2)))
    assert ok, stat


# --------------------------------------------------------------------------
# mutation (Sec. 2: applied across all genomes of the next population)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p32", [P10, 0xFFFFFFFF])
def test_mutation_law(p32):
    c = cfg(width=64, height=64, pop=32, p32=p32, migration=0, seed=21)
    run = oracle.OracleRun(c)
    run.step(1)
    f = run.population()[0]
    p = p32 / 2.0 ** 32
    vals = np.array([-1.0, -0.5, 0.0, 0.5, 1.0], dtype=np.float32)
    counts = np.array([(f == v).sum() for v in vals])
    assert counts.sum() == f.size
    expect = np.array([p / 5, p / 5, 1 - p + p / 5, p / 5, p / 5]) * f.size
    ok, stat = _chi2_ok(counts, expect)
    assert ok, stat


def test_no_mutation_keeps_fitness():
    run = oracle.OracleRun(cfg(p32=0))
    run.step(50)
    f, T, _ = run.population()
    assert np.all(f == 0.0)


# --------------------------------------------------------------------------
# migration (Sec. 2: immigrants replace random members, emigrants are copies
# sent to cardinal neighbours). With one agent per island and no mutation the
# whole dynamics is a deterministic function of the emitted directions.
# --------------------------------------------------------------------------
def _neighbour(i, d, W, H):
    x, y = i % W, i // W
    if d == 0:
        y = (y - 1) % H
    elif d == 1:
        x = (x + 1) % W
    elif d == 2:
        y = (y + 1) % H
    else:
        x = (x - 1) % W
    return y * W + x


@pytest.mark.parametrize("W,H", [(6, 5), (1, 7), (2, 3), (9, 1)])
def test_migration_one_agent_islands_brute_force(W, H):
    c = cfg(width=W, height=H, pop=1, p32=0, seed=4)
    run = oracle.OracleRun(c)
    I = W * H
    marks = np.arange(I, dtype=np.float32) * 2 + 1
    run.set_population(f=marks)
    value = marks.copy()          # model of each island's single agent
    pending = None                # model of the outbox (valid, dir, value)
    for t in range(12):
        post = value.copy()
        if pending is not None:
            for i in range(I):
                for q in range(4):             # later direction wins
                    j = _neighbour(i, q, W, H)
                    if pending[0][j] and pending[1][j] == (q ^ 2):
                        post[i] = pending[2][j]
        run.step(1)
        ob = run.outbox()
        assert ob["valid"].all()
        # the emitted copy is the post-immigration agent
        assert np.array_equal(ob["f"], post)
        value = post
        pending = (ob["valid"].astype(bool), ob["dir"].astype(int), ob["f"].copy())
        f, T, _ = run.population()
        assert np.array_equal(f, value)
    # each island's agent is marked by an island it could have come from
    assert set(np.unique(f)).issubset(set(marks))


def test_migration_off_keeps_islands_closed():
    c = cfg(width=5, height=4, pop=8, p32=0, migration=0, selection=0, seed=2)
    run = oracle.OracleRun(c)
    marks = np.repeat(np.arange(20, dtype=np.float32), 8)
    run.set_population(f=marks)
    run.step(30)
    f, T, _ = run.population()
    assert np.array_equal(f, marks)
    assert np.all(T == 30)
    assert not run.outbox()["valid"].any()


def test_arrivals_per_island_bounded_and_sourced():
    # Island-unique marks, neutral selection, no mutation: after two
    # generations every agent of island i carries its own mark or the mark of
    # a neighbour that emitted toward i; at most 4 foreign marks per island.
    W, H, N = 7, 6, 8
    c = cfg(width=W, height=H, pop=N, p32=0, selection=0, seed=8)
    run = oracle.OracleRun(c)
    run.set_population(f=np.repeat(np.arange(W * H, dtype=np.float32), N))
    run.step(1)
    ob = run.outbox()
    run.step(1)
    f = run.population()[0].reshape(W * H, N)
    for i in range(W * H):
        senders = {j for q in range(4) for j in [_neighbour(i, q, W, H)]
                   if ob["valid"][j] and ob["dir"][j] == (q ^ 2)}
        allowed = {float(i)} | {float(j) for j in senders}
        assert set(f[i].tolist()) <= allowed
        assert len(set(f[i].tolist()) - {float(i)}) <= 4


# --------------------------------------------------------------------------
# lineage: every parent link must be consistent with one generation's
# operations (T + 1, fitness moved by one delta, surface differing at most
# in the deposited site).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("selection", [0, 1])
def test_lineage_links_are_single_generation_steps(selection):
    c = cfg(width=6, height=6, pop=16, sites=32, seed=12, selection=selection)
    run = oracle.OracleRun(c, lineage=True)
    hist = [run.population()]
    for _ in range(120):
        run.step(1)
        hist.append(run.population())
    N = c["pop"]
    deltas = set()
    changed = 0
    links = 0
    ups = downs = 0
    for a in range(0, run.agents, 5):
        gens, isl, slt = run.ancestry(a)
        assert np.all(np.diff(gens.astype(np.int64)) < 0)
        assert gens[-1] == 0
        f_now, T_now, _ = hist[-1]
        assert T_now[a] == len(gens) - 1
        for (gc, ic, sc), (gp, ip, sp) in zip(zip(gens[:-1], isl[:-1], slt[:-1]),
                                              zip(gens[1:], isl[1:], slt[1:])):
            fc, Tc, Dc = (h[ic * N + sc] for h in hist[gc])
            fp, Tp, Dp = (h[ip * N + sp] for h in hist[gp])
            assert Tc == Tp + 1
            d = float(fc) - float(fp)
            deltas.add(d)
            changed += d != 0
            ups += d > 0
            downs += d < 0
            links += 1
            diff = np.bitwise_xor(Dc, Dp)
            site = oracle.site_of(int(Tp), 32)
            if site == oracle.DISCARD:
                assert not diff.any()
            else:
                mask = np.zeros_like(diff)
                mask[site >> 5] = 1 << (site & 31)
                assert not (diff & ~mask).any()
    assert deltas <= {-1.0, -0.5, 0.0, 0.5, 1.0}
    if selection:
        # surviving lineages are enriched for beneficial mutations
        assert ups > 2 * downs
    else:
        # neutral: lineages are blind to mutations, nonzero deltas at 4p/5
        assert 0.05 < changed / links < 0.11


def test_wright_fisher_pair_coalescence_is_geometric():
    # Neutral selection, no migration: each island is a Wright-Fisher
    # population, so two distinct agents coalesce tau generations back with
    # tau ~ Geometric(1/N).
    N = 16
    c = cfg(width=64, height=64, pop=N, selection=0, migration=0, p32=0, seed=31)
    run = oracle.OracleRun(c, lineage=True)
    G = 300
    run.step(G)
    taus = []
    for i in range(64 * 64):
        g = run.true_mrca(i * N + 0, i * N + 1)
        assert g >= 0
        taus.append(G - g)
    taus = np.array(taus)
    assert taus.min() >= 1
    edges = list(range(1, 40)) + [G + 1]
    obs = np.histogram(taus, bins=edges)[0]
    cdf = stats.geom.cdf(np.array(edges) - 1, 1.0 / N)
    exp = np.diff(cdf) * len(taus)
    ok, stat = _chi2_ok(obs, exp)
    assert ok, stat
    assert abs(taus.mean() - N) < 5 * np.sqrt((1 - 1 / N) * N * N / len(taus))


def test_siblings_mrca_is_parent():
    c = cfg(width=4, height=4, pop=32, sites=32, seed=17)
    run = oracle.OracleRun(c, lineage=True)
    run.step(60)
    f, T, D = run.population()
    parents = {}
    found = 0
    for a in range(run.agents):
        g, i, s = run.ancestry(a)
        key = (int(g[1]), int(i[1]), int(s[1]))
        if key in parents:
            b = parents[key]
            assert run.true_mrca(a, b) == T[a] - 1 == T[b] - 1
            L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], 32)
            assert U >= T[a] - 1
            found += 1
        else:
            parents[key] = a
    assert found > 100


def test_mrca_interval_brackets_true_mrca():
    S, kc = 32, 5
    c = cfg(width=12, height=10, pop=16, sites=S, seed=41)
    run = oracle.OracleRun(c, lineage=True)
    run.step(1500)
    f, T, D = run.population()
    rng = np.random.default_rng(3)
    sample = rng.choice(run.agents, size=160, replace=False)
    viol_hi = 0
    viol_lo = 0
    eligible = 0
    pairs = 0
    related = 0
    for x in range(len(sample)):
        for y in range(x + 1, len(sample)):
            a, b = int(sample[x]), int(sample[y])
            g = run.true_mrca(a, b)
            g = max(g, 0)
            L, U = oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], S, kc)
            pairs += 1
            viol_hi += g > U
            viol_lo += g < L
            eligible += L > 0
            related += g > 0
    assert viol_hi == 0
    assert eligible > 1000 and related > 1000
    # P(g < L) <= 2^-kc for each pair, so the rate is over all pairs; pairs
    # share ancestry, so allow slack beyond the binomial
    bound = 2.0 ** -kc
    assert viol_lo <= 1.25 * bound * pairs + 4 * np.sqrt(bound * pairs) + 1


def test_mrca_interval_special_cases():
    S = 32
    D = np.array([0x12345678], dtype=np.uint32)
    # identical surfaces: no mismatch, U = min(T)
    L, U = oracle.mrca_interval(1000, D, 900, D, S, 5)
    assert U == 900
    # mismatch at rank 0 (site 0): MRCA before any common deposit
    D2 = D ^ np.uint32(1)
    L, U = oracle.mrca_interval(1000, D, 1000, D2, S, 5)
    assert (L, U) == (0, 0)


# --------------------------------------------------------------------------
# determinism, resume, sampling
# --------------------------------------------------------------------------
def test_determinism_and_split_steps():
    a = oracle.OracleRun(cfg(seed=5))
    b = oracle.OracleRun(cfg(seed=5))
    a.step(300)
    b.step(100)
    b.step(200)
    for x, y in zip(a.population(), b.population()):
        assert np.array_equal(x, y)
    c = oracle.OracleRun(cfg(seed=6))
    c.step(300)
    assert not np.array_equal(a.population()[2], c.population()[2])


def test_resume_from_state():
    a = oracle.OracleRun(cfg(seed=9, sites=32))
    a.step(150)
    pop = a.population()
    ob = a.outbox()
    b = oracle.OracleRun(cfg(seed=9, sites=32))
    b.set_population(*pop)
    b.set_outbox(ob["valid"], ob["dir"], ob["f"], ob["T"], ob["D"])
    b.set_generation(150)
    a.step(150)
    b.step(150)
    for x, y in zip(a.population(), b.population()):
        assert np.array_equal(x, y)


def test_sample_one_per_island():
    run = oracle.OracleRun(cfg(width=32, height=32))
    run.step(3)
    ids = run.sample_one_per_island()
    assert np.array_equal(ids // 32, np.arange(32 * 32))
    counts = np.bincount((ids % 32).astype(int), minlength=32)
    ok, stat = _chi2_ok(counts, np.full(32, 1024 / 32))
    assert ok, stat


def test_validation():
    assert oracle.validate(cfg())
    assert not oracle.validate(cfg(pop=24))
    assert not oracle.validate(cfg(sites=48))
    assert not oracle.validate(cfg(k=9))
    assert not oracle.validate(cfg(k=0))
    assert not oracle.validate(cfg(width=0))


def test_bulk_mrca_functions_match_pairwise():
    S = 32
    c = cfg(width=6, height=5, pop=16, sites=S, seed=44)
    run = oracle.OracleRun(c, lineage=True)
    run.step(300)
    f, T, D = run.population()
    ids = np.array([0, 3, 17, 100, 101, 250, 479, 333], dtype=np.uint64)
    G = run.true_mrca_matrix(ids)
    Lm, Um = oracle.mrca_interval_matrix(T[ids.astype(int)], D[ids.astype(int)], S, 5)
    for x in range(len(ids)):
        for y in range(len(ids)):
            a, b = int(ids[x]), int(ids[y])
            if x != y:
                assert G[x, y] == run.true_mrca(a, b)
            else:
                assert G[x, x] == T[a]
            assert (Lm[x, y], Um[x, y]) == oracle.mrca_interval(int(T[a]), D[a], int(T[b]), D[b], S, 5)
