"""Pins for the paper's two mutation treatments in the oracle (Sec. 3:
purifying-only, where 33% of replications lower fitness by a normally
distributed amount, and adaptation-enabled, which adds beneficial normally
distributed increments with probability 0.3%). Sizes are |Z| with Z the
variance-matched sum of eight uniform 16-bit draws."""
import numpy as np
import pytest
from scipy import stats

import oracle

P33 = int(0.33 * 2 ** 32)
P03 = int(0.003 * 2 ** 32)


def cfg(**kw):
    base = dict(width=64, height=64, pop=32, sites=32, k=5, selection=0, p32=P33,
                migration=0, seed=77, run_id=3, law=1, p_ben32=0)
    base.update(kw)
    return base


def one_generation(c):
    run = oracle.OracleRun(c)
    run.step(1)
    return run.population()[0]


def test_purifying_rate_sign_and_moments():
    f = one_generation(cfg())
    n = f.size
    neg = f[f < 0]
    assert (f > 0).sum() == 0
    p = P33 / 2 ** 32
    assert abs(neg.size / n - p) < 5 * np.sqrt(p * (1 - p) / n)
    z = -neg.astype(np.float64)
    m2, m4 = (z ** 2).mean(), (z ** 4).mean()
    # Irwin-Hall(8) standardised: variance 1, kurtosis 3 - 6/(5*8) = 2.85
    assert abs(m2 - 1.0) < 5 * np.sqrt((2.85 - 1.0) / z.size)
    assert abs(m4 - 2.85) < 0.3
    assert z.max() < 2 * np.sqrt(6.0)
    # indistinguishable from a half-normal at this sample size
    assert stats.kstest(z, stats.halfnorm.cdf).pvalue > 1e-4


def test_adaptive_rates():
    p_ben = 0.3
    f = one_generation(cfg(p_ben32=int(p_ben * 2 ** 32)))
    n = f.size
    for frac, p in (((f > 0).mean(), p_ben), ((f < 0).mean(), P33 / 2 ** 32)):
        assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / n)
    assert stats.kstest(f[f > 0].astype(np.float64), stats.halfnorm.cdf).pvalue > 1e-4


def test_no_mutation_special_case_matches_discrete_law():
    a = oracle.OracleRun(cfg(width=8, height=8, law=1, p32=0, p_ben32=0, selection=1, migration=1))
    b = oracle.OracleRun(cfg(width=8, height=8, law=0, p32=0, selection=1, migration=1))
    a.step(50)
    b.step(50)
    for x, y in zip(a.population(), b.population()):
        assert np.array_equal(x, y)


def test_treatment_lineages_move_by_bounded_sizes():
    c = cfg(width=6, height=6, pop=16, p_ben32=P03 * 50, selection=1, migration=1)
    run = oracle.OracleRun(c, lineage=True)
    hist = [run.population()]
    for _ in range(60):
        run.step(1)
        hist.append(run.population())
    sizes = []
    for a in range(0, run.agents, 3):
        gens, isl, slt = run.ancestry(a)
        for (gc, ic, sc), (gp, ip, sp) in zip(zip(gens[:-1], isl[:-1], slt[:-1]),
                                              zip(gens[1:], isl[1:], slt[1:])):
            fc = hist[gc][0][ic * 16 + sc]
            fp = hist[gp][0][ip * 16 + sp]
            assert hist[gc][1][ic * 16 + sc] == hist[gp][1][ip * 16 + sp] + 1
            sizes.append(abs(float(fc) - float(fp)))
    sizes = np.array(sizes)
    assert sizes.max() < 2 * np.sqrt(6.0) + 1e-3
    assert (sizes > 0).mean() > 0.2


@pytest.mark.parametrize("bad", [dict(law=2), dict(p32=2 ** 32 - 10, p_ben32=100)])
def test_treatment_validation(bad):
    assert not oracle.validate(cfg(**bad))
