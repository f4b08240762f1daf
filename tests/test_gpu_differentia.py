"""GPU parity for the surface variants: wider differentia (b = 2, 4, 8 bits per
site at the surface's 32- or 64-bit footprint), the tilted
(recency-proportional) policy and the hybrid (steady + tilted halves) policy. Surfaces, T, fitness and generation equal the
CPU oracle bit for bit across shapes, launch forms, edge shapes and the
asynchronous schedule (batches refuse them); the all-pairs MRCA intervals
equal the oracle's."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import (ASYNC_UNPACED, FORM_RESIDENT, FORM_STREAMING, GABatch, GAError,
                                  GARun, phylo)
from paper_2405_03605_amd.workloads import run_config

pytestmark = pytest.mark.gpu

SHAPES = [(32, 2), (16, 4), (8, 8), (16, 2), (8, 4), (4, 8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("sites,bits", SHAPES)
@pytest.mark.parametrize("form", [FORM_STREAMING, FORM_RESIDENT])
def test_wide_parity(sites, bits, form):
    cfg = run_config(width=9, height=7, pop=16, sites=sites, dbits=bits, k=3)
    say(f"S={sites} b={bits} form {form}")
    run = GARun(cfg)
    run.set_launch(0, 0, form)
    for n in (1, 60, 239):
        run.step(n)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 300), f"S={sites} b={bits} form {form}")


@pytest.mark.parametrize("kw", [dict(pop=1, width=20, height=5), dict(pop=64, width=5, height=4),
                                dict(pop=8, width=1, height=11, selection=0),
                                dict(pop=32, width=40, height=30, law=1, p_ben32=12884902,
                                     p32=1417339207, k=5),
                                dict(pop=32, width=12, height=12, model=2)])
def test_wide_edges(kw):
    cfg = run_config(sites=8, dbits=8, **kw)
    run = GARun(cfg)
    run.step(400)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 400), f"S=8 b=8 {kw}")


def test_wide_async_and_batch_refusal():
    run = GARun(run_config(width=7, height=5, pop=8, sites=16, dbits=4))
    batch = GABatch()
    with pytest.raises(GAError):
        batch.add(run, 10)
    batch.close()
    run.close()
    cfg = run_config(width=17, height=9, pop=16, sites=16, dbits=4, schedule=1)
    run = GARun(cfg)
    run.set_launch(4)
    run.set_async(1, ASYNC_UNPACED, 2)
    run.step(120)
    ref = oracle.OracleRun({k: v for k, v in cfg.items() if k != "schedule"})
    ref.step_async(120, 4, 2)
    assert_same_state(run.read(), ref, "async skewed S=16 b=4")
    run.close()


@pytest.mark.parametrize("sites,bits", SHAPES)
def test_wide_mrca_matrix(sites, bits):
    cfg = run_config(width=24, height=16, pop=16, sites=sites, dbits=bits, seed=77)
    run = GARun(cfg)
    run.step(700)
    ids, T, D = run.extract()
    run.close()
    rng = np.random.default_rng(sites * bits)
    T2 = np.concatenate([T, rng.integers(0, 2 ** 31, 40).astype(np.uint32), [0, 1, sites - 1, sites]
                         ]).astype(np.uint32)
    D2 = np.concatenate([D, rng.integers(0, 2 ** 32, (44, D.shape[1]), dtype=np.uint64)
                         .astype(np.uint32)])
    for kc in (1, 3):
        L, U = phylo.mrca_matrix(T2, D2, sites, kc, bits=bits)
        L0, U0 = oracle.mrca_interval_matrix(T2, D2, sites, kc, bits)
        assert np.array_equal(U, U0) and np.array_equal(L, L0), (sites, bits, kc)


TILTED = [(32, 1), (64, 1), (32, 2)]


@pytest.mark.parametrize("sites,bits", TILTED)
@pytest.mark.parametrize("form", [FORM_STREAMING, FORM_RESIDENT])
def test_tilted_parity(sites, bits, form):
    cfg = run_config(width=9, height=7, pop=16, sites=sites, dbits=bits, policy=1, k=3)
    say(f"tilted S={sites} b={bits} form {form}")
    run = GARun(cfg)
    run.set_launch(0, 0, form)
    for n in (1, 200, 599):
        run.step(n)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 800), f"tilted S={sites} b={bits} form {form}")


def test_tilted_mid_run_async_and_strings():
    cfg = run_config(width=96, height=64, pop=32, sites=64, policy=1, model=1)
    run = GARun(cfg)
    run.step(500)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 500), "tilted 96x64x32 OneMax")
    cfg = run_config(width=17, height=9, pop=16, sites=32, policy=1, schedule=1)
    run = GARun(cfg)
    run.set_launch(4)
    run.set_async(1, ASYNC_UNPACED, 3)
    run.step(150)
    ref = oracle.OracleRun({k: v for k, v in cfg.items() if k != "schedule"})
    ref.step_async(150, 4, 3)
    assert_same_state(run.read(), ref, "async skewed tilted")
    run.close()
    with pytest.raises(GAError):
        GABatch().add(GARun(run_config(policy=1)), 5)


@pytest.mark.parametrize("sites,bits", TILTED)
def test_tilted_mrca_matrix(sites, bits):
    cfg = run_config(width=24, height=16, pop=16, sites=sites, dbits=bits, policy=1, seed=79)
    run = GARun(cfg)
    run.step(1500)
    ids, T, D = run.extract()
    run.close()
    rng = np.random.default_rng(sites + bits)
    extra = np.array([0, 1, 2, 3, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1, 2 ** 32 - 1], np.uint32)
    T2 = np.concatenate([T, rng.integers(0, 2 ** 32, 40, dtype=np.uint64).astype(np.uint32),
                         extra]).astype(np.uint32)
    D2 = np.concatenate([D, rng.integers(0, 2 ** 32, (48, D.shape[1]), dtype=np.uint64)
                         .astype(np.uint32)])
    # a copy of each run surface at an older count shares ranks with it
    T2 = np.concatenate([T2, (T // 3).astype(np.uint32)])
    D2 = np.concatenate([D2, D])
    for kc in (1, 4):
        L, U = phylo.mrca_matrix(T2, D2, sites, kc, bits=bits, policy=1)
        L0, U0 = oracle.mrca_interval_matrix(T2, D2, sites, kc, bits, policy=1)
        assert np.array_equal(U, U0) and np.array_equal(L, L0), (sites, bits, kc)


@pytest.mark.parametrize("form", [FORM_STREAMING, FORM_RESIDENT])
@pytest.mark.parametrize("kw", [dict(width=9, height=7, pop=16, k=3),
                                dict(width=5, height=3, pop=1), dict(width=4, height=4, pop=64)])
def test_hybrid_parity(form, kw):
    cfg = run_config(sites=64, policy=2, **kw)
    run = GARun(cfg)
    run.set_launch(0, 0, form)
    for n in (1, 200, 799):
        run.step(n)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 1000), f"hybrid {kw} form {form}")


def test_hybrid_async_and_mrca_matrix():
    cfg = run_config(width=17, height=9, pop=16, sites=64, policy=2, schedule=1)
    run = GARun(cfg)
    run.set_launch(4)
    run.set_async(1, ASYNC_UNPACED, 2)
    run.step(300)
    ref = oracle.OracleRun({k: v for k, v in cfg.items() if k != "schedule"})
    ref.step_async(300, 4, 2)
    assert_same_state(run.read(), ref, "async skewed hybrid")
    run.close()
    cfg = run_config(width=24, height=16, pop=16, sites=64, policy=2, seed=81)
    run = GARun(cfg)
    run.step(1500)
    ids, T, D = run.extract()
    run.close()
    rng = np.random.default_rng(64)
    extra = np.array([0, 1, 2, 3, 64, 65, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1], np.uint32)
    T2 = np.concatenate([T, rng.integers(0, 2 ** 32, 40, dtype=np.uint64).astype(np.uint32),
                         extra, (T // 3).astype(np.uint32)]).astype(np.uint32)
    D2 = np.concatenate([D, rng.integers(0, 2 ** 32, (49, 2), dtype=np.uint64).astype(np.uint32),
                         D])
    for kc in (1, 4):
        L, U = phylo.mrca_matrix(T2, D2, 64, kc, policy=2)
        L0, U0 = oracle.mrca_interval_matrix(T2, D2, 64, kc, 1, policy=2)
        assert np.array_equal(U, U0) and np.array_equal(L, L0), kc


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130])
@pytest.mark.parametrize("sites,bits,policy", [(32, 1, 1), (64, 1, 1), (32, 2, 1), (64, 1, 2)])
def test_tilted_and_hybrid_mrca_block_edges(n, sites, bits, policy):
    # the tiled kernels take 64 x 64 blocks on and above the diagonal and
    # mirror them: one partial block, exactly one block, one block and a
    # ragged row/column, two blocks and a ragged one; counters near each other
    # (many common ranks) and far apart
    say(f"MRCA blocks n={n} S={sites} b={bits} policy={policy}")
    rng = np.random.default_rng(1000 * n + 10 * sites + bits + policy)
    base = rng.integers(1, 2 ** 20, n, dtype=np.int64)
    base[::3] = rng.integers(0, 2 ** 32, len(base[::3]), dtype=np.uint64).astype(np.int64)
    T = base.astype(np.uint32)
    words = sites * bits // 32
    D = rng.integers(0, 2 ** 32, (n, words), dtype=np.uint64).astype(np.uint32)
    D[1::2] = D[0:n - 1:2]      # identical pairs of surfaces
    for kc in (1, 5):
        L, U = phylo.mrca_matrix(T, D, sites, kc, bits=bits, policy=policy)
        L0, U0 = oracle.mrca_interval_matrix(T, D, sites, kc, bits, policy=policy)
        assert np.array_equal(U, U0) and np.array_equal(L, L0), (n, sites, bits, policy, kc)
