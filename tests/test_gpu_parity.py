"""GPU parity: the HIP generation step against the CPU oracle, bit for bit, on
the same seeded configurations (fitness bits, T, surfaces, outboxes and the
generation counter), across launch forms, launch shapes, edge configurations
and the full-size workloads."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import FORM_RESIDENT, FORM_STREAMING, GARun
from paper_2405_03605_amd.workloads import MID, MID_NEUTRAL, PAPER, TINY, run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _gpu_run(cfg, gens, form=0, ipw=0, wpg=0, graph_block=None, steps=None):
    run = GARun(cfg)
    if form or ipw or wpg:
        run.set_launch(ipw, wpg, form)
    if graph_block is not None:
        run.set_graph_block(graph_block)
    for n in (steps or [gens]):
        run.step(n)
    got = run.read()
    run.close()
    return got


@pytest.mark.parametrize("form", [0, FORM_STREAMING, FORM_RESIDENT])
def test_tiny_full_run(form):
    say(f"tiny 8x8x32 S=64, 1000 generations, form {form}")
    got = _gpu_run(TINY, 1000, form=form)
    assert_same_state(got, oracle_after(TINY, 1000), f"tiny form {form}")


EDGE = [
    dict(pop=1, width=5, height=3),
    dict(pop=2, width=7, height=1),
    dict(pop=4, width=1, height=9, sites=32),
    dict(pop=8, width=2, height=2, k=8),
    dict(pop=16, width=3, height=5, k=5, sites=32),
    dict(pop=64, width=4, height=3, k=4),
    dict(pop=64, width=9, height=7, sites=32, selection=0),
    dict(pop=32, width=6, height=6, k=1),
    dict(pop=32, width=6, height=6, migration=0),
    dict(pop=32, width=6, height=6, p32=0),
    dict(pop=32, width=6, height=6, p32=0xFFFFFFFF),
    dict(pop=8, width=33, height=3, k=3, seed=12345, run_id=77),
    dict(pop=32, width=1, height=1),
    dict(pop=32, width=7, height=5, sites=32, k=5, law=1, p32=1417339207, p_ben32=0),
    dict(pop=32, width=7, height=5, sites=32, k=5, law=1, p32=1417339207, p_ben32=12884901),
    dict(pop=16, width=5, height=9, sites=64, k=3, law=1, p32=1417339207, p_ben32=1288490188),
    dict(pop=8, width=9, height=4, sites=32, k=8, law=1, p32=0xFFFFFFFF - 1288490188, p_ben32=1288490188),
]


@pytest.mark.parametrize("edge", EDGE, ids=lambda e: "-".join(f"{k}{v}" for k, v in e.items()))
@pytest.mark.parametrize("form", [FORM_STREAMING, FORM_RESIDENT])
def test_edge_configurations(edge, form):
    cfg = run_config(**edge)
    say(f"edge {cfg} form {form}")
    got = _gpu_run(cfg, 230, form=form, steps=[1, 100, 129])
    assert_same_state(got, oracle_after(cfg, 230), f"edge {edge} form {form}")


@pytest.mark.parametrize("ipw,wpg,gb", [(2, 1, 0), (8, 3, 7), (32, 16, 100), (64, 4, 50), (64, 1, 0)])
def test_launch_shapes_give_identical_bits(ipw, wpg, gb):
    cfg = run_config(width=23, height=17, pop=32, sites=32, k=3, seed=3)
    say(f"launch shape ipw {ipw} wpg {wpg} graph block {gb}")
    got = _gpu_run(cfg, 260, form=FORM_STREAMING, ipw=ipw, wpg=wpg, graph_block=gb,
                   steps=[60, 200])
    assert_same_state(got, oracle_after(cfg, 260), f"shape {ipw}/{wpg}/{gb}")


def test_ragged_tail_over_many_waves():
    # 1,601 islands of 16 agents: 25 full 64-island chunks plus a 1-island tail
    cfg = run_config(width=1601, height=1, pop=16, sites=64, k=2, seed=9)
    say("ragged tail 1601x1x16")
    got = _gpu_run(cfg, 150, form=FORM_STREAMING)
    assert_same_state(got, oracle_after(cfg, 150), "ragged")


@pytest.mark.parametrize("cfg,name", [(MID, "mid selection"), (MID_NEUTRAL, "mid neutral")])
def test_mid_full_size_prefix(cfg, name):
    gens = 12
    say(f"{name}: 256x256x32, {gens} generations")
    got = _gpu_run(cfg, gens, steps=[5, 7])
    assert_same_state(got, oracle_after(cfg, gens), name)


def test_paper_scale_prefix_in_bench_configuration():
    # 16.8M agents; the benchmark's launch (streaming, graph blocks) for 3 generations
    gens = 3
    say("paper scale 1024x512x32, 3 generations")
    got = _gpu_run(PAPER, gens)
    assert_same_state(got, oracle_after(PAPER, gens), "paper scale")


def test_resume_through_host_state():
    cfg = run_config(width=10, height=7, pop=16, sites=64, k=4, seed=21)
    a = GARun(cfg)
    a.set_launch(form=FORM_STREAMING)
    a.step(120)
    snap = a.read()
    b = GARun(cfg)
    b.set_launch(form=FORM_STREAMING)
    b.write(snap["f"], snap["T"], snap["D"], snap["outbox"], snap["generation"])
    b.step(90)
    a.step(90)
    ga_, gb_ = a.read(), b.read()
    for key in ("f", "T", "D"):
        assert np.array_equal(ga_[key], gb_[key])
    assert_same_state(gb_, oracle_after(cfg, 210), "resumed")


def test_generation_counter_high_word():
    # generations cross 2^32: the counter's high word feeds the RNG
    cfg = run_config(width=6, height=5, pop=8, sites=32, seed=5)
    ref = oracle.OracleRun(cfg)
    ref.step(10)
    f, T, D = ref.population()
    ob = ref.outbox()
    start = (1 << 32) - 3
    ref.set_generation(start)
    run = GARun(cfg)
    run.set_launch(form=FORM_STREAMING)
    run.write(f, T, D, ob, start)
    run.step(7)
    ref.step(7)
    assert_same_state(run.read(), ref, "high word")


@pytest.mark.parametrize("sites", [32, 64])
def test_deposits_at_large_T(sites):
    # arbitrary T up to 2^31 and random surfaces: exercises every epoch of the
    # surface policy, including the multi-step site walk
    cfg = run_config(width=16, height=16, pop=32, sites=sites, seed=8)
    rng = np.random.default_rng(sites)
    A = 16 * 16 * 32
    T = rng.integers(0, 1 << 31, size=A, dtype=np.uint64).astype(np.uint32)
    T[::7] = (T[::7] >> np.uint32(12)) << np.uint32(12)   # many written deposits
    T[::11] = rng.integers(0, 300, size=T[::11].size)
    D = rng.integers(0, 1 << 32, size=(A, sites // 32), dtype=np.uint64).astype(np.uint32)
    f = (rng.integers(-40, 40, size=A) * 0.5).astype(np.float32)
    ref = oracle.OracleRun(cfg)
    ref.set_population(f, T, D)
    run = GARun(cfg)
    run.set_launch(form=FORM_STREAMING)
    run.write(f, T, D, None, 0)
    for _ in range(3):
        run.step(1)
        ref.step(1)
        assert_same_state(run.read(), ref, f"large T S={sites}")


def test_extract_surfaces():
    cfg = run_config(width=20, height=12, pop=16, sites=64, seed=4)
    run = GARun(cfg)
    run.step(77)
    ref = oracle_after(cfg, 77)
    f, T, D = ref.population()
    ids, Tx, Dx = run.extract()
    assert np.array_equal(ids, ref.sample_one_per_island())
    assert np.array_equal(Tx, T[ids.astype(np.int64)])
    assert np.array_equal(Dx, D[ids.astype(np.int64)])
    pick = np.random.default_rng(1).integers(0, run.agents, size=1000)
    ids2, T2, D2 = run.extract(pick)
    assert np.array_equal(ids2, pick.astype(np.uint64))
    assert np.array_equal(T2, T[pick])
    assert np.array_equal(D2, D[pick])
