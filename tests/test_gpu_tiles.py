"""GPU parity of the LDS-resident tile form: populations held in LDS across
generations, one workgroup per tile, edge emissions exchanged through the HBM
outbox with per-tile progress words. Every result is compared with the oracle
bit for bit (fitness bits, T, surfaces, outbox, generation), across launches
(steps split so generations cross launch boundaries), forced tile shapes
(ragged tiles, one-wide and one-high tiles, two tiles across a torus side),
island sizes, surface sizes, the 256x256x32 workloads at full size and a resume
through host state."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import FORM_RESIDENT, FORM_STREAMING, GAError, GARun
from paper_2405_03605_amd.workloads import MID, MID_NEUTRAL, TINY, run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _tiled(cfg, tiles=None, steps=(1, 100, 129)):
    run = GARun(cfg)
    run.set_launch(form=FORM_RESIDENT)
    if tiles:
        run.set_tiles(*tiles)
    shape = run.tiles()
    assert shape[2] >= 1, "resident form did not choose tiles"
    for n in steps:
        run.step(n)
    got = run.read()
    run.close()
    return got, shape


def test_mid_chooses_one_tile_per_cu():
    run = GARun(MID)
    assert run.tiles() == (16, 16, 256)
    run.set_launch(form=FORM_STREAMING)
    assert run.tiles() == (0, 0, 0)
    run.close()


SHAPES = [
    # (config, tile shape): ragged tiles, strips, two tiles across a side
    (dict(width=23, height=17, pop=32, sites=32, k=3, seed=3), (4, 4)),
    (dict(width=23, height=17, pop=32, sites=32, k=3, seed=3), (23, 1)),
    (dict(width=23, height=17, pop=32, sites=32, k=3, seed=3), (1, 17)),
    (dict(width=23, height=17, pop=32, sites=32, k=3, seed=3), (12, 9)),
    (dict(width=23, height=17, pop=32, sites=32, k=3, seed=3), (5, 3)),
    (dict(width=20, height=12, pop=8, sites=64, k=2, seed=11), (7, 5)),
    (dict(width=20, height=12, pop=1, sites=32, k=1, seed=12), (3, 2)),
    (dict(width=9, height=8, pop=64, sites=64, k=8, seed=13), (2, 3)),
    (dict(width=9, height=8, pop=64, sites=32, selection=0, seed=14), (9, 4)),
    (dict(width=16, height=16, pop=16, sites=64, k=5, migration=0, seed=15), (4, 8)),
    (dict(width=16, height=16, pop=4, sites=32, k=2, p32=0xFFFFFFFF, seed=16), (8, 16)),
    (dict(width=1, height=40, pop=32, sites=32, k=2, seed=17), (1, 7)),
    (dict(width=40, height=1, pop=32, sites=64, k=2, seed=18), (13, 1)),
    (dict(width=2, height=2, pop=32, sites=64, k=2, seed=19), (1, 1)),
    (dict(width=7, height=5, pop=32, sites=32, k=5, law=1, p32=1417339207, p_ben32=12884901,
          seed=20), (3, 3)),
]


@pytest.mark.parametrize("edge,tiles", SHAPES,
                         ids=lambda e: "-".join(f"{k}{v}" for k, v in e.items())
                         if isinstance(e, dict) else f"t{e[0]}x{e[1]}")
def test_forced_tiles_match_oracle(edge, tiles):
    cfg = run_config(**edge)
    say(f"tiles {tiles} on {cfg}")
    got, shape = _tiled(cfg, tiles)
    assert shape[:2] == tiles
    assert_same_state(got, oracle_after(cfg, 230), f"tiles {tiles} {edge}")


def test_tiny_resident_1000_generations():
    say("tiny 8x8x32 S=64, 1000 generations, resident tiles")
    got, _ = _tiled(TINY, steps=(1000,))
    assert_same_state(got, oracle_after(TINY, 1000), "tiny resident")


def test_tiny_split_over_four_tiles():
    say("tiny 8x8x32 S=64 on four 4x4 tiles, 1000 generations")
    got, shape = _tiled(TINY, (4, 4), steps=(1, 499, 500))
    assert shape == (4, 4, 4)
    assert_same_state(got, oracle_after(TINY, 1000), "tiny on 4 tiles")


@pytest.mark.parametrize("cfg,name", [(MID, "mid selection"), (MID_NEUTRAL, "mid neutral")])
def test_mid_full_size_across_launches(cfg, name):
    # 2,097,152 agents on 256 tiles of 16x16 islands; 250 generations in three
    # launches (a launch boundary after generation 1 and 100)
    say(f"{name}: 256x256x32 resident tiles, 250 generations")
    got, shape = _tiled(cfg, steps=(1, 99, 150))
    assert shape == (16, 16, 256)
    assert_same_state(got, oracle_after(cfg, 250), f"{name} resident")


def test_mid_resume_through_host_state():
    # streaming to 120, resident from the host copy to 260, against the oracle
    a = GARun(MID)
    a.set_launch(form=FORM_STREAMING)
    a.step(120)
    snap = a.read()
    a.close()
    b = GARun(MID)
    b.write(snap["f"], snap["T"], snap["D"], snap["outbox"], snap["generation"])
    assert b.tiles()[2] == 256
    b.step(140)
    ref = oracle.OracleRun(MID)
    ref.set_population(snap["f"], snap["T"], snap["D"])
    ob = snap["outbox"]
    ref.set_outbox(ob["valid"], ob["dir"], ob["f"], ob["T"], ob["D"])
    ref.set_generation(120)
    ref.step(140)
    assert_same_state(b.read(), ref, "mid resumed resident")
    b.close()


def test_generation_counter_high_word_resident():
    cfg = run_config(width=6, height=5, pop=8, sites=32, seed=5)
    ref = oracle.OracleRun(cfg)
    ref.step(10)
    f, T, D = ref.population()
    ob = ref.outbox()
    start = (1 << 32) - 3
    ref.set_generation(start)
    run = GARun(cfg)
    run.set_launch(form=FORM_RESIDENT)
    run.set_tiles(2, 5)
    run.write(f, T, D, ob, start)
    run.step(7)
    ref.step(7)
    assert_same_state(run.read(), ref, "high word resident")


def test_streaming_and_resident_alternate():
    cfg = run_config(width=30, height=20, pop=16, sites=32, k=4, seed=23)
    run = GARun(cfg)
    for i, n in enumerate((37, 63, 1, 80, 19)):
        run.set_launch(form=FORM_RESIDENT if i % 2 == 0 else FORM_STREAMING)
        if i % 2 == 0:
            run.set_tiles(*((7, 6) if i == 0 else (30, 4)))
        run.step(n)
    assert_same_state(run.read(), oracle_after(cfg, 200), "alternating forms")


def test_tile_errors():
    from paper_2405_03605_amd.workloads import PAPER
    run = GARun(run_config(width=64, height=64, pop=64, sites=64))
    with pytest.raises(GAError):
        run.set_tiles(4, 0)                  # one side without the other
    with pytest.raises(GAError):
        run.set_tiles(64, 64)                # 262,144 agents: far more than a CU's LDS
    run.set_tiles(8, 8)                      # a failed call kept the run usable
    assert run.tiles() == (8, 8, 64)
    run.close()
    big = GARun(PAPER)                       # 16.8M agents: no tiling fits 256 CUs
    with pytest.raises(GAError):
        big.set_launch(form=FORM_RESIDENT)
    assert big.tiles() == (0, 0, 0)
    big.close()
    asy = GARun(run_config(width=8, height=8, schedule=1))
    with pytest.raises(GAError):
        asy.set_tiles(4, 4)
    asy.close()
