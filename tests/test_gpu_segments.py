"""Segment parity at depth on the full-size workloads: the GPU runs to a
generation t0 near the end of the workload's length, its whole state
(population, pending outbox, generation counter) is loaded into the CPU
oracle, both sides step the same number of generations, and every field is
compared bit for bit.

The RNG is counter-based (keyed by seed, run, island, generation and slot), so
a segment from any t0 is the same computation the oracle would make after a
full-length run from generation 0; a segment near the end exercises the
deepest surface epochs the workload reaches (T about 1e5 on the 32-site
surface: epoch 12, 25 retained ranks) in the launch configuration the
benchmark times."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, say
from paper_2405_03605_amd import FORM_STREAMING, GARun
from paper_2405_03605_amd.workloads import (MID, MID_GENS, MID_NEUTRAL, PAPER, PAPER_GENS)

pytestmark = pytest.mark.gpu

SEGMENT = 100


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _check_invariants(snap, t0, what):
    # every counter lags the generation (migration copies lag); fitness moves
    # by multiples of 1/2 under the discrete law, so it stays on that grid
    assert snap["generation"] == t0
    assert int(snap["T"].max()) <= t0, f"{what}: T above the generation"
    twice = snap["f"].astype(np.float64) * 2.0
    assert np.array_equal(twice, np.round(twice)), f"{what}: fitness off the half-integer grid"


def _segment(cfg, t0, what, form=0):
    run = GARun(cfg)
    if form:
        run.set_launch(form=form)
    say(f"{what}: GPU to generation {t0}")
    run.step(t0)
    snap = run.read()
    _check_invariants(snap, t0, what)
    say(f"{what}: T spans {int(snap['T'].min())}..{int(snap['T'].max())}; oracle from GPU state")
    ref = oracle.OracleRun(cfg)
    ref.set_population(snap["f"], snap["T"], snap["D"])
    ob = snap["outbox"]
    ref.set_outbox(ob["valid"], ob["dir"], ob["f"], ob["T"], ob["D"])
    ref.set_generation(t0)
    del snap
    run.step(SEGMENT)
    ref.step(SEGMENT)
    say(f"{what}: comparing generation {t0 + SEGMENT}")
    assert_same_state(run.read(), ref, what)
    run.close()


def test_paper_scale_segment_at_depth():
    # 16,777,216 agents; the last 100 of the workload's 100,000 generations
    _segment(PAPER, PAPER_GENS - SEGMENT, "paper scale 1024x512x32")


@pytest.mark.parametrize("cfg,name", [(MID, "mid selection"), (MID_NEUTRAL, "mid neutral")])
def test_mid_segment_at_depth(cfg, name):
    # 2,097,152 agents; the last 100 of the workload's 10,000 generations
    _segment(cfg, MID_GENS - SEGMENT, f"{name} 256x256x32")


@pytest.mark.parametrize("cfg,name", [(MID, "mid selection"), (MID_NEUTRAL, "mid neutral")])
def test_mid_segment_at_depth_streaming(cfg, name):
    # the per-generation launch form on the same workload, whatever the default
    _segment(cfg, MID_GENS - SEGMENT, f"{name} 256x256x32 streaming", form=FORM_STREAMING)
