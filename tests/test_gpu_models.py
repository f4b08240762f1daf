"""GPU parity for the genome models with a string (OneMax and Trap-4 on a
64-bit string; Sec. 2 Methods: any fixed-length genome through initialize,
mutate and evaluate): strings, fitness, T, surfaces and generation equal the
CPU oracle bit for bit, in both launch forms, several launch shapes, edge
shapes, both schedules and across a resume."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import (ASYNC_UNPACED, FORM_RESIDENT, FORM_STREAMING, GABatch, GAError,
                                  GARun, _lib)
from paper_2405_03605_amd.workloads import run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _oracle_cfg(cfg):
    return {k: v for k, v in cfg.items() if k != "schedule"}


@pytest.mark.parametrize("model", [1, 2])
def test_founders(model):
    cfg = run_config(width=13, height=7, pop=16, model=model)
    run = GARun(cfg)
    got = run.read()
    run.close()
    assert_same_state(got, oracle.OracleRun(cfg), f"founders model {model}")


SHAPES = [
    dict(),
    dict(width=5, height=3, pop=1, sites=32),
    dict(width=7, height=1, pop=2, k=5),
    dict(width=1, height=9, pop=4, sites=32, selection=0),
    dict(width=9, height=7, pop=64, k=8),
    dict(width=33, height=3, pop=8, sites=32, k=3, seed=12345, run_id=77),
    dict(width=6, height=6, pop=32, migration=0),
    dict(width=6, height=6, pop=32, p32=0xFFFFFFFF),
]


@pytest.mark.parametrize("model", [1, 2])
@pytest.mark.parametrize("kw", SHAPES)
@pytest.mark.parametrize("form", [FORM_STREAMING, FORM_RESIDENT])
def test_model_parity(model, kw, form):
    cfg = run_config(model=model, **kw)
    say(f"model {model} {kw} form {form}")
    run = GARun(cfg)
    run.set_launch(0, 0, form)
    for n in (1, 100, 129):
        run.step(n)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 230), f"model {model} {kw} form {form}")


def test_launch_shape_beyond_lds_is_rejected():
    # 64 islands per wavefront x 16 wavefronts of 32-byte entries: 164 KiB
    run = GARun(run_config(width=40, height=24, model=2))
    with pytest.raises(GAError):
        run.set_launch(64, 16)
    run.close()


@pytest.mark.parametrize("ipw,wpg", [(2, 1), (16, 4), (64, 8)])
def test_launch_shapes_agree(ipw, wpg):
    cfg = run_config(width=40, height=24, pop=32, sites=64, k=5, model=2)
    run = GARun(cfg)
    run.set_launch(ipw, wpg, FORM_STREAMING)
    run.step(300)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(cfg, 300), f"trap-4 ipw {ipw} wpg {wpg}")


@pytest.mark.parametrize("model", [1, 2])
def test_mid_size_run(model):
    cfg = run_config(width=128, height=64, pop=32, sites=32, k=4, model=model)
    say(f"model {model} 128x64x32, 400 generations")
    run = GARun(cfg)
    run.step(400)
    got = run.read()
    run.close()
    ref = oracle_after(cfg, 400)
    assert_same_state(got, ref, f"model {model} 128x64x32")
    if model == 1:
        assert got["f"].mean() > 40          # selection climbs OneMax


@pytest.mark.parametrize("model", [1, 2])
def test_async_schedules(model):
    # one wavefront with a skew: the oracle's skewed interleaving; paced on the
    # whole GPU: the synchronous schedule
    cfg = run_config(width=17, height=9, pop=16, model=model, schedule=1)
    run = GARun(cfg)
    run.set_launch(4)
    run.set_async(1, ASYNC_UNPACED, 3)
    ref = oracle.OracleRun(_oracle_cfg(cfg))
    for n in (1, 60):
        run.step(n)
        ref.step_async(n, 4, 3)
    assert_same_state(run.read(), ref, f"model {model} async skew 3")
    run.close()
    cfg = run_config(width=64, height=48, pop=32, sites=32, model=model, schedule=1)
    run = GARun(cfg)
    run.step(250)
    got = run.read()
    assert run.async_waits() == 0
    run.close()
    assert_same_state(got, oracle_after(_oracle_cfg(cfg), 250), f"model {model} async paced")


def test_resume_with_strings():
    cfg = run_config(width=10, height=6, pop=16, model=1, k=3)
    run = GARun(cfg)
    run.step(90)
    mid = run.read()
    ref = oracle_after(cfg, 90)
    assert_same_state(mid, ref, "onemax at 90")
    # a fresh run written from the state continues identically (the pending
    # outbox is not exchanged, so both sides drop it)
    run2 = GARun(cfg)
    run2.write(mid["f"], mid["T"], mid["D"], generation=90)
    run2.write_strings(mid["P"])
    run2.step(70)
    ref.set_outbox(np.zeros(ref.islands, np.uint8), np.zeros(ref.islands, np.uint8),
                   np.zeros(ref.islands, np.float32), np.zeros(ref.islands, np.uint32),
                   np.zeros((ref.islands, ref.words), np.uint32))
    # the fresh run has no outbox pending; the oracle's is cleared to match
    ref.step(70)
    assert_same_state(run2.read(), ref, "onemax resumed at 160")
    run.close()
    run2.close()


def test_string_model_errors():
    run = GARun(run_config(width=8, height=8, model=2))
    lib = _lib.load()
    box = (_lib.OutboxEntry * run.islands)()
    assert lib.ga_read_population(run.handle, None, None, None,
                                  ctypes.cast(box, ctypes.c_void_p), None) == _lib.GA_EINVAL
    batch = GABatch()
    with pytest.raises(GAError):
        batch.add(run, 10)
    batch.close()
    plain = GARun(run_config(width=8, height=8))
    with pytest.raises(GAError):
        plain.read_strings()
    plain.close()
    run.close()
