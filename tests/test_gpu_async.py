"""GPU checks of the asynchronous schedule (Sec. 2 Methods: per-neighbour
buffers consumed and refilled without a global step).

Bit for bit against the oracle: the one-wavefront launch (the sequential
interleaving of chunks) for many shapes and chunk sizes, resume, and the cases
that reduce to the synchronous schedule (migration off; every island in one
chunk). The free-running launch is not reproducible; it is checked for
invariants every interleaving keeps and, statistically, against the
synchronous schedule and a no-migration control."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import ASYNC_UNPACED, GABatch, GARun, GAError
from paper_2405_03605_amd import async_stats
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


def _async(**kw):
    return run_config(schedule=1, **kw)


def _oracle_cfg(cfg):
    return {k: v for k, v in cfg.items() if k != "schedule"}


ONE_WAVE = [
    (dict(), 2, 0),
    (dict(), 16, 3),
    (dict(), 64, 0),
    (dict(width=5, height=3, pop=8, sites=32, k=5), 8, 1),
    (dict(width=13, height=11, pop=8, sites=32, k=5), 16, 2),
    (dict(width=1, height=9, pop=4, selection=0), 16, 0),
    (dict(width=33, height=1, pop=16, law=1, p_ben32=12884902, p32=1417339207, k=5), 4, 5),
    (dict(width=20, height=10, pop=1, sites=32), 64, 1),
    (dict(width=9, height=7, pop=64, k=8), 1, 7),
    (dict(width=9, height=7, pop=64, k=8, sites=32), 3, 2),
    (dict(width=2, height=2, pop=32, p32=0xFFFFFFFF), 2, 1),
    (dict(width=17, height=9, pop=32, seed=777, run_id=5), 6, 4),
]


@pytest.mark.parametrize("kw,ipw,skew", ONE_WAVE)
def test_one_wavefront_is_the_oracle_interleaving(kw, ipw, skew):
    # One wavefront runs the chunks in order; with a skew it runs the
    # oracle's skewed interleaving (genomes late or overwritten), without one
    # (paced, as by default) the synchronous schedule.
    cfg = _async(**kw)
    say(f"async one wavefront {kw} ipw {ipw} skew {skew}")
    run = GARun(cfg)
    run.set_launch(ipw)
    run.set_async(1, ASYNC_UNPACED if skew else 0, skew)
    ref = oracle.OracleRun(_oracle_cfg(cfg))
    for n in (1, 40, 59):
        run.step(n)
        ref.step_async(n, ipw, skew)
    got = run.read()
    assert run.async_waits() == 0
    run.close()
    assert "outbox" not in got
    assert_same_state(got, ref, f"async one wavefront {kw} ipw {ipw} skew {skew}")
    if not skew:
        assert_same_state(got, oracle_after(_oracle_cfg(cfg), 100), "equals synchronous")


def test_long_skewed_run_and_resume():
    cfg = _async(width=12, height=8, pop=32, sites=64, k=5)
    say("async skewed 12x8x32, 1500 generations with a resume")
    run = GARun(cfg)
    run.set_launch(16)
    run.set_async(1, ASYNC_UNPACED, 2)
    run.step(700)
    mid = run.read()
    ref = oracle.OracleRun(_oracle_cfg(cfg))
    ref.step_async(700, 16, 2)
    assert_same_state(mid, ref, "async at 700")
    # resume into a fresh run from the population alone: buffers start empty
    run2 = GARun(cfg)
    run2.set_launch(16)
    run2.set_async(1, ASYNC_UNPACED, 2)
    run2.write(mid["f"], mid["T"], mid["D"], generation=700)
    run2.step(800)
    ref.clear_mailboxes()
    ref.step_async(800, 16, 2)
    assert_same_state(run2.read(), ref, "async resumed at 1500")
    run.close()
    run2.close()


@pytest.mark.parametrize("kw,gens", [(dict(width=64, height=64, pop=32, sites=64, k=5), 1000),
                                     (dict(width=100, height=37, pop=8, sites=32, k=3), 800),
                                     (dict(width=256, height=256, pop=32, sites=32), 200)])
def test_paced_free_running_is_synchronous(kw, gens):
    # Default pacing: an island starts generation t only once its neighbours
    # have finished t-1, and takes only genomes sent before t, so with no
    # barrier across the grid the result is the synchronous schedule's.
    cfg = _async(**kw)
    say(f"async paced free-running {kw}, {gens} generations")
    run = GARun(cfg)
    run.step(gens // 2)
    run.step(gens - gens // 2)
    got = run.read()
    waits = run.async_waits()
    run.close()
    assert waits == 0, f"{waits} pacing waits gave up"
    assert_same_state(got, oracle_after(_oracle_cfg(cfg), gens), f"async paced {kw}")


@pytest.mark.parametrize("kw,max_waves", [(dict(width=48, height=16), 5),
                                          (dict(width=48, height=16), 24),
                                          (dict(width=48, height=16), 0),
                                          (dict(width=1, height=300), 9),
                                          (dict(width=300, height=1), 0),
                                          (dict(width=2, height=2), 0)])
def test_lockstep_with_several_chunks_per_wavefront(kw, max_waves):
    # No lead and no skew is the lockstep exchange: an island waits for its
    # four neighbours' headers of the previous generation. With chunks of 4
    # islands over a few wavefronts, each wavefront runs many chunks in turn,
    # and neighbouring chunks often belong to one wavefront; on a torus one
    # island wide or high an island is its own east-west (north-south)
    # neighbour.
    cfg = _async(pop=16, sites=32, k=3, **kw)
    say(f"async lockstep {kw}, ipw 4, max_waves {max_waves}")
    run = GARun(cfg)
    run.set_launch(4)
    run.set_async(max_waves, 0)
    for n in (1, 150, 149):
        run.step(n)
    got = run.read()
    waits = run.async_waits()
    run.close()
    assert waits == 0, f"{waits} waits gave up"
    assert_same_state(got, oracle_after(_oracle_cfg(cfg), 300), f"lockstep {kw} {max_waves}")


@pytest.mark.parametrize("lead,migration", [(0, 1), (ASYNC_UNPACED, 0)])
def test_mail_offsets_beyond_32_bits(lead, migration):
    # 4100 x 4100 one-agent islands with 64-site surfaces: past 2^24 islands
    # the mail plane (eight 32-byte entries per island, 4.3 GB here) needs
    # 64-bit offsets in both exchanges
    cfg = _async(width=4100, height=4100, pop=1, sites=64, k=2, migration=migration)
    say(f"async 4100x4100x1 S=64, lead {lead}, migration {migration}, 3 generations")
    run = GARun(cfg)
    run.set_async(0, lead)
    run.step(3)
    got = run.read()
    waits = run.async_waits()
    run.close()
    assert waits == 0
    assert_same_state(got, oracle_after(_oracle_cfg(cfg), 3), f"4100x4100x1 lead {lead}")


def test_lockstep_and_general_exchange_alternate():
    # Skewed one-wavefront launches (the general exchange; genomes late,
    # overwritten or still pending at the end of a launch) alternate with
    # lockstep launches, on one and on several wavefronts. A lockstep launch
    # starts by applying the general rule once (a pending older genome is
    # taken in its first generation), so every segment matches the oracle's
    # interleaving, down to the last genome taken from each side.
    cfg = _async(width=24, height=16, pop=16, sites=64, k=4, seed=31)
    ipw = 8
    run = GARun(cfg)
    run.set_launch(ipw)
    ref = oracle.OracleRun(_oracle_cfg(cfg))
    plan = [((1, ASYNC_UNPACED, 3), 37, 3), ((0, 0, 0), 25, 0), ((1, ASYNC_UNPACED, 2), 31, 2),
            ((5, 0, 0), 40, 0), ((1, ASYNC_UNPACED, 5), 23, 5), ((1, 0, 0), 30, 0)]
    for (mw, lead, skew), n, ref_skew in plan:
        say(f"async segment max_waves {mw} lead {lead} skew {skew}, {n} generations")
        run.set_async(mw, lead, skew)
        run.step(n)
        ref.step_async(n, ipw, ref_skew)
        assert_same_state(run.read(), ref, f"after segment {mw, lead, skew}")
        seen = ref.mailboxes()["seen"].astype(np.int64) - 1
        assert np.array_equal(run.async_last_taken(), seen), f"last taken after {mw, lead, skew}"
    assert run.async_waits() == 0
    run.close()


def test_lockstep_resume_from_a_written_population():
    cfg = _async(width=40, height=12, pop=32, sites=32, k=2)
    run = GARun(cfg)
    run.step(120)
    mid = run.read()
    run.close()
    ref = oracle_after(_oracle_cfg(cfg), 120)
    assert_same_state(mid, ref, "lockstep at 120")
    run2 = GARun(cfg)
    run2.set_launch(4)
    run2.set_async(7, 0)
    run2.write(mid["f"], mid["T"], mid["D"], generation=120)
    run2.step(90)
    ref.set_outbox(np.zeros(ref.islands, np.uint8), np.zeros(ref.islands, np.uint8),
                   np.zeros(ref.islands, np.float32), np.zeros(ref.islands, np.uint32),
                   np.zeros((ref.islands, ref.words), np.uint32))
    ref.step(90)
    assert_same_state(run2.read(), ref, "lockstep resumed at 210")
    assert run2.async_waits() == 0
    run2.close()


@pytest.mark.parametrize("kw,gens", [(dict(width=1024, height=512), (500, 500)),
                                     (dict(width=256, height=256), (1000, 2000))])
def test_lockstep_equals_the_synchronous_kernel_at_full_size(kw, gens):
    # the synchronous kernel is pinned to the oracle at these sizes; the
    # lockstep launch (several of them, crossing launch boundaries) must give
    # the same bits with no barrier across the grid
    cfg = run_config(pop=32, sites=32, k=2, **kw)
    say(f"lockstep vs synchronous {kw}, {sum(gens)} generations")
    sync = GARun(cfg)
    sync.step(sum(gens))
    want = sync.read(outbox=False)
    sync.close()
    run = GARun(dict(cfg, schedule=1))
    for n in gens:
        run.step(n)
    got = run.read()
    waits = run.async_waits()
    run.close()
    assert waits == 0
    assert got["generation"] == want["generation"]
    for key in ("f", "T", "D"):
        a, b = got[key], want[key]
        if key == "f":
            a, b = a.view(np.uint32), b.view(np.uint32)
        assert np.array_equal(a, b), f"{key} differs at {np.flatnonzero(a != b)[:5]}"


def test_paced_last_taken_follows_the_migration_draws():
    # Equal to the synchronous schedule, the last genome island i took from
    # side q was sent in the last generation g <= t-2 in which the neighbour
    # there drew the direction toward i (Philox MIGRATE stream, computed here).
    cfg = _async(width=32, height=24, pop=16, sites=32)
    t = 150
    say("async paced last-taken generations 32x24x16")
    run = GARun(cfg)
    run.step(t)
    got = run.async_last_taken()
    assert run.async_waits() == 0
    run.close()
    W, H = cfg["width"], cfg["height"]
    I = W * H
    key = [cfg["seed"], cfg["run_id"]]
    dirs = np.array([[int(oracle.philox([0, i, g, 1], key)[1] >> 30) for g in range(t - 1)]
                     for i in range(I)])
    for i in range(I):
        x, y = i % W, i // W
        nbrs = [((y - 1) % H) * W + x, y * W + (x + 1) % W, ((y + 1) % H) * W + x,
                y * W + (x - 1) % W]
        for q, j in enumerate(nbrs):
            sent = np.nonzero(dirs[j] == (q ^ 2))[0]
            assert got[i, q] == (sent[-1] if sent.size else -1), (i, q)


@pytest.mark.parametrize("lead", [ASYNC_UNPACED, 0])
@pytest.mark.parametrize("kw", [dict(width=64, height=64, pop=32, sites=32),
                                dict(width=100, height=37, pop=8, sites=64, k=5)])
def test_unpaced_without_migration_is_synchronous(kw, lead):
    cfg = _async(migration=0, **kw)
    say(f"async lead {lead}, no migration {kw}")
    run = GARun(cfg)
    run.set_async(0, lead)
    run.step(300)
    got = run.read()
    run.close()
    assert_same_state(got, oracle_after(_oracle_cfg(cfg), 300), f"async no migration {kw}")


@pytest.mark.parametrize("lead", [ASYNC_UNPACED, 3])
def test_free_running_invariants(lead):
    # Until T reaches S every deposit fills a fresh site (rank r at site r), so a
    # genome with T deposits has no bit set at sites T..S-1: a genome read torn
    # between two buffer contents would likely break that. Fitness under the
    # discrete law stays a multiple of 1/2. A genome is taken only after the
    # generation it was sent in, so T never exceeds the generation, even when
    # it comes from a neighbour that is further along.
    cfg = _async(width=256, height=128, pop=32, sites=64, p32=2 ** 31)
    say(f"async free-running invariants 256x128x32, lead {lead}, 60 generations x 5")
    run = GARun(cfg)
    run.set_async(0, lead)
    for rep in range(5):
        run.step(12)
        got = run.read()
        t = got["generation"]
        T = got["T"].astype(np.uint64)
        assert (T >= 1).all() and (T <= t).all()
        bits = got["D"][:, 0].astype(np.uint64) | (got["D"][:, 1].astype(np.uint64) << np.uint64(32))
        above = np.where(T < 64, bits >> T, np.uint64(0))
        assert (above == 0).all(), f"surface bits above T at {np.flatnonzero(above)[:5]}"
        twice = got["f"] * 2
        assert np.array_equal(twice, np.round(twice))
    run.close()


def test_async_errors():
    cfg = _async(width=8, height=8)
    run = GARun(cfg)
    from paper_2405_03605_amd import _lib
    import ctypes
    lib = _lib.load()
    box = (_lib.OutboxEntry * run.islands)()
    assert lib.ga_read_population(run.handle, None, None, None,
                                  ctypes.cast(box, ctypes.c_void_p), None) == _lib.GA_EINVAL
    with pytest.raises(GAError):
        run.set_launch(16, 4, 2)          # resident form is synchronous
    batch = GABatch()
    with pytest.raises(GAError):
        batch.add(run, 10)
    batch.close()
    with pytest.raises(GAError):
        run.set_async(2, ASYNC_UNPACED, 3)   # a skew needs one wavefront
    with pytest.raises(GAError):
        run.set_async(1, 0, 3)               # ... and no pacing
    sync = GARun(run_config(width=8, height=8))
    with pytest.raises(GAError):
        sync.set_async(1)
    with pytest.raises(GAError):
        sync.async_waits()
    sync.close()
    run.close()


# --------------------------------------------------------------------------
# statistics of the free-running schedule (the acceptance rule of
# paper_2405_03605_amd.async_stats, fixed before these runs)
# --------------------------------------------------------------------------
_REPS = {}


def _reps(kind):
    if kind not in _REPS:
        n = async_stats.CONTROL_REPS if kind == "control" else async_stats.REPS
        say(f"{n} replicates of {kind}, 64x64x32 x {async_stats.GENS} generations")
        _REPS[kind] = [async_stats.replicate(kind, r) for r in range(n)]
    return _REPS[kind]


def _judged(kind):
    res = async_stats.judge(_reps("sync"), _reps(kind), _reps("control"))
    lost = np.mean([x["lost"] for x in _reps(kind)])
    for key, v in res.items():
        say(f"{kind} {key}: sync {v['sync_mean']:.4g} +- {v['sync_sd']:.3g}, async "
            f"{v['async_mean']:.4g} +- {v['async_sd']:.3g}, control {v['control_mean']:.4g}; "
            f"shift {v['shift_over_effect']:.3f} of the migration effect, "
            f"{v['shift_over_se']:.2f} SE, KS p {v['ks_p']:.3g} -> "
            f"{'pass' if v['pass'] else 'MISS'}")
    say(f"{kind}: {lost:.4f} of sent genomes never absorbed")
    return res


def test_lead2_statistics_match_synchronous():
    res = _judged("lead2")
    assert all(v["pass"] for v in res.values()), {k: v["pass"] for k, v in res.items()}


@pytest.mark.xfail(strict=True, reason=(
    "finding: unpaced, about 18% of sent genomes are overwritten before they are read and "
    "mean fitness falls 0.31 of the migration effect below the synchronous schedule "
    "(85 standard errors); both tree metrics pass the rule"))
def test_unpaced_statistics_match_synchronous():
    res = _judged("unpaced")
    assert all(v["pass"] for v in res.values()), {k: v["pass"] for k, v in res.items()}


def test_statistics_have_power():
    # without migration the islands share no ancestor since the founders: the
    # trees are far longer, and fitness differs, by much more than the noise
    sync, control = _reps("sync"), _reps("control")
    for key in ("sum_branch_length", "mean_evolutionary_distinctiveness"):
        a = np.array([x[key] for x in sync])
        c = np.array([x[key] for x in control])
        assert c.min() > a.max(), key


def test_lockstep_absorbs_every_genome():
    # paced (the lockstep exchange) with every wait met, each island takes the
    # one genome each neighbour sent it, as the synchronous schedule does: one
    # per island and generation, except in generation 0 (nothing was sent
    # before it; what generation 299 sends is still in flight)
    cfg = run_config(schedule=1, width=37, height=23, pop=16, sites=32)
    run = GARun(cfg)
    run.step(300)
    assert run.async_waits() == 0
    assert run.async_taken() == 37 * 23 * 299
    run.close()
    with pytest.raises(GAError):
        sync = GARun(run_config(width=4, height=4, pop=8))
        try:
            sync.async_taken()
        finally:
            sync.close()


def test_lockstep_matches_the_oracle_at_paper_scale():
    # the paper-scale grid (16.8M agents) in the lockstep launch against the
    # oracle itself, three generations
    cfg = run_config(pop=32, sites=32, k=2, width=1024, height=512)
    say("lockstep vs oracle at 1024x512x32, 3 generations")
    run = GARun(dict(cfg, schedule=1))
    run.step(3)
    got = run.read()
    assert run.async_waits() == 0
    run.close()
    assert_same_state(got, oracle_after(cfg, 3), "lockstep 1024x512x32")
