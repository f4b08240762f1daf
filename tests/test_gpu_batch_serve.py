"""GPU parity of the batched and served forms: every member of a batch, and
every served request, must give the bits it gives alone and the oracle's bits."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_state, oracle_after, say
from paper_2405_03605_amd import FORM_STREAMING, GABatch, GAError, GARun
from paper_2405_03605_amd.autotune import (apply, autotune, autotune_batch, batch_candidates,
                                           candidates, class_of)
from paper_2405_03605_amd.serve import Server
from paper_2405_03605_amd.workloads import batched_configs, run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


UNEVEN = [
    run_config(width=5, height=3, pop=8, sites=32, k=3, selection=1, run_id=11),
    run_config(width=17, height=9, pop=16, sites=64, k=8, selection=0, run_id=12),
    run_config(width=12, height=12, pop=32, sites=32, k=2, run_id=13),
    run_config(width=3, height=40, pop=64, sites=64, k=5, run_id=14),
    run_config(width=33, height=2, pop=4, sites=32, k=2, run_id=15),
    run_config(width=1, height=1, pop=1, sites=64, k=1, run_id=16),
    run_config(width=20, height=20, pop=8, sites=64, k=7, selection=0, run_id=17),
    run_config(width=9, height=11, pop=32, sites=64, migration=0, run_id=18),
    run_config(width=14, height=6, pop=16, sites=32, k=5, law=1, p32=1417339207,
               p_ben32=12884901, run_id=19),
]
BUDGETS = [150, 230, 100, 99, 305, 1, 320, 200, 175]


@pytest.mark.parametrize("graph_block,ipw,wpg", [(100, 0, 0), (0, 0, 1), (64, 8, 8), (100, 64, 2)])
def test_batch_members_match_oracle(graph_block, ipw, wpg):
    say(f"batch of {len(UNEVEN)} uneven runs, graph block {graph_block}, ipw {ipw}")
    runs = [GARun(c) for c in UNEVEN]
    batch = GABatch()
    batch.set_graph_block(graph_block)
    if ipw or wpg:
        batch.set_launch(ipw, wpg)
    for r, b in zip(runs, BUDGETS):
        batch.add(r, b)
    batch.step(120)
    batch.step(200)
    for r, b in zip(runs, BUDGETS):
        assert batch.remaining(r) == 0
    for r, c, b in zip(runs, UNEVEN, BUDGETS):
        assert_same_state(r.read(), oracle_after(c, b), f"member {c['run_id']}")
    batch.close()


def test_membership_changes_between_blocks():
    a, b, c = (GARun(cfg) for cfg in UNEVEN[:3])
    batch = GABatch()
    batch.add(a, 500)
    batch.add(b, 500)
    batch.step(100)
    batch.remove(b)          # b continues alone
    b.set_launch(form=FORM_STREAMING)
    b.step(37)
    batch.add(c, 80)         # c joins late
    batch.step(150)
    batch.add(b, 13)         # b rejoins
    batch.step(100)
    batch.close()
    assert_same_state(a.read(), oracle_after(UNEVEN[0], 350), "a")
    assert_same_state(b.read(), oracle_after(UNEVEN[1], 150), "b")
    assert_same_state(c.read(), oracle_after(UNEVEN[2], 80), "c")


def test_placement_with_odd_group_sizes_and_grid_growth():
    """The launch's slots are laid out per XCD in whole rounds of eight
    groups: group sizes that are no power of two, and a member whose tiles
    outgrow the captured grid (new tables, a new graph) mid-run, must leave
    every member's bits as the oracle's."""
    small = UNEVEN[:4]
    big = run_config(width=256, height=64, pop=8, sites=32, k=3, selection=1, run_id=21)
    runs = [GARun(c) for c in small]
    batch = GABatch()
    batch.set_launch(0, 3)
    for r in runs:
        batch.add(r, 400)
    say("odd group sizes: 3 waves per group, small members")
    batch.step(100)
    rb = GARun(big)
    batch.add(rb, 150)       # 256 more tiles: past the first grid
    say("odd group sizes: a large member joins")
    batch.step(100)
    batch.set_launch(0, 5)
    say("odd group sizes: 5 waves per group")
    batch.step(100)
    batch.step(100)
    for r in runs + [rb]:
        assert batch.remaining(r) == 0
    batch.close()
    for r, c in zip(runs, small):
        assert_same_state(r.read(), oracle_after(c, 400), f"member {c['run_id']}")
    assert_same_state(rb.read(), oracle_after(big, 150), "large member")


def test_batched_workload_equals_alone():
    cfgs = batched_configs()
    gens = 130
    say(f"64-run batched workload, {gens} generations, batch vs alone")
    alone = []
    for c in cfgs:
        r = GARun(c)
        r.step(gens)
        alone.append(r.read(outbox=False))
        r.close()
    runs = [GARun(c) for c in cfgs]
    batch = GABatch()
    for r in runs:
        batch.add(r, gens)
    batch.step(gens)
    for r, c, ref in zip(runs, cfgs, alone):
        got = r.read(outbox=False)
        for key in ("f", "T", "D"):
            assert np.array_equal(got[key], ref[key]), (c, key)
    # the smallest members against the oracle as well
    order = np.argsort([c["width"] * c["height"] * c["pop"] for c in cfgs])
    for i in order[:4]:
        assert_same_state(runs[i].read(), oracle_after(cfgs[i], gens), f"batched {i}")
    batch.close()


def test_autotune_candidates_are_bit_identical():
    cfg = run_config(width=40, height=30, pop=16, sites=64, k=3, seed=2)
    ref = oracle_after(cfg, 60)
    cands = candidates(cfg)
    assert len(cands) >= 8
    for cand in cands:
        run = GARun(cfg)
        try:
            apply(run, cand)
        except GAError:      # a tiling the GPU cannot hold at once
            run.close()
            continue
        run.step(60)
        assert_same_state(run.read(), ref, f"candidate {cand}")
        run.close()
    best = autotune(cfg, gens=10, use_cache=False)
    assert best in cands


def test_batch_class_candidates_are_bit_identical():
    # every islands-per-wavefront candidate of every class present, the j-th
    # candidate of each class in the j-th batch with the j-th group size,
    # against the oracle; then the autotuner's choice
    from paper_2405_03605_amd.autotune import WPG_CANDIDATES
    refs = [oracle_after(c, b) for c, b in zip(UNEVEN, BUDGETS)]
    classes = sorted({class_of(c) for c in UNEVEN})
    cands = {k: batch_candidates(k[0]) for k in classes}
    rounds = max(len(v) for v in cands.values())
    say(f"{len(classes)} classes, up to {rounds} candidates each")
    for j in range(rounds):
        runs = [GARun(c) for c in UNEVEN]
        batch = GABatch()
        for r, b in zip(runs, BUDGETS):
            batch.add(r, b)
        batch.set_launch(0, WPG_CANDIDATES[j % len(WPG_CANDIDATES)])
        for (log2n, words), cl in cands.items():
            ipw = cl[j % len(cl)]
            batch.set_class_launch(log2n, words, ipw)
            assert batch.class_launch(log2n, words)[0] == ipw
        batch.step(120)
        batch.step(200)
        for r, c, ref in zip(runs, UNEVEN, refs):
            assert_same_state(r.read(), ref, f"round {j} member {c['run_id']}")
        batch.close()
        for r in runs:
            r.close()
    runs = [GARun(c) for c in UNEVEN]
    batch = GABatch()
    for r, b in zip(runs, BUDGETS):
        batch.add(r, b)
    chosen = autotune_batch(batch, UNEVEN, gens=20, use_cache=False)
    assert chosen["waves_per_group"] in WPG_CANDIDATES
    for k in classes:
        assert chosen[k] in cands[k]
    batch.step(320)
    for r, c, ref in zip(runs, UNEVEN, refs):
        assert_same_state(r.read(), ref, f"autotuned member {c['run_id']}")
    batch.close()


def test_settled_follows_the_gpu():
    # a member whose budget ran out is settled once its last block has run
    import torch
    run = GARun(UNEVEN[2])
    batch = GABatch()
    batch.add(run, 150)
    assert not batch.settled(run)
    batch.step(200)
    torch.cuda.synchronize()
    assert batch.remaining(run) == 0 and batch.settled(run)
    assert run.generation == 150
    batch.remove(run)
    assert run.generation == 150
    assert_same_state(run.read(), oracle_after(UNEVEN[2], 150), "settled member")
    batch.close()


def test_settled_with_many_step_calls_enqueued():
    # a member that finished in the first of many step calls reads settled once
    # that call has run, however many calls were enqueued after it (a call
    # returns once the call two before it has run, so after the third call the
    # first has); its samples then equal the oracle's
    short, long_ = GARun(UNEVEN[0]), GARun(UNEVEN[1])
    batch = GABatch()
    batch.add(short, 3)
    batch.add(long_, 10 ** 6)
    for _ in range(20):
        batch.step(3)
    assert batch.remaining(short) == 0 and batch.settled(short)
    assert not batch.settled(long_)
    batch.remove(short)
    assert_same_state(short.read(), oracle_after(UNEVEN[0], 3), "member settled early")
    batch.close()
    for r in (short, long_):
        r.close()


@pytest.mark.parametrize("shapes", [None, {"waves_per_group": 2, (3, 1): 16, (3, 2): 64,
                                             (4, 1): 4, (4, 2): 32, (5, 1): 2, (5, 2): 16}])
def test_served_results_equal_alone_and_oracle(shapes):
    # also with a launch shape applied to the pool as the autotuner would
    rng = np.random.default_rng(5)
    stream = []
    for i in range(10):
        cfg = run_config(width=int(rng.integers(3, 30)), height=int(rng.integers(3, 20)),
                         pop=int(rng.choice([8, 16, 32])), sites=int(rng.choice([32, 64])),
                         k=int(rng.integers(2, 9)), selection=int(rng.integers(0, 2)),
                         seed=1, run_id=500 + i)
        stream.append((0.002 * i, cfg, int(rng.integers(50, 400))))
    import paper_2405_03605_amd as ga
    biggest = max(ga.state_bytes(c) for _, c, _ in stream)
    srv = Server(budget_bytes=3 * biggest, max_slots=4, block=64, shapes=shapes)
    done = srv.drain(stream)
    srv.close()
    assert len(done) == len(stream)
    assert max(srv.used, 0) == 0
    for req in done:
        ids, T, D = req.result
        ref = oracle_after(req.cfg, req.gens)
        f0, T0, D0 = ref.population()
        assert np.array_equal(ids, ref.sample_one_per_island())
        assert np.array_equal(T, T0[ids.astype(np.int64)])
        assert np.array_equal(D, D0[ids.astype(np.int64)])


def test_pool_first_fit_release_merging_and_results():
    # three runs fill the pool exactly; a larger run fits only once the run
    # between the two freed blocks is gone and all three blocks have merged
    import paper_2405_03605_amd as ga
    from paper_2405_03605_amd import GAError, GAPool
    a = run_config(width=8, height=6, pop=16, sites=32, seed=1, run_id=900)
    b = run_config(width=20, height=12, pop=32, sites=64, k=4, seed=1, run_id=901)
    c = run_config(width=9, height=7, pop=8, sites=32, seed=1, run_id=902)
    big = run_config(width=16, height=12, pop=32, sites=64, seed=1, run_id=903)
    al = lambda x: (x + 255) // 256 * 256
    sa, sb, sc, sbig = (al(ga.state_bytes(x)) for x in (a, b, c, big))
    assert max(sa, sc) < sbig <= sa + sb + sc
    pool = GAPool(sa + sb + sc, max_slots=3)
    ta, tb, tc = pool.admit(a, 50), pool.admit(b, 80), pool.admit(c, 50)
    assert None not in (ta, tb, tc)
    assert pool.usage() == {"used": sa + sb + sc, "largest_free": 0, "live": 3}
    assert pool.admit(c, 10) is None             # no slot and no memory
    pool.step(50)
    assert pool.done() == [ta, tc] and pool.remaining(tb) == 30
    ra = pool.retire(ta)
    assert pool.usage()["largest_free"] == sa
    assert pool.admit(big, 40) is None           # a's block alone is too small
    rc = pool.retire(tc)                         # not adjacent to a's block
    assert pool.usage() == {"used": sb, "largest_free": max(sa, sc), "live": 1}
    assert pool.admit(big, 40) is None
    pool.step(30)
    rb = pool.retire(tb)
    assert pool.usage() == {"used": 0, "largest_free": sa + sb + sc, "live": 0}
    tbig = pool.admit(big, 40)
    assert tbig is not None
    pool.step(40)
    rbig = pool.retire(tbig)
    for cfg, gens, (ids, T, D) in ((a, 50, ra), (c, 50, rc), (b, 80, rb), (big, 40, rbig)):
        ref = oracle_after(cfg, gens)
        f0, T0, D0 = ref.population()
        assert np.array_equal(ids, ref.sample_one_per_island()), cfg["run_id"]
        assert np.array_equal(T, T0[ids.astype(np.int64)]), cfg["run_id"]
        assert np.array_equal(D, D0[ids.astype(np.int64)]), cfg["run_id"]
    # a run retired before its budget is spent, without sampling
    t = pool.admit(a, 1000)
    pool.step(5)
    assert pool.remaining(t) == 995 and pool.done() == []
    pool.retire(t, sample=False)
    with pytest.raises(GAError):
        pool.remaining(t)
    with pytest.raises(GAError):
        pool.retire(t)
    with pytest.raises(GAError):
        pool.retire(t, sample=False)
    with pytest.raises(GAError):
        pool.admit(run_config(width=100, height=100, pop=32), 10)   # larger than the pool
    assert pool.usage()["used"] == 0
    pool.close()


def test_pool_churn_keeps_runs_apart():
    # runs of uneven sizes admitted, stepped and retired in a random order
    # until the pool has fragmented and merged many times; every retired
    # run's sample must be the oracle's (overlapping blocks would corrupt one)
    import paper_2405_03605_amd as ga
    from paper_2405_03605_amd import GAPool
    rng = np.random.default_rng(77)
    al = lambda x: (x + 255) // 256 * 256
    cfgs = [run_config(width=int(rng.integers(3, 10)), height=int(rng.integers(2, 8)),
                       pop=int(rng.choice([4, 8, 16])), sites=int(rng.choice([32, 64])),
                       k=int(rng.integers(1, 5)), seed=3, run_id=2000 + i) for i in range(60)]
    budget = 6 * max(al(ga.state_bytes(c)) for c in cfgs)
    pool = GAPool(budget, max_slots=8)
    pool.set_graph_block(7)
    pending = list(range(len(cfgs)))
    live, results = {}, {}
    gens = {i: int(rng.integers(5, 60)) for i in pending}
    for _ in range(400):
        while pending:
            t = pool.admit(cfgs[pending[0]], gens[pending[0]])
            if t is None:
                break
            live[t] = pending.pop(0)
        if not live:
            break
        pool.step(int(rng.integers(1, 25)))
        for t in pool.done():
            results[live.pop(t)] = pool.retire(t)
        u = pool.usage()
        assert u["used"] <= budget and u["live"] == len(live)
    assert not pending and not live and len(results) == len(cfgs)
    assert pool.usage() == {"used": 0, "largest_free": budget, "live": 0}
    for i in range(len(cfgs)):
        ids, T, D = results[i]
        ref = oracle_after(cfgs[i], gens[i])
        f0, T0, D0 = ref.population()
        assert np.array_equal(ids, ref.sample_one_per_island()), i
        assert np.array_equal(T, T0[ids.astype(np.int64)]), i
        assert np.array_equal(D, D0[ids.astype(np.int64)]), i
    pool.close()


def test_pool_argument_errors():
    import ctypes
    import torch
    from paper_2405_03605_amd._lib import GA_EINVAL, load
    lib = load()
    mem = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    P = ctypes.c_void_p
    base = mem.data_ptr()
    assert lib.ga_pool_create(P(base + 1), 1 << 19, 4, P(stream.cuda_stream), ctypes.byref(h)) == GA_EINVAL
    assert lib.ga_pool_create(P(base), 1 << 19, 0, P(stream.cuda_stream), ctypes.byref(h)) == GA_EINVAL
    assert lib.ga_pool_create(None, 1 << 19, 4, P(stream.cuda_stream), ctypes.byref(h)) == GA_EINVAL
    assert lib.ga_pool_create(P(base), 1 << 19, 4, P(stream.cuda_stream), None) == GA_EINVAL
    # a pool smaller than one 256-byte block holds nothing
    assert lib.ga_pool_create(P(base), 255, 4, P(stream.cuda_stream), ctypes.byref(h)) == 0
    left = ctypes.c_uint64()
    assert lib.ga_pool_remaining(h, 1, ctypes.byref(left)) == GA_EINVAL
    used, big, live = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_uint32()
    assert lib.ga_pool_usage(h, ctypes.byref(used), ctypes.byref(big), ctypes.byref(live)) == 0
    assert (used.value, big.value, live.value) == (0, 0, 0)
    lib.ga_pool_destroy(h)
    lib.ga_pool_destroy(None)
