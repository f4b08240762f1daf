"""Host logic of the continuous-batching server on the CPU, with a stand-in for
the device run pool: admission in arrival order while the pool takes runs
(memory and slots), retirement when a budget is spent, memory returned,
latency report. The native pool's allocator is checked on the GPU."""
import pytest

from paper_2405_03605_amd.serve import Server


class FakePool:
    """Budget and slot accounting by sums (no fragmentation), budgets counted
    down per step, results tagged with the run id."""

    def __init__(self, budget, slots):
        self.budget, self.slots = budget, slots
        self.left, self.size, self.cfgs, self.finished = {}, {}, {}, {}
        self.next = 1
        self.steps = 0
        self.block = None
        self.closed = False

    def set_graph_block(self, n):
        self.block = n

    def set_launch(self, ipw=0, wpg=0):
        self.launch = (ipw, wpg)

    def set_class_launch(self, log2n, words, ipw=0):
        self.classes = getattr(self, "classes", {})
        self.classes[(log2n, words)] = ipw

    @property
    def used(self):
        return sum(self.size.values())

    def admit(self, cfg, gens):
        need = sb(cfg)
        if len(self.left) >= self.slots or self.used + need > self.budget:
            return None
        t = self.next
        self.next += 1
        self.left[t], self.size[t], self.cfgs[t] = gens, need, cfg
        return t

    def remaining(self, t):
        return self.left[t]

    def step(self, n):
        self.steps += 1
        for t in self.left:
            before = self.left[t]
            self.left[t] -= min(n, before)
            if before and not self.left[t]:
                self.finished[t] = self.steps

    def done(self, settled=False):
        # a run settles once a later step has been enqueued after its last one
        return sorted(t for t, v in self.left.items()
                      if v == 0 and (not settled or self.finished.get(t, 0) < self.steps))

    def retire(self, t, sample=True):
        cfg = self.cfgs.pop(t)
        del self.left[t], self.size[t]
        return ("ids", cfg["run_id"]) if sample else None

    def close(self):
        self.closed = True


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t


def cfg(rid, agents=64):
    return dict(width=agents // 8, height=1, pop=8, sites=32, k=2, selection=1, p32=0,
                migration=1, seed=1, run_id=rid)


def sb(c):
    return c["width"] * c["height"] * c["pop"] * 100


def make_server(budget, slots=8, block=10):
    return Server(budget, max_slots=slots, block=block, make_pool=FakePool, state_bytes=sb,
                  clock=Clock())


def test_autotuned_shapes_reach_the_pool():
    shapes = {"waves_per_group": 8, (3, 1): 32, (5, 2): 8}
    srv = Server(10_000, max_slots=2, block=10, make_pool=FakePool, state_bytes=sb,
                 clock=Clock(), shapes=shapes)
    assert srv.pool.launch == (0, 8)
    assert srv.pool.classes == {(3, 1): 32, (5, 2): 8}
    plain = make_server(10_000)
    assert not hasattr(plain.pool, "launch")


def test_admission_respects_memory_and_order():
    srv = make_server(budget=64 * 100 * 2)      # room for two 64-agent runs
    for i in range(4):
        srv.submit(cfg(i), gens=25)
    assert srv.admit() == 2
    assert [r.rid for r in srv.waiting] == [2, 3]
    assert srv.used == 2 * 6400
    srv.advance()            # 10 gens
    assert srv.retire() == 0
    srv.advance()
    srv.advance()            # 30 >= 25
    assert srv.retire() == 2
    assert srv.used == 0
    assert srv.admit() == 2


def test_slots_limit_and_head_of_line_order():
    srv = make_server(budget=10 ** 9, slots=3)
    big = srv.submit(cfg(0, agents=512), gens=5)
    for i in range(1, 6):
        srv.submit(cfg(i), gens=5)
    assert srv.admit() == 3
    assert len(srv.live) == 3 and any(req is big for req, _ in srv.live.values())
    # a head-of-line request that does not fit holds back those behind it
    srv2 = make_server(budget=64 * 100 * 2, slots=8)
    srv2.submit(cfg(0), gens=5)
    srv2.submit(cfg(1, agents=128), gens=5)     # needs the whole budget
    srv2.submit(cfg(2), gens=5)
    assert srv2.admit() == 1 and [r.rid for r in srv2.waiting] == [1, 2]


def test_oversized_and_invalid_requests_rejected():
    srv = make_server(budget=1000)
    with pytest.raises(ValueError):
        srv.submit(cfg(0, agents=64), gens=5)     # needs 6400 > 1000


def test_drain_completes_everything_and_reports():
    srv = make_server(budget=64 * 100 * 3, slots=2, block=7)
    arrivals = [(0.0, cfg(i), 10 + 5 * i) for i in range(6)]
    done = srv.drain(arrivals)
    assert sorted(r.rid for r in done) == list(range(6))
    assert all(r.result == ("ids", r.cfg["run_id"]) for r in done)
    assert all(r.finished >= r.admitted >= r.arrival for r in done)
    assert srv.used == 0 and not srv.live and not srv.waiting
    assert srv.pool.block == 7
    rep = srv.report(wall=1.0)
    assert rep["completed"] == 6
    assert rep["agent_gens"] == sum(64 * (10 + 5 * i) for i in range(6))
    assert rep["latency_p99_s"] >= rep["latency_p50_s"] > 0
    srv.close()
    assert srv.pool.closed
