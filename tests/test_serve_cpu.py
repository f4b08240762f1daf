"""Host logic of the continuous-batching server on the CPU, with stand-ins for
the device runs: admission by footprint and slot count in arrival order,
retirement when a budget is spent, memory returned, latency report."""
import pytest

from paper_2405_03605_amd.serve import Server


class FakeRun:
    def __init__(self, cfg):
        self.cfg = cfg
        self.closed = False

    def extract(self):
        return ("ids", self.cfg["run_id"])

    def close(self):
        self.closed = True


class FakeBatch:
    def __init__(self):
        self.left = {}
        self.block = None
        self.steps = 0

    def set_graph_block(self, n):
        self.block = n

    def add(self, run, budget):
        assert run not in self.left
        self.left[run] = budget

    def remove(self, run):
        del self.left[run]

    def remaining(self, run):
        return self.left[run]

    def step(self, n):
        self.steps += 1
        for r in self.left:
            self.left[r] -= min(n, self.left[r])

    def close(self):
        pass


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
    return Server(budget, max_slots=slots, block=block, make_run=FakeRun,
                  make_batch=FakeBatch, state_bytes=sb, clock=Clock())


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
    assert len(srv.live) == 3 and big.rid in srv.live


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
    rep = srv.report(wall=1.0)
    assert rep["completed"] == 6
    assert rep["agent_gens"] == sum(64 * (10 + 5 * i) for i in range(6))
    assert rep["latency_p99_s"] >= rep["latency_p50_s"] > 0
