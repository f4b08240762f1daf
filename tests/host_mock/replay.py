"""Replay of the C ABI's host paths against the host-only runtime
(tests/host_mock): single runs in both forms and schedules, genome strings,
wide differentia, resume through host state, argument errors; a batch of the
64 uneven runs with launch-shape changes and membership churn; the served
stream through the run pool and the server; the relatedness calls. Run in a
child interpreter with the library built with AddressSanitizer and
UndefinedBehaviorSanitizer preloaded (tests/test_host_sanitized.py); any report
aborts it. Nothing here checks a generation's arithmetic (the kernels are
stubs): only that the host code stays in bounds, defined and consistent.

    python tests/host_mock/replay.py <path of the mock-built library>
"""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2405_03605_amd import _lib  # noqa: E402
from paper_2405_03605_amd.autotune import batch_candidates, class_of  # noqa: E402
from paper_2405_03605_amd.run import GAPool, GARun, _fields, make_config  # noqa: E402
from paper_2405_03605_amd.serve import Server  # noqa: E402
from paper_2405_03605_amd.workloads import batched_configs, run_config, served_requests  # noqa: E402

lib = ctypes.CDLL(sys.argv[1])
for name, (res, args) in _lib.SIGNATURES.items():
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
_lib._lib = lib
check = _lib.check
P = ctypes.c_void_p
_keep = []


def aligned(n):
    raw = np.zeros(n + 256, dtype=np.uint8)
    _keep.append(raw)
    off = (-raw.ctypes.data) % 256
    return raw[off:off + n]


def host_run(cfg):
    """A GARun whose state is a host buffer (the binding's methods need only
    the handle and the sizes)."""
    r = GARun.__new__(GARun)
    r.cfg = _fields(cfg)
    r._c = make_config(r.cfg)
    n = lib.ga_state_bytes(ctypes.byref(r._c))
    assert n > 0, cfg
    r.mem = aligned(n)
    h = P()
    check(lib.ga_init(ctypes.byref(r._c), P(r.mem.ctypes.data), n, None, ctypes.byref(h)))
    r._h = h
    r.state_bytes = n
    r.islands = r.cfg["width"] * r.cfg["height"]
    r.agents = r.islands * r.cfg["pop"]
    r.words = r.cfg["sites"] * r.cfg["dbits"] // 32
    return r


def single_runs():
    shapes = [dict(), dict(width=1, height=9, pop=4, selection=0), dict(width=20, height=10, pop=1),
              dict(width=9, height=7, pop=64, k=8, sites=64), dict(model=1, sites=32),
              dict(model=2, k=5), dict(dbits=4, sites=16), dict(policy=1, sites=64),
              dict(policy=2, sites=64), dict(law=1, p_ben32=12884901, p32=1417339207)]
    for kw in shapes:
        for schedule in (0, 1):
            cfg = run_config(**dict(dict(width=13, height=11), **kw, schedule=schedule))
            r = host_run(cfg)
            forms = (0, 1) if schedule else (0, 1, 2)
            for form in forms:
                r.set_launch(0, 0, form)
                r.set_graph_block(100)
                r.step(250)
                r.set_graph_block(0)
                r.step(7)
            r.set_launch(max(1, 64 // r.cfg["pop"]), 2, 1)
            r.step(130)
            assert r.generation == 257 * len(forms) + 130, r.generation
            st = r.read(outbox=not schedule and not r.cfg["model"])
            r.write(st["f"], st["T"], st["D"], generation=int(st["generation"]))
            if r.cfg["model"]:
                w = r.read_strings()
                r.write_strings(w)
            r.extract()
            r.extract(np.arange(0, r.agents, 3, dtype=np.uint64))
            if schedule:
                for lead in (0, 2, 0xFFFFFFFF):
                    r.set_async(0, lead)
                    r.step(40)
                r.set_async(1, 0xFFFFFFFF, 2)
                r.step(20)
                assert lib.ga_set_async(r._h, 1, 3, 2) != 0
                r.step(20)
                r.async_waits()
                r.async_taken()
                r.async_last_taken()
            else:
                r.set_tiles(4, 4)
                r.set_launch(0, 0, 2)
                r.step(30)
                r.tiles()
                r.set_tiles(0, 0)
            r.close()
    # argument errors answer an error code and leave nothing behind
    bad = [dict(pop=3), dict(sites=3), dict(k=0), dict(width=0), dict(model=9), dict(law=1, model=1)]
    for kw in bad:
        c = make_config(_fields(run_config(**kw)))
        assert lib.ga_state_bytes(ctypes.byref(c)) == 0, kw
    r = host_run(run_config())
    for call in (lambda: lib.ga_set_launch(r._h, 100, 0, 0), lambda: lib.ga_set_launch(r._h, 0, 99, 0),
                 lambda: lib.ga_set_tiles(r._h, 0, 3), lambda: lib.ga_set_graph_block(r._h, 10 ** 6),
                 lambda: lib.ga_async_taken(r._h, None)):
        assert call() != 0
    r.close()
    print("single runs ok", flush=True)


def batched(gens=2000):
    cfgs = batched_configs()
    runs = [host_run(c) for c in cfgs]
    h = P()
    check(lib.ga_batch_create(None, ctypes.byref(h)))
    for r in runs:
        check(lib.ga_batch_add(h, r._h, gens + 100))
    classes = sorted({class_of(c) for c in cfgs})
    for wpg in (2, 4, 8, 16):
        check(lib.ga_batch_set_launch(h, 0, wpg))
        check(lib.ga_batch_step(h, 100))
    for (l, w) in classes:
        for ipw in batch_candidates(l):
            check(lib.ga_batch_set_class_launch(h, l, w, ipw))
            check(lib.ga_batch_step(h, 100))
    check(lib.ga_batch_set_graph_block(h, 64))
    check(lib.ga_batch_step(h, 1000))
    # membership churn between steps, settled queries, then the rest
    for i, r in enumerate(runs[::3]):
        check(lib.ga_batch_remove(h, r._h))
        check(lib.ga_batch_add(h, r._h, 50 + i))
    s = ctypes.c_int()
    for _ in range(12):
        check(lib.ga_batch_step(h, 30))
        for r in runs:
            check(lib.ga_batch_settled(h, r._h, ctypes.byref(s)))
    check(lib.ga_batch_step(h, gens))
    lib.ga_batch_destroy(h)
    for r in runs:
        r.close()
    print("batched ok", flush=True)


class HostPool(GAPool):
    """GAPool over a host buffer."""

    def __init__(self, budget, slots):
        self.mem = aligned(budget)
        h = P()
        check(lib.ga_pool_create(P(self.mem.ctypes.data), budget, slots, None, ctypes.byref(h)))
        self._h = h
        self.budget = budget
        self._shape = {}


def served(n=300, budget=1 << 30):
    reqs = served_requests(n, rate=1.0)
    # every request at once, in order: admission churn against a small pool
    arrivals = [(0.0, c, g) for t, c, g in reqs]

    def sb(cfg):
        return lib.ga_state_bytes(ctypes.byref(make_config(_fields(cfg))))
    shapes = {"waves_per_group": 2, (3, 1): 16, (5, 2): 8, (6, 1): 16}
    srv = Server(budget, max_slots=64, block=100, make_pool=HostPool, state_bytes=sb, shapes=shapes)
    done = srv.drain(arrivals)
    srv.close()
    assert len(done) == n
    print("served ok", len(done), flush=True)


def relatedness():
    rng = np.random.default_rng(1)
    for n in (1, 2, 65, 300):
        T = rng.integers(0, 1 << 20, n, dtype=np.uint32)
        D = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
        L = np.empty((n, n), np.uint32)
        U = np.empty((n, n), np.uint32)
        ws = aligned(max(1, lib.ga_mrca_workspace_bytes(n)))
        check(lib.ga_mrca_matrix(P(T.ctypes.data), P(D.ctypes.data), n, 64, 5, P(ws.ctypes.data),
                                 ws.size, P(L.ctypes.data), P(U.ctypes.data), None))
        check(lib.ga_mrca_matrix_noalloc(P(T.ctypes.data), P(D.ctypes.data), n, 64, 1, 0, 5,
                                         P(L.ctypes.data), P(U.ctypes.data), None))
    print("relatedness ok", flush=True)


if __name__ == "__main__":
    single_runs()
    batched()
    served()
    relatedness()
