"""Continuous-batching server for GA runs.

Requests (a run configuration and a generation budget) arrive over time. The
server keeps every admitted run's state on the device and advances all of them
together in the batched form (one launch per generation over every member's
islands, blocks of generations replayed from a HIP graph). Between blocks it
retires runs whose budget is spent (their end-population surfaces are sampled,
one agent per island, as in the paper's Sec. 3 end-state sampling), which frees
their memory, and admits waiting requests in arrival order for as long as the
pool takes them. Each run's result is bit-identical to running it alone,
because its random stream depends only on (seed, run_id, island, generation,
slot).

Each round enqueues the next block before it retires anything, and retires
only runs whose last block has already run (their sampling waits for no
block still on the GPU), so the host's bookkeeping overlaps the GPU's work.

Memory, slots and the batch belong to the pool: by default the native run pool
(`GAPool`, ga_pool_* in the C ABI: runs sub-allocated first fit from one device
buffer of the budget's size). The pool is injected (`make_pool`), so the
arrival-order policy here can be exercised on the CPU with a stand-in.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    cfg: dict
    gens: int
    arrival: float
    admitted: float | None = None
    finished: float | None = None
    result: tuple | None = None     # (ids, T, surfaces) of the sampled end population
    footprint: int = 0


class Server:
    def __init__(self, budget_bytes: int, max_slots: int = 64, block: int = 100,
                 make_pool=None, state_bytes=None, clock=time.perf_counter, shapes=None):
        if make_pool is None or state_bytes is None:
            from .run import GAPool, state_bytes as sb
            make_pool = make_pool or GAPool
            state_bytes = state_bytes or sb
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.block = int(block)
        self._state_bytes = state_bytes
        self.pool = make_pool(self.budget, self.max_slots)
        self.pool.set_graph_block(self.block)
        if shapes:
            # the launch shape the autotuner chose for a batch of this mix
            from .autotune import apply_shapes
            apply_shapes(self.pool, shapes)
        self.clock = clock
        self.waiting: deque[Request] = deque()
        self.live: dict[int, tuple[Request, int]] = {}   # ticket -> (request, ticket)
        self.done: list[Request] = []
        self.agent_gens = 0
        self._next_id = 0

    @property
    def used(self) -> int:
        """Device bytes held by live runs."""
        return self.pool.used

    # -- requests ---------------------------------------------------------
    def submit(self, cfg: dict, gens: int, arrival: float | None = None) -> Request:
        fp = int(self._state_bytes(cfg))
        if fp <= 0:
            raise ValueError(f"invalid configuration {cfg}")
        if fp > self.budget:
            raise ValueError(f"run needs {fp} bytes, more than the whole budget {self.budget}")
        req = Request(self._next_id, dict(cfg), int(gens),
                      self.clock() if arrival is None else arrival, footprint=fp)
        self._next_id += 1
        self.waiting.append(req)
        return req

    # -- one scheduling round ---------------------------------------------
    def admit(self) -> int:
        """Admit waiting requests in arrival order while the pool takes them."""
        n = 0
        while self.waiting:
            req = self.waiting[0]
            ticket = self.pool.admit(req.cfg, req.gens)
            if ticket is None:
                break
            self.waiting.popleft()
            req.admitted = self.clock()
            self.live[ticket] = (req, ticket)
            n += 1
        return n

    def retire(self, settled: bool = False) -> int:
        """Retire runs whose generation budget is spent; sample their surfaces.
        With settled, only runs whose last generation has already run on the
        GPU: their sampling then waits for no block still running."""
        n = 0
        for ticket in (self.pool.done(settled=True) if settled else self.pool.done()):
            req, _ = self.live.pop(ticket)
            req.result = self.pool.retire(ticket)
            req.finished = self.clock()
            self.done.append(req)
            n += 1
        return n

    def advance(self):
        """One block of generations for every live run."""
        if not self.live:
            return
        for ticket, (req, _) in self.live.items():
            self.agent_gens += min(self.block, self.pool.remaining(ticket)) * (
                req.cfg["width"] * req.cfg["height"] * req.cfg["pop"])
        self.pool.step(self.block)

    def drain(self, arrivals=None, time_limit: float | None = None, progress=None,
              progress_every: float = 10.0):
        """Serve until every request is done. `arrivals` is an optional list of
        (arrival_offset_s, cfg, gens) submitted when the clock reaches them;
        `progress(server, elapsed_s)` is called about every progress_every s."""
        start = self.clock()
        next_report = progress_every
        pending = deque(sorted(arrivals or [], key=lambda a: a[0]))
        while pending or self.waiting or self.live:
            now = self.clock() - start
            if progress is not None and now >= next_report:
                progress(self, now)
                next_report = now + progress_every
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0][0] <= now:
                off, cfg, gens = pending.popleft()
                self.submit(cfg, gens, arrival=start + off)
            self.admit()
            if not self.live:
                if pending:
                    time.sleep(min(0.001, max(0.0, pending[0][0] - now)))
                continue
            if any(self.pool.remaining(t) for t in self.live):
                # the next block goes in before this round's retirements, so
                # the GPU runs it while the host samples the runs the block
                # before finished and admits the next requests
                self.advance()
                self.retire(settled=True)
            else:
                self.retire()
        return self.done

    def close(self):
        for ticket in list(self.live):
            self.live.pop(ticket)
            self.pool.retire(ticket, sample=False)
        self.pool.close()

    # -- reporting ----------------------------------------------------------
    def report(self, wall: float) -> dict:
        lat = np.array([r.finished - r.arrival for r in self.done]) if self.done else np.zeros(1)
        return {"completed": len(self.done), "waiting": len(self.waiting), "live": len(self.live),
                "agent_gens": int(self.agent_gens), "wall_s": wall,
                "agent_gens_per_s": self.agent_gens / wall if wall > 0 else 0.0,
                "latency_p50_s": float(np.percentile(lat, 50)),
                "latency_p99_s": float(np.percentile(lat, 99))}


def main():
    import argparse
    import json
    import os
    import sys

    import torch

    from .workloads import served_requests
    ap = argparse.ArgumentParser(description="serve a Poisson stream of GA run requests")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=None, help="arrivals per second (default: 80%% of capacity)")
    ap.add_argument("--budget-gb", type=float, default=None, help="HBM budget (default: free memory less 8 GB)")
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--block", type=int, default=100)
    ap.add_argument("--capacity", type=float, default=1.0e11,
                    help="batched agent-generations/s used to set the default rate")
    ap.add_argument("--time-limit", type=float, default=None)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    reqs = served_requests(args.requests, rate=1.0)
    mean_work = np.mean([c["width"] * c["height"] * c["pop"] * g for _, c, g in reqs])
    rate = args.rate or 0.8 * args.capacity / mean_work
    arrivals = [(t / rate, c, g) for t, c, g in reqs]
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * 1e9) if args.budget_gb else int(free - 8e9)
    srv = Server(budget, max_slots=args.slots, block=args.block)

    def progress(server, elapsed):
        print(f"[serve] {elapsed:.0f} s: done {len(server.done)}, live {len(server.live)}, "
              f"waiting {len(server.waiting)}, used {server.used / 1e9:.2f} GB", file=sys.stderr,
              flush=True)

    t0 = time.perf_counter()
    srv.drain(arrivals, time_limit=args.time_limit, progress=progress)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = srv.report(wall)
    rep.update({"requests": args.requests, "rate_per_s": rate, "budget_bytes": budget,
                "mean_work_agent_gens": mean_work})
    srv.close()
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
