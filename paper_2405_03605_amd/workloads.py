"""Seeded synthetic workloads (run configurations) shared by the tests, the
benchmark and the serving loop. Inputs only: this module holds none of the
method's arithmetic.

Run configurations use the fields width, height, pop (agents per island),
sites (surface size), k (tournament size), selection (1 tournament, 0 neutral),
p32 (mutation probability times 2^32), migration (0/1), seed, run_id.
"""
from __future__ import annotations

import math

import numpy as np

P10 = 429496729  # floor(0.1 * 2^32): mutation probability 0.1


def run_config(**kw) -> dict:
    base = dict(width=8, height=8, pop=32, sites=64, k=2, selection=1, p32=P10, migration=1,
                seed=1, run_id=0)
    base.update(kw)
    return base


# The three plain workloads: 8x8x32 with 64-site surfaces (1,000 generations),
# 256x256x32 with 32-site surfaces (10,000 generations, selection on and off),
# and the 16.8M-agent 1024x512x32 grid with 32-site surfaces (100,000 generations).
TINY = run_config(width=8, height=8, pop=32, sites=64)
TINY_GENS = 1000
MID = run_config(width=256, height=256, pop=32, sites=32)
MID_NEUTRAL = run_config(width=256, height=256, pop=32, sites=32, selection=0, run_id=1)
MID_GENS = 10000
PAPER = run_config(width=1024, height=512, pop=32, sites=32)
PAPER_GENS = 100000


# The paper's two treatments (Sec. 3), tournament size 5: purifying-only (33%
# of replications lose a normally distributed amount) and adaptation-enabled
# (additionally 0.3% gain one).
P33 = 1417339207   # floor(0.33 * 2^32)
P003 = 12884901    # floor(0.003 * 2^32)
PURIFYING = dict(k=5, law=1, p32=P33, p_ben32=0)
ADAPTIVE = dict(k=5, law=1, p32=P33, p_ben32=P003)


def batched_configs(n_runs: int = 64, seed: int = 20240503) -> list[dict]:
    """64 uneven runs: grids log-uniform 16..256 x 16..128, agents per island
    uniform over {8,16,32,64}, 32 or 64 sites, tournament 2..8, selection on or
    off with equal odds, mutation p = 0.1, seed 1 and run_id 0..63."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_runs):
        W = int(round(math.exp(rng.uniform(math.log(16), math.log(256)))))
        H = int(round(math.exp(rng.uniform(math.log(16), math.log(128)))))
        out.append(run_config(width=W, height=H, pop=int(rng.choice([8, 16, 32, 64])),
                              sites=int(rng.choice([32, 64])), k=int(rng.integers(2, 9)),
                              selection=int(rng.integers(0, 2)), seed=1, run_id=r))
    return out


BATCHED_GENS = 20000


def served_requests(n: int = 2000, seed: int = 20240504, rate: float = 10.0):
    """Poisson request stream: agents per run log-uniform 1e3..4e6, N uniform
    over {8,16,32,64}, islands = agents / N laid out near-square, generation
    budgets log-uniform 1e3..1e5; other parameters as in the batched workload.
    Returns a list of (arrival_time_s, config, generations)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n):
        t += rng.exponential(1.0 / rate)
        agents = math.exp(rng.uniform(math.log(1e3), math.log(4e6)))
        N = int(rng.choice([8, 16, 32, 64]))
        islands = max(1, int(round(agents / N)))
        W = int(math.ceil(math.sqrt(islands)))
        H = max(1, int(round(islands / W)))
        gens = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e5)))))
        cfg = run_config(width=W, height=H, pop=N, sites=int(rng.choice([32, 64])),
                         k=int(rng.integers(2, 9)), selection=int(rng.integers(0, 2)),
                         seed=1, run_id=1000 + r)
        reqs.append((t, cfg, gens))
    return reqs
