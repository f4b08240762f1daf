"""Benchmark: agent-generations per second of the island-model GA generation
step on one MI355X, at 16.8M agents (1024 x 512 islands x 32 agents, 32-site
surfaces, tournament 2, mutation p = 0.1), plus batched vs plain throughput on
64 uneven runs.

A step is one generation of the whole population: absorb, emit, evaluate,
tournament, copy, mutate and deposit for every island and agent. The state is
resident in HBM before timing starts. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--batched-gens G]
                  [--no-cpu-baseline] [--no-batched] [--workload paper|shard]
                  [--schedule async [--max-lead N|unpaced]]

The default is the synchronous schedule. --schedule async times the
barrier-free asynchronous schedule on the same workload instead (and adds the
freshness of the exchanged genomes to the line). --workload shard times the
256 x 256-island tile one GPU would hold if the 16.8M grid were cut over eight.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_LANE_OPS = CUS * LANES_PER_CU * CLOCK_HZ   # full-rate 32-bit VALU lane-ops/s
KERNEL_SRC = os.path.join(ROOT, "paper_2405_03605_amd", "csrc", "ga_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_generation_kernel_paper.json")


def algorithmic_bytes_per_generation(cfg: dict) -> int:
    """HBM bytes one generation must move: every agent's genome read and
    written once (fitness, T, S/32 surface words), and per island one outbox
    entry written and one read (header, fitness, T, surface words)."""
    I = cfg["width"] * cfg["height"]
    A = I * cfg["pop"]
    genome = 8 + cfg["sites"] // 8
    return 2 * genome * A + 2 * (4 + genome) * I


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    if the kernel source has changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def bench_single(args, torch):
    from paper_2405_03605_amd import GARun
    from paper_2405_03605_amd.workloads import MID, PAPER

    cfg = dict(PAPER if args.workload == "paper" else MID)
    if args.schedule == "async":
        cfg["schedule"] = 1
    run = GARun(cfg)
    if args.ipw or args.wpg:
        run.set_launch(args.ipw, args.wpg)
    if args.schedule == "async":
        run.set_async(0, args.max_lead)
    if args.graph_block is not None:
        run.set_graph_block(args.graph_block)
    stream = torch.cuda.current_stream()
    run.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    run.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    gen = run.read(outbox=False)["generation"]
    assert gen == args.warmup + args.steps, (gen, args.warmup, args.steps)
    extra = None
    if args.schedule == "async":
        import numpy as np
        age = gen - 1 - run.async_last_taken()
        extra = {"max_lead": "unpaced" if args.max_lead == 0xFFFFFFFF else args.max_lead,
                 "waits_given_up": run.async_waits(),
                 "last_taken_age_p50_p99_max": [float(np.percentile(age, 50)),
                                                float(np.percentile(age, 99)), int(age.max())]}
    run.close()
    return cfg, wall, ev_ms, extra


def bench_batched(gens: int, torch):
    from paper_2405_03605_amd import GABatch, GARun
    from paper_2405_03605_amd.workloads import batched_configs

    cfgs = batched_configs()
    agents = sum(c["width"] * c["height"] * c["pop"] for c in cfgs)
    # plain: one run per launch sequence, runs one after another
    runs = [GARun(c) for c in cfgs]
    for r in runs:
        r.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in runs:
        r.step(gens)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    for r in runs:
        r.close()
    # batched: every run in one launch per generation, 100-generation graph blocks
    runs = [GARun(c) for c in cfgs]
    batch = GABatch()
    for r in runs:
        batch.add(r, gens + 100)
    batch.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(gens)
    torch.cuda.synchronize()
    batched = time.perf_counter() - t0
    batch.close()
    for r in runs:
        r.close()
    # every member's algorithmic bytes per generation over the batched wall time
    # (graph replays and the per-block advance included)
    bytes_gen = sum(algorithmic_bytes_per_generation(c) for c in cfgs)
    achieved = bytes_gen * gens / batched / 1e9
    return {"runs": len(cfgs), "agents": agents, "generations": gens,
            "batched_agent_gens_per_s": agents * gens / batched,
            "plain_agent_gens_per_s": agents * gens / plain,
            "speedup": plain / batched,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                         "bytes_per_generation": bytes_gen,
                         "kernel": "batch_generation_kernel"}}


def bench_served(n_requests: int, capacity: float, torch):
    """The served workload's Poisson stream (its first n_requests requests) at
    80% of the measured batched capacity, full free HBM as budget."""
    import numpy as np

    from paper_2405_03605_amd.serve import Server
    from paper_2405_03605_amd.workloads import served_requests

    reqs = served_requests(n_requests, rate=1.0)
    mean_work = float(np.mean([c["width"] * c["height"] * c["pop"] * g for _, c, g in reqs]))
    rate = 0.8 * capacity / mean_work
    arrivals = [(t / rate, c, g) for t, c, g in reqs]
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - 8e9)
    srv = Server(budget, max_slots=256, block=100)
    t0 = time.perf_counter()
    srv.drain(arrivals)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = srv.report(wall)
    srv.close()
    rep.update({"requests": n_requests, "rate_per_s": rate, "budget_bytes": budget,
                "mean_work_agent_gens": mean_work})
    return rep


def cpu_baseline(cfg: dict, budget_s: float = 12.0):
    import oracle
    run = oracle.OracleRun(cfg)
    t0 = time.perf_counter()
    run.step(1)
    first = time.perf_counter() - t0
    gens = max(1, min(40, int(budget_s / max(first, 1e-3))))
    t0 = time.perf_counter()
    run.step(gens)
    dt = time.perf_counter() - t0
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    return {"value": agents * gens / dt, "unit": "agent-generations/s", "cores": 1,
            "kind": "oracle",
            "sample": f"single-threaded CPU oracle, generations 1 to {gens} (generation 0 "
                      f"untimed) of the {cfg['width']}x{cfg['height']}x{cfg['pop']} run "
                      f"({agents} agents), generation loop only, {dt:.1f} s",
            "host": host_cpu()}


def host_cpu() -> dict:
    """CPU model and logical CPU count of the machine the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--batched-gens", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--served-requests", type=int, default=150,
                    help="requests of the served stream to run (0 skips the served leg)")
    ap.add_argument("--ipw", type=int, default=0, help="islands per wavefront (0: library default)")
    ap.add_argument("--wpg", type=int, default=0, help="wavefronts per workgroup (0: default)")
    ap.add_argument("--graph-block", type=int, default=None,
                    help="generations per HIP graph replay (default 100; 0 disables)")
    ap.add_argument("--workload", choices=("paper", "shard"), default="paper",
                    help="paper: 1024x512 islands x 32 (16.8M agents); shard: 256x256 x 32 "
                         "(2.1M agents), one GPU's tile of the paper grid cut 4 x 2")
    ap.add_argument("--schedule", choices=("sync", "async"), default="sync")
    ap.add_argument("--max-lead", default="0",
                    help="async: generations an island may lead a neighbour, or 'unpaced'")
    args = ap.parse_args()
    args.max_lead = 0xFFFFFFFF if args.max_lead == "unpaced" else int(args.max_lead)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the island grid "
              "would shard as 2D tiles with a per-generation halo exchange, which is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    cfg, wall, ev_ms, async_info = bench_single(args, torch)
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    value = agents * args.steps / wall
    kernel_s = ev_ms * 1e-3 / args.steps
    bytes_gen = algorithmic_bytes_per_generation(cfg)
    achieved = bytes_gen / kernel_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                "traffic": measured_traffic() if args.workload == "paper" else None,
                "kernel": "generation_kernel<5,1>", "bytes_per_launch": bytes_gen,
                "launch_us": round(kernel_s * 1e6, 2)}
    if async_info is not None:
        # one persistent launch covers many generations: per-generation figures
        kernel = "lockstep_kernel<5,1>" if args.max_lead == 0 else "async_kernel<5,1>"
        roofline.update({"kernel": kernel, "traffic": None,
                         "bytes_per_launch": None, "bytes_per_generation": bytes_gen,
                         "launch_us": None, "us_per_generation": round(kernel_s * 1e6, 2)})
    shape = (f"{cfg['width']}x{cfg['height']} islands x {cfg['pop']} agents "
             f"({agents / 1e6:.1f}M)")
    metric = ("agent-generations/sec at 16.8M agents; batched vs plain throughput"
              if args.workload == "paper" else
              "agent-generations/sec at 2.1M agents (one GPU's 256x256 tile of the 16.8M grid)")
    out = {"metric": metric,
           "value": value, "unit": "agent-generations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"island GA {shape}, 32-site surface, tournament 2, "
                                  "mutation p=0.1, migration 1/island/gen",
                      "islands": cfg["width"] * cfg["height"], "agents": agents,
                      "step": "one generation", "schedule": args.schedule},
           "roofline": roofline}
    if async_info is not None:
        out["async"] = async_info
    if not args.no_batched:
        out["batched"] = bench_batched(args.batched_gens, torch)
        if args.served_requests > 0:
            out["served"] = bench_served(args.served_requests,
                                         out["batched"]["batched_agent_gens_per_s"], torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
