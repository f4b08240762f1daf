"""Benchmark: agent-generations per second of the island-model GA generation
step on one MI355X, at 16.8M agents (1024 x 512 islands x 32 agents, 32-site
surfaces, tournament 2, mutation p = 0.1), plus batched vs plain throughput on
64 uneven runs, the served stream, and the LDS-resident tile form on one GPU's
256 x 256 tile.

A step is one generation of the whole population: absorb, emit, evaluate,
tournament, copy, mutate and deposit for every island and agent. The state is
resident in HBM before timing starts. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--batched-gens G]
                  [--served-requests R] [--resident-gens G] [--no-cpu-baseline]
                  [--no-batched] [--no-resident] [--workload paper|shard]
                  [--form auto|streaming|resident] [--schedule async [--max-lead N|unpaced]]

The default is the synchronous schedule. --schedule async times the
barrier-free asynchronous schedule on the same workload instead (and adds the
freshness of the exchanged genomes to the line). --workload shard times the
256 x 256-island tile one GPU would hold if the 16.8M grid were cut over eight.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_LANE_OPS = CUS * LANES_PER_CU * CLOCK_HZ   # full-rate 32-bit VALU lane-ops/s
PROFILES = os.path.join(ROOT, "profiles")
COUNTER_FILES = {"paper-streaming": os.path.join(PROFILES, "counters_generation_kernel_paper.json"),
                 "mid-tiles": os.path.join(PROFILES, "counters_tile_kernel_mid.json"),
                 "batch": os.path.join(PROFILES, "counters_batch_all_kernel_64runs.json")}


def algorithmic_bytes_per_generation(cfg: dict) -> int:
    """HBM bytes one generation of the streaming form must move: every agent's
    genome read and written once (fitness, T, S/32 surface words), and per
    island one outbox entry written and one read (header, fitness, T, surface
    words)."""
    I = cfg["width"] * cfg["height"]
    A = I * cfg["pop"]
    genome = 8 + cfg["sites"] // 8
    return 2 * genome * A + 2 * (4 + genome) * I


def algorithmic_lane_ops_per_agent_generation(cfg: dict) -> float:
    """32-bit VALU lane operations one agent-generation needs at least, the
    work of the LDS-resident form (its memory traffic is the population once
    per launch plus the tiles' edge emissions):
      per child: one Philox4x32-10 block, 10 rounds of two 32x32->64 products
        and two three-input XORs (40); k entrant indices (k) and k-1 strict
        comparisons each selecting fitness and address (3 (k-1)); the mutation
        test, delta index, conversion and add (5); the deposit's rank test
        (4), bit insert (3) and T + 1 (1);
      per island (1/N of it per agent): the migration block (40), four arrival
        tests and slot extractions (8), the emigrant's slot and header (2)."""
    k = cfg["k"] if cfg.get("selection", 1) else 1
    child = 40 + k + 3 * (k - 1) + 5 + 8
    island = 40 + 8 + 2
    return child + island / cfg["pop"]


def counter_record(mode: str, tiles=None):
    """The committed counter record of a kernel, or None if its sources have
    changed since the counters were taken (or, for a tile kernel, they were
    taken on another tiling)."""
    from paper_2405_03605_amd.counters import source_hash
    try:
        with open(COUNTER_FILES[mode]) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != source_hash(mode):
        return None
    if tiles is not None and rec.get("tiles") != f"{tiles[0]}x{tiles[1]}":
        return None
    return rec


def progress(msg: str):
    """One progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _timed(run, steps, warmup, torch):
    """Wall time and HIP-event time (on the launch stream) of `steps`
    generations after `warmup` untimed ones."""
    stream = torch.cuda.current_stream()
    run.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    run.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ev0.elapsed_time(ev1)


def bench_single(args, torch):
    from paper_2405_03605_amd import FORM_AUTO, FORM_RESIDENT, FORM_STREAMING, GARun
    from paper_2405_03605_amd.workloads import MID, PAPER

    cfg = dict(PAPER if args.workload == "paper" else MID)
    if args.schedule == "async":
        cfg["schedule"] = 1
    run = GARun(cfg)
    form = {"auto": FORM_AUTO, "streaming": FORM_STREAMING, "resident": FORM_RESIDENT}[args.form]
    if args.ipw or args.wpg or form:
        run.set_launch(args.ipw, args.wpg, form)
    if args.schedule == "async":
        run.set_async(0, args.max_lead)
    if args.graph_block is not None:
        run.set_graph_block(args.graph_block)
    tiles = run.tiles() if args.schedule == "sync" else (0, 0, 0)
    wall, ev_ms = _timed(run, args.steps, args.warmup, torch)
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
    return cfg, wall, ev_ms, extra, tiles


def roofline_streaming(cfg, us_per_gen, counters):
    bytes_gen = algorithmic_bytes_per_generation(cfg)
    achieved = bytes_gen / (us_per_gen * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": counters["bytes_per_generation"] if counters else None,
            "valu_issue_frac": counters["valu_issue_frac"] if counters else None,
            "kernel": "generation_kernel<5,1,FitnessModel,false>", "bytes_per_launch": bytes_gen,
            "launch_us": round(us_per_gen, 2)}


def roofline_tiles(cfg, us_per_gen, counters, tiles):
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    ops = algorithmic_lane_ops_per_agent_generation(cfg)
    achieved = ops * agents / (us_per_gen * 1e-6) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2),
            "unit": "T lane-op/s", "frac": round(achieved / peak, 4),
            "traffic": counters["bytes_per_generation"] if counters else None,
            "valu_issue_frac": counters["valu_issue_frac"] if counters else None,
            "kernel": "tile_kernel<5,1,FitnessModel,false>",
            "lane_ops_per_agent_generation": round(ops, 2),
            "tiles": {"tile_w": tiles[0], "tile_h": tiles[1], "count": tiles[2]},
            "us_per_generation": round(us_per_gen, 2)}


def bench_resident(gens: int, torch):
    """The 256 x 256 x 32 workload (one GPU's tile of the 16.8M grid) in the
    LDS-resident tile form against the per-generation streaming form."""
    from paper_2405_03605_amd import FORM_RESIDENT, FORM_STREAMING, GARun
    from paper_2405_03605_amd.workloads import MID

    agents = MID["width"] * MID["height"] * MID["pop"]
    out = {"workload": "256x256 islands x 32 agents (2.1M), 32-site surface, tournament 2",
           "generations": gens}
    from paper_2405_03605_amd.autotune import autotune
    choice = autotune(MID, forms=(FORM_RESIDENT,))
    for name, form in (("resident", FORM_RESIDENT), ("streaming", FORM_STREAMING)):
        run = GARun(MID)
        run.set_launch(form=form)
        if form == FORM_RESIDENT:
            run.set_tiles(choice[0], choice[1])      # the autotuner's tiling
        tiles = run.tiles()
        wall, ev_ms = _timed(run, gens, 100, torch)
        run.close()
        us = ev_ms * 1e3 / gens
        out[f"{name}_agent_gens_per_s"] = agents * gens / wall
        out[f"{name}_us_per_generation"] = round(us, 3)
        if name == "resident":
            out["roofline"] = roofline_tiles(MID, us, counter_record("mid-tiles", tiles), tiles)
        else:
            out["streaming_hbm_frac"] = round(
                algorithmic_bytes_per_generation(MID) / (us * 1e-6) / 1e9 / PEAK_HBM_GBPS, 4)
    out["speedup"] = out["resident_agent_gens_per_s"] / out["streaming_agent_gens_per_s"]
    return out


def bench_batched(gens: int, torch, tune: bool = True):
    from paper_2405_03605_amd import GABatch, GARun
    from paper_2405_03605_amd.workloads import batched_configs

    cfgs = batched_configs()
    agents = sum(c["width"] * c["height"] * c["pop"] for c in cfgs)
    progress(f"batched leg: 64 runs alone, {gens} generations each")
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
    # batched: one launch per generation over every member's islands in
    # 100-generation graph blocks, launch shape chosen by the autotuner (timed
    # on scratch runs of the same shapes before the timed region)
    from paper_2405_03605_amd.autotune import autotune_batch
    progress(f"batched leg: plain {agents * gens / plain:.3e} agent-gen/s; autotuning the batch")
    runs = [GARun(c) for c in cfgs]
    batch = GABatch()
    for r in runs:
        batch.add(r, gens + 100)
    chosen = autotune_batch(batch, cfgs) if tune else dict(
        {k: batch.class_launch(*k)[0] for k in batch.classes()}, waves_per_group=4)
    progress(f"batched leg: shapes {chosen}; timing {gens} generations")
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
    counters = counter_record("batch")
    shapes = shape_names(chosen)
    return chosen, {"runs": len(cfgs), "agents": agents, "generations": gens,
            "plain_form": "each run alone in the library's default form (LDS-resident tiles "
                          "where it fits, else streaming)",
            "autotuned_shapes": shapes,
            "batched_agent_gens_per_s": agents * gens / batched,
            "plain_agent_gens_per_s": agents * gens / plain,
            "speedup": plain / batched,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                         "bytes_per_generation": bytes_gen,
                         "traffic": counters["bytes_per_generation"] if counters else None,
                         "valu_issue_frac": counters["valu_issue_frac"] if counters else None,
                         "kernel": "batch_all_kernel"}}


def shape_names(chosen: dict) -> dict:
    """autotune_batch's choice with readable class names."""
    out = {"waves_per_group": chosen["waves_per_group"]}
    out.update({f"N={1 << k[0]},words={k[1]}": {"islands_per_wave": v}
                for k, v in sorted((k, v) for k, v in chosen.items() if k != "waves_per_group")})
    return out


def bench_served(n_requests: int, capacity: float, torch, tune: bool = True):
    """The served workload's Poisson stream (its first n_requests requests) at
    80% of the measured batched capacity, full free HBM as budget, the pool's
    launch shape chosen by the autotuner on a batch of the stream's first 64
    requests (the served mix, not the batched one)."""
    import numpy as np

    from paper_2405_03605_amd.serve import Server
    from paper_2405_03605_amd.workloads import served_requests

    reqs = served_requests(n_requests, rate=1.0)
    mean_work = float(np.mean([c["width"] * c["height"] * c["pop"] * g for _, c, g in reqs]))
    rate = 0.8 * capacity / mean_work
    arrivals = [(t / rate, c, g) for t, c, g in reqs]
    free, _ = torch.cuda.mem_get_info()
    budget = int(free - 8e9)
    shapes = None
    if tune:
        from paper_2405_03605_amd.autotune import autotune_batch

        class _Keep:      # collects the choice; the server applies it to its pool
            def set_launch(self, ipw, wpg):
                pass

            def set_class_launch(self, log2n, words, ipw):
                pass
        shapes = autotune_batch(_Keep(), [c for _, c, _ in reqs[:64]])
        progress(f"served leg: shapes {shapes}")
    srv = Server(budget, max_slots=256, block=100, shapes=shapes)
    progress(f"served leg: {n_requests} requests at {rate:.2f}/s")

    def report(server, elapsed):
        progress(f"served leg: {elapsed:.0f} s, done {len(server.done)}, live "
                 f"{len(server.live)}, waiting {len(server.waiting)}")

    t0 = time.perf_counter()
    srv.drain(arrivals, progress=report, progress_every=10.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = srv.report(wall)
    srv.close()
    rep.update({"requests": n_requests, "rate_per_s": rate, "budget_bytes": budget,
                "mean_work_agent_gens": mean_work})
    if shapes:
        rep["autotuned_shapes"] = shape_names(shapes)
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
    ap.add_argument("--batched-gens", type=int, default=20000,
                    help="generations of the 64-run batched workload (its full length)")
    ap.add_argument("--resident-gens", type=int, default=2000,
                    help="generations of the 256x256 tile in each form (0 skips that leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="batched leg: the default launch shape of every class")
    ap.add_argument("--no-resident", action="store_true")
    ap.add_argument("--served-requests", type=int, default=2000,
                    help="requests of the served stream to run (0 skips the served leg)")
    ap.add_argument("--ipw", type=int, default=0, help="islands per wavefront (0: library default)")
    ap.add_argument("--wpg", type=int, default=0, help="wavefronts per workgroup (0: default)")
    ap.add_argument("--graph-block", type=int, default=None,
                    help="generations per HIP graph replay (default 100; 0 disables)")
    ap.add_argument("--workload", choices=("paper", "shard"), default="paper",
                    help="paper: 1024x512 islands x 32 (16.8M agents); shard: 256x256 x 32 "
                         "(2.1M agents), one GPU's tile of the paper grid cut 4 x 2")
    ap.add_argument("--form", choices=("auto", "streaming", "resident"), default="auto",
                    help="launch form of the main line (auto: resident when the run fits LDS)")
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

    progress(f"main line: {args.workload} workload, {args.steps} generations")
    cfg, wall, ev_ms, async_info, tiles = bench_single(args, torch)
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    value = agents * args.steps / wall
    us_per_gen = ev_ms * 1e3 / args.steps
    if async_info is not None:
        roofline = roofline_streaming(cfg, us_per_gen, None)
        kernel = "lockstep_kernel<5,1>" if args.max_lead == 0 else "async_kernel<5,1>"
        roofline.update({"kernel": kernel, "bytes_per_launch": None,
                         "bytes_per_generation": roofline["bytes_per_launch"],
                         "launch_us": None, "us_per_generation": round(us_per_gen, 2)})
    elif tiles[2]:
        mode = "mid-tiles" if args.workload == "shard" else None
        roofline = roofline_tiles(cfg, us_per_gen, counter_record(mode, tiles) if mode else None,
                                  tiles)
    else:
        mode = "paper-streaming" if args.workload == "paper" else None
        roofline = roofline_streaming(cfg, us_per_gen, counter_record(mode) if mode else None)
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
                      "step": "one generation", "schedule": args.schedule,
                      "form": "resident" if tiles[2] else "streaming"},
           "roofline": roofline}
    if async_info is not None:
        out["async"] = async_info
    if not args.no_resident and args.resident_gens > 0:
        progress("resident leg: 256x256x32, tiles and streaming")
        out["resident"] = bench_resident(args.resident_gens, torch)
    if not args.no_batched:
        _, out["batched"] = bench_batched(args.batched_gens, torch,
                                          tune=not args.no_batch_autotune)
        if args.served_requests > 0:
            out["served"] = bench_served(args.served_requests,
                                         out["batched"]["batched_agent_gens_per_s"], torch,
                                         tune=not args.no_batch_autotune)
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
