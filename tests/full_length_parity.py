"""Full-length parity and lineage check on one GPU (a long one-off run, not
collected by pytest).

Runs a named workload for G generations on the GPU (in the benchmark's launch
configuration) and on the CPU oracle from the same seed, compares the whole end
state bit for bit (fitness bits, T, surfaces, outbox), and optionally checks
pairwise MRCA intervals estimated from GPU-extracted surfaces against the
oracle's true lineages for a uniform sample of agents and for every agent of a
sample of islands.

    python tests/full_length_parity.py --config paper --gens 1000 --mrca-samples 4096
    python tests/full_length_parity.py --config mid --gens 10000
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2405_03605_amd import workloads  # noqa: E402

CONFIGS = {"tiny": workloads.TINY, "mid": workloads.MID, "mid_neutral": workloads.MID_NEUTRAL,
           "paper": workloads.PAPER}


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def compare(got, ref):
    f, T, D = ref.population()
    ob = ref.outbox()
    v = ob["valid"].astype(bool)
    res = {
        "generation": got["generation"] == ref.generation,
        "fitness_bits": bool(np.array_equal(got["f"].view(np.uint32), f.view(np.uint32))),
        "T": bool(np.array_equal(got["T"], T)),
        "surfaces": bool(np.array_equal(got["D"], D)),
        "outbox_valid": bool(np.array_equal(got["outbox"]["valid"], ob["valid"])),
        "outbox_genomes": bool(np.array_equal(got["outbox"]["dir"][v], ob["dir"][v])
                               and np.array_equal(got["outbox"]["f"][v].view(np.uint32),
                                                  ob["f"][v].view(np.uint32))
                               and np.array_equal(got["outbox"]["T"][v], ob["T"][v])
                               and np.array_equal(got["outbox"]["D"][v], ob["D"][v])),
    }
    res["all"] = all(res.values())
    res["T_range"] = [int(T.min()), int(T.max())]
    res["fitness_range"] = [float(f.min()), float(f.max())]
    return res


def mrca_check(run, ref, ids, sites, kc=5):
    _, T, D = run.extract(ids)
    _, T0, D0 = ref.population()
    idx = ids.astype(np.int64)
    same = bool(np.array_equal(T, T0[idx]) and np.array_equal(D, D0[idx]))
    G = ref.true_mrca_matrix(ids)
    L, U = oracle.mrca_interval_matrix(T, D, sites, kc)
    iu = np.triu_indices(len(ids), 1)
    g = np.maximum(G[iu].astype(np.int64), 0)
    Lp, Up = L[iu].astype(np.int64), U[iu].astype(np.int64)
    lo = int((g < Lp).sum())
    # per pair P(g < L) <= 2^-kc, so the rate is taken over all pairs
    return {"samples": int(len(ids)), "pairs": int(g.size), "surfaces_equal_oracle": same,
            "related_pairs": int((G[iu] > 0).sum()), "upper_bound_violations": int((g > Up).sum()),
            "lower_bound_violations": lo, "pairs_with_lower_bound": int((Lp > 0).sum()),
            "lower_violation_rate": lo / g.size, "allowed_rate": 2.0 ** -kc,
            "mean_interval_width": float((Up - Lp).mean())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=sorted(CONFIGS), required=True)
    ap.add_argument("--gens", type=int, required=True)
    ap.add_argument("--mrca-samples", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    cfg = dict(CONFIGS[args.config])

    import torch
    from paper_2405_03605_amd import GARun
    torch.cuda.set_device(0)
    log(f"gpu: {args.config} {cfg['width']}x{cfg['height']}x{cfg['pop']}, {args.gens} generations")
    run = GARun(cfg)
    t0 = time.perf_counter()
    run.step(args.gens)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    got = run.read()
    log(f"gpu done in {gpu_s:.3f} s")

    lineage = args.mrca_samples > 0
    ref = oracle.OracleRun(cfg, lineage=lineage)
    if lineage:
        ref.reserve_lineage(args.gens)
    t0 = time.perf_counter()
    done = 0
    while done < args.gens:
        n = min(args.chunk, args.gens - done)
        ref.step(n)
        done += n
        log(f"oracle generation {done}/{args.gens} ({time.perf_counter() - t0:.0f} s)")
    cpu_s = time.perf_counter() - t0
    agents = run.agents
    out = {"config": args.config, "cfg": cfg, "generations": args.gens, "agents": agents,
           "gpu_s": gpu_s, "oracle_s": cpu_s,
           "oracle_agent_gens_per_s": agents * args.gens / cpu_s,
           "parity": compare(got, ref)}
    log(f"parity {out['parity']}")
    if lineage:
        rng = np.random.default_rng(4096)
        uni = np.sort(rng.choice(agents, size=args.mrca_samples, replace=False)).astype(np.uint64)
        n_isl = max(1, args.mrca_samples // cfg["pop"])
        isl = np.sort(rng.choice(run.islands, size=n_isl, replace=False))
        clu = (isl[:, None] * cfg["pop"] + np.arange(cfg["pop"])[None, :]).ravel().astype(np.uint64)
        out["mrca_uniform"] = mrca_check(run, ref, uni, cfg["sites"])
        log(f"uniform sample {out['mrca_uniform']}")
        out["mrca_island_clustered"] = mrca_check(run, ref, clu, cfg["sites"])
        log(f"clustered sample {out['mrca_island_clustered']}")
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    ok = out["parity"]["all"] and all(
        out[k]["upper_bound_violations"] == 0 and out[k]["surfaces_equal_oracle"]
        for k in ("mrca_uniform", "mrca_island_clustered") if k in out)
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
