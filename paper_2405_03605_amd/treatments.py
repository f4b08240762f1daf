"""The paper's treatment comparison (Sec. 3, Fig. 2a): purifying-only versus
adaptation-enabled runs with tournament size 5, one genome sampled per island
at the end, phylogenies reconstructed from (up to) 10k sampled surfaces, and
sum branch length and mean evolutionary distinctiveness compared. The paper
reports larger values for purifying-only runs, the branch-length effect
particularly strong.

    python -m paper_2405_03605_amd.treatments --width 100 --height 100 --gens 1000000
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import phylo
from .run import GARun
from .workloads import ADAPTIVE, PURIFYING, run_config


def one_run(treatment: str, width: int, height: int, gens: int, sites: int, samples: int,
            replicate: int, torch) -> dict:
    law = PURIFYING if treatment == "purifying" else ADAPTIVE
    cfg = run_config(width=width, height=height, pop=32, sites=sites, seed=2024 + replicate,
                     run_id=(0 if treatment == "purifying" else 1000) + replicate, **law)
    run = GARun(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(gens)
    torch.cuda.synchronize()
    sim_s = time.perf_counter() - t0
    ids, T, D = run.extract()          # one genome per island
    f = run.read(outbox=False)["f"]
    run.close()
    if ids.size > samples:
        pick = np.sort(np.random.default_rng(replicate).choice(ids.size, samples, replace=False))
        ids, T, D = ids[pick], T[pick], D[pick]
    t0 = time.perf_counter()
    Z, m = phylo.reconstruct(T, D, sites)
    m.update({"treatment": treatment, "replicate": replicate, "gens": gens,
              "agents": run.agents, "sim_s": sim_s, "reconstruct_s": time.perf_counter() - t0,
              "mean_fitness": float(f.mean()), "T_min": int(T.min()), "T_max": int(T.max())})
    return m


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--width", type=int, default=100)
    ap.add_argument("--height", type=int, default=100)
    ap.add_argument("--gens", type=int, default=1000000)
    ap.add_argument("--sites", type=int, default=64)
    ap.add_argument("--samples", type=int, default=10000)
    ap.add_argument("--replicates", type=int, default=4)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    rows = []
    for rep in range(args.replicates):
        for treatment in ("purifying", "adaptive"):
            m = one_run(treatment, args.width, args.height, args.gens, args.sites, args.samples,
                        rep, torch)
            rows.append(m)
            print(json.dumps(m), flush=True)
    summary = {}
    for key in ("sum_branch_length", "mean_evolutionary_distinctiveness"):
        p = [r[key] for r in rows if r["treatment"] == "purifying"]
        a = [r[key] for r in rows if r["treatment"] == "adaptive"]
        summary[key] = {"purifying_mean": float(np.mean(p)), "adaptive_mean": float(np.mean(a)),
                        "purifying_greater_in_every_pair": bool(all(x > y for x, y in zip(p, a)))}
    print(json.dumps({"summary": summary, "config": vars(args)}), flush=True)


if __name__ == "__main__":
    main()
