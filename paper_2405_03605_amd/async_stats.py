"""Statistical comparison of the asynchronous schedule (Sec. 2 Methods: islands
exchange genomes through per-neighbour buffers with no global step) against the
synchronous one. The free-running schedule is a different random process (a
genome can arrive late or be overwritten unread), so it is judged by effect
size over replicates: for mean fitness and two phylometrics of the tree
reconstructed from one agent per island (Sec. 3, Fig. 2: sum branch length,
mean evolutionary distinctiveness), the shift from the synchronous mean must
be at most a quarter of what migration itself changes (synchronous against a
no-migration control), or within three standard errors.

  python -m paper_2405_03605_amd.async_stats --out profiles/async_statistics.json
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import phylo
from ._lib import ASYNC_UNPACED
from .run import GARun
from .workloads import run_config

CFG = dict(width=64, height=64, pop=32, sites=64, k=5, p32=429496729)
GENS = 1500
REPS = 10
CONTROL_REPS = 4
METRICS = ("mean_fitness", "sum_branch_length", "mean_evolutionary_distinctiveness")
SEEDS = {"sync": 1000, "lead2": 2000, "unpaced": 3000, "control": 900}


def replicate(kind: str, r: int) -> dict:
    """One replicate: kind is "sync", "lead2", "unpaced" or "control"."""
    seed = SEEDS[kind] + r
    schedule = 1 if kind in ("lead2", "unpaced") else 0
    cfg = run_config(schedule=schedule, migration=0 if kind == "control" else 1, seed=seed,
                     run_id=seed * 7, **CFG)
    run = GARun(cfg)
    if schedule:
        run.set_async(0, 2 if kind == "lead2" else ASYNC_UNPACED)
    run.step(GENS)
    f = run.read(outbox=False)["f"]
    out = {"mean_fitness": float(f.mean())}
    if schedule:
        islands = CFG["width"] * CFG["height"]
        # every island sends one genome per generation; those of the last
        # generation are still in flight
        out["lost"] = 1.0 - run.async_taken() / (islands * (GENS - 1))
        age = GENS - 1 - run.async_last_taken()
        out["last_taken_age_p50_p99_max"] = [float(np.percentile(age, 50)),
                                             float(np.percentile(age, 99)), int(age.max())]
        out["waits_given_up"] = run.async_waits()
    ids, T, D = run.extract()
    run.close()
    _, m = phylo.reconstruct(T, D, CFG["sites"])
    out["sum_branch_length"] = m["sum_branch_length"]
    out["mean_evolutionary_distinctiveness"] = m["mean_evolutionary_distinctiveness"]
    return out


def judge(sync: list, other: list, control: list) -> dict:
    """Per metric: shift, migration effect, Welch SE, KS p and the verdict."""
    from scipy import stats
    res = {}
    for key in METRICS:
        a = np.array([x[key] for x in sync])
        b = np.array([x[key] for x in other])
        c = float(np.mean([x[key] for x in control]))
        d = abs(b.mean() - a.mean())
        effect = abs(a.mean() - c)
        se = float(np.sqrt(a.var(ddof=1) / a.size + b.var(ddof=1) / b.size))
        res[key] = {"sync_mean": float(a.mean()), "sync_sd": float(a.std(ddof=1)),
                    "async_mean": float(b.mean()), "async_sd": float(b.std(ddof=1)),
                    "control_mean": c, "shift": float(d), "migration_effect": float(effect),
                    "shift_over_effect": float(d / effect) if effect else None,
                    "shift_over_se": float(d / se) if se else None,
                    "ks_p": float(stats.ks_2samp(a, b).pvalue),
                    "pass": bool(d <= 0.25 * effect or d <= 3 * se)}
    return res


def summary(reps: dict) -> dict:
    out = {"workload": "64x64 islands x 32 agents, 64-site surface, tournament 5, p = 0.1, "
                       f"{GENS} generations",
           "replicates": {k: len(v) for k, v in reps.items()},
           "rule": "pass on a metric if |mean(async) - mean(sync)| <= 0.25 |mean(sync) - "
                   "mean(control)| or <= 3 Welch SE"}
    for kind in ("lead2", "unpaced"):
        j = judge(reps["sync"], reps[kind], reps["control"])
        out[kind] = {"metrics": j, "pass": all(v["pass"] for v in j.values()),
                     "lost_mean": float(np.mean([x["lost"] for x in reps[kind]])),
                     "last_taken_age_p50_p99_max": reps[kind][0]["last_taken_age_p50_p99_max"],
                     "waits_given_up": int(sum(x["waits_given_up"] for x in reps[kind]))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("async_stats needs an MI355X GPU")
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    reps = {}
    for kind, n in (("sync", REPS), ("control", CONTROL_REPS), ("lead2", REPS), ("unpaced", REPS)):
        reps[kind] = []
        for r in range(n):
            reps[kind].append(replicate(kind, r))
        print(f"[async_stats {time.perf_counter() - t0:.0f}s] {kind}: {n} replicates", flush=True)
    out = summary(reps)
    out["per_replicate"] = reps
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "per_replicate"}), flush=True)


if __name__ == "__main__":
    main()
