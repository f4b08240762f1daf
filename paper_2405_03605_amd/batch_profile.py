"""Short batched-form runs with HIP graphs off, so that a profiler's counters
see one dispatch per generation (workload of the batched form: 64 uneven runs
advanced together, one launch per generation).

  python -m paper_2405_03605_amd.batch_profile              # the 64-run workload, 12 generations
  python -m paper_2405_03605_amd.batch_profile --single     # one 1024x256x32 run: plain, then batched
"""
from __future__ import annotations

import argparse

from ._lib import FORM_STREAMING
from .run import GABatch, GARun
from .workloads import batched_configs, run_config


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gens", type=int, default=12)
    ap.add_argument("--single", action="store_true",
                    help="one 1024x256x32 run through the plain kernel, then as a one-member batch")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("batch_profile needs an MI355X GPU")
    torch.cuda.set_device(0)
    if args.single:
        cfg = run_config(width=1024, height=256, pop=32, sites=32, seed=1)
        run = GARun(cfg)
        run.set_launch(16, 4, FORM_STREAMING)
        run.set_graph_block(0)
        run.step(args.gens)
        torch.cuda.synchronize()
        run.close()
        runs = [GARun(cfg)]
    else:
        runs = [GARun(c) for c in batched_configs()]
    batch = GABatch()
    for r in runs:
        batch.add(r, 10 ** 6)
    batch.set_graph_block(0)
    batch.step(args.gens)
    torch.cuda.synchronize()
    batch.close()
    for r in runs:
        r.close()
    print(f"batched: {len(runs)} runs x {args.gens} generations", flush=True)


if __name__ == "__main__":
    main()
