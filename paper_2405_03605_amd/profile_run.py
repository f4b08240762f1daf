"""Short runs with a fixed number of generations per kernel launch, so that a
profiler's per-dispatch counters compare across dispatches (graphs off).

  python -m paper_2405_03605_amd.profile_run paper-streaming   # 16.8M agents, one launch per generation
  python -m paper_2405_03605_amd.profile_run mid-tiles         # 256x256x32, LDS-resident tiles
  python -m paper_2405_03605_amd.profile_run mid-streaming     # 256x256x32, one launch per generation
  python -m paper_2405_03605_amd.profile_run batch             # the 64-run batched workload
  python -m paper_2405_03605_amd.profile_run batch-single      # one 1024x256x32 run, plain then batched
  python -m paper_2405_03605_amd.profile_run batch-classes     # per class: one run plain, then batched

--gens is the generations per dispatch for mid-tiles (default 200) and the
dispatch count otherwise (default 12); --launches the tile launches (default 4);
--tiles WxH the tile shape of mid-tiles.
"""
from __future__ import annotations

import argparse

from ._lib import FORM_RESIDENT, FORM_STREAMING
from .run import GABatch, GARun
from .workloads import MID, PAPER, batched_configs, run_config

MODES = ("paper-streaming", "mid-tiles", "mid-streaming", "batch", "batch-single", "batch-classes")

# One run per batch class (log2 N, surface words) of the batched workload,
# 256 x 128 islands each, for the per-class instruction counts.
CLASS_RUNS = [(l, w) for l in (3, 4, 5, 6) for w in (1, 2)]


def class_config(log2n: int, words: int) -> dict:
    return run_config(width=256, height=128, pop=1 << log2n, sites=32 * words, seed=1)


def _streaming(cfg, gens, torch, ipw=0, wpg=0):
    run = GARun(cfg)
    run.set_launch(ipw, wpg, FORM_STREAMING)
    run.set_graph_block(0)
    run.step(gens)
    torch.cuda.synchronize()
    run.close()


def _batch(runs, gens, torch):
    batch = GABatch()
    for r in runs:
        batch.add(r, 10 ** 6)
    batch.set_graph_block(0)
    batch.step(gens)
    torch.cuda.synchronize()
    batch.close()
    for r in runs:
        r.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=MODES)
    ap.add_argument("--gens", type=int, default=None)
    ap.add_argument("--launches", type=int, default=4)
    ap.add_argument("--tiles", default=None, help="mid-tiles: tile shape WxH (default: the library's)")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("profile_run needs an MI355X GPU")
    torch.cuda.set_device(0)
    if args.mode == "paper-streaming":
        gens = args.gens or 12
        _streaming(PAPER, gens, torch)
    elif args.mode == "mid-streaming":
        gens = args.gens or 12
        _streaming(MID, gens, torch)
    elif args.mode == "mid-tiles":
        gens = args.gens or 200
        run = GARun(MID)
        run.set_launch(form=FORM_RESIDENT)
        if args.tiles:
            tw, th = (int(x) for x in args.tiles.split("x"))
            run.set_tiles(tw, th)
        assert run.tiles()[2] > 0
        for _ in range(args.launches):
            run.step(gens)          # one tile launch of `gens` generations each
        torch.cuda.synchronize()
        run.close()
    elif args.mode == "batch":
        gens = args.gens or 12
        _batch([GARun(c) for c in batched_configs()], gens, torch)
    elif args.mode == "batch-classes":
        # per class, in this order: `gens` plain dispatches, then `gens` batched,
        # both with the batch's default shape (512 agents per wavefront, four
        # wavefronts per group)
        gens = args.gens or 12
        for l, w in CLASS_RUNS:
            cfg = class_config(l, w)
            _streaming(cfg, gens, torch, ipw=512 >> l, wpg=4)
            _batch([GARun(cfg)], gens, torch)
    else:
        gens = args.gens or 12
        cfg = run_config(width=1024, height=256, pop=32, sites=32, seed=1)
        _streaming(cfg, gens, torch)
        _batch([GARun(cfg)], gens, torch)
    print(f"{args.mode}: {gens} generations per dispatch", flush=True)


if __name__ == "__main__":
    main()
