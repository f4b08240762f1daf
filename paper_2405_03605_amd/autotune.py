"""Launch-shape autotuner: islands per wavefront, wavefronts per workgroup and
launch form for a run shape, chosen by timing a scratch run of the same shape.

Every candidate computes the same bits (the RNG is keyed by island, generation
and slot, never by the launch shape), so the choice only moves time.
"""
from __future__ import annotations

import time

from ._lib import FORM_RESIDENT, FORM_STREAMING
from .run import GARun

SHAPE_FIELDS = ("width", "height", "pop", "sites", "k", "selection", "migration")
_cache: dict = {}


def shape_key(cfg: dict) -> tuple:
    return tuple(int(cfg[f]) for f in SHAPE_FIELDS)


def candidates(cfg: dict) -> list[tuple[int, int, int]]:
    """(islands_per_wave, waves_per_group, form) candidates for a run shape."""
    per_iter = 64 // cfg["pop"]
    islands = cfg["width"] * cfg["height"]
    out = []
    ipw = per_iter
    while ipw <= 64:
        for wpg in (1, 2, 4, 8):
            out.append((ipw, wpg, FORM_STREAMING))
        ipw *= 2
    # resident: one workgroup, only for runs that fit 16 wavefronts
    res_ipw = max(per_iter, -(-islands // 16))
    res_ipw = -(-res_ipw // per_iter) * per_iter
    if res_ipw <= 64 and -(-islands // res_ipw) <= 16:
        out.append((0, 0, FORM_RESIDENT))
    return out


def time_candidate(run: GARun, cand, gens: int, torch) -> float:
    ipw, wpg, form = cand
    run.set_launch(ipw, wpg, form)
    run.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.step(gens)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / gens


def autotune(cfg: dict, gens: int | None = None, use_cache: bool = True):
    """Fastest (islands_per_wave, waves_per_group, form) for cfg's shape."""
    import torch
    key = shape_key(cfg)
    if use_cache and key in _cache:
        return _cache[key]
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    if gens is None:
        gens = max(4, min(200, int(2e8 // max(agents, 1))))
    scratch = GARun(dict(cfg, seed=0x5eed, run_id=0xA070))
    best, best_t = None, float("inf")
    for cand in candidates(cfg):
        t = time_candidate(scratch, cand, gens, torch)
        if t < best_t:
            best, best_t = cand, t
    scratch.close()
    _cache[key] = best
    return best


def apply(run: GARun, choice):
    ipw, wpg, form = choice
    run.set_launch(ipw, wpg, form)
