"""Launch-shape autotuner. Every candidate computes the same bits (the RNG is
keyed by island, generation and slot, never by the launch shape), so the
choice only moves time.

Single runs: islands per wavefront and wavefronts per workgroup of the
streaming form, the LDS-resident form (its tile shapes), chosen by timing a
scratch run of the same shape.

Batches: per class of members (log2 N, surface words), the class kernel's
islands per wavefront and wavefronts per workgroup, chosen by timing a scratch
batch of that class's member shapes; cached by the class and its shapes.
"""
from __future__ import annotations

import time

from ._lib import FORM_RESIDENT, FORM_STREAMING
from .run import GABatch, GARun

SHAPE_FIELDS = ("width", "height", "pop", "sites", "k", "selection", "migration")
_cache: dict = {}
_batch_cache: dict = {}


def shape_key(cfg: dict) -> tuple:
    return tuple(int(cfg[f]) for f in SHAPE_FIELDS)


def candidates(cfg: dict) -> list[tuple]:
    """Candidates for a single run: (islands_per_wave, waves_per_group,
    FORM_STREAMING) and (tile_w, tile_h, FORM_RESIDENT) (0, 0: the library's
    tiling)."""
    per_iter = 64 // cfg["pop"]
    out = []
    ipw = per_iter
    while ipw <= 64:
        for wpg in (1, 2, 4, 8):
            out.append((ipw, wpg, FORM_STREAMING))
        ipw *= 2
    out.append((0, 0, FORM_RESIDENT))
    W, H = cfg["width"], cfg["height"]
    shapes = [(W, H), (max(1, W // 2), max(1, H // 2)), (max(1, W // 4), max(1, H // 4))]
    # one tile per CU (256), square and at half and twice, four times the width
    area = -(-W * H // 256)
    side = 1
    while side * side < area:
        side *= 2
    for tw in (side // 4, side // 2, side, side * 2, side * 4):
        if tw >= 1:
            shapes.append((min(tw, W), min(-(-area // tw), H)))
    for tw, th in shapes:
        if tile_lds_estimate(tw, th, cfg) <= 160 * 1024 and (tw, th, FORM_RESIDENT) not in out:
            out.append((tw, th, FORM_RESIDENT))
    return out


def tile_lds_estimate(tw: int, th: int, cfg: dict) -> int:
    """LDS bytes of a tile of tw x th islands (16-byte agent records, 8 more
    with a string; the island tables, both outbox parities, the halo)."""
    words = cfg["sites"] * cfg.get("dbits", 1) // 32
    strings = cfg.get("model", 0) != 0
    ob = 4 if words == 1 and not strings else 8
    agents = -(-tw * th * cfg["pop"] // 64) * 64 + 2   # and two scratch records
    return agents * (24 if strings else 16) + 8 * tw * th + 8 * tw * th * ob + 8 * (tw + th) * (ob + 1) + 16


def apply(run: GARun, choice):
    a, b, form = choice
    if form == FORM_RESIDENT:
        run.set_launch(form=FORM_RESIDENT)
        run.set_tiles(a, b)
    else:
        run.set_launch(a, b, form)


def time_candidate(run: GARun, cand, gens: int, torch, reps: int = 3) -> float:
    """Seconds per generation of one candidate, the best of reps timings (the
    candidates of a shape differ by a percent or so, about what one timing
    varies by)."""
    apply(run, cand)
    run.step(2)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        run.step(gens)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / gens)
    return best


def autotune(cfg: dict, gens: int | None = None, use_cache: bool = True, forms=None):
    """Fastest candidate for cfg's shape (candidates that do not fit are
    skipped), among those of the given forms (None: all)."""
    import torch
    from ._lib import GAError
    key = (shape_key(cfg), tuple(forms) if forms else None)
    if use_cache and key in _cache:
        return _cache[key]
    agents = cfg["width"] * cfg["height"] * cfg["pop"]
    if gens is None:            # a few milliseconds per timing
        gens = max(4, min(400, int(8e8 // max(agents, 1))))
    scratch = GARun(dict(cfg, seed=0x5eed, run_id=0xA070))
    best, best_t = None, float("inf")
    for cand in candidates(cfg):
        if forms and cand[2] not in forms:
            continue
        try:
            t = time_candidate(scratch, cand, gens, torch)
        except GAError:
            continue            # a tiling that does not fit
        if t < best_t:
            best, best_t = cand, t
    scratch.close()
    _cache[key] = best
    return best


# ---- batches -----------------------------------------------------------------

def class_of(cfg: dict) -> tuple:
    return ((cfg["pop"]).bit_length() - 1, cfg["sites"] * cfg.get("dbits", 1) // 32)


def batch_candidates(log2n: int) -> list[int]:
    """Islands-per-wavefront candidates of one class: 64 to 2,048 agents per
    wavefront, multiples of one iteration (64/N islands)."""
    per_iter = 64 >> log2n
    out = []
    ipw = per_iter
    while ipw <= 64:
        if 64 <= ipw << log2n <= 2048:
            out.append(ipw)
        ipw *= 2
    return out


WPG_CANDIDATES = (2, 4, 8)


def _batch_key(cfgs: list) -> tuple:
    return tuple(sorted((c["width"], c["height"], c["pop"], c["sites"]) for c in cfgs))


def _time_batch(batch: GABatch, gens: int, torch, reps: int = 2) -> float:
    batch.step(gens)                 # new tables (and graph, if the shape changed), warm
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        batch.step(gens)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


# A candidate replaces the shape in place only if it is this much faster: one
# class's shape moves a mixed batch's step by a percent or so, about what two
# timings of the same shape differ by.
BATCH_MARGIN = 0.01


def autotune_batch(batch: GABatch, cfgs: list, gens: int = 300, use_cache: bool = True) -> dict:
    """Choose and apply the launch shape of a batch of runs with configurations
    cfgs: the batch-wide wavefronts per workgroup, then each class's islands
    per wavefront with the others held (coordinate descent), every candidate
    timed (best of two) on a scratch batch of the same shapes in one launch
    per generation, as the batch runs, and taken only if it beats the shape in
    place by BATCH_MARGIN. Returns {"waves_per_group": w, (log2 N, words): ipw}."""
    import torch
    key = _batch_key(cfgs)
    if not (use_cache and key in _batch_cache):
        classes = sorted({class_of(c) for c in cfgs})
        runs = [GARun(dict(c, seed=0x5eed, run_id=0xB000 + i)) for i, c in enumerate(cfgs)]
        scratch = GABatch()
        for r in runs:
            scratch.add(r, 1 << 40)
        chosen = {k: scratch.class_launch(*k)[0] for k in classes}
        best_w = 4
        scratch.set_launch(0, best_w)
        best_t = _time_batch(scratch, gens, torch)
        for w in WPG_CANDIDATES:
            if w == best_w:
                continue
            scratch.set_launch(0, w)
            t = _time_batch(scratch, gens, torch)
            if t < best_t * (1 - BATCH_MARGIN):
                best_w, best_t = w, t
        scratch.set_launch(0, best_w)
        for k in classes:
            best_i = chosen[k]
            for ipw in batch_candidates(k[0]):
                if ipw == best_i:
                    continue
                scratch.set_class_launch(k[0], k[1], ipw)
                t = _time_batch(scratch, gens, torch)
                if t < best_t * (1 - BATCH_MARGIN):
                    best_i, best_t = ipw, t
            scratch.set_class_launch(k[0], k[1], best_i)
            chosen[k] = best_i
        chosen["waves_per_group"] = best_w
        scratch.close()
        for r in runs:
            r.close()
        _batch_cache[key] = chosen
    chosen = _batch_cache[key]
    apply_shapes(batch, chosen)
    return dict(chosen)


def apply_shapes(target, chosen: dict):
    """Apply autotune_batch's choice to a GABatch or a GAPool (whose runs fall
    in the same classes): the group size, then each class's islands per
    wavefront."""
    target.set_launch(0, chosen["waves_per_group"])
    for k, ipw in chosen.items():
        if k != "waves_per_group":
            target.set_class_launch(k[0], k[1], ipw)
