"""Throughput of the all-pairs MRCA interval kernels (reconstruction, Sec. 2:
pairwise MRCA estimates over a sample of end-state genomes).

Samples n surfaces from a run of one GPU's 256 x 256-island tile after
`--gens` generations (n = 10,000 by default, about 5e7 unordered pairs), then
times ga_mrca_matrix_ex on device-resident inputs with HIP events on the
launch stream, for each surface variant. Prints one JSON line per variant:
pairs per second, and the algorithmic bytes (the two n x n u32 outputs, 8 B
per ordered pair, plus the inputs) per second against MI355X's 8 TB/s.

  python -m paper_2405_03605_amd.mrca_bench [--n 10000] [--reps 10] [--gens 3000]
"""
from __future__ import annotations

import argparse
import ctypes
import json

import numpy as np

from ._lib import check, load
from .run import GARun
from .workloads import run_config

PEAK_HBM_GBPS = 8000.0
VARIANTS = [  # (name, sites, bits, policy)
    ("steady S=32", 32, 1, 0),
    ("steady S=64", 64, 1, 0),
    ("steady S=16 b=4", 16, 4, 0),
    ("tilted S=32", 32, 1, 1),
    ("tilted S=64", 64, 1, 1),
    ("tilted S=32 b=2", 32, 2, 1),
    ("hybrid S=64", 64, 1, 2),
]


def sample(sites: int, bits: int, policy: int, n: int, gens: int, seed: int = 5):
    """n surfaces (T, D) sampled without replacement from a run's end state."""
    cfg = run_config(width=256, height=256, pop=32, sites=sites, dbits=bits, policy=policy,
                     seed=seed)
    run = GARun(cfg)
    run.step(gens)
    ids = np.random.default_rng(seed).choice(run.agents, size=n, replace=False)
    _, T, D = run.extract(ids.astype(np.uint64))
    run.close()
    return T, D


def time_matrix(T, D, sites, bits, policy, kc, reps, torch):
    lib = load()
    n = T.size
    dev = torch.device("cuda", torch.cuda.current_device())
    t_dev = torch.from_numpy(np.ascontiguousarray(T).view(np.int32)).to(dev)
    d_dev = torch.from_numpy(np.ascontiguousarray(D).view(np.int32)).to(dev)
    ws_bytes = int(lib.ga_mrca_workspace_bytes(n))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    L = torch.empty((n, n), dtype=torch.int32, device=dev)
    U = torch.empty((n, n), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    P = ctypes.c_void_p
    args = (P(t_dev.data_ptr()), P(d_dev.data_ptr()), n, sites, bits, policy, kc,
            P(ws.data_ptr()), ws_bytes, P(L.data_ptr()), P(U.data_ptr()), P(stream.cuda_stream))
    check(lib.ga_mrca_matrix_ex(*args))  # warm-up
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        check(lib.ga_mrca_matrix_ex(*args))
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--gens", type=int, default=3000)
    ap.add_argument("--kc", type=int, default=5)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("mrca_bench needs an MI355X GPU")
    torch.cuda.set_device(0)
    # practical write ceiling: a plain fill of the same two n x n u32 outputs
    n = args.n
    out = torch.empty((2, n, n), dtype=torch.int32, device="cuda")
    out.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        out.zero_()
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / args.reps
    print(json.dumps({"variant": "fill of both outputs (write ceiling)", "n": n,
                      "us_per_matrix": round(sec * 1e6, 1),
                      "GB_per_s": round(8 * n * n / sec / 1e9, 1)}), flush=True)
    del out
    for name, sites, bits, policy in VARIANTS:
        T, D = sample(sites, bits, policy, args.n, args.gens)
        sec = time_matrix(T, D, sites, bits, policy, args.kc, args.reps, torch)
        n = args.n
        words = sites * bits // 32
        algo = 8 * n * n + 4 * n * (1 + words)
        line = {"variant": name, "n": n, "ordered_pairs": n * n,
                "us_per_matrix": round(sec * 1e6, 1), "pairs_per_s": n * (n - 1) / 2 / sec}
        if policy == 0:
            # O(1) per pair: bound by writing the two outputs
            line["roofline"] = {"bound": "hbm", "achieved": round(algo / sec / 1e9, 1),
                                "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                "frac": round(algo / sec / 1e9 / PEAK_HBM_GBPS, 4),
                                "bytes_per_matrix": algo}
        else:
            # a walk over the S sites per pair: bound by instruction issue, not
            # by the output bytes (their HBM fraction is given for reference)
            line["roofline"] = {"bound": "alu",
                                "hbm_frac": round(algo / sec / 1e9 / PEAK_HBM_GBPS, 4)}
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
