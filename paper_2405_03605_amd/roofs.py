"""Roof microbenchmarks of the generation step on one MI355X (through the C
ABI's ga_roof_* calls, timed with HIP events on the launch stream):

* HBM: an in-place update of three planes of 16,777,216 + padding words (the
  fitness, T and surface planes of the 16.8M-agent run, 201 MB), read and
  written once per launch;
* RNG: full Philox4x32-10 blocks per second (the block each child draws);
* issue rates: wave64 instructions per second of a three-input XOR and of a
  32x32->64 multiply-add (with its XOR), over every SIMD.

    python -m paper_2405_03605_amd.roofs [--json]
"""
from __future__ import annotations

import argparse
import ctypes
import json

CUS, SIMDS_PER_CU, CLOCK_HZ = 256, 4, 2.4e9


def _time(fn, stream, torch, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


INPLACE_WORDS = 16777216  # per plane: the 16.8M-agent population, one word per agent
INPLACE_BYTES_EACH_WAY = 3 * 4 * INPLACE_WORDS


def measure(reps: int = 20, only: str | None = None) -> dict:
    import torch
    from ._lib import check, load
    lib = load()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    s = ctypes.c_void_p(stream.cuda_stream)
    P = ctypes.c_void_p
    out = {}

    # HBM: three planes of the 16.8M-agent population
    words = INPLACE_WORDS
    planes = torch.zeros(3 * words, dtype=torch.int32, device=dev)
    t = _time(lambda: check(lib.ga_roof_inplace(P(planes.data_ptr()), words, 3, s)), stream,
              torch, reps)
    moved = 2 * INPLACE_BYTES_EACH_WAY
    out["hbm_inplace"] = {"bytes_per_launch": moved, "us": t * 1e6, "GB_per_s": moved / t / 1e9}
    del planes
    if only == "inplace":
        return out

    # RNG and issue rates: 2,048 threads per CU, enough wavefronts to hide latency
    threads = CUS * 2048
    buf = torch.empty(threads, dtype=torch.int32, device=dev)
    blocks = 64
    t = _time(lambda: check(lib.ga_roof_philox(P(buf.data_ptr()), threads, blocks, s)), stream,
              torch, reps)
    out["philox"] = {"blocks_per_s": threads * blocks / t, "us": t * 1e6,
                     "threads": threads, "blocks_per_thread": blocks}
    iters = 256
    waves = threads / 64
    for kind, name, per_step in ((0, "xor3", 1), (1, "mad_u64_u32+xor", 2)):
        t = _time(lambda: check(lib.ga_roof_valu(P(buf.data_ptr()), threads, iters, kind, s)),
                  stream, torch, reps)
        insts = waves * iters * 8 * per_step
        simd_cycles = CUS * SIMDS_PER_CU * CLOCK_HZ * t
        out[name] = {"wave_insts_per_s": insts / t, "us": t * 1e6,
                     "cycles_per_wave_inst": simd_cycles / insts}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--only", choices=("inplace",), default=None,
                    help="only the in-place update (counter calibration: its bytes are exact)")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(measure(args.reps, args.only)), flush=True)


if __name__ == "__main__":
    main()
