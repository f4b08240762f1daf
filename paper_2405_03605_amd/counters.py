"""Hardware-counter record of one kernel on one workload, for the roofline
fields of bench.py: HBM bytes per dispatch (FETCH_SIZE, WRITE_SIZE, each
scaled by what the counter reads for an in-place update of known size) and VALU
issue (SQ counters). Each counter set is one rocprofv3 pass over a committed
command, run as a child process (this process never touches the GPU). The
scale factors come from the library's in-place update roof kernel, whose
bytes are exact.

  python -m paper_2405_03605_amd.counters paper-streaming --out profiles/counters_generation_kernel_paper.json
  python -m paper_2405_03605_amd.counters mid-tiles --out profiles/counters_tile_kernel_mid.json
  python -m paper_2405_03605_amd.counters batch --out profiles/counters_batch_all_kernel_64runs.json
  python -m paper_2405_03605_amd.counters batch-classes --out profiles/counters_batch_classes.json

The record holds the sha256 of the kernel's sources; bench.py reports its
figures only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import shutil
import subprocess
import sys
import tempfile

from .roofs import INPLACE_BYTES_EACH_WAY

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")

# Sources each kernel family is compiled from (the hash bench.py compares).
COMMON = ["ga_device.hpp", "ga_internal.hpp", "models/models.hpp", "models/fitness.hpp",
          "models/strings.hpp", "models/onemax.hpp", "models/trap4.hpp"]
KERNELS = {
    "paper-streaming": {"kernel": "generation_kernel", "sources": ["ga_kernels.hip"] + COMMON,
                        "name": "generation_kernel<5,1,FitnessModel,false>",
                        "workload": "1024x512 islands x 32 agents, 32-site surface, tournament 2",
                        "gens_per_dispatch": 1},
    "mid-tiles": {"kernel": "tile_kernel", "sources": ["ga_tile.hip"] + COMMON,
                  "name": "tile_kernel<5,1,FitnessModel,false>",
                  "workload": "256x256 islands x 32 agents, 32-site surface, tournament 2, "
                              "the autotuner's tiling (one tile per CU)",
                  "gens_per_dispatch": 200, "autotuned_tiles": True},
    "batch": {"kernel": "batch_all_kernel", "sources": ["ga_kernels.hip"] + COMMON,
              "name": "batch_all_kernel",
              "workload": "64 uneven runs, 8,597,368 agents, one launch per generation",
              "gens_per_dispatch": 1},
}
SQ_SET = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_VALU",
          "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU_INT64", "GRBM_GUI_ACTIVE"]
SIMDS = 1024


def source_hash(mode: str) -> str:
    h = hashlib.sha256()
    for name in KERNELS[mode]["sources"]:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pass(counters, cmd, kernel, tmp, tag):
    """One rocprofv3 pass: per-dispatch counter values of `kernel` dispatches."""
    out_dir = os.path.join(tmp, tag)
    prof = ["rocprofv3", "--pmc"] + counters + ["--output-format", "csv", "-d", out_dir,
                                                "-o", "run", "--"]
    print(f"[counters] {tag}: {' '.join(counters)}", flush=True)
    subprocess.run(prof + cmd, check=True, timeout=300, cwd=ROOT)
    files = glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise RuntimeError(f"no counter file under {out_dir}")
    per = {}
    for path in files:
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if kernel not in row.get("Kernel_Name", ""):
                    continue
                d = per.setdefault(row["Dispatch_Id"], {})
                name = row["Counter_Name"]
                d[name] = d.get(name, 0.0) + float(row["Counter_Value"])
    if not per:
        raise RuntimeError(f"no {kernel} dispatch in {files}")
    return [per[k] for k in sorted(per, key=int)]


def _mean(dispatches, name, skip_first=True):
    vals = [d[name] for d in dispatches]
    if skip_first and len(vals) > 1:
        vals = vals[1:]
    return sum(vals) / len(vals)


def autotuned_tiles() -> str:
    """The tile shape the autotuner picks for the 256 x 256 x 32 workload in
    the LDS-resident form, found in a child process outside the profiler."""
    code = ("import torch; torch.cuda.set_device(0); "
            "from paper_2405_03605_amd.autotune import autotune; "
            "from paper_2405_03605_amd.workloads import MID; "
            "from paper_2405_03605_amd import FORM_RESIDENT, GARun; "
            "c = autotune(MID, forms=(FORM_RESIDENT,)); r = GARun(MID); "
            "r.set_launch(form=FORM_RESIDENT); r.set_tiles(c[0], c[1]); "
            "w, h, n = r.tiles(); print(f'{w}x{h}')")
    out = subprocess.run([sys.executable, "-c", code], check=True, capture_output=True, text=True,
                         timeout=300, cwd=ROOT)
    return out.stdout.strip().splitlines()[-1]


def collect(mode: str) -> dict:
    spec = KERNELS[mode]
    py = sys.executable
    cmd = [py, "-m", "paper_2405_03605_amd.profile_run", mode]
    tiles = None
    if spec.get("autotuned_tiles"):
        tiles = autotuned_tiles()
        print(f"[counters] autotuned tiles {tiles}", flush=True)
        cmd += ["--tiles", tiles]
    calib = [py, "-m", "paper_2405_03605_amd.roofs", "--only", "inplace", "--reps", "2"]
    tmp = tempfile.mkdtemp(prefix="counters_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        # the in-place update reads and writes exactly INPLACE_BYTES_EACH_WAY
        cf = _pass(["FETCH_SIZE"], calib, "inplace_kernel", tmp, "calib_fetch")
        cw = _pass(["WRITE_SIZE"], calib, "inplace_kernel", tmp, "calib_write")
        kib = INPLACE_BYTES_EACH_WAY / 1024.0
        fetch_scale = kib / _mean(cf, "FETCH_SIZE")
        write_scale = kib / _mean(cw, "WRITE_SIZE")
        f = _pass(["FETCH_SIZE"], cmd, spec["kernel"], tmp, "fetch")
        w = _pass(["WRITE_SIZE"], cmd, spec["kernel"], tmp, "write")
        sq = _pass(SQ_SET, cmd, spec["kernel"], tmp, "sq")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    gens = spec["gens_per_dispatch"]
    fetch_kib, write_kib = _mean(f, "FETCH_SIZE"), _mean(w, "WRITE_SIZE")
    read_b = fetch_kib * 1024.0 * fetch_scale
    write_b = write_kib * 1024.0 * write_scale
    valu = _mean(sq, "SQ_INSTS_VALU")
    gui = _mean(sq, "GRBM_GUI_ACTIVE")
    # GRBM_GUI_ACTIVE sums the busy cycles of the 8 XCDs: per-XCD cycles x 1,024 SIMDs
    simd_cycles = gui / 8.0 * SIMDS
    rec = {
        "kernel": spec["name"], "workload": spec["workload"], "mode": mode,
        "kernel_source_sha256": source_hash(mode),
        "tiles": tiles,
        "generations_per_dispatch": gens, "dispatches": len(sq),
        "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
        "fetch_kib_per_dispatch": round(fetch_kib, 1), "write_kib_per_dispatch": round(write_kib, 1),
        "read_bytes_per_generation": round(read_b / gens),
        "write_bytes_per_generation": round(write_b / gens),
        "bytes_per_generation": round((read_b + write_b) / gens),
        "sq_per_dispatch": {n: _mean(sq, n) for n in SQ_SET},
        "valu_wave_insts_per_generation": round(valu / gens),
        # issue slots used: a wave64 VALU instruction holds a SIMD for 4 cycles
        "valu_issue_frac": round(4.0 * valu / simd_cycles, 4),
        "commands": {"workload": " ".join(["python3"] + cmd[1:]),
                     "calibration": "python3 -m paper_2405_03605_amd.roofs --only inplace --reps 2",
                     "passes": ["rocprofv3 --pmc FETCH_SIZE", "rocprofv3 --pmc WRITE_SIZE",
                                "rocprofv3 --pmc " + " ".join(SQ_SET)]},
    }
    return rec


CLASS_SET = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_SMEM", "SQ_INSTS_LDS",
             "SQ_INSTS_VALU_INT64", "GRBM_GUI_ACTIVE"]


def collect_classes(gens: int = 12) -> dict:
    """Instruction counts of the batch kernel against the kernel compiled for
    one run, class by class: one run per class advanced alone, then as a batch
    of one (profile_run batch-classes), one SQ pass."""
    from .profile_run import CLASS_RUNS, class_config
    py = sys.executable
    cmd = [py, "-m", "paper_2405_03605_amd.profile_run", "batch-classes", "--gens", str(gens)]
    tmp = tempfile.mkdtemp(prefix="counters_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        out_dir = os.path.join(tmp, "classes")
        prof = ["rocprofv3", "--pmc"] + CLASS_SET + ["--output-format", "csv", "-d", out_dir,
                                                     "-o", "run", "--"]
        print(f"[counters] classes: {' '.join(CLASS_SET)}", flush=True)
        subprocess.run(prof + cmd, check=True, timeout=300, cwd=ROOT)
        files = glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True)
        per = {}
        for path in files:
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    name = row.get("Kernel_Name", "")
                    if "generation_kernel" not in name and "batch_all_kernel" not in name:
                        continue
                    d = per.setdefault(int(row["Dispatch_Id"]), {"kernel": name})
                    c = row["Counter_Name"]
                    d[c] = d.get(c, 0.0) + float(row["Counter_Value"])
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    seq = [per[k] for k in sorted(per)]
    if len(seq) != 2 * gens * len(CLASS_RUNS):
        raise RuntimeError(f"expected {2 * gens * len(CLASS_RUNS)} dispatches, got {len(seq)}")
    rows = []
    for i, (l, w) in enumerate(CLASS_RUNS):
        plain = seq[2 * gens * i: 2 * gens * i + gens]
        batch = seq[2 * gens * i + gens: 2 * gens * (i + 1)]
        assert all("generation_kernel" in d["kernel"] for d in plain)
        assert all("batch_all_kernel" in d["kernel"] for d in batch)
        cfg = class_config(l, w)
        row = {"N": 1 << l, "surface_words": w,
               "run": f"{cfg['width']}x{cfg['height']}x{cfg['pop']}, S={cfg['sites']}",
               "plain_kernel": plain[0]["kernel"].split("(")[0]}
        for name in CLASS_SET:
            row["plain_" + name] = _mean(plain, name)
            row["batch_" + name] = _mean(batch, name)
        row["valu_ratio"] = round(row["batch_SQ_INSTS_VALU"] / row["plain_SQ_INSTS_VALU"], 4)
        row["salu_ratio"] = round(row["batch_SQ_INSTS_SALU"] / row["plain_SQ_INSTS_SALU"], 4)
        rows.append(row)
    return {"kernel": "batch_all_kernel", "mode": "batch-classes",
            "kernel_source_sha256": source_hash("batch"), "generations_per_class": gens,
            "classes": rows,
            "commands": {"workload": " ".join(["python3"] + cmd[1:]),
                         "pass": "rocprofv3 --pmc " + " ".join(CLASS_SET)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=sorted(KERNELS) + ["batch-classes"])
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    rec = collect_classes() if args.mode == "batch-classes" else collect(args.mode)
    with open(args.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
