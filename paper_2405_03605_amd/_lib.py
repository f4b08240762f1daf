"""ctypes binding of libga_hip.so (include/ga.h). Argument marshalling only:
every generation step runs in the library's HIP kernels. There is no CPU
fallback; loading fails loudly when the library is missing."""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libga_hip.so")
HEADER = os.path.join(ROOT, "include", "ga.h")
SOURCES = [os.path.join(_HERE, "csrc", n)
           for n in ("ga_kernels.hip", "ga_tile.hip", "ga_mrca.hip", "ga_roofs.hip", "ga_api.hip")]
BUILD_DIR = os.path.join(_HERE, "_build")
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per source: the tile kernel's LDS counters are bumped by one lane at a time;
# the compiler's atomic optimizer would turn each such bump into a wavefront
# scan that waits for its result on the spot.
EXTRA_FLAGS = {"ga_tile.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}
# roctx ranges around the host calls that submit generations
ROCTX = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]

GA_OK, GA_EINVAL, GA_ENOMEM, GA_EDEVICE, GA_ESTATE = 0, -1, -2, -3, -4
FORM_AUTO, FORM_STREAMING, FORM_RESIDENT = 0, 1, 2
SCHEDULE_SYNC, SCHEDULE_ASYNC = 0, 1
ASYNC_UNPACED = 0xFFFFFFFF
MODEL_FITNESS, MODEL_ONEMAX, MODEL_TRAP4 = 0, 1, 2
POLICY_STEADY, POLICY_TILTED, POLICY_HYBRID = 0, 1, 2


class GAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def build(hipcc: str = "hipcc") -> str:
    """Compile libga_hip.so for gfx950 in-tree (one object per source, in
    parallel, then one link)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    quiet = subprocess.DEVNULL if os.environ.get("GA_QUIET_BUILD") else None
    objs = [os.path.join(BUILD_DIR, os.path.basename(src) + ".o") for src in SOURCES]

    def compile_one(src_obj):
        src, obj = src_obj
        extra = EXTRA_FLAGS.get(os.path.basename(src), [])
        subprocess.run([hipcc] + HIPCC_FLAGS + extra + ["-c", src, "-o", obj], check=True,
                       stderr=quiet)

    with ThreadPoolExecutor(len(SOURCES)) as pool:
        list(pool.map(compile_one, zip(SOURCES, objs)))
    tmp = LIB_PATH + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ROCTX,
                   check=True, stderr=quiet)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "struct_size", "width", "height", "pop_per_island", "surface_sites",
        "tournament_size", "selection", "mutation_threshold", "migration", "seed", "run_id",
        "mutation_law", "beneficial_threshold", "schedule", "genome_model",
        "differentia_bits", "surface_policy")]


class OutboxEntry(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_uint32), ("dir", ctypes.c_uint32), ("fitness", ctypes.c_float),
                ("T", ctypes.c_uint32), ("surface", ctypes.c_uint32 * 2)]


# name -> (restype, argtypes); every symbol declared in include/ga.h
P = ctypes.c_void_p
u32, u64, sz, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
SIGNATURES = {
    "ga_state_bytes": (sz, [P]),
    "ga_init": (i32, [P, P, sz, P, ctypes.POINTER(P)]),
    "ga_step": (i32, [P, u64]),
    "ga_read_population": (i32, [P, P, P, P, P, P]),
    "ga_write_population": (i32, [P, P, P, P, P, u64]),
    "ga_extract_surfaces": (i32, [P, P, sz, P, P, P]),
    "ga_read_strings": (i32, [P, P]),
    "ga_write_strings": (i32, [P, P]),
    "ga_generation": (u64, [P]),
    "ga_destroy": (None, [P]),
    "ga_set_launch": (i32, [P, u32, u32, u32]),
    "ga_set_graph_block": (i32, [P, u32]),
    "ga_set_tiles": (i32, [P, u32, u32]),
    "ga_get_tiles": (i32, [P, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
    "ga_set_async": (i32, [P, u32, u32, u32]),
    "ga_async_waits": (i32, [P, ctypes.POINTER(u64)]),
    "ga_async_taken": (i32, [P, ctypes.POINTER(u64)]),
    "ga_async_last_taken": (i32, [P, P]),
    "ga_batch_create": (i32, [P, ctypes.POINTER(P)]),
    "ga_batch_add": (i32, [P, P, u64]),
    "ga_batch_remove": (i32, [P, P]),
    "ga_batch_step": (i32, [P, u64]),
    "ga_batch_remaining": (u64, [P, P]),
    "ga_batch_size": (sz, [P]),
    "ga_batch_set_graph_block": (i32, [P, u32]),
    "ga_batch_set_launch": (i32, [P, u32, u32]),
    "ga_batch_set_class_launch": (i32, [P, u32, u32, u32]),
    "ga_batch_class_launch": (i32, [P, u32, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)]),
    "ga_batch_settled": (i32, [P, P, ctypes.POINTER(i32)]),
    "ga_batch_destroy": (None, [P]),
    "ga_pool_create": (i32, [P, sz, u32, P, ctypes.POINTER(P)]),
    "ga_pool_admit": (i32, [P, P, u64, ctypes.POINTER(u64)]),
    "ga_pool_step": (i32, [P, u64]),
    "ga_pool_set_graph_block": (i32, [P, u32]),
    "ga_pool_set_launch": (i32, [P, u32, u32]),
    "ga_pool_set_class_launch": (i32, [P, u32, u32, u32]),
    "ga_pool_remaining": (i32, [P, u64, ctypes.POINTER(u64)]),
    "ga_pool_poll": (i32, [P, P, sz, ctypes.POINTER(sz)]),
    "ga_pool_poll_settled": (i32, [P, P, sz, ctypes.POINTER(sz), i32]),
    "ga_pool_retire": (i32, [P, u64, P, P, P]),
    "ga_pool_usage": (i32, [P, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(u32)]),
    "ga_pool_destroy": (None, [P]),
    "ga_mrca_workspace_bytes": (sz, [sz]),
    "ga_mrca_matrix": (i32, [P, P, sz, u32, u32, P, sz, P, P, P]),
    "ga_mrca_matrix_ex": (i32, [P, P, sz, u32, u32, u32, u32, P, sz, P, P, P]),
    "ga_mrca_matrix_noalloc": (i32, [P, P, sz, u32, u32, u32, u32, P, P, P]),
    "ga_roof_inplace": (i32, [P, sz, u32, P]),
    "ga_roof_philox": (i32, [P, u32, u32, P]),
    "ga_roof_valu": (i32, [P, u32, u32, u32, P]),
    "ga_strerror": (ctypes.c_char_p, [i32]),
    "ga_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != GA_OK:
        lib = load()
        raise GAError(code, lib.ga_last_error().decode() or lib.ga_strerror(code).decode())
