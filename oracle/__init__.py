"""CPU oracle for the island-model GA generation step (ctypes binding).

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. The GPU library
never imports, links or calls it, and it imports nothing from the GPU library.

The arithmetic lives in ``ga_oracle.c`` (plain single-threaded C). This module
only marshals arguments. Every function cites the passage of the paper it
follows in the C source (Sec. 2 Methods for the generation cycle, Sec. 3 for the
genome layout, Fig. 1 for post hoc relatedness estimation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GA_ORACLE_LIB names another build of the same source to load instead (the
# sanitizer test's instrumented copy).
LIB_PATH = os.environ.get("GA_ORACLE_LIB") or os.path.join(_HERE, "libga_oracle.so")
SOURCES = [os.path.join(_HERE, "ga_oracle.c")]
DISCARD = 0xFFFFFFFF
_FLAGS = ["-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-fno-fast-math",
          "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math) into oracle/libga_oracle.so."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2"] + _FLAGS + ["-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_sanitized(out: str) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), into `out`; load it through GA_ORACLE_LIB with the
    sanitizer runtimes preloaded."""
    cmd = (["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"] + _FLAGS + ["-o", str(out)] + SOURCES + ["-lm"])
    subprocess.run(cmd, check=True)
    return str(out)


class _Config(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "width", "height", "pop", "sites", "k", "selection", "p32", "migration",
        "seed", "run_id", "law", "p_ben32", "model", "dbits", "policy")]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u32, u64, sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    lib.orc_philox.argtypes = [P, P, P]
    lib.orc_site_of.argtypes = [u64, u32]
    lib.orc_site_of.restype = u32
    lib.orc_epoch.argtypes = [u64, u32]
    lib.orc_epoch.restype = u32
    lib.orc_site_of_range.argtypes = [u64, sz, u32, P]
    lib.orc_validate.argtypes = [ctypes.POINTER(_Config)]
    lib.orc_validate.restype = ctypes.c_int
    lib.orc_create.argtypes = [ctypes.POINTER(_Config), ctypes.c_int]
    lib.orc_create.restype = P
    lib.orc_free.argtypes = [P]
    lib.orc_reserve_lineage.argtypes = [P, u64]
    lib.orc_reserve_lineage.restype = ctypes.c_int
    lib.orc_step.argtypes = [P, u64]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_step_async.argtypes = [P, u64, u64, u32]
    lib.orc_step_async.restype = ctypes.c_int
    lib.orc_clear_mailboxes.argtypes = [P]
    lib.orc_get_mailboxes.argtypes = [P, P, P, P, P, P]
    lib.orc_generation.argtypes = [P]
    lib.orc_generation.restype = u64
    lib.orc_agents.argtypes = [P]
    lib.orc_agents.restype = u64
    lib.orc_get_population.argtypes = [P, P, P, P]
    lib.orc_set_population.argtypes = [P, P, P, P]
    lib.orc_get_outbox.argtypes = [P, P, P, P, P, P]
    lib.orc_set_outbox.argtypes = [P, P, P, P, P, P]
    lib.orc_set_generation.argtypes = [P, u64]
    lib.orc_set_generation.restype = ctypes.c_int
    lib.orc_sample_one_per_island.argtypes = [P, P]
    lib.orc_true_mrca.argtypes = [P, u64, u64]
    lib.orc_true_mrca.restype = ctypes.c_int64
    lib.orc_ancestry.argtypes = [P, u64, P, P, P, sz]
    lib.orc_ancestry.restype = sz
    lib.orc_mrca_interval.argtypes = [u32, P, u32, P, u32, u32, P, P]
    lib.orc_true_mrca_matrix.argtypes = [P, P, sz, P]
    lib.orc_true_mrca_matrix.restype = ctypes.c_int
    lib.orc_mrca_interval_matrix.argtypes = [P, P, sz, u32, u32, P, P]
    lib.orc_mrca_interval_bits.argtypes = [u32, P, u32, P, u32, u32, u32, P, P]
    lib.orc_site_of_tilted.argtypes = [u64, u32]
    lib.orc_site_of_tilted.restype = u32
    lib.orc_site_of_hybrid.argtypes = [u64]
    lib.orc_site_of_hybrid.restype = u32
    lib.orc_site_of_policy.argtypes = [u64, u32, u32]
    lib.orc_site_of_policy.restype = u32
    lib.orc_retained.argtypes = [u64, u32, u32, P]
    lib.orc_retained.restype = sz
    lib.orc_mrca_interval_policy.argtypes = [u32, P, u32, P, u32, u32, u32, u32, P, P]
    lib.orc_mrca_interval_matrix_policy.argtypes = [P, P, sz, u32, u32, u32, u32, P, P]
    lib.orc_mrca_interval_matrix_bits.argtypes = [P, P, sz, u32, u32, u32, P, P]
    lib.orc_get_payload.argtypes = [P, P]
    lib.orc_set_payload.argtypes = [P, P]
    lib.orc_evaluate.argtypes = [u32, u32, u32]
    lib.orc_evaluate.restype = ctypes.c_float
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def evaluate(model: int, p0: int, p1: int) -> float:
    """Fitness genome model 1 (OneMax) or 2 (Trap-4) gives the 64-bit string (p0, p1)."""
    return float(_load().orc_evaluate(model, p0, p1))


def site_of(rank: int, sites: int) -> int:
    """Surface site written by the deposit of stratum ``rank`` (DISCARD if none)."""
    return int(_load().orc_site_of(rank, sites))


def epoch(n: int, sites: int) -> int:
    return int(_load().orc_epoch(n, sites))


def site_of_range(first: int, count: int, sites: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    _load().orc_site_of_range(first, count, sites, _ptr(out))
    return out


def mrca_interval(Ta: int, Da, Tb: int, Db, sites: int, kc: int = 5, bits: int = 1,
                  policy: int = 0, general: bool = False):
    """(L, U) bounds on the MRCA's deposit counter from two surfaces of
    ``sites`` differentia of ``bits`` bits each under a surface policy (0
    steady, 1 tilted). The steady policy uses its closed form unless
    ``general`` asks for the retained-rank estimator every policy uses."""
    a = np.ascontiguousarray(Da, dtype=np.uint32)
    b = np.ascontiguousarray(Db, dtype=np.uint32)
    L = ctypes.c_uint32()
    U = ctypes.c_uint32()
    if policy == 0 and not general:
        _load().orc_mrca_interval_bits(Ta, _ptr(a), Tb, _ptr(b), sites, bits, kc,
                                       ctypes.byref(L), ctypes.byref(U))
    else:
        _load().orc_mrca_interval_policy(Ta, _ptr(a), Tb, _ptr(b), sites, bits, policy, kc,
                                         ctypes.byref(L), ctypes.byref(U))
    return int(L.value), int(U.value)


def site_of_tilted(rank: int, sites: int) -> int:
    return int(_load().orc_site_of_tilted(rank, sites))


def site_of_policy(rank: int, sites: int, policy: int) -> int:
    """Site a deposit of ``rank`` writes under policy 0 (steady), 1 (tilted)
    or 2 (hybrid), or DISCARD."""
    return int(_load().orc_site_of_policy(rank, sites, policy))


def retained(n: int, sites: int, policy: int) -> np.ndarray:
    """Ranks a surface holds after n deposits, ascending."""
    out = np.empty(64, dtype=np.uint64)
    c = _load().orc_retained(n, sites, policy, _ptr(out))
    return out[:c].copy()


def mrca_interval_matrix(T, D, sites: int, kc: int = 5, bits: int = 1, policy: int = 0):
    """(L, U) matrices for every pair of the n surfaces (T[n], D[n, S*bits/32])."""
    Ta = np.ascontiguousarray(T, dtype=np.uint32)
    Da = np.ascontiguousarray(D, dtype=np.uint32)
    n = Ta.size
    L = np.empty((n, n), dtype=np.uint32)
    U = np.empty((n, n), dtype=np.uint32)
    if policy == 0:
        _load().orc_mrca_interval_matrix_bits(_ptr(Ta), _ptr(Da), n, sites, bits, kc, _ptr(L),
                                              _ptr(U))
    else:
        _load().orc_mrca_interval_matrix_policy(_ptr(Ta), _ptr(Da), n, sites, bits, policy, kc,
                                                _ptr(L), _ptr(U))
    return L, U


CONFIG_FIELDS = ("width", "height", "pop", "sites", "k", "selection", "p32",
                 "migration", "seed", "run_id", "law", "p_ben32", "model", "dbits", "policy")
OPTIONAL_FIELDS = {"law": 0, "p_ben32": 0, "model": 0, "dbits": 1, "policy": 0}


def _fields(cfg: dict) -> dict:
    return {f: int(cfg.get(f, OPTIONAL_FIELDS.get(f, 0)) if f in OPTIONAL_FIELDS else cfg[f])
            for f in CONFIG_FIELDS}


def validate(cfg: dict) -> bool:
    c = _Config(**_fields(cfg))
    return _load().orc_validate(ctypes.byref(c)) == 0


class OracleRun:
    """One GA run on the CPU oracle. ``cfg`` holds the fields of CONFIG_FIELDS."""

    def __init__(self, cfg: dict, lineage: bool = False):
        lib = _load()
        self.cfg = _fields(cfg)
        c = _Config(**self.cfg)
        h = lib.orc_create(ctypes.byref(c), 1 if lineage else 0)
        if not h:
            raise ValueError(f"oracle rejected configuration {self.cfg}")
        self._h = ctypes.c_void_p(h)
        self.words = self.cfg["sites"] * self.cfg["dbits"] // 32
        self.islands = self.cfg["width"] * self.cfg["height"]
        self.agents = self.islands * self.cfg["pop"]

    def close(self):
        if getattr(self, "_h", None):
            _load().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def generation(self) -> int:
        return int(_load().orc_generation(self._h))

    def reserve_lineage(self, gens: int):
        if _load().orc_reserve_lineage(self._h, int(gens)) != 0:
            raise MemoryError("cannot reserve lineage storage")

    def step(self, n: int):
        if _load().orc_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle step failed (lineage buffer)")

    def step_async(self, n: int, group: int, skew: int = 0):
        """n generations of the asynchronous schedule in the reproducible
        interleaving: groups of ``group`` islands, group c running generation t
        at step t + (c mod (skew + 1)); skew 0 equals the synchronous schedule."""
        if _load().orc_step_async(self._h, int(n), int(group), int(skew)) != 0:
            raise RuntimeError("oracle async step failed (lineage on, group 0, or memory)")

    def clear_mailboxes(self):
        _load().orc_clear_mailboxes(self._h)

    def mailboxes(self):
        """Asynchronous buffers: stamp, f, T with shape (islands, 4, 2) (sender,
        direction, parity of the sending generation), D (islands, 4, 2, words),
        and seen (islands, 4)."""
        n = self.islands * 8
        stamp = np.empty(n, dtype=np.uint64)
        seen = np.empty(self.islands * 4, dtype=np.uint64)
        f = np.empty(n, dtype=np.float32)
        T = np.empty(n, dtype=np.uint32)
        D = np.empty((n, self.words), dtype=np.uint32)
        _load().orc_get_mailboxes(self._h, _ptr(stamp), _ptr(seen), _ptr(f), _ptr(T), _ptr(D))
        sh = (self.islands, 4, 2)
        return {"stamp": stamp.reshape(sh), "seen": seen.reshape(self.islands, 4),
                "f": f.reshape(sh), "T": T.reshape(sh), "D": D.reshape(sh + (self.words,))}

    def payload(self) -> np.ndarray:
        """Genome strings of models 1 and 2, shape (agents, 2) uint32."""
        P = np.empty((self.agents, 2), dtype=np.uint32)
        _load().orc_get_payload(self._h, _ptr(P))
        return P

    def set_payload(self, P):
        a = np.ascontiguousarray(P, dtype=np.uint32).reshape(self.agents, 2)
        _load().orc_set_payload(self._h, _ptr(a))

    def population(self):
        f = np.empty(self.agents, dtype=np.float32)
        T = np.empty(self.agents, dtype=np.uint32)
        D = np.empty((self.agents, self.words), dtype=np.uint32)
        _load().orc_get_population(self._h, _ptr(f), _ptr(T), _ptr(D))
        return f, T, D

    def set_population(self, f=None, T=None, D=None):
        args = []
        for a, dt in ((f, np.float32), (T, np.uint32), (D, np.uint32)):
            if a is None:
                args.append(None)
            else:
                args.append(np.ascontiguousarray(a, dtype=dt))
        _load().orc_set_population(self._h, *[(_ptr(a) if a is not None else None) for a in args])

    def outbox(self):
        n = self.islands
        valid = np.empty(n, dtype=np.uint8)
        d = np.empty(n, dtype=np.uint8)
        f = np.empty(n, dtype=np.float32)
        T = np.empty(n, dtype=np.uint32)
        D = np.empty((n, self.words), dtype=np.uint32)
        _load().orc_get_outbox(self._h, _ptr(valid), _ptr(d), _ptr(f), _ptr(T), _ptr(D))
        return {"valid": valid, "dir": d, "f": f, "T": T, "D": D}

    def set_outbox(self, valid, d, f, T, D):
        arrs = [np.ascontiguousarray(valid, dtype=np.uint8), np.ascontiguousarray(d, dtype=np.uint8),
                np.ascontiguousarray(f, dtype=np.float32), np.ascontiguousarray(T, dtype=np.uint32),
                np.ascontiguousarray(D, dtype=np.uint32)]
        _load().orc_set_outbox(self._h, *[_ptr(a) for a in arrs])

    def set_generation(self, t: int):
        if _load().orc_set_generation(self._h, int(t)) != 0:
            raise RuntimeError("cannot move the generation counter of a lineage-recording run")

    def sample_one_per_island(self) -> np.ndarray:
        ids = np.empty(self.islands, dtype=np.uint64)
        _load().orc_sample_one_per_island(self._h, _ptr(ids))
        return ids

    def true_mrca(self, a: int, b: int) -> int:
        g = int(_load().orc_true_mrca(self._h, int(a), int(b)))
        if g == -2:
            raise RuntimeError("lineage was not recorded from generation 0")
        return g

    def true_mrca_matrix(self, ids) -> np.ndarray:
        """T of the MRCA for every pair of the listed agents (-1: different founders)."""
        a = np.ascontiguousarray(ids, dtype=np.uint64)
        out = np.empty((a.size, a.size), dtype=np.int32)
        if _load().orc_true_mrca_matrix(self._h, _ptr(a), a.size, _ptr(out)) != 0:
            raise RuntimeError("lineage not recorded from generation 0, or out of memory")
        return out

    def ancestry(self, agent: int):
        cap = self.generation + 1
        g = np.empty(cap, dtype=np.uint64)
        i = np.empty(cap, dtype=np.uint32)
        s = np.empty(cap, dtype=np.uint32)
        n = _load().orc_ancestry(self._h, int(agent), _ptr(g), _ptr(i), _ptr(s), cap)
        return g[:n], i[:n], s[:n]
