"""Python handles over the C ABI: GARun (one GA run) and GABatch (many runs
advanced together). PyTorch provides the device memory and the stream; every
generation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (FORM_AUTO, GA_EINVAL, GA_ENOMEM, Config, GAError, OutboxEntry, check, load)

CONFIG_FIELDS = ("width", "height", "pop", "sites", "k", "selection", "p32", "migration",
                 "seed", "run_id", "law", "p_ben32", "schedule", "model", "dbits", "policy")
OPTIONAL_FIELDS = {"law": 0, "p_ben32": 0, "schedule": 0, "model": 0, "dbits": 1, "policy": 0}


def _fields(cfg: dict) -> dict:
    return {f: int(cfg.get(f, OPTIONAL_FIELDS[f]) if f in OPTIONAL_FIELDS else cfg[f])
            for f in CONFIG_FIELDS}


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_config(cfg: dict) -> Config:
    return Config(struct_size=ctypes.sizeof(Config), width=cfg["width"], height=cfg["height"],
                  pop_per_island=cfg["pop"], surface_sites=cfg["sites"],
                  tournament_size=cfg["k"], selection=cfg["selection"],
                  mutation_threshold=cfg["p32"], migration=cfg["migration"],
                  seed=cfg["seed"], run_id=cfg["run_id"],
                  mutation_law=cfg.get("law", 0), beneficial_threshold=cfg.get("p_ben32", 0),
                  schedule=cfg.get("schedule", 0), genome_model=cfg.get("model", 0),
                  differentia_bits=cfg.get("dbits", 1), surface_policy=cfg.get("policy", 0))


def state_bytes(cfg: dict) -> int:
    """Device footprint of a run (0 if the configuration is invalid)."""
    c = make_config(cfg)
    return int(load().ga_state_bytes(ctypes.byref(c)))


class GARun:
    """One island-model GA run whose state lives in a torch uint8 CUDA tensor."""

    def __init__(self, cfg: dict, device=None, stream=None):
        import torch
        lib = load()
        self.cfg = _fields(cfg)
        self._c = make_config(self.cfg)
        nbytes = int(lib.ga_state_bytes(ctypes.byref(self._c)))
        if nbytes == 0:
            raise GAError(GA_EINVAL, f"invalid configuration {self.cfg}")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        check(lib.ga_init(ctypes.byref(self._c), ctypes.c_void_p(self.mem.data_ptr()), nbytes,
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.state_bytes = nbytes
        self.islands = self.cfg["width"] * self.cfg["height"]
        self.agents = self.islands * self.cfg["pop"]
        self.words = self.cfg["sites"] * self.cfg["dbits"] // 32

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        check(load().ga_step(self._h, int(n)))

    @property
    def generation(self) -> int:
        return int(load().ga_generation(self._h))

    def set_launch(self, islands_per_wave: int = 0, waves_per_group: int = 0, form: int = FORM_AUTO):
        check(load().ga_set_launch(self._h, islands_per_wave, waves_per_group, form))

    def set_graph_block(self, gens: int):
        check(load().ga_set_graph_block(self._h, gens))

    def set_tiles(self, tile_w: int = 0, tile_h: int = 0):
        """Tile shape of the LDS-resident form (0, 0: the library's choice)."""
        check(load().ga_set_tiles(self._h, int(tile_w), int(tile_h)))

    def tiles(self) -> tuple:
        """(tile_w, tile_h, tiles) that ga_step uses; zeros for the streaming form."""
        w, h, n = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        check(load().ga_get_tiles(self._h, ctypes.byref(w), ctypes.byref(h), ctypes.byref(n)))
        return int(w.value), int(h.value), int(n.value)

    def set_async(self, max_wavefronts: int = 0, max_lead: int = 0, skew: int = 0):
        """Asynchronous runs: cap on wavefronts (0 = fill the GPU), how many
        generations an island may lead a neighbour (ASYNC_UNPACED = no bound),
        and a reproducible skewed interleaving (one wavefront, unpaced)."""
        check(load().ga_set_async(self._h, int(max_wavefronts), int(max_lead), int(skew)))

    def async_last_taken(self) -> np.ndarray:
        """(islands, 4): generation in which the last genome each island took
        from each side was sent (-1: none yet)."""
        out = np.empty((self.islands, 4), dtype=np.int64)
        check(load().ga_async_last_taken(self._h, _ptr(out)))
        return out

    def async_waits(self) -> int:
        """How many pacing waits gave up so far (0: every wait was met)."""
        n = ctypes.c_uint64()
        check(load().ga_async_waits(self._h, ctypes.byref(n)))
        return int(n.value)

    def async_taken(self) -> int:
        """Genomes absorbed from the neighbours' buffers since creation."""
        n = ctypes.c_uint64()
        check(load().ga_async_taken(self._h, ctypes.byref(n)))
        return int(n.value)

    @property
    def asynchronous(self) -> bool:
        return self.cfg["schedule"] == 1

    @property
    def has_strings(self) -> bool:
        return self.cfg["model"] != 0

    def read_strings(self) -> np.ndarray:
        """Genome strings (models 1 and 2), shape (agents, 2) uint32."""
        out = np.empty((self.agents, 2), dtype=np.uint32)
        check(load().ga_read_strings(self._h, _ptr(out)))
        return out

    def write_strings(self, words):
        a = np.ascontiguousarray(words, dtype=np.uint32).reshape(self.agents, 2)
        check(load().ga_write_strings(self._h, _ptr(a)))

    def read(self, outbox: bool = True) -> dict:
        """Population, generation, the strings of a genome model that has them,
        and (synchronous fitness-valued runs) the pending outbox."""
        outbox = outbox and not self.asynchronous and not self.has_strings
        A, I, W = self.agents, self.islands, self.words
        f = np.empty(A, dtype=np.float32)
        T = np.empty(A, dtype=np.uint32)
        D = np.empty((A, W), dtype=np.uint32)
        ob = (OutboxEntry * I)() if outbox else None
        gen = ctypes.c_uint64()
        obp = ctypes.cast(ob, ctypes.c_void_p) if ob is not None else None
        check(load().ga_read_population(self._h, _ptr(f), _ptr(T), _ptr(D), obp, ctypes.byref(gen)))
        out = {"f": f, "T": T, "D": D, "generation": int(gen.value)}
        if self.has_strings:
            out["P"] = self.read_strings()
        if ob is not None:
            raw = np.frombuffer(ob, dtype=np.uint32).reshape(I, 6)
            out["outbox"] = {
                "valid": raw[:, 0].astype(np.uint8), "dir": raw[:, 1].astype(np.uint8),
                "f": raw[:, 2].copy().view(np.float32), "T": raw[:, 3].copy(),
                "D": raw[:, 4:4 + W].copy()}
        return out

    def write(self, f=None, T=None, D=None, outbox: dict | None = None, generation: int = 0):
        A, I, W = self.agents, self.islands, self.words
        fa = None if f is None else np.ascontiguousarray(f, dtype=np.float32)
        Ta = None if T is None else np.ascontiguousarray(T, dtype=np.uint32)
        Da = None if D is None else np.ascontiguousarray(np.asarray(D, dtype=np.uint32).reshape(A, W))
        for a, n in ((fa, A), (Ta, A)):
            if a is not None and a.size != n:
                raise ValueError("population array has the wrong size")
        ob = None
        if outbox is not None:
            raw = np.zeros((I, 6), dtype=np.uint32)
            raw[:, 0] = outbox["valid"]
            raw[:, 1] = outbox["dir"]
            raw[:, 2] = np.asarray(outbox["f"], dtype=np.float32).view(np.uint32)
            raw[:, 3] = outbox["T"]
            raw[:, 4:4 + W] = np.asarray(outbox["D"], dtype=np.uint32).reshape(I, W)
            ob = (OutboxEntry * I).from_buffer_copy(raw.tobytes())
        obp = ctypes.cast(ob, ctypes.c_void_p) if ob is not None else None
        check(load().ga_write_population(self._h, _ptr(fa), _ptr(Ta), _ptr(Da), obp, int(generation)))

    def extract(self, agent_ids=None):
        """(ids, T, D) for one agent per island (agent_ids None) or the listed agents."""
        W = self.words
        if agent_ids is None:
            n = self.islands
            ids_in = None
        else:
            ids_in = np.ascontiguousarray(agent_ids, dtype=np.uint64)
            n = ids_in.size
        ids = np.empty(n, dtype=np.uint64)
        T = np.empty(n, dtype=np.uint32)
        D = np.empty((n, W), dtype=np.uint32)
        check(load().ga_extract_surfaces(self._h, _ptr(ids_in), n, _ptr(ids), _ptr(T), _ptr(D)))
        return ids, T, D


class GABatch:
    """Many runs advanced together: one launch per generation over every
    member's islands, blocks of generations replayed from a HIP graph."""

    def __init__(self, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(load().ga_batch_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.members = []

    def add(self, run: GARun, budget: int):
        check(load().ga_batch_add(self._h, run.handle, int(budget)))
        self.members.append(run)

    def remove(self, run: GARun):
        check(load().ga_batch_remove(self._h, run.handle))
        self.members.remove(run)

    def step(self, n: int):
        check(load().ga_batch_step(self._h, int(n)))

    def remaining(self, run: GARun) -> int:
        return int(load().ga_batch_remaining(self._h, run.handle))

    def __len__(self):
        return int(load().ga_batch_size(self._h))

    def set_graph_block(self, gens: int):
        check(load().ga_batch_set_graph_block(self._h, gens))

    def set_launch(self, islands_per_wave: int = 0, waves_per_group: int = 0):
        check(load().ga_batch_set_launch(self._h, islands_per_wave, waves_per_group))

    def set_class_launch(self, log2n: int, words: int, islands_per_wave: int = 0):
        """Islands per wavefront of one class (log2 N, surface words); 0 = the batch's rule."""
        check(load().ga_batch_set_class_launch(self._h, int(log2n), int(words),
                                               int(islands_per_wave)))

    def class_launch(self, log2n: int, words: int) -> tuple:
        """(islands_per_wave, tiles) of a class."""
        i, t = ctypes.c_uint32(), ctypes.c_uint32()
        check(load().ga_batch_class_launch(self._h, int(log2n), int(words), ctypes.byref(i),
                                           ctypes.byref(t)))
        return int(i.value), int(t.value)

    def classes(self) -> list:
        """(log2 N, surface words) of every class with members."""
        out = []
        for log2n in range(7):
            for words in (1, 2):
                if self.class_launch(log2n, words)[1]:
                    out.append((log2n, words))
        return out

    def settled(self, run: GARun) -> bool:
        s = ctypes.c_int()
        check(load().ga_batch_settled(self._h, run.handle, ctypes.byref(s)))
        return bool(s.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_batch_destroy(self._h)
            self._h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GAPool:
    """Runs created inside one device buffer and advanced together (ga_pool_*):
    admission fails softly (None) while no slot or free block fits the run."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, device=None, stream=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.mem = torch.empty(int(budget_bytes), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        check(load().ga_pool_create(ctypes.c_void_p(self.mem.data_ptr()), int(budget_bytes),
                                    int(max_slots), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h)))
        self._h = h
        self.budget = int(budget_bytes)
        self._shape = {}

    def admit(self, cfg: dict, gens: int):
        """Ticket of the new run, or None if it does not fit now."""
        c = _fields(cfg)
        ticket = ctypes.c_uint64()
        code = load().ga_pool_admit(self._h, ctypes.byref(make_config(c)), int(gens),
                                    ctypes.byref(ticket))
        if code == GA_ENOMEM:
            return None
        check(code)
        self._shape[ticket.value] = (c["width"] * c["height"], c["sites"] * c["dbits"] // 32)
        return ticket.value

    def step(self, n: int):
        check(load().ga_pool_step(self._h, int(n)))

    def set_graph_block(self, gens: int):
        check(load().ga_pool_set_graph_block(self._h, int(gens)))

    def set_launch(self, islands_per_wave: int = 0, waves_per_group: int = 0):
        check(load().ga_pool_set_launch(self._h, int(islands_per_wave), int(waves_per_group)))

    def set_class_launch(self, log2n: int, words: int, islands_per_wave: int = 0):
        """Islands per wavefront of one class (log2 N, surface words) of the pool's batch."""
        check(load().ga_pool_set_class_launch(self._h, int(log2n), int(words),
                                              int(islands_per_wave)))

    def remaining(self, ticket: int) -> int:
        left = ctypes.c_uint64()
        check(load().ga_pool_remaining(self._h, int(ticket), ctypes.byref(left)))
        return int(left.value)

    def done(self, settled: bool = False) -> list:
        """Tickets of the runs whose budget is spent (with settled, only those
        whose last generation has already run on the GPU)."""
        n = ctypes.c_size_t()
        lib = load()
        check(lib.ga_pool_poll_settled(self._h, None, 0, ctypes.byref(n), int(settled)))
        out = np.empty(n.value, dtype=np.uint64)
        check(lib.ga_pool_poll_settled(self._h, _ptr(out), out.size, ctypes.byref(n),
                                       int(settled)))
        return [int(t) for t in out[:n.value]]

    def retire(self, ticket: int, sample: bool = True):
        """Remove a run; with sample, return (ids, T, surfaces) of one agent per island."""
        if not sample:
            check(load().ga_pool_retire(self._h, int(ticket), None, None, None))
            self._shape.pop(int(ticket), None)
            return None
        # an unknown ticket is refused by the library (GAError), as for the other calls
        islands, words = self._shape.get(int(ticket), (0, 0))
        ids = np.empty(islands, dtype=np.uint64)
        T = np.empty(islands, dtype=np.uint32)
        D = np.empty((islands, words), dtype=np.uint32)
        check(load().ga_pool_retire(self._h, int(ticket), _ptr(ids), _ptr(T), _ptr(D)))
        self._shape.pop(int(ticket), None)   # a failed retire leaves the run in the pool
        return ids, T, D

    def usage(self) -> dict:
        if getattr(self, "_h", None) is None:
            return {"used": 0, "largest_free": 0, "live": 0}   # closed
        used, big, live = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_uint32()
        check(load().ga_pool_usage(self._h, ctypes.byref(used), ctypes.byref(big),
                                   ctypes.byref(live)))
        return {"used": int(used.value), "largest_free": int(big.value), "live": int(live.value)}

    @property
    def used(self) -> int:
        return self.usage()["used"]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
