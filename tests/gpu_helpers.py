"""Shared helpers for the GPU parity tests: run a configuration on the HIP
library and on the CPU oracle and compare every field bit for bit."""
import sys

import numpy as np

import oracle


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same_state(got: dict, ref: "oracle.OracleRun", what: str = ""):
    """Bit-exact comparison of a GPU read() against the oracle's state."""
    f, T, D = ref.population()
    gen = ref.generation
    assert got["generation"] == gen, f"{what}: generation {got['generation']} != {gen}"
    gf = got["f"].view(np.uint32)
    rf = f.view(np.uint32)
    if not np.array_equal(gf, rf):
        bad = np.flatnonzero(gf != rf)
        raise AssertionError(f"{what}: fitness differs at {bad.size} agents, first {bad[:5]} "
                             f"gpu {got['f'][bad[:5]]} oracle {f[bad[:5]]}")
    if not np.array_equal(got["T"], T):
        bad = np.flatnonzero(got["T"] != T)
        raise AssertionError(f"{what}: T differs at {bad.size} agents, first {bad[:5]} "
                             f"gpu {got['T'][bad[:5]]} oracle {T[bad[:5]]}")
    if not np.array_equal(got["D"], D):
        bad = np.flatnonzero((got["D"] != D).any(axis=1))
        raise AssertionError(f"{what}: surfaces differ at {bad.size} agents, first {bad[:5]}")
    if "P" in got:
        P = ref.payload()
        if not np.array_equal(got["P"], P):
            bad = np.flatnonzero((got["P"] != P).any(axis=1))
            raise AssertionError(f"{what}: genome strings differ at {bad.size} agents, first {bad[:5]}")
    if "outbox" in got:
        ob = ref.outbox()
        g = got["outbox"]
        assert np.array_equal(g["valid"], ob["valid"]), f"{what}: outbox valid flags differ"
        v = ob["valid"].astype(bool)
        assert np.array_equal(g["dir"][v], ob["dir"][v]), f"{what}: outbox directions differ"
        assert np.array_equal(g["f"][v].view(np.uint32), ob["f"][v].view(np.uint32)), \
            f"{what}: outbox fitness differs"
        assert np.array_equal(g["T"][v], ob["T"][v]), f"{what}: outbox T differs"
        assert np.array_equal(g["D"][v], ob["D"][v]), f"{what}: outbox surfaces differ"


def oracle_after(cfg: dict, gens: int) -> "oracle.OracleRun":
    ref = oracle.OracleRun(cfg)
    ref.step(gens)
    return ref
