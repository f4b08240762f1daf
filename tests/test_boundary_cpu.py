"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/ga.h declares, and rejects bad configurations and
buffers before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2405_03605_amd as ga
from paper_2405_03605_amd import _lib
from paper_2405_03605_amd.run import make_config
from paper_2405_03605_amd.workloads import MID, PAPER, TINY, run_config


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libga_hip.so not built (run __graft_entry__.build())")
    return _lib.load()


def _declared_functions():
    text = open(_lib.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ga_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_state_bytes_layout(lib):
    # SoA planes: fitness, T, surface words per agent; 2 AoS outboxes of
    # (fitness, T, surface words, header) per island; counters; extraction staging.
    # Planes are padded to roundup(islands, 64) + 128 islands.
    # The asynchronous schedule has eight buffers (direction x parity), four
    # stamps, a progress word and eight lockstep headers per island instead of
    # the two outboxes; the synchronous one a progress word per resident-form
    # tile (at most 8,192 tiles, never more than islands).
    def expect(c):
        I = (c["width"] * c["height"] + 63) // 64 * 64 + 128
        A = I * c["pop"]
        W = c["sites"] * c.get("dbits", 1) // 32
        al = lambda b: (b + 255) // 256 * 256
        ob = 4 if W == 1 else 8   # AoS outbox entry words
        # a genome model with a string adds two string planes and uses 32-byte
        # entries
        strings = c.get("model", 0) != 0
        if strings:
            ob = 8
        exchange = ((al(4 * 8 * I * ob) + al(4 * 4 * I) + al(4 * I) + al(4 * 8 * I))
                    if c.get("schedule")
                    else 2 * al(4 * I * ob) + al(4 * min(8192, c["width"] * c["height"])))
        return (al(4 * A) * 2 + al(4 * A * W) + (al(4 * A * 2) if strings else 0) + exchange
                + 256 + 2 * al(4 * I) + al(4 * I * W))
    for c in (TINY, MID, PAPER, run_config(width=3, height=5, pop=1, sites=32)):
        assert ga.state_bytes(c) == expect(c)
        a = dict(c, schedule=1)
        assert ga.state_bytes(a) == expect(a) > ga.state_bytes(c)
        for sites, bits in ((16, 4), (8, 8), (16, 2), (4, 8)):
            w = dict(c, sites=sites, dbits=bits)
            assert ga.state_bytes(w) == expect(w)
        # the surface policy does not change the layout
        assert ga.state_bytes(dict(c, policy=1)) == expect(c)
        for model in (1, 2):
            m = dict(c, model=model)
            assert ga.state_bytes(m) == expect(m) > ga.state_bytes(c)
            ma = dict(m, schedule=1)
            assert ga.state_bytes(ma) == expect(ma)
    # paper-scale run: 16.8M agents, 12 B each
    assert 200e6 < ga.state_bytes(PAPER) < 230e6


@pytest.mark.parametrize("bad", [
    dict(pop=24), dict(pop=128), dict(pop=0), dict(sites=48), dict(sites=16), dict(k=0),
    dict(k=9), dict(width=0), dict(height=0), dict(width=70000), dict(selection=2),
    dict(migration=3), dict(width=65535, height=65535, pop=64), dict(width=65535, height=8193, pop=2),
    dict(law=2), dict(law=1, p32=2 ** 32 - 10, p_ben32=100), dict(schedule=2), dict(model=3),
    dict(model=1, law=1, p_ben32=5), dict(sites=32, dbits=4), dict(sites=64, dbits=2),
    dict(sites=16, dbits=3), dict(sites=2, dbits=16), dict(sites=12, dbits=4),
    dict(policy=1, sites=16, dbits=4), dict(policy=2, sites=32), dict(policy=2, sites=32, dbits=2),
    dict(policy=3)])
def test_invalid_configs_rejected(lib, bad):
    c = make_config(run_config(**bad))
    assert lib.ga_state_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    rc = lib.ga_init(ctypes.byref(c), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert rc == _lib.GA_EINVAL
    assert h.value is None
    assert lib.ga_last_error()


def test_init_argument_checks(lib):
    c = make_config(TINY)
    need = lib.ga_state_bytes(ctypes.byref(c))
    h = ctypes.c_void_p()
    assert lib.ga_init(ctypes.byref(c), None, need, None, ctypes.byref(h)) == _lib.GA_EINVAL
    assert lib.ga_init(ctypes.byref(c), ctypes.c_void_p(4096 + 8), need, None,
                       ctypes.byref(h)) == _lib.GA_EINVAL
    assert lib.ga_init(ctypes.byref(c), ctypes.c_void_p(4096), need - 1, None,
                       ctypes.byref(h)) == _lib.GA_ENOMEM
    c.struct_size = 8
    assert lib.ga_init(ctypes.byref(c), ctypes.c_void_p(4096), need, None,
                       ctypes.byref(h)) == _lib.GA_EINVAL


def test_null_handles_rejected(lib):
    assert lib.ga_step(None, 5) == _lib.GA_EINVAL
    assert lib.ga_read_population(None, None, None, None, None, None) == _lib.GA_EINVAL
    assert lib.ga_extract_surfaces(None, None, 0, None, None, None) == _lib.GA_EINVAL
    assert lib.ga_batch_step(None, 1) == _lib.GA_EINVAL
    assert lib.ga_generation(None) == 0
    lib.ga_destroy(None)
    lib.ga_batch_destroy(None)
    for code in (0, -1, -2, -3, -4, -99):
        assert lib.ga_strerror(code)


def test_first_release_config_size_accepted(lib):
    import ctypes as ct
    c = make_config(run_config(law=1, p_ben32=5))
    full = lib.ga_state_bytes(ct.byref(c))
    c.struct_size = _lib.Config.mutation_law.offset     # size before the treatment fields
    assert lib.ga_state_bytes(ct.byref(c)) == full
    # size before the schedule field: synchronous, whatever the field would say
    c = make_config(run_config(law=1, p_ben32=5, schedule=1))
    c.struct_size = _lib.Config.schedule.offset
    assert lib.ga_state_bytes(ct.byref(c)) == full
    c.schedule = 7                                      # not read at that size
    assert lib.ga_state_bytes(ct.byref(c)) == full
    # size before the genome model: fitness-valued, whatever the field says
    c = make_config(run_config(schedule=1, model=2))
    async_bytes = lib.ga_state_bytes(ct.byref(make_config(run_config(schedule=1))))
    c.struct_size = _lib.Config.genome_model.offset
    assert lib.ga_state_bytes(ct.byref(c)) == async_bytes
    # size before the differentia width: one bit per site, so 16 sites is invalid
    c = make_config(run_config(sites=16, dbits=4))
    assert lib.ga_state_bytes(ct.byref(c)) > 0
    c.struct_size = _lib.Config.differentia_bits.offset
    assert lib.ga_state_bytes(ct.byref(c)) == 0
    # size before the surface policy: steady, whatever the field says
    c = make_config(run_config(policy=9))
    assert lib.ga_state_bytes(ct.byref(c)) == 0
    c.struct_size = _lib.Config.surface_policy.offset
    assert lib.ga_state_bytes(ct.byref(c)) > 0
