"""Surfaces produced on the GPU against the oracle's true lineages: the MRCA
interval estimated from two GPU-extracted surfaces must contain the true MRCA's
deposit counter (hard upper bound for every pair; the lower bound may fail with
probability at most 2^-kc per pair)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import say
from paper_2405_03605_amd import GARun
from paper_2405_03605_amd.workloads import run_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("sample", ["uniform", "island-clustered"])
def test_gpu_surfaces_bracket_true_mrca(sample):
    S, kc, G = 32, 5, 1000
    cfg = run_config(width=32, height=16, pop=32, sites=S, seed=3)
    say(f"MRCA intervals, 32x16x32, {G} generations, {sample} sample")
    ref = oracle.OracleRun(cfg, lineage=True)
    ref.step(G)
    run = GARun(cfg)
    run.step(G)
    rng = np.random.default_rng(2024)
    A = run.agents
    if sample == "uniform":
        ids = np.sort(rng.choice(A, size=200, replace=False))
    else:
        isl = rng.choice(A // 32, size=6, replace=False)
        ids = np.concatenate([i * 32 + np.arange(32) for i in isl])
    got_ids, T, D = run.extract(ids)
    f0, T0, D0 = ref.population()
    assert np.array_equal(T, T0[ids]) and np.array_equal(D, D0[ids])
    hi_viol = lo_viol = pairs = related = 0
    for x in range(len(ids)):
        for y in range(x + 1, len(ids)):
            a, b = int(ids[x]), int(ids[y])
            g = max(ref.true_mrca(a, b), 0)
            L, U = oracle.mrca_interval(int(T[x]), D[x], int(T[y]), D[y], S, kc)
            hi_viol += g > U
            lo_viol += g < L
            pairs += 1
            related += g > 0
    assert hi_viol == 0
    assert related > 0
    # P(g < L) <= 2^-kc for each pair; pairs are correlated, so allow slack
    bound = 2.0 ** -kc
    assert lo_viol <= 1.25 * bound * pairs + 4 * np.sqrt(bound * pairs) + 1


# n = 300 takes the 16-byte row stores; 301..303 the ragged tail of each row
@pytest.mark.parametrize("sites,kc,n", [(32, 5, 300), (64, 5, 303), (32, 1, 301), (64, 3, 302)])
def test_gpu_mrca_matrix_equals_oracle_on_random_surfaces(sites, kc, n):
    from paper_2405_03605_amd import phylo
    rng = np.random.default_rng(sites * 10 + kc)
    special = [0, 1, 2, sites - 1, sites, sites + 1, 2 * sites, 2 * sites + 1, 100, 1000,
               100000, (1 << 31) - 1, 1 << 31, 4000000000]
    T = np.concatenate([special, rng.integers(0, 1 << 20, size=n // 2),
                        rng.integers(0, 1 << 32, size=n - n // 2 - len(special), dtype=np.uint64)])
    T = T.astype(np.uint32)
    D = rng.integers(0, 1 << 32, size=(n, sites // 32), dtype=np.uint64).astype(np.uint32)
    # make many pairs share long prefixes: copy surfaces between random pairs
    for _ in range(200):
        a, b = rng.integers(0, n, size=2)
        D[b] = D[a]
    L, U = phylo.mrca_matrix(T, D, sites, kc)
    L0, U0 = oracle.mrca_interval_matrix(T, D, sites, kc)
    assert np.array_equal(U, U0)
    assert np.array_equal(L, L0)


def test_gpu_mrca_matrix_on_run_surfaces():
    from paper_2405_03605_amd import phylo
    cfg = run_config(width=32, height=16, pop=32, sites=64, seed=5)
    run = GARun(cfg)
    run.step(700)
    ids = np.arange(0, run.agents, 29)[:520]
    _, T, D = run.extract(ids)
    L, U = phylo.mrca_matrix(T, D, 64, 5)
    L0, U0 = oracle.mrca_interval_matrix(T, D, 64, 5)
    assert np.array_equal(U, U0) and np.array_equal(L, L0)
    Z, m = phylo.reconstruct(T, D, 64)
    assert m["tips"] == len(ids) and m["sum_branch_length"] > 0


@pytest.mark.parametrize("sites,bits,policy", [(32, 1, 0), (16, 4, 0), (32, 1, 1), (64, 1, 1),
                                               (32, 2, 1), (64, 1, 2)])
def test_mrca_matrix_full_size_sampled(sites, bits, policy):
    # the benchmark's size: 10,000 surfaces sampled from a 256 x 256-island run
    # after 3,000 generations, the whole n x n matrix on the GPU in the
    # launch the benchmark times; a sample of rows x columns (first and last
    # included, both sides of the diagonal) against the oracle
    import ctypes
    import torch
    from paper_2405_03605_amd._lib import check, load
    say(f"MRCA full size S={sites} b={bits} policy={policy}")
    cfg = run_config(width=256, height=256, pop=32, sites=sites, dbits=bits, policy=policy,
                     seed=5)
    run = GARun(cfg)
    run.step(3000)
    n = 10000
    ids = np.random.default_rng(5).choice(run.agents, size=n, replace=False)
    _, T, D = run.extract(ids.astype(np.uint64))
    run.close()
    lib = load()
    dev = torch.device("cuda", 0)
    t_dev = torch.from_numpy(np.ascontiguousarray(T).view(np.int32)).to(dev)
    d_dev = torch.from_numpy(np.ascontiguousarray(D).view(np.int32)).to(dev)
    ws_bytes = int(lib.ga_mrca_workspace_bytes(n))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    L = torch.empty((n, n), dtype=torch.int32, device=dev)
    U = torch.empty((n, n), dtype=torch.int32, device=dev)
    P = ctypes.c_void_p
    stream = torch.cuda.current_stream(dev)
    check(lib.ga_mrca_matrix_ex(P(t_dev.data_ptr()), P(d_dev.data_ptr()), n, sites, bits, policy,
                                5, P(ws.data_ptr()), ws_bytes, P(L.data_ptr()), P(U.data_ptr()),
                                P(stream.cuda_stream)))
    torch.cuda.synchronize()
    pick = np.unique(np.concatenate([[0, 1, 63, 64, n - 2, n - 1],
                                     np.random.default_rng(6).choice(n, 90, replace=False)]))
    idx = torch.from_numpy(pick).to(dev)
    Lg = L[idx][:, idx].cpu().numpy().view(np.uint32)
    Ug = U[idx][:, idx].cpu().numpy().view(np.uint32)
    L0, U0 = oracle.mrca_interval_matrix(T[pick], D[pick], sites, 5, bits, policy=policy)
    assert np.array_equal(Ug, U0) and np.array_equal(Lg, L0), (sites, bits, policy)
