"""Post hoc phylogenetic analysis of sampled end-state surfaces (paper Fig. 1:
hereditary-stratigraphy markers support estimating relatedness between
lineages after the run; Sec. 3 reconstructs phylogenies from 10k sampled
end-state genomes and compares sum branch length and mean evolutionary
distinctiveness between treatments; Fig. 2).

The all-pairs MRCA intervals run on the GPU (`ga_mrca_matrix`). From them:
    estimated MRCA counter  g = (L + U) / 2
    time since the MRCA     d/2 = (Tx + Ty) / 2 - g    (generations, per lineage)
The tree is the average-linkage (UPGMA) clustering of d, an ultrametric tree
whose merge heights are the estimated times back to each common ancestor.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import check, load


def mrca_matrix(T, D, sites: int, kc: int = 5, device=None, bits: int = 1, policy: int = 0):
    """(L, U) interval matrices for every pair of the n sampled surfaces, on the GPU.
    T: (n,) deposit counters; D: (n, sites * bits / 32) surface words; policy 0
    steady, 1 tilted."""
    import torch
    lib = load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    Tn = np.ascontiguousarray(T, dtype=np.uint32)
    Dn = np.ascontiguousarray(np.asarray(D, dtype=np.uint32).reshape(Tn.size, sites * bits // 32))
    n = Tn.size
    if n == 0:
        return np.zeros((0, 0), np.uint32), np.zeros((0, 0), np.uint32)
    t_dev = torch.from_numpy(Tn.view(np.int32)).to(dev)
    d_dev = torch.from_numpy(Dn.view(np.int32)).to(dev)
    ws_bytes = int(lib.ga_mrca_workspace_bytes(n))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L = torch.empty((n, n), dtype=torch.int32, device=dev)
    U = torch.empty((n, n), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    P = ctypes.c_void_p
    check(lib.ga_mrca_matrix_ex(P(t_dev.data_ptr()), P(d_dev.data_ptr()), n, sites, bits, policy,
                                kc, P(ws.data_ptr()), ws_bytes, P(L.data_ptr()),
                                P(U.data_ptr()), P(stream.cuda_stream)))
    return L.cpu().numpy().view(np.uint32), U.cpu().numpy().view(np.uint32)


def estimated_distance(T, L, U) -> np.ndarray:
    """Pairwise distance (twice the estimated generations back to the MRCA)."""
    T = np.asarray(T, dtype=np.float64)
    g = (L.astype(np.float64) + U.astype(np.float64)) / 2.0
    d = (T[:, None] + T[None, :]) - 2.0 * g
    np.fill_diagonal(d, 0.0)
    return np.maximum(d, 0.0)


def upgma(dist: np.ndarray) -> np.ndarray:
    """Average-linkage clustering (UPGMA) of a symmetric distance matrix, as a
    SciPy linkage matrix; merge heights are half the distances (tip-to-node)."""
    from scipy.cluster.hierarchy import linkage
    from scipy.spatial.distance import squareform
    Z = linkage(squareform(dist, checks=False), method="average")
    Z[:, 2] = Z[:, 2] / 2.0
    return Z


def phylometrics(Z: np.ndarray) -> dict:
    """Sum branch length and mean evolutionary distinctiveness (fair
    proportion: each edge's length shared equally by the tips below it) of an
    ultrametric tree given as a linkage matrix with node heights in Z[:, 2]."""
    n = Z.shape[0] + 1
    height = np.zeros(2 * n - 1)
    count = np.ones(2 * n - 1)
    parent = np.full(2 * n - 1, -1, dtype=np.int64)
    for m, (a, b, h, c) in enumerate(Z):
        node = n + m
        height[node] = h
        count[node] = c
        parent[int(a)] = node
        parent[int(b)] = node
    edge = np.zeros(2 * n - 1)
    has_parent = parent >= 0
    edge[has_parent] = np.maximum(height[parent[has_parent]] - height[has_parent], 0.0)
    sbl = float(edge.sum())
    share = edge / count                     # per-tip share of each edge
    # parents are created after their children, so a pass from the root down
    # accumulates each node's shares of all edges above it
    acc = np.zeros(2 * n - 1)
    for node in range(2 * n - 2, -1, -1):
        acc[node] = share[node] + (acc[parent[node]] if parent[node] >= 0 else 0.0)
    ed = acc[:n]
    return {"tips": n, "sum_branch_length": sbl, "mean_evolutionary_distinctiveness": float(ed.mean()),
            "root_height": float(height[2 * n - 2]) if n > 1 else 0.0}


def reconstruct(T, D, sites: int, kc: int = 5, device=None, bits: int = 1, policy: int = 0):
    """Tree (linkage matrix) and phylometrics for sampled surfaces."""
    L, U = mrca_matrix(T, D, sites, kc, device, bits, policy)
    Z = upgma(estimated_distance(T, L, U))
    return Z, phylometrics(Z)
