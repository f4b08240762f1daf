"""Host-side reconstruction pieces: phylometrics on trees worked by hand, the
distance transform, and UPGMA against brute-force average linkage."""
import numpy as np

from paper_2405_03605_amd import phylo


def test_phylometrics_hand_worked_tree():
    # ((0:1, 1:1):3, 2:4) with node heights 1 and 4: edges 1, 1, 3, 4 -> SBL 9;
    # fair proportion: tip0 = 1 + 3/2, tip1 = 1 + 3/2, tip2 = 4 -> mean 3.
    Z = np.array([[0, 1, 1.0, 2], [2, 3, 4.0, 3]])
    m = phylo.phylometrics(Z)
    assert m["sum_branch_length"] == 9.0
    assert m["mean_evolutionary_distinctiveness"] == 3.0
    assert m["root_height"] == 4.0


def test_star_tree_and_fair_proportion_identity():
    rng = np.random.default_rng(1)
    n = 40
    pts = np.sort(rng.random(n)) * 100
    d = np.abs(pts[:, None] - pts[None, :])
    Z = phylo.upgma(d)
    m = phylo.phylometrics(Z)
    # fair-proportion ED sums to the tree length over the tips
    assert np.isclose(m["mean_evolutionary_distinctiveness"] * n, m["sum_branch_length"])


def test_upgma_matches_brute_force_average_linkage():
    rng = np.random.default_rng(2)
    n = 12
    x = rng.random((n, 3))
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    Z = phylo.upgma(d)
    # brute force: repeatedly merge the closest pair, distances averaged over members
    clusters = {i: [i] for i in range(n)}
    heights = []
    while len(clusters) > 1:
        keys = list(clusters)
        best = None
        for a in range(len(keys)):
            for b in range(a + 1, len(keys)):
                ca, cb = clusters[keys[a]], clusters[keys[b]]
                dd = d[np.ix_(ca, cb)].mean()
                if best is None or dd < best[0]:
                    best = (dd, keys[a], keys[b])
        dd, ka, kb = best
        heights.append(dd / 2)
        new = max(clusters) + 1
        clusters[new] = clusters.pop(ka) + clusters.pop(kb)
    assert np.allclose(sorted(heights), sorted(Z[:, 2]))


def test_estimated_distance():
    T = np.array([100, 100, 90])
    L = np.array([[0, 40, 10], [40, 0, 10], [10, 10, 0]], dtype=np.uint32)
    U = np.array([[100, 60, 30], [60, 100, 30], [30, 30, 90]], dtype=np.uint32)
    d = phylo.estimated_distance(T, L, U)
    assert d[0, 1] == 200 - 100 and d[0, 2] == 190 - 40 and d[1, 1] == 0
