"""Pins of the oracle's minimum spanning tree (dense Prim, Sec. 3.5 / Algorithm 3).

Each test checks the oracle against something other than itself: Kruskal's
algorithm under the same total edge order, scipy's MST on the dense FP64
distance matrix, closed forms (collinear points, integer lattices) and the
cycle property of minimum spanning trees.
"""
import numpy as np
import pytest
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.spatial.distance import cdist

from paper_1702_04739_amd import datagen
from tests import brute


@pytest.mark.parametrize("n,d,seed", [(2, 1, 0), (3, 2, 1), (17, 3, 2), (120, 5, 3), (400, 16, 4)])
def test_prim_equals_kruskal_random(orc, n, d, seed):
    X = np.random.default_rng(seed).standard_normal((n, d)).astype(np.float32)
    parent, length, depth, _ = orc.prim_mst(X)
    edges, S = brute.kruskal(X)
    assert brute.edge_set(parent) == edges
    assert parent[0] == -1 and length[0] == 0.0
    np.testing.assert_array_equal(depth, orc.tree_depth(parent))
    for v in range(1, n):
        assert length[v] == np.sqrt(S[v, parent[v]])


@pytest.mark.parametrize("maker", [lambda: datagen.lattice(6, 2), lambda: datagen.lattice(4, 3),
                                   lambda: datagen.with_duplicates(120, 4, 15)])
def test_prim_equals_kruskal_ties(orc, maker):
    """Tie-heavy inputs: the (D^2, min id, max id) order makes the MST unique."""
    X = maker()
    parent, _, _, _ = orc.prim_mst(X)
    edges, _ = brute.kruskal(X)
    assert brute.edge_set(parent) == edges


@pytest.mark.parametrize("threads", [2, 5])
@pytest.mark.parametrize("maker", [lambda: np.random.default_rng(8).standard_normal((700, 6)).astype(np.float32),
                                   lambda: datagen.lattice(5, 3), lambda: datagen.with_duplicates(300, 5, 40)])
def test_prim_threads_equal_kruskal(orc, maker, threads):
    """The threaded key update (used for the large golden digests) gives Kruskal's tree, ties included."""
    X = maker()
    parent, length, depth, added = orc.prim_mst(X, threads=threads)
    edges, S = brute.kruskal(X)
    assert brute.edge_set(parent) == edges
    ref = orc.prim_mst(X)
    for got, want in zip((parent, length, depth, added), ref):
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,d,seed", [(50, 2, 5), (800, 8, 6), (2500, 16, 7)])
def test_weight_matches_scipy(orc, n, d, seed):
    X = np.random.default_rng(seed).random((n, d)).astype(np.float32)
    _, length, _, _ = orc.prim_mst(X)
    D = cdist(X.astype(np.float64), X.astype(np.float64))
    W_ref = minimum_spanning_tree(D).sum()
    assert abs(length.sum() - W_ref) <= 1e-12 * W_ref


def test_collinear_closed_form(orc):
    """Points on a line: the MST joins consecutive points, W = max - min exactly,
    and the tree rooted at vertex 0 is a path."""
    X = datagen.collinear(n=97)
    parent, length, depth, _ = orc.prim_mst(X)
    pos = X[:, 0].astype(np.float64) / 3.0
    srt = np.argsort(pos)
    expect = {(min(int(a), int(b)), max(int(a), int(b))) for a, b in zip(srt[:-1], srt[1:])}
    assert brute.edge_set(parent) == expect
    assert length.sum() == 5.0 * (pos.max() - pos.min())
    r = int(np.where(srt == 0)[0][0])
    assert depth.max() == max(r, len(srt) - 1 - r)


def test_lattice_closed_form(orc):
    X = datagen.lattice(side=7, dim=2)
    _, length, _, _ = orc.prim_mst(X)
    assert np.all(length[1:] == 1.0)
    assert length.sum() == X.shape[0] - 1


def test_cycle_property(orc):
    """No non-tree pair is shorter than the longest edge on its tree path."""
    X = datagen.config(1, n=150)
    parent, length, _, _ = orc.prim_mst(X)
    S = brute.sqdist_matrix(X)
    tree = brute.edge_set(parent)
    n = X.shape[0]
    for i in range(n):
        for j in range(i + 1, n):
            if (i, j) in tree:
                continue
            assert np.sqrt(S[i, j]) >= brute.tree_path_max(parent, length, i, j)


def test_sqdist_left_to_right(orc):
    X = np.array([[1.0, 2.0, 3.0], [0.5, -1.0, 7.25]], np.float32)
    assert orc.sqdist(X, 0, 1) == 0.25 + 9.0 + 18.0625
    assert orc.sqdist(X, 1, 0) == orc.sqdist(X, 0, 1)
