"""Pins of the oracle's tree search (Sec. 2.2: Algorithm 1 inside Algorithm 2,
labelled as in Algorithm 4).

The oracle's i_k is compared with the exhaustive minimum over all
k-subpartitions (eq. 2.6) on tiny trees, with closed forms on paths and stars,
and with structural invariants of its output.
"""
import math

import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import brute


def _lengths(n, rng, lo=0.2, hi=3.0):
    length = rng.uniform(lo, hi, size=n)
    length[0] = 0.0
    return length


@pytest.mark.parametrize("seed", range(60))
def test_exhaustive_tree_reading(orc, seed):
    """i_k equals the brute-force minimum over D_k (n <= 8, k <= 3)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 9))
    k = int(rng.integers(2, min(3, n) + 1))
    parent = brute.random_tree(n, rng)
    length = _lengths(n, rng)
    res = orc.subpartition(parent, length, k, sigma=float(rng.uniform(0.5, 2.0)))
    phi = np.where(parent >= 0, np.exp(-length / res.sigma), 0.0)
    om = brute.tree_degree_weights(parent, phi)
    best = brute.exhaustive_miso(k, parent, phi, om, np.zeros(n))
    assert abs(res.i_k - best) <= 1e-12 * best
    # the returned subpartition attains i_k
    c, _ = brute.cost_of(res.labels, k, parent, phi, om, np.zeros(n))
    assert abs(c - res.i_k) <= 1e-12 * res.i_k


@pytest.mark.parametrize("seed", range(25))
def test_exhaustive_with_potential_and_full_omega(orc, seed):
    """Same with the full-graph omega of eq. 2.2 and a positive potential
    (eq. 2.3) on an actual point set's MST."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 8))
    k = int(rng.integers(2, min(3, n) + 1))
    X = rng.standard_normal((n, 2)).astype(np.float32)
    alpha_pot = float(rng.choice([0.0, 0.05, 0.3]))
    parent, length, res = orc.run(X, k, omega="full", alpha_pot=alpha_pot)
    S = brute.sqdist_matrix(X)
    Dm = np.sqrt(S)
    phi = np.where(parent >= 0, np.exp(-length / res.sigma), 0.0)
    F = np.exp(-Dm / res.sigma)
    np.fill_diagonal(F, 0.0)
    om = F.sum(axis=1)
    p0 = alpha_pot * Dm.sum(axis=1)
    best = brute.exhaustive_miso(k, parent, phi, om, p0)
    assert abs(res.i_k - best) <= 1e-12 * best


@pytest.mark.parametrize("n,k", [(n, k) for n in range(3, 11) for k in range(2, 5) if k <= n])
def test_uniform_path_closed_form(orc, n, k):
    """Uniform path P_n (tree-degree omega): MISO_k = (k-1)/(n-1) exactly when
    (n-1)/(k-1) is an odd integer, and strictly more otherwise."""
    parent = np.arange(-1, n - 1, dtype=np.int32)   # 0 - 1 - 2 - ... - (n-1)
    length = np.ones(n)
    length[0] = 0.0
    res = orc.subpartition(parent, length, k, sigma=1.0)
    q = (n - 1) / (k - 1)
    target = (k - 1) / (n - 1)
    if q == int(q) and int(q) % 2 == 1:
        assert abs(res.i_k - target) <= 1e-12
    else:
        assert res.i_k > target * (1 + 1e-9)
    phi = np.where(parent >= 0, math.exp(-1.0), 0.0)
    om = brute.tree_degree_weights(parent, phi)
    best = brute.exhaustive_miso(k, parent, phi, om, np.zeros(n)) if n <= 9 else None
    if best is not None:
        assert abs(res.i_k - best) <= 1e-12


@pytest.mark.parametrize("m,k", [(3, 2), (5, 2), (5, 4), (7, 8), (40, 10)])
def test_star_closed_form(orc, m, k):
    """Star K_{1,m} with equal weights: MISO_k = 1 for 2 <= k <= m+1."""
    n = m + 1
    parent = np.zeros(n, np.int32)
    parent[0] = -1
    length = np.full(n, 1.5)
    length[0] = 0.0
    res = orc.subpartition(parent, length, k, sigma=1.0)
    assert abs(res.i_k - 1.0) <= 1e-12


def test_tree_invariants_on_data(orc):
    """Exactly k disjoint nonempty clusters, each connected in T, each of cost <=
    beta; i_k = max cost <= 1 for the tree-degree omega; the bisection ends at
    FP64 resolution; the cut count is monotone in N."""
    X = datagen.config(1, n=600)
    k = 5
    parent, length, res = orc.run(X, k)
    phi = np.where(parent >= 0, np.exp(-length / res.sigma), 0.0)
    om = brute.tree_degree_weights(parent, phi)
    labs = res.labels
    assert set(np.unique(labs)) <= set(range(-1, k))
    costs = []
    for j in range(k):
        members = np.where(labs == j)[0]
        assert members.size == res.cl_size[j] > 0
        assert brute.is_connected_in_tree(members, parent)
        c = brute.cost_of(np.where(labs == j, 0, -1), 1, parent, phi, om, np.zeros(len(parent)))[0]
        assert c <= res.beta
        assert abs(c - res.cl_num[j] / res.cl_den[j]) <= 1e-12 * c
        costs.append(c)
    assert abs(max(costs) - res.i_k) <= 1e-12 * res.i_k
    assert int(np.argmax(costs)) == res.jstar
    assert res.i_k <= 1.0
    mid = (res.alpha + res.beta) / 2
    assert mid in (res.alpha, res.beta)
    assert res.alpha0 <= res.alpha0_raw and res.beta0 > res.beta0_raw
    assert math.frexp(res.alpha0)[0] == 0.5 and math.frexp(res.beta0)[0] == 0.5
    # monotone decision (Algorithm 1 as a function of N)
    depth = orc.tree_depth(parent)
    order = orc.tree_order(depth)
    p0 = np.zeros(len(parent))
    Ns = np.geomspace(res.alpha0, res.beta0, 200)
    counts = [orc.decide(parent, order, phi, om, p0, len(parent), N) for N in Ns]
    assert all(a <= b for a, b in zip(counts, counts[1:]))
    assert orc.decide(parent, order, phi, om, p0, k, res.beta) == k
    assert orc.decide(parent, order, phi, om, p0, k, res.alpha) < k


def test_separated_blobs(orc):
    """Two blobs 100 sigma apart, k = 2: the two clusters are the two blobs."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 3))
    B = rng.standard_normal((50, 3)) + 400.0
    X = np.vstack([A, B]).astype(np.float32)
    truth = np.r_[np.zeros(40, int), np.ones(50, int)]
    _, _, res = orc.run(X, 2)
    for j in range(2):
        members = truth[res.labels == j]
        assert members.size > 0 and np.all(members == members[0])
    assert set(truth[res.labels >= 0]) == {0, 1}


def test_paper_bracket_agrees(orc):
    X = datagen.config(1, n=300)
    parent, length, r1 = orc.run(X, 4)
    r2 = orc.subpartition(parent, length, 4, bracket="paper")
    assert abs(r1.i_k - r2.i_k) <= 1e-12 * r1.i_k
    assert r2.alpha0 == r2.alpha0_raw and r2.beta0 > r2.beta0_raw
    assert r1.t_paper == r2.t_paper


def test_lower_median(orc):
    rng = np.random.default_rng(9)
    for n in (2, 3, 10, 11):
        parent = brute.random_tree(n, rng)
        length = _lengths(n, rng)
        m = n - 1
        assert orc.lower_median(parent, length) == np.sort(length[1:])[(m - 1) // 2]


def test_rejects_bad_input(orc):
    parent = np.array([-1, 0, 1], np.int32)
    length = np.array([0.0, 1.0, 1.0])
    with pytest.raises(RuntimeError):
        orc.subpartition(parent, length, 1)
    with pytest.raises(RuntimeError):
        orc.subpartition(parent, length, 4)
    with pytest.raises(RuntimeError):
        orc.subpartition(np.array([-1, 2, 1], np.int32), length, 2)  # cycle 1 <-> 2
    with pytest.raises(ValueError):
        orc.tree_depth(np.array([0, 0, 1], np.int32))
