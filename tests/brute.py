"""Independent brute-force checkers used to pin the oracle (CPU only).

Nothing here calls the oracle: Kruskal's algorithm with a union-find, the
exhaustive enumeration of k-subpartitions, the cost function written from its
definition (Sec. 2.1, eq. 2.4) and tree-path maxima for the cycle property.
"""
from __future__ import annotations

import itertools

import numpy as np


def sqdist_matrix(X):
    """FP64 squared distances, accumulated left to right over coordinates."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    S = np.zeros((n, n))
    for t in range(d):
        diff = X[:, None, t] - X[None, :, t]
        S = S + diff * diff
    return S


def kruskal(X):
    """MST edge set under the total order (D^2, min id, max id)."""
    S = sqdist_matrix(X)
    n = S.shape[0]
    iu, ju = np.triu_indices(n, 1)
    keys = np.lexsort((ju, iu, S[iu, ju]))  # primary D^2, then min id, then max id
    par = list(range(n))

    def find(a):
        while par[a] != a:
            par[a] = par[par[a]]
            a = par[a]
        return a

    edges = []
    for e in keys:
        a, b = int(iu[e]), int(ju[e])
        ra, rb = find(a), find(b)
        if ra != rb:
            par[ra] = rb
            edges.append((a, b))
            if len(edges) == n - 1:
                break
    return set(edges), S


def edge_set(parent):
    return {(min(v, int(p)), max(v, int(p))) for v, p in enumerate(parent) if p >= 0}


def tree_path_max(parent, length, i, j):
    """Largest edge length on the tree path between i and j (parent-array tree)."""
    anc = {}
    a, m = i, 0.0
    while a >= 0:
        anc[a] = m
        if parent[a] >= 0:
            m = max(m, length[a])
        a = parent[a]
    b, mb = j, 0.0
    while b not in anc:
        mb = max(mb, length[b])
        b = parent[b]
    return max(anc[b], mb)


def cost_of(labels, k, parent, phi, omega0, p0):
    """max_j (phi(delta A_j) + p(A_j)) / omega(A_j) over the tree's edges (eq. 2.4),
    with A_j = {v : labels[v] == j}."""
    labels = np.asarray(labels)
    out = []
    for j in range(k):
        inA = labels == j
        if not inA.any():
            return np.inf, []
        bnd = 0.0
        for v, u in enumerate(parent):
            if u >= 0 and inA[v] != inA[u]:
                bnd += phi[v]
        out.append((bnd + p0[inA].sum()) / omega0[inA].sum())
    return max(out), out


def exhaustive_miso(k, parent, phi, omega0, p0):
    """min over all k-subpartitions (disjoint nonempty sets, need not cover X)
    of the cost, by enumerating every labelling in {-1, 0..k-1}^n (Sec. 2.1, eq. 2.6)."""
    parent = np.asarray(parent)
    n = parent.shape[0]
    phi = np.asarray(phi, np.float64)
    omega0 = np.asarray(omega0, np.float64)
    p0 = np.asarray(p0, np.float64)
    child = np.array([v for v in range(n) if parent[v] >= 0])
    par = parent[child]
    labs = np.array(list(itertools.product(range(-1, k), repeat=n)), dtype=np.int8)  # (M, n)
    # vectorised over labellings
    costs = np.zeros(labs.shape[0])
    valid = np.ones(labs.shape[0], bool)
    for j in range(k):
        inA = labs == j
        nonempty = inA.any(axis=1)
        valid &= nonempty
        cross = inA[:, child] != inA[:, par]
        bnd = cross.astype(np.float64) @ phi[child]
        num = bnd + inA.astype(np.float64) @ p0
        den = inA.astype(np.float64) @ omega0
        with np.errstate(divide="ignore", invalid="ignore"):
            c = np.where(nonempty, num / np.where(den > 0, den, 1.0), np.inf)
        costs = np.maximum(costs, c)
    costs[~valid] = np.inf
    return float(costs.min())


def random_tree(n, rng):
    """Random recursive tree rooted at 0 (parent[v] < v), then relabelled."""
    parent = np.full(n, -1, np.int64)
    for v in range(1, n):
        parent[v] = rng.integers(0, v)
    perm = np.concatenate([[0], 1 + rng.permutation(n - 1)])  # the root keeps id 0
    newp = np.full(n, -1, np.int64)
    for v in range(n):
        if parent[v] >= 0:
            newp[perm[v]] = perm[parent[v]]
    return newp.astype(np.int32)


def tree_degree_weights(parent, phi):
    """omega0(v) = sum of phi over v's tree edges (the tree-degree reading of eq. 2.2)."""
    n = len(parent)
    om = np.zeros(n)
    for v, u in enumerate(parent):
        if u >= 0:
            om[v] += phi[v]
            om[u] += phi[v]
    return om


def is_connected_in_tree(members, parent):
    members = set(int(m) for m in members)
    if not members:
        return False
    # a vertex set is connected in a rooted tree iff exactly one member has its parent outside
    tops = [m for m in members if parent[m] < 0 or int(parent[m]) not in members]
    return len(tops) == 1
