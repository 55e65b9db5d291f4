"""Helpers for the GPU parity tests: comparisons of a GPU tree / subpartition
with the oracle's, and certification of near-tie edge swaps."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def edge_set(parent):
    parent = np.asarray(parent)
    v = np.where(parent >= 0)[0]
    p = parent[v]
    return set(zip(np.minimum(v, p).tolist(), np.maximum(v, p).tolist()))


def d2_64(X, i, j):
    a = X[i].astype(np.float64)
    b = X[j].astype(np.float64)
    s = 0.0
    for t in range(a.shape[0]):
        df = a[t] - b[t]
        s = s + df * df
    return s


def path_edges(parent, a, b):
    """Edges (min, max) on the tree path between a and b in a parent-array tree."""
    anc = []
    x = a
    seen = {}
    while x >= 0:
        seen[x] = len(anc)
        anc.append(x)
        x = parent[x]
    y, tail = b, []
    while y not in seen:
        tail.append(y)
        y = parent[y]
    lca = y
    up = anc[: seen[lca] + 1]
    nodes = up + tail[::-1]
    return [(min(u, w), max(u, w)) for u, w in zip(nodes[:-1], nodes[1:])]


def check_tree_vs_oracle(X, gpu_parent, orc_parent, tol_rel):
    """Edge sets equal, except GPU edges whose swap with an oracle-tree edge on
    their cycle is a certified near tie: |D^2(e) - D^2(f)| <= tol_rel * (D^2(e) + D^2(f)).
    Returns the number of certified swaps."""
    ge, oe = edge_set(gpu_parent), edge_set(orc_parent)
    assert len(ge) == len(oe) == len(gpu_parent) - 1
    extra = ge - oe
    swaps = 0
    orc_parent = np.asarray(orc_parent)
    for (a, b) in sorted(extra):
        de = d2_64(X, a, b)
        ok = False
        for (u, w) in path_edges(orc_parent, a, b):
            df = d2_64(X, u, w)
            if abs(de - df) <= tol_rel * (de + df):
                ok = True
                break
        assert ok, "GPU edge (%d,%d) D2=%r is not a near tie of the oracle tree" % (a, b, de)
        swaps += 1
    return swaps


def screen_tol(d):
    """Relative tolerance between the FP32 recheck order and the FP64 order."""
    return 4.0 * (d + 2) * 2.0 ** -24


def check_subpartition_structure(parent, length, labels, k, sigma, beta, i_k, jstar=None, root=0):
    """k disjoint nonempty clusters, each connected in the tree, each of cost
    <= beta (tree-degree omega), i_k = max cost."""
    parent = np.asarray(parent)
    labels = np.asarray(labels)
    n = len(parent)
    phi = np.where(parent >= 0, np.exp(-np.asarray(length) / sigma), 0.0)
    om = np.zeros(n)
    v = np.where(parent >= 0)[0]
    np.add.at(om, v, phi[v])
    np.add.at(om, parent[v], phi[v])
    costs = []
    for j in range(k):
        inA = labels == j
        assert inA.any(), "cluster %d empty" % j
        tops = np.where(inA & ((parent < 0) | ~inA[np.maximum(parent, 0)]))[0]
        assert len(tops) == 1, "cluster %d not connected" % j
        cross = inA[v] != inA[parent[v]]
        num = phi[v][cross].sum()
        den = om[inA].sum()
        costs.append(num / den)
    costs = np.array(costs)
    assert np.all(costs <= beta * (1 + 1e-12))
    assert abs(costs.max() - i_k) <= 1e-9 * i_k
    if jstar is not None:
        assert abs(costs[jstar] - i_k) <= 1e-9 * i_k
    return costs
