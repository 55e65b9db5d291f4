"""Pins of the oracle's adjoint: gradient of the total tree length W and of the
optimal cluster's cost I (eq. 2.4 with the tree-degree omega) with respect to
the points and sigma, holding the tree and the subpartition fixed.

Checked against closed forms and FP64 central differences of W and I
evaluated here from their definitions (numpy, no oracle call)."""
import numpy as np
import pytest

from paper_1702_04739_amd import datagen


def _W_I(X, parent, labels, jstar, sigma, phi_kind=0):
    X = np.asarray(X, np.float64)
    v = np.where(parent >= 0)[0]
    u = parent[v]
    D = np.sqrt(((X[v] - X[u]) ** 2).sum(axis=1))
    phi = np.exp(-D / sigma) if phi_kind == 0 else np.exp(-D * D / (2 * sigma * sigma))
    inv, inu = labels[v] == jstar, labels[u] == jstar
    num = phi[inv != inu].sum()
    inner = phi[inv & inu].sum()
    return D.sum(), num / (2 * inner + num)


def test_two_points_closed_form(orc):
    X = np.array([[0.0, 0.0], [3.0, 4.0]], np.float32)
    parent = np.array([-1, 0], np.int32)
    labels = np.array([0, 1], np.int32)
    gX, gs, W, I, nd = orc.backward(X, parent, labels, 0, 2.0, gW=1.0, gI=0.0)
    assert W == 5.0 and nd == 0
    np.testing.assert_allclose(gX, [[-0.6, -0.8], [0.6, 0.8]], rtol=0, atol=1e-15)
    assert gs == 0.0
    # single boundary edge: I = phi/phi = 1 regardless of geometry
    gX, gs, W, I, nd = orc.backward(X, parent, labels, 0, 2.0, gW=0.0, gI=1.0)
    assert I == 1.0
    np.testing.assert_allclose(gX, 0.0, atol=1e-15)
    assert abs(gs) < 1e-15


def test_dW_is_sum_of_unit_vectors(orc):
    X = datagen.config(5, n=300)
    parent, _, _, _ = orc.prim_mst(X)
    labels = np.zeros(len(parent), np.int32)
    gX, gs, W, _, _ = orc.backward(X, parent, labels, 0, 1.0, gW=1.0, gI=0.0)
    Xd = X.astype(np.float64)
    ref = np.zeros_like(Xd)
    for v, u in enumerate(parent):
        if u < 0:
            continue
        e = Xd[v] - Xd[u]
        e /= np.linalg.norm(e)
        ref[v] += e
        ref[u] -= e
    np.testing.assert_allclose(gX, ref, rtol=0, atol=1e-12)
    assert gs == 0.0


@pytest.mark.parametrize("phi_kind", [0, 1])
def test_central_differences(orc, phi_kind):
    """64 random unit directions, h = 1e-4, on the fixed-structure function."""
    X = datagen.config(5, n=400)
    parent, length, res = orc.run(X, 6, phi="exp" if phi_kind == 0 else "gauss_sq")
    labels, jstar, sigma = res.labels, res.jstar, res.sigma
    gW, gI = 0.7, 3.0
    gX, gs, W, I, nd = orc.backward(X, parent, labels, jstar, sigma, gW=gW, gI=gI,
                                    phi="exp" if phi_kind == 0 else "gauss_sq")
    W0, I0 = _W_I(X, parent, labels, jstar, sigma, phi_kind)
    assert abs(W - W0) <= 1e-12 * W0 and abs(I - I0) <= 1e-12 * I0
    assert abs(I - res.i_k) <= 1e-9 * res.i_k
    rng = np.random.default_rng(1005)
    Xd = X.astype(np.float64)
    h = 1e-4
    for _ in range(64):
        V = rng.standard_normal(Xd.shape)
        V /= np.linalg.norm(V)
        Wp, Ip = _W_I(Xd + h * V, parent, labels, jstar, sigma, phi_kind)
        Wm, Im = _W_I(Xd - h * V, parent, labels, jstar, sigma, phi_kind)
        fd = (gW * (Wp - Wm) + gI * (Ip - Im)) / (2 * h)
        an = float((gX * V).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    Wp, Ip = _W_I(Xd, parent, labels, jstar, sigma + h, phi_kind)
    Wm, Im = _W_I(Xd, parent, labels, jstar, sigma - h, phi_kind)
    fd = gI * (Ip - Im) / (2 * h)
    assert abs(fd - gs) <= 1e-7 * max(1.0, abs(gs))
