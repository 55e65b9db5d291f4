"""GPU adjoint (iso_backward / MSTIsoCost) on the 20,000 x 128 blob workload:
against the FP64 oracle's adjoint on the same tree and subpartition, and against
FP64 central differences (h = 1e-4, 64 random unit directions) of the
fixed-structure function evaluated in numpy."""
import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


@pytest.fixture(scope="module")
def forward():
    import paper_1702_04739_amd as iso
    X = datagen.config(5)  # n = 20000, d = 128
    Xg = torch.from_numpy(X).cuda()
    labels, ik, info = iso.cluster(Xg, 16)
    return iso, X, Xg, labels, ik, info


@pytest.mark.parametrize("phi", ["exp", "gauss_sq"])
def test_adjoint_matches_oracle(forward, phi):
    import oracle
    iso, X, Xg, labels, ik, info = forward
    H.log("adjoint vs oracle n=%d d=%d phi=%s" % (*X.shape, phi))
    sigma = info["sub"]["sigma"]
    jstar = info["sub"]["jstar"]
    parent = info["parent"]
    gX, gs, I = iso.adjoint(Xg, parent, labels, jstar, sigma, gW=0.7, gI=3.0, phi=phi)
    rX, rs, rW, rI, nd = oracle.backward(X, parent.cpu().numpy(), labels.cpu().numpy(), jstar, sigma, gW=0.7, gI=3.0,
                                         phi=phi)
    g = gX.cpu().numpy().astype(np.float64)
    scale = np.abs(rX).max()
    assert np.abs(g - rX).max() <= 1e-6 * scale
    assert abs(gs - rs) <= 1e-10 * max(abs(rs), 1e-300)
    assert abs(I - rI) <= 1e-12 * rI
    if phi == "exp":
        assert abs(I - ik) <= 1e-9 * ik


def test_adjoint_central_differences(forward):
    iso, X, Xg, labels, ik, info = forward
    H.log("adjoint vs central differences, 64 directions")
    sigma = info["sub"]["sigma"]
    jstar = info["sub"]["jstar"]
    parent = info["parent"].cpu().numpy()
    lab = labels.cpu().numpy()
    gW, gI = 0.7, 3.0
    gX, gs, _ = iso.adjoint(Xg, info["parent"], labels, jstar, sigma, gW=gW, gI=gI)
    g = gX.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(1005)
    Xd = X.astype(np.float64)
    h = 1e-4
    for _ in range(64):
        V = rng.standard_normal(Xd.shape)
        V /= np.linalg.norm(V)
        Wp, Ip = _W_I(Xd + h * V, parent, lab, jstar, sigma)
        Wm, Im = _W_I(Xd - h * V, parent, lab, jstar, sigma)
        fd = (gW * (Wp - Wm) + gI * (Ip - Im)) / (2 * h)
        an = float((g * V).sum())
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)
    Wp, Ip = _W_I(Xd, parent, lab, jstar, sigma + h)
    Wm, Im = _W_I(Xd, parent, lab, jstar, sigma - h)
    fd = gI * (Ip - Im) / (2 * h)
    assert abs(fd - gs) <= 1e-6 * max(1.0, abs(gs))


def test_autograd_function(forward):
    iso, X, Xg, labels, ik, info = forward
    H.log("MSTIsoCost autograd")
    sigma = torch.tensor(info["sub"]["sigma"], dtype=torch.float64, device="cuda", requires_grad=True)
    pts = Xg.clone().requires_grad_(True)
    W, I, lab = iso.MSTIsoCost.apply(pts, sigma, 16)
    assert abs(W.item() - info["mst"]["mst_weight"]) <= 1e-12 * W.item()
    assert abs(I.item() - ik) <= 1e-12 * ik
    assert torch.equal(lab, labels)
    (0.7 * W + 3.0 * I).backward()
    gX, gs, _ = iso.adjoint(Xg, info["parent"], labels, info["sub"]["jstar"], info["sub"]["sigma"], 0.7, 3.0)
    assert torch.equal(pts.grad, gX)
    assert sigma.grad.item() == gs
