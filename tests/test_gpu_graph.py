"""GPU parity of the full-graph weights (eq. 2.2 read literally, eq. 2.3 with
alpha > 0) and of the tree search that uses them, against the FP64 oracle.

Both sides form every distance as the square root of the same FP64
left-to-right sum and add the row terms in ascending j, so D, the potential
p and the distance sums are bit-identical; phi = exp(.) differs by at most an
ulp between the device libm and glibc, so omega0 is compared to 1e-13
relative, and the tree search to the bars of the tree-degree case (labels
identical, i_k within 1e-12, final bracket within 4 ulp).
"""
import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "c1-n2000-d16": lambda: datagen.config(1),
    "c5-n1500-d128": lambda: datagen.config(5, n=1500),
    "c2-n1200-d64": lambda: datagen.config(2, n=1200),
    "ragged-n129-d17": lambda: datagen.uniform(129, 17),
}

_cache = {}


def _tree(orc, name):
    if name not in _cache:
        X = CASES[name]()
        p, l, _, _ = orc.prim_mst(X)
        _cache[name] = (X, p, l, orc.lower_median(p, l))
    return _cache[name]


@pytest.fixture(scope="module")
def iso():
    import paper_1702_04739_amd as iso
    return iso


@pytest.mark.parametrize("phi", ["exp", "gauss_sq"])
@pytest.mark.parametrize("name", list(CASES))
def test_graph_weights_match_oracle(iso, orc, name, phi):
    X, p, l, sigma = _tree(orc, name)
    alpha = 0.05
    H.log("graph weights %s phi=%s" % (name, phi))
    om, p0 = iso.graph_weights(torch.from_numpy(X).cuda(), sigma, phi=phi, alpha=alpha)
    _, ref_om, ref_p0 = orc.tree_weights(p, l, sigma, omega="full", phi=phi, alpha_pot=alpha, X=X)
    np.testing.assert_allclose(om.cpu().numpy(), ref_om, rtol=1e-13, atol=0)
    np.testing.assert_array_equal(p0.cpu().numpy(), ref_p0)


def test_sigma_median(iso, orc):
    X, p, l, sigma = _tree(orc, "c1-n2000-d16")
    assert iso.sigma_median(torch.from_numpy(p).cuda(), torch.from_numpy(l).cuda()) == sigma


@pytest.mark.parametrize("name,k", [("c1-n2000-d16", 5), ("c5-n1500-d128", 16), ("c2-n1200-d64", 20),
                                    ("ragged-n129-d17", 3)])
@pytest.mark.parametrize("omega,alpha", [("full", 0.0), ("full", 0.05), ("tree", 0.05)])
def test_subpartition_full_weights(iso, orc, name, k, omega, alpha):
    X, p, l, sigma = _tree(orc, name)
    H.log("subpartition %s k=%d omega=%s alpha=%g" % (name, k, omega, alpha))
    ref = orc.subpartition(p, l, k, omega=omega, alpha_pot=alpha, X=X)
    Xg = torch.from_numpy(X).cuda()
    om, p0 = iso.graph_weights(Xg, sigma, alpha=alpha, omega=(omega == "full"))
    labels, ik, info = iso.isoperimetric_subpartition(torch.from_numpy(p).cuda(), torch.from_numpy(l).cuda(), k,
                                                      omega0=om, p0=p0, return_clusters=True)
    assert info["sigma"] == ref.sigma
    assert abs(ik - ref.i_k) <= 1e-12 * ref.i_k
    np.testing.assert_array_equal(labels.cpu().numpy(), ref.labels)
    assert info["alpha0"] == ref.alpha0 and info["beta0"] == ref.beta0
    assert abs(info["beta"] - ref.beta) <= 4 * np.spacing(ref.beta)
    np.testing.assert_array_equal(info["cluster_size"].cpu().numpy(), ref.cl_size)


def test_cluster_full_end_to_end(iso, orc):
    X, p, l, sigma = _tree(orc, "c1-n2000-d16")
    H.log("cluster c1 omega=full alpha=0.05 fp64 recheck")
    ref = orc.subpartition(p, l, 5, omega="full", alpha_pot=0.05, X=X)
    labels, ik, info = iso.cluster(torch.from_numpy(X).cuda(), 5, precision="bf16", recheck="fp64", omega="full",
                                   alpha=0.05)
    np.testing.assert_array_equal(info["parent"].cpu().numpy(), p)
    assert abs(ik - ref.i_k) <= 1e-12 * ref.i_k
    np.testing.assert_array_equal(labels.cpu().numpy(), ref.labels)


def test_graph_weights_errors(iso):
    from paper_1702_04739_amd._lib import IsoError
    X = torch.zeros(10, 3, device="cuda")
    with pytest.raises(IsoError):
        iso.graph_weights(X, 0.0)
    with pytest.raises(IsoError):
        iso.graph_weights(X, 1.0, alpha=-1.0)
