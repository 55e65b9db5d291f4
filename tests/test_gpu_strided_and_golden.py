"""GPU entry points on strided inputs (row stride ld > d) and on the hand-worked
golden trees.

Strided inputs: the points are the first d columns of a wider array whose
extra columns hold NaN, so a kernel that read past column d - 1 of a row would
fail the non-finite check or change a result.  Every output must equal the
output for the same points stored contiguously (same kernels, same order of
operations).

Golden trees (tests/golden/*.json, derived by hand from the paper's
definitions): the tree stage alone reproduces their closed forms, including
the printed iteration count t of Algorithm 2 and the branch where the smallest
flow underflows so that the bracket starts at alpha0 = 0."""
import json
import math
import os

import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def iso():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1702_04739_amd as iso
    return iso


def _strided(X, extra=13):
    n, d = X.shape
    W = torch.full((n, d + extra), float("nan"), dtype=torch.float32, device="cuda")
    W[:, :d] = torch.from_numpy(X).cuda()
    S = W[:, :d]
    assert S.stride(0) == d + extra and S.stride(1) == 1
    return S


STRIDED_CASES = {
    "c3-n1500-d784": lambda: datagen.config(3, n=1500),
    "c1-n2000-d16": lambda: datagen.config(1),
    "ragged-n129-d17": lambda: datagen.uniform(129, 17),
}


@pytest.mark.parametrize("precision,recheck", [("fp32", "fp32"), ("bf16", "fp32"), ("bf16", "fp64"),
                                               ("fp8", "fp64"), ("int8", "fp32")])
@pytest.mark.parametrize("name", list(STRIDED_CASES))
def test_mst_strided_equals_contiguous(iso, name, precision, recheck):
    X = STRIDED_CASES[name]()
    if precision == "int8" and not name.startswith("c3"):
        pytest.skip("the INT8 screen takes 8-bit data only")
    H.log("strided mst %s %s + %s" % (name, precision, recheck))
    Xc = torch.from_numpy(X).cuda()
    Xs = _strided(X)
    pc, lc, ic = iso.mst(Xc, precision=precision, recheck=recheck)
    ps, ls, is_ = iso.mst(Xs, precision=precision, recheck=recheck)
    assert torch.equal(pc, ps) and torch.equal(lc, ls)
    assert ic["mst_weight"] == is_["mst_weight"]


def test_mst_prim_strided_equals_contiguous(iso):
    X = datagen.config(5, n=700)
    H.log("strided mst_prim n=700 d=128")
    pc, lc = iso.mst_prim(torch.from_numpy(X).cuda())
    ps, ls = iso.mst_prim(_strided(X))
    assert torch.equal(pc, ps) and torch.equal(lc, ls)


def test_graph_weights_strided_equals_contiguous(iso):
    X = datagen.config(2, n=900)
    H.log("strided graph_weights n=900 d=64")
    om_c, p_c = iso.graph_weights(torch.from_numpy(X).cuda(), 3.0, alpha=0.5)
    om_s, p_s = iso.graph_weights(_strided(X), 3.0, alpha=0.5)
    assert torch.equal(om_c, om_s) and torch.equal(p_c, p_s)


def test_adjoint_strided_equals_contiguous(iso):
    X = datagen.config(5, n=3000)
    H.log("strided adjoint n=3000 d=128")
    Xc = torch.from_numpy(X).cuda()
    labels, ik, info = iso.cluster(Xc, 16)
    sig, js, parent = info["sub"]["sigma"], info["sub"]["jstar"], info["parent"]
    gc, sc, Ic = iso.adjoint(Xc, parent, labels, js, sig, gW=0.7, gI=3.0)
    gs, ss, Is = iso.adjoint(_strided(X), parent, labels, js, sig, gW=0.7, gI=3.0)
    assert torch.equal(gc, gs) and sc == ss and Ic == Is


def _closed(expr):
    return eval(expr, {"exp": math.exp})


def _golden_tree(name):
    g = json.load(open(os.path.join(GOLDEN, name)))
    parent = torch.tensor(g["parent"], dtype=torch.int32, device="cuda")
    length = torch.tensor(g["length"], dtype=torch.float64, device="cuda")
    return g, parent, length


def test_hand_tree4_on_gpu(iso):
    g, parent, length = _golden_tree("hand_tree4.json")
    H.log("golden hand_tree4 on the GPU")
    labels, ik, info = iso.isoperimetric_subpartition(parent, length, g["k"], sigma=g["sigma"],
                                                      return_clusters=True)
    ref = _closed(g["i_k_closed_form"])
    assert abs(ik - ref) <= 1e-15 * ref
    assert labels.cpu().tolist() == g["labels"]
    assert info["t_paper"] == g["t_paper"]
    assert abs(info["alpha0_raw"] - _closed(g["alpha0_raw_closed_form"])) <= 1e-15 * info["alpha0_raw"]
    assert abs(info["beta0_raw"] - _closed(g["beta0_raw_closed_form"])) <= 1e-15 * info["beta0_raw"]
    assert info["jstar"] == g["jstar"]
    costs = (info["cluster_num"] / info["cluster_den"]).cpu().numpy()
    np.testing.assert_allclose(costs, [_closed(c) for c in g["cluster_costs_closed_form"]], rtol=1e-15)


def test_underflow_alpha0_zero_on_gpu(iso, orc_lib):
    """phi_* underflows: bracket [0, 4], 1076 bisection steps to the smallest
    subnormal, i_k = 0 exactly, the same labels and bracket as the oracle."""
    g, parent, length = _golden_tree("underflow_path4.json")
    H.log("golden underflow_path4 on the GPU")
    labels, ik, info = iso.isoperimetric_subpartition(parent, length, g["k"], sigma=g["sigma"],
                                                      return_clusters=True)
    assert info["alpha0_raw"] == 0.0 and info["alpha0"] == g["alpha0"] and info["beta0"] == g["beta0"]
    assert info["t_paper"] == g["t_paper"]
    assert info["iters"] == g["iters"]
    assert info["alpha"] == g["alpha"] and info["beta"] == g["beta"]
    assert ik == g["i_k"]
    assert labels.cpu().tolist() == g["labels"]
    assert info["jstar"] == g["jstar"]
    np.testing.assert_allclose(info["cluster_den"].cpu().numpy(),
                               [_closed(c) for c in g["cluster_den_closed_form"]], rtol=1e-15)
    ref = orc_lib.subpartition(np.array(g["parent"], np.int32), np.array(g["length"]), g["k"], sigma=g["sigma"])
    assert ref.iters == info["iters"] and ref.beta == info["beta"]


@pytest.fixture(scope="module")
def orc_lib():
    import oracle
    return oracle
