"""GPU: the bounding-ball test that lets a Boruvka round skip tile pairs.

A skipped tile pair provably holds no pair that the round needs, so the tree
must be the one every-tile-pair screening builds, bit for bit (parent array and
FP64 lengths), for every screen precision, with and without the neighbour lists
and the final round, with pair bounds, and with tiles that hold no point.  On
clustered data (the image-like recipe: ten separated centres) most tile pairs
are skipped; against the oracle the pruned tree is checked here on a case whose
final round is pruned, on a lattice (ties everywhere) and on a mixture with
outliers, and at full size by the digest tests.  Below 8,192 points (32 tiles)
every pair is screened.
"""
import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def iso():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1702_04739_amd as iso
    return iso


CASES = {
    "c3-n20000-d784": lambda: datagen.config(3, n=20000),
    "c2-n20000-d64": lambda: datagen.config(2, n=20000),
    "c5-n20000-d128": lambda: datagen.config(5, n=20000),
    "c1-n10000-d16": lambda: datagen.config(1, n=10000),
    "uniform-n9000-d8": lambda: datagen.uniform(9000, 8),
    "duplicates-n9000": lambda: datagen.with_duplicates(9000, 5, 1800),
    # n a multiple of the tile: the padded order ends with a tile of padding only
    "c3-n8192-d784": lambda: datagen.config(3, n=8192),
    # ties everywhere (every lattice edge has length 1) and a degenerate set
    "lattice-96x96": lambda: datagen.lattice(96, 2),
    "constant-n9000": lambda: np.full((9000, 6), 0.25, np.float32),
}


def _run(iso, X, **kw):
    parent, length, info = iso.mst(X, **kw)
    return parent.cpu().numpy(), length.cpu().numpy(), info


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8", "int8"])
@pytest.mark.parametrize("name", list(CASES))
def test_pruned_tree_equals_full_screen(iso, name, precision):
    Xh = CASES[name]()
    if precision == "int8" and not name.startswith("c3"):
        pytest.skip("INT8 screen: 8-bit data only (the image-like recipe)")
    X = torch.from_numpy(Xh).cuda()
    H.log("case %s n=%d d=%d %s screen, pruned vs every tile pair" % (name, *Xh.shape, precision))
    p0, l0, i0 = _run(iso, X, precision=precision, recheck="fp32", prune=False)
    p1, l1, i1 = _run(iso, X, precision=precision, recheck="fp32", prune=True)
    H.log("  full %s" % i0)
    H.log("  pruned %s" % i1)
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(l1, l0)
    assert i0["tile_pairs"] == i0["tile_pairs_full"]
    assert i1["tile_pairs"] <= i1["tile_pairs_full"]
    if name.startswith("c3-n20000"):
        # ten separated centres: most tile pairs are skipped
        assert i1["tile_pairs"] < 0.6 * i1["tile_pairs_full"]


@pytest.mark.parametrize("rounds", ["plain", "no-final", "no-lists"])
def test_pruned_plain_rounds(iso, rounds):
    """Every round a screened round (no lists, no final round), or one of the
    two off: the same tree with and without the test."""
    Xh = datagen.config(3, n=12000)
    X = torch.from_numpy(Xh).cuda()
    kw = dict(precision="bf16", recheck="fp32", escalate=False,
              lists=rounds == "no-final", final_round=rounds == "no-lists")
    H.log("c3 n=12000 bf16, %s rounds" % rounds)
    p0, l0, _ = _run(iso, X, prune=False, **kw)
    p1, l1, i1 = _run(iso, X, prune=True, **kw)
    H.log("  pruned %s" % i1)
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(l1, l0)
    assert i1["tile_pairs"] < i1["tile_pairs_full"]


def test_pruned_pair_bounds(iso):
    """Heavy-tailed norms (the communities recipe): the BF16 screen with pair
    bounds, where a point's reach is its running upper bound."""
    Xh = datagen.config(4, n=9000)
    X = torch.from_numpy(Xh).cuda()
    H.log("c4 n=9000 d=4096 bf16 pair bounds")
    p0, l0, i0 = _run(iso, X, precision="bf16", recheck="fp32", pair_bounds=True, escalate=False, prune=False)
    p1, l1, i1 = _run(iso, X, precision="bf16", recheck="fp32", pair_bounds=True, escalate=False, prune=True)
    H.log("  full %s" % i0)
    H.log("  pruned %s" % i1)
    assert i1["pair_bounds"]
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(l1, l0)


def test_pruned_final_round_matches_oracle(iso):
    """A case whose final round is pruned per pair of components, against the
    oracle's FP64 tree."""
    import oracle
    Xh = datagen.config(5, n=9000)
    op, ol, _, _ = oracle.prim_mst(Xh)
    parent, length, info = iso.mst(torch.from_numpy(Xh).cuda(), precision="bf16", recheck="fp64")
    H.log("  c5 n=9000 info %s" % info)
    assert info["final_components"] > 1
    assert info["tile_pairs"] < info["tile_pairs_full"]
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    np.testing.assert_allclose(length.cpu().numpy(), ol, rtol=1e-15, atol=0)


@pytest.mark.parametrize("name", ["lattice-96x96", "c1-n10000-d16"])
def test_pruned_ties_match_oracle(iso, name):
    """Many equal distances (a square lattice) and a mixture with outliers,
    FP64 recheck: the pruned tree is the oracle's, edge for edge."""
    import oracle
    Xh = CASES[name]()
    op, ol, _, _ = oracle.prim_mst(Xh)
    parent, length, info = iso.mst(torch.from_numpy(Xh).cuda(), precision="fp32", recheck="fp64")
    H.log("  %s info %s" % (name, info))
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    np.testing.assert_allclose(length.cpu().numpy(), ol, rtol=1e-15, atol=0)


def test_pruned_strided_input(iso):
    """Rows with a stride larger than d (a column slice of a wider array): the
    pruning kernels read X through ld like the screen and the recheck."""
    Xw = datagen.config(5, n=9000)
    wide = np.concatenate([Xw, np.ones((Xw.shape[0], 7), np.float32)], axis=1)
    Xs = torch.from_numpy(wide).cuda()[:, :Xw.shape[1]]
    assert Xs.stride(0) == Xw.shape[1] + 7
    p0, l0, _ = _run(iso, torch.from_numpy(Xw).cuda(), precision="bf16", recheck="fp32", prune=False)
    p1, l1, i1 = _run(iso, Xs, precision="bf16", recheck="fp32", prune=True)
    H.log("  strided info %s" % i1)
    assert i1["tile_pairs"] < i1["tile_pairs_full"]
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(l1, l0)
