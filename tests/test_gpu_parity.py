"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars (floating point decides the tree's edges and the labels, integers are
compared exactly):
  - FP64 recheck: edge set identical to the oracle's Prim tree.
  - FP32 recheck: edge set identical except certified near ties (an edge swap
    whose two squared lengths differ by less than the FP32 evaluation error).
  - edge lengths and MST weight: relative 1e-12 (both sides compute the same
    FP64 left-to-right sums; sqrt may differ by an ulp).
  - tree search on an identical tree: labels identical, i_k relative 1e-12.
  - end to end: labels identical when the trees are, i_k relative 1e-9.
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


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


CASES = {
    "c1-n2000-d16": lambda: datagen.config(1),
    "c2-n2500-d64": lambda: datagen.config(2, n=2500),
    "c3-n1500-d784": lambda: datagen.config(3, n=1500),
    "c4-n1000-d4096": lambda: datagen.config(4, n=1000),
    "c5-n3000-d128": lambda: datagen.config(5, n=3000),
    "uniform-n333-d3": lambda: datagen.uniform(333, 3),
    "lattice-12x12": lambda: datagen.lattice(12, 2),
    "lattice-5^3": lambda: datagen.lattice(5, 3),
    "duplicates-n400": lambda: datagen.with_duplicates(400, 5, 60),
    "collinear-n300": lambda: datagen.collinear(300),
    "star-m200": lambda: datagen.star_points(200, 6),
    "tiny-n2": lambda: np.array([[0.0, 1.0], [2.0, -1.0]], np.float32),
    "tiny-n3": lambda: np.array([[0.0], [1.0], [3.0]], np.float32),
    "ragged-n129-d17": lambda: datagen.uniform(129, 17),
}

_cache = {}


def _oracle_tree(orc, name):
    if name not in _cache:
        X = CASES[name]()
        p, l, _, _ = orc.prim_mst(X)
        _cache[name] = (X, p, l)
    return _cache[name]


@pytest.mark.parametrize("rounds", ["default", "plain"])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("name", list(CASES))
def test_mst_fp64_recheck_identical(iso, orc, name, precision, rounds):
    """Same tree as the oracle; "plain" screens every round in the requested
    precision (no neighbour lists, no final round, no escalation to FP32),
    "default" lets rounds skip the full screen and a loose screen escalate."""
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s n=%d d=%d %s screen + fp64 recheck, %s rounds" % (name, *X.shape, precision, rounds))
    plain = rounds == "plain"
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision=precision, recheck="fp64",
                                   lists=not plain, final_round=not plain, escalate=not plain)
    if plain:
        assert info["list_rounds"] == 0 and info["final_components"] == 0
        assert info["screen_precision"] == precision
    gp = parent.cpu().numpy()
    gl = length.cpu().numpy()
    assert H.edge_set(gp) == H.edge_set(op)
    np.testing.assert_array_equal(gp, op)  # same tree rooted at 0 => same parent array
    np.testing.assert_allclose(gl, ol, rtol=1e-15, atol=0)
    W = ol.sum()
    assert abs(info["mst_weight"] - W) <= 1e-12 * max(W, 1e-300)


@pytest.mark.parametrize("recheck", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_mst_pair_bounds(iso, orc, name, recheck):
    """BF16 screen with each pair's own error bound in every capture threshold
    (forced; every round screened, no escalation): the oracle's tree with the
    FP64 recheck, the oracle's tree up to certified near ties with FP32."""
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s n=%d d=%d bf16 pair-bound screen + %s recheck" % (name, *X.shape, recheck))
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision="bf16", recheck=recheck, escalate=False,
                                   pair_bounds=True)
    H.log("  info %s" % info)
    assert info["pair_bounds"] and info["screen_precision"] == "bf16"
    assert info["list_rounds"] == 0 and info["final_components"] == 0
    gp = parent.cpu().numpy()
    if recheck == "fp64":
        np.testing.assert_array_equal(gp, op)
        np.testing.assert_allclose(length.cpu().numpy(), ol, rtol=1e-15, atol=0)
    else:
        swaps = H.check_tree_vs_oracle(X, gp, op, H.screen_tol(X.shape[1]))
        if swaps == 0:
            np.testing.assert_array_equal(gp, op)
        W = ol.sum()
        assert abs(info["mst_weight"] - W) <= 1e-6 * max(W, 1e-300)


def test_pair_bounds_chosen_for_heavy_tailed_norms(iso, orc):
    """Lognormal sparse rows (the communities recipe) have heavy-tailed norms:
    a BF16 request switches to pair bounds by itself and keeps the BF16 screen
    (no hand-over to FP32), with the oracle's tree; grid-valued image-like
    rows (light tails) keep the separable bound."""
    X, op, ol = _oracle_tree(orc, "c4-n1000-d4096")
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision="bf16", recheck="fp64")
    H.log("  c4 info %s" % info)
    assert info["pair_bounds"] and info["screen_precision"] == "bf16" and info["rescanned_rows"] == 0
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    X3, op3, _ = _oracle_tree(orc, "c3-n1500-d784")
    parent, _, info = iso.mst(torch.from_numpy(X3).cuda(), precision="bf16", recheck="fp64")
    H.log("  c3 info %s" % info)
    assert not info["pair_bounds"] and info["screen_precision"] == "bf16"
    np.testing.assert_array_equal(parent.cpu().numpy(), op3)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("name", list(CASES))
def test_mst_fp32_recheck_near_ties_only(iso, orc, name, precision):
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s n=%d d=%d %s screen + fp32 recheck" % (name, *X.shape, precision))
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision=precision, recheck="fp32")
    gp = parent.cpu().numpy()
    swaps = H.check_tree_vs_oracle(X, gp, op, H.screen_tol(X.shape[1]))
    W = ol.sum()
    assert abs(info["mst_weight"] - W) <= 1e-6 * max(W, 1e-300)
    if swaps == 0:
        np.testing.assert_array_equal(gp, op)


@pytest.mark.parametrize("name,k", [("c1-n2000-d16", 5), ("c5-n3000-d128", 16), ("c2-n2500-d64", 20),
                                    ("collinear-n300", 4), ("star-m200", 7), ("lattice-12x12", 3),
                                    ("tiny-n2", 2), ("tiny-n3", 3)])
@pytest.mark.parametrize("phi,bracket", [("exp", "pow2"), ("gauss_sq", "pow2"), ("exp", "paper")])
def test_subpartition_on_oracle_tree(iso, orc, name, k, phi, bracket):
    """Tree stage alone, fed the oracle's tree: identical labels and bracket."""
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s k=%d phi=%s bracket=%s" % (name, k, phi, bracket))
    ref = orc.subpartition(op, ol, k, phi=phi, bracket=bracket)
    labels, ik, info = iso.isoperimetric_subpartition(torch.from_numpy(op).cuda(), torch.from_numpy(ol).cuda(), k,
                                                      phi=phi, bracket=bracket, return_clusters=True)
    assert info["sigma"] == ref.sigma
    assert abs(ik - ref.i_k) <= 1e-12 * ref.i_k
    np.testing.assert_array_equal(labels.cpu().numpy(), ref.labels)
    assert info["max_depth"] == ref.max_depth
    assert info["t_paper"] == ref.t_paper or bracket == "paper"
    if bracket == "pow2":
        # identical power-of-two bracket and step count; the final bracket may
        # move by an ulp because phi = exp(.) is evaluated by the device libm
        # on one side and by glibc on the other (each within 1 ulp)
        assert info["alpha0"] == ref.alpha0 and info["beta0"] == ref.beta0
        assert abs(info["iters"] - ref.iters) <= 2
        assert abs(info["beta"] - ref.beta) <= 4 * np.spacing(ref.beta)
        assert abs(info["alpha"] - ref.alpha) <= 4 * np.spacing(ref.beta)
    np.testing.assert_array_equal(info["cluster_size"].cpu().numpy(), ref.cl_size)
    np.testing.assert_allclose(info["cluster_num"].cpu().numpy(), ref.cl_num, rtol=1e-12)
    np.testing.assert_allclose(info["cluster_den"].cpu().numpy(), ref.cl_den, rtol=1e-12)
    assert info["jstar"] == ref.jstar
    for key in ("alpha0_raw", "beta0_raw"):
        assert abs(info[key] - getattr(ref, key)) <= 1e-13 * abs(getattr(ref, key))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("name,k", [("c1-n2000-d16", 5), ("c5-n3000-d128", 16), ("c3-n1500-d784", 10),
                                    ("c2-n2500-d64", 20), ("c4-n1000-d4096", 50)])
def test_end_to_end(iso, orc, name, k, precision):
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s end to end k=%d %s screen" % (name, k, precision))
    ref = orc.subpartition(op, ol, k)
    labels, ik, info = iso.cluster(torch.from_numpy(X).cuda(), k, precision=precision, recheck="fp32")
    gp = info["parent"].cpu().numpy()
    assert abs(ik - ref.i_k) <= 1e-9 * ref.i_k
    if H.edge_set(gp) == H.edge_set(op):
        np.testing.assert_array_equal(labels.cpu().numpy(), ref.labels)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_determinism(iso, precision):
    X = torch.from_numpy(datagen.config(5, n=4000)).cuda()
    H.log("determinism n=4000 d=128 %s" % precision)
    a = iso.cluster(X, 16, precision=precision)
    b = iso.cluster(X, 16, precision=precision)
    assert torch.equal(a[0], b[0]) and a[1] == b[1]
    assert torch.equal(a[2]["parent"], b[2]["parent"]) and torch.equal(a[2]["length"], b[2]["length"])


def test_errors(iso):
    from paper_1702_04739_amd._lib import IsoError
    X = torch.zeros(10, 3, device="cuda")
    X[3, 1] = float("nan")
    with pytest.raises(IsoError) as e:
        iso.mst(X)
    assert e.value.code == -2
    parent = torch.tensor([-1, 0, 3, 2], dtype=torch.int32, device="cuda")  # 2 <-> 3 cycle
    length = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(IsoError) as e:
        iso.isoperimetric_subpartition(parent, length, 2)
    assert e.value.code == -1
    parent = torch.tensor([-1, 0, 0, 5], dtype=torch.int32, device="cuda")  # out of range
    with pytest.raises(IsoError) as e:
        iso.isoperimetric_subpartition(parent, length, 2)
    assert e.value.code == -1


@pytest.mark.parametrize("cfg,n", [(3, 3000), (4, 3000)])
def test_screen_precision_does_not_change_tree(iso, cfg, n):
    """The screen only proposes candidates: FP32, BF16 and FP8 screens give
    the same tree under the same recheck."""
    X = torch.from_numpy(datagen.config(cfg, n=n)).cuda()
    H.log("screen precision invariance config %d n=%d" % (cfg, n))
    a = iso.mst(X, precision="fp32")
    for prec in ("bf16", "fp8") + (("int8",) if cfg == 3 else ()):
        b = iso.mst(X, precision=prec)
        H.log("  %s: candidates %d rescanned %d (fp32: %d, %d)" % (prec, b[2]["candidates"], b[2]["rescanned_rows"],
                                                                   a[2]["candidates"], a[2]["rescanned_rows"]))
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("name", ["c3-n1500-d784", "lattice-12x12", "lattice-5^3"])
@pytest.mark.parametrize("recheck", ["fp64", "fp32"])
def test_int8_screen_8bit_data(iso, orc, name, recheck):
    """8-bit data (q/256 coordinates, integer lattices): the INT8 screen's
    exact integer distances give the same tree as the oracle (FP64 recheck)
    and the same tree as the FP32 screen (either recheck)."""
    X, op, ol = _oracle_tree(orc, name)
    H.log("case %s int8 screen + %s recheck" % (name, recheck))
    Xg = torch.from_numpy(X).cuda()
    parent, length, info = iso.mst(Xg, precision="int8", recheck=recheck)
    p32, l32, _ = iso.mst(Xg, precision="fp32", recheck=recheck)
    assert torch.equal(parent, p32) and torch.equal(length, l32)
    if recheck == "fp64":
        np.testing.assert_array_equal(parent.cpu().numpy(), op)


def test_int8_rejects_other_data(iso):
    from paper_1702_04739_amd._lib import IsoError
    X = torch.from_numpy(datagen.config(1, n=300)).cuda()
    with pytest.raises(IsoError) as e:
        iso.mst(X, precision="int8")
    assert e.value.code == -1


def test_identical_points(iso, orc):
    """All points equal: every edge has length 0 (a valid tree, zero weight);
    sigma = 0 is degenerate and the tree search rejects it cleanly."""
    from paper_1702_04739_amd._lib import IsoError
    X = np.full((300, 7), 0.25, np.float32)
    p, l, _, _ = orc.prim_mst(X)
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision="bf16", recheck="fp64")
    np.testing.assert_array_equal(parent.cpu().numpy(), p)
    assert info["mst_weight"] == 0.0
    with pytest.raises(IsoError) as e:
        iso.isoperimetric_subpartition(parent, length, 3)
    assert e.value.code == -1


LIST_CASES = {
    # 8-bit image-like rows (values q/256): the BF16 and INT8 screens are exact
    # there, so the second round's neighbour lists decide the later rounds
    "c3-n4000-d784": lambda: datagen.config(3, n=4000),
    "c3-n2600-d784-seed9": lambda: datagen.config(3, n=2600, seed=9),
}


@pytest.mark.parametrize("precision", ["bf16", "int8", "fp32"])
@pytest.mark.parametrize("name", list(LIST_CASES))
def test_neighbour_list_rounds_match_oracle(iso, orc, name, precision):
    """Rounds decided by the neighbour lists give the oracle's tree (FP64
    recheck: identical edges, lengths to 1e-12), and the lists are used."""
    if name not in _cache:
        X = LIST_CASES[name]()
        p, l, _, _ = orc.prim_mst(X)
        _cache[name] = (X, p, l)
    X, op, ol = _cache[name]
    H.log("list rounds %s %s" % (name, precision))
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision=precision, recheck="fp64",
                                   final_round=False)
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    np.testing.assert_allclose(length.cpu().numpy(), ol, rtol=1e-12, atol=0)
    H.log("  info %s" % info)
    assert info["rounds"] >= 3
    if precision != "fp32":
        assert info["list_rounds"] >= 1, info


def _cube_grid(side=6, dim=5, gap=3):
    """side x side unit cubes {0,1}^dim, cube (a, b) shifted by gap (a e_1 + b e_2):
    the first round joins each cube; between neighbouring cubes 2^(dim-1)
    pairs tie at distance gap - 1 and every neighbouring pair of cubes ties,
    so the final round's choices are all made by the id order."""
    v = np.stack(np.meshgrid(*[np.arange(2)] * dim, indexing="ij"), -1).reshape(-1, dim)
    pts = []
    for a in range(side):
        for b in range(side):
            o = np.zeros(dim)
            o[0], o[1] = gap * a, gap * b
            pts.append(v + o)
    return np.concatenate(pts).astype(np.float32)


def _two_clusters(n=600, d=12, seed=21):
    """Two tight clusters far apart: the tree's last edge is much longer than the rest."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d))
    X[n // 2:, 0] += 60.0
    return X[rng.permutation(n)].astype(np.float32)


FINAL_CASES = {
    "cubes-6x6-2^5": lambda: _cube_grid(),
    "uniform-n512-d8": lambda: datagen.uniform(512, 8),  # n a multiple of the 256-point tile
    "uniform-n256-d5": lambda: datagen.uniform(256, 5),  # exactly one tile
    "two-clusters-n600": lambda: _two_clusters(),
    "c3-n4000-d784": lambda: datagen.config(3, n=4000),
    "c1-n2000-d16": lambda: datagen.config(1),
    "c5-n3000-d128": lambda: datagen.config(5, n=3000),
}


@pytest.mark.parametrize("precision", ["fp32", "bf16", "int8"])
@pytest.mark.parametrize("name", list(FINAL_CASES))
def test_final_round_matches_oracle(iso, orc, name, precision):
    """The final round (all remaining components joined from their pairwise
    lightest edges) gives the oracle's tree under the FP64 recheck."""
    key = "final-" + name
    if key not in _cache:
        X = FINAL_CASES[name]()
        p, l, _, _ = orc.prim_mst(X)
        _cache[key] = (X, p, l)
    X, op, ol = _cache[key]
    if precision == "int8" and name.startswith(("c1", "c5", "uniform", "two-clusters")):
        pytest.skip("the INT8 screen takes 8-bit data only")
    H.log("final round %s %s" % (name, precision))
    parent, length, info = iso.mst(torch.from_numpy(X).cuda(), precision=precision, recheck="fp64")
    H.log("  info %s" % info)
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    np.testing.assert_allclose(length.cpu().numpy(), ol, rtol=1e-12, atol=0)
    # the final round runs when the screen's bound is tight (exact
    # representation: FP32, or BF16/INT8 on grid-valued data); with a loose
    # bound its recheck would be too large and the rounds stay plain
    if precision == "fp32" or name.startswith(("cubes", "c3")):
        assert info["final_components"] >= 2, info


def test_loose_screen_escalates_to_fp32(iso, orc):
    """Lognormal sparse data (the communities recipe): the FP8 bound is so
    loose that rows fall through to the exact rescan, so the call hands over
    to the FP32 screen; without escalation FP8 builds the same tree."""
    X, op, ol = _oracle_tree(orc, "c4-n1000-d4096")
    Xg = torch.from_numpy(X).cuda()
    H.log("escalation c4-n1000-d4096 fp8")
    parent, length, info = iso.mst(Xg, precision="fp8", recheck="fp64")
    H.log("  info %s" % info)
    assert info["screen_precision"] == "fp32"
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
    parent, length, info = iso.mst(Xg, precision="fp8", recheck="fp64", escalate=False)
    H.log("  strict %s" % info)
    assert info["screen_precision"] == "fp8" and info["rescanned_rows"] > 0
    np.testing.assert_array_equal(parent.cpu().numpy(), op)
