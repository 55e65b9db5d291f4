"""The paper's MST construction (Algorithm 3, GPU Prim) against the FP64
oracle's Prim: identical parent arrays, lengths and insertion order (both
use the FP64 left-to-right distances and the edge order (D^2, min id, max
id)), and the same tree as the Boruvka path with the FP64 recheck."""
import numpy as np
import pytest

from paper_1702_04739_amd import datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "c1-n2000-d16": lambda: datagen.config(1),
    "c5-n1000-d128": lambda: datagen.config(5, n=1000),
    "lattice-12x12": lambda: datagen.lattice(12, 2),
    "duplicates-n400": lambda: datagen.with_duplicates(400, 5, 60),
    "tiny-n2": lambda: np.array([[0.0, 1.0], [2.0, -1.0]], np.float32),
    "ragged-n129-d17": lambda: datagen.uniform(129, 17),
}


@pytest.mark.parametrize("name", list(CASES))
def test_prim_matches_oracle(orc, name):
    import paper_1702_04739_amd as iso
    X = CASES[name]()
    H.log("gpu prim %s n=%d d=%d" % (name, *X.shape))
    p, l, _, order = orc.prim_mst(X)
    Xg = torch.from_numpy(X).cuda()
    gp, gl, go = iso.mst_prim(Xg, return_order=True)
    np.testing.assert_array_equal(gp.cpu().numpy(), p)
    np.testing.assert_array_equal(gl.cpu().numpy(), l)
    np.testing.assert_array_equal(go.cpu().numpy(), order)
    bp, bl, _ = iso.mst(Xg, precision="bf16", recheck="fp64")
    assert torch.equal(bp, gp)
