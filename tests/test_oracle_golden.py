"""Hand-worked fixtures under tests/golden/ (derivations inside each file)."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_tree4(orc):
    g = json.load(open(os.path.join(GOLDEN, "hand_tree4.json")))
    res = orc.subpartition(np.array(g["parent"], np.int32), np.array(g["length"]), g["k"], sigma=g["sigma"])
    ik = eval(g["i_k_closed_form"], {"exp": math.exp})
    assert abs(res.i_k - ik) <= 1e-15 * ik
    np.testing.assert_array_equal(res.labels, g["labels"])
    costs = [eval(c, {"exp": math.exp}) for c in g["cluster_costs_closed_form"]]
    np.testing.assert_allclose(res.cl_num / res.cl_den, costs, rtol=1e-15)
    assert res.jstar == g["jstar"]
