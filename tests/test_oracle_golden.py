"""Hand-worked fixtures under tests/golden/ (derivations inside each file)."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _closed(expr):
    return eval(expr, {"exp": math.exp})


def test_hand_tree4(orc):
    g = json.load(open(os.path.join(GOLDEN, "hand_tree4.json")))
    res = orc.subpartition(np.array(g["parent"], np.int32), np.array(g["length"]), g["k"], sigma=g["sigma"])
    ik = _closed(g["i_k_closed_form"])
    assert abs(res.i_k - ik) <= 1e-15 * ik
    np.testing.assert_array_equal(res.labels, g["labels"])
    costs = [_closed(c) for c in g["cluster_costs_closed_form"]]
    np.testing.assert_allclose(res.cl_num / res.cl_den, costs, rtol=1e-15)
    assert res.jstar == g["jstar"]


def test_hand_tree4_bracket_and_printed_iteration_count(orc):
    """Algorithm 2's printed bracket and iteration count t (log base 2,
    rounded up), derived by hand in the fixture."""
    g = json.load(open(os.path.join(GOLDEN, "hand_tree4.json")))
    res = orc.subpartition(np.array(g["parent"], np.int32), np.array(g["length"]), g["k"], sigma=g["sigma"])
    a0, b0 = _closed(g["alpha0_raw_closed_form"]), _closed(g["beta0_raw_closed_form"])
    assert abs(res.alpha0_raw - a0) <= 1e-15 * a0
    assert abs(res.beta0_raw - b0) <= 1e-15 * b0
    assert res.t_paper == g["t_paper"]
    # the power-of-two bracket encloses the printed one
    assert res.alpha0 <= res.alpha0_raw and res.beta0 > res.beta0_raw
    assert res.alpha0 == 2.0 ** math.floor(math.log2(a0)) and res.beta0 == 2.0 ** math.ceil(math.log2(b0))


def test_underflow_path4(orc):
    """phi_* underflows to 0, so alpha0 = 0: the bisection runs to the smallest
    subnormal and MISO_2 = 0 exactly (hand derivation in the fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "underflow_path4.json")))
    res = orc.subpartition(np.array(g["parent"], np.int32), np.array(g["length"]), g["k"], sigma=g["sigma"])
    assert res.phi_min == 0.0
    assert res.alpha0_raw == 0.0 and res.alpha0 == g["alpha0"] and res.beta0 == g["beta0"]
    assert res.t_paper == g["t_paper"]
    assert res.iters == g["iters"]
    assert res.alpha == g["alpha"] and res.beta == g["beta"] == math.ldexp(1.0, -1074)
    assert res.i_k == g["i_k"]
    np.testing.assert_array_equal(res.labels, g["labels"])
    np.testing.assert_allclose(res.cl_den, [_closed(c) for c in g["cluster_den_closed_form"]], rtol=1e-15)
    assert res.jstar == g["jstar"]
