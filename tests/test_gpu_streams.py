"""GPU: MST calls on several streams at once.

A pruned MST call uses a second stream, its events and a pinned staging
buffer, which the library keeps per device and lends to one call at a time.
Calls issued together from two host threads on two streams (and calls on a
stream other than the default one) must each take their own set and return
the tree of a call made alone, bit for bit; the same holds for repeated calls,
which reuse the sets.
"""
import threading

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


def _mst(iso, X, stream=None):
    if stream is None:
        parent, length, info = iso.mst(X, precision="bf16", recheck="fp32")
    else:
        with torch.cuda.stream(stream):
            parent, length, info = iso.mst(X, precision="bf16", recheck="fp32")
        stream.synchronize()
    return parent.cpu().numpy(), length.cpu().numpy(), info


def test_concurrent_calls_on_two_streams(iso):
    Xa = torch.from_numpy(datagen.config(3, n=20000)).cuda()
    Xb = torch.from_numpy(datagen.config(5, n=12000)).cuda()
    H.log("reference calls (default stream): c3 n=20000, c5 n=12000")
    pa, la, ia = _mst(iso, Xa)
    pb, lb, ib = _mst(iso, Xb)
    assert ia["tile_pairs"] < ia["tile_pairs_full"] and ib["tile_pairs"] < ib["tile_pairs_full"]  # pruned calls
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]
    err = []

    def run(slot, X):
        try:
            for _ in range(3):
                out[slot] = _mst(iso, X, streams[slot])
        except Exception as e:  # reported by the main thread
            err.append(e)

    H.log("two host threads, two streams, three calls each")
    th = [threading.Thread(target=run, args=(0, Xa)), threading.Thread(target=run, args=(1, Xb))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in th), "a thread did not finish"
    assert not err, err
    np.testing.assert_array_equal(out[0][0], pa)
    np.testing.assert_array_equal(out[0][1], la)
    np.testing.assert_array_equal(out[1][0], pb)
    np.testing.assert_array_equal(out[1][1], lb)
    H.log("  both threads' trees equal the calls made alone")
