"""The allocation-free subpartition entry point (iso_subpartition_noalloc,
workspace in the library's fixed device array) against iso_subpartition with a
caller workspace, called through the C ABI: identical labels, i_k, per-cluster
sums and bisection record, on consecutive calls that reuse the array with a
smaller input each time (the largest input it takes first)."""
import ctypes

import numpy as np
import pytest

from paper_1702_04739_amd import _lib, datagen
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_N = 32768  # ISO_SUB_NOALLOC_MAX_N


def _random_tree(n, seed):
    rng = np.random.default_rng(seed)
    parent = np.empty(n, np.int32)
    parent[0] = -1
    parent[1:] = [rng.integers(0, v) for v in range(1, n)]
    length = rng.lognormal(0.0, 0.5, n)
    length[0] = 0.0
    return parent, length


def _run(lib, parent, length, k, noalloc):
    n = parent.shape[0]
    dev = parent.device
    labels = torch.full((n,), -7, dtype=torch.int32, device=dev)
    cnum = torch.empty(k, dtype=torch.float64, device=dev)
    cden = torch.empty(k, dtype=torch.float64, device=dev)
    csize = torch.empty(k, dtype=torch.int32, device=dev)
    info = _lib.SubInfo()
    ik = ctypes.c_double(0.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    args = (ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(length.data_ptr()), n, 0, k, 0.0, None,
            ctypes.c_void_p(labels.data_ptr()), ctypes.byref(ik), ctypes.c_void_p(cnum.data_ptr()),
            ctypes.c_void_p(cden.data_ptr()), ctypes.c_void_p(csize.data_ptr()), ctypes.byref(info))
    if noalloc:
        _lib.check(lib.iso_subpartition_noalloc(*args, stream), "iso_subpartition_noalloc")
    else:
        need = ctypes.c_size_t(0)
        _lib.check(lib.iso_sub_workspace_size(n, k, ctypes.byref(need)), "iso_sub_workspace_size")
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
        _lib.check(lib.iso_subpartition(*args, ctypes.c_void_p(ws.data_ptr()), int(need.value), stream),
                   "iso_subpartition")
    torch.cuda.synchronize()
    rec = {f: getattr(info, f) for f, _ in _lib.SubInfo._fields_ if f != "reserved0"}
    return labels.cpu().numpy(), ik.value, cnum.cpu().numpy(), cden.cpu().numpy(), csize.cpu().numpy(), rec


def _cases():
    import paper_1702_04739_amd as iso
    # largest first, then smaller inputs into the same array
    X = torch.from_numpy(datagen.config(5, n=MAX_N)).cuda()
    p, l, _ = iso.mst(X)
    yield "blobs n=%d (MST), k=16" % MAX_N, p, l, 16
    p, l = _random_tree(5000, 11)
    yield "random tree n=5000, k=40", torch.from_numpy(p).cuda(), torch.from_numpy(l).cuda(), 40
    X = torch.from_numpy(datagen.config(1)).cuda()
    p, l, _ = iso.mst(X)
    yield "gaussian mixture n=2000 (MST), k=5", p, l, 5
    p, l = _random_tree(3, 12)
    yield "random tree n=3, k=3", torch.from_numpy(p).cuda(), torch.from_numpy(l).cuda(), 3


def test_noalloc_equals_workspace_entry_point():
    lib = _lib.load(build_if_missing=False)
    for name, parent, length, k in _cases():
        H.log("noalloc subpartition: %s" % name)
        ref = _run(lib, parent, length, k, noalloc=False)
        got = _run(lib, parent, length, k, noalloc=True)
        np.testing.assert_array_equal(got[0], ref[0])
        assert got[1] == ref[1]
        np.testing.assert_array_equal(got[2], ref[2])
        np.testing.assert_array_equal(got[3], ref[3])
        np.testing.assert_array_equal(got[4], ref[4])
        assert got[5] == ref[5]
        assert (got[0] >= -1).all() and (got[0] < k).all()


def test_noalloc_rejects_beyond_maximum():
    lib = _lib.load(build_if_missing=False)
    n = MAX_N + 1
    parent = torch.full((n,), 0, dtype=torch.int32, device="cuda")
    parent[0] = -1
    length = torch.ones(n, dtype=torch.float64, device="cuda")
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    ik = ctypes.c_double(0.0)
    rc = lib.iso_subpartition_noalloc(ctypes.c_void_p(parent.data_ptr()), ctypes.c_void_p(length.data_ptr()), n, 0,
                                      4, 0.0, None, ctypes.c_void_p(labels.data_ptr()), ctypes.byref(ik), None, None,
                                      None, None, None)
    assert rc == -1
    assert b"maximum" in lib.iso_last_error()
