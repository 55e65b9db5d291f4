"""The C-ABI library loads on the CPU-only host, exports every symbol the
header declares, sizes workspaces, and rejects invalid arguments before any
device work (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

from paper_1702_04739_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isoclust.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(iso_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    declared = _declared()
    assert declared, "no declarations parsed"
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_last_error():
    lib = _lib.load()
    assert b"gfx950" in lib.iso_version()
    assert isinstance(lib.iso_last_error(), bytes)


def test_workspace_sizes():
    lib = _lib.load()
    sz = ctypes.c_size_t(0)
    assert lib.iso_mst_workspace_size(200_000, 784, 0, ctypes.byref(sz)) == 0
    big = sz.value
    assert big > 200_000 * 784 * 4
    assert lib.iso_mst_workspace_size(2000, 16, 0, ctypes.byref(sz)) == 0
    assert 0 < sz.value < big
    assert lib.iso_sub_workspace_size(1000, 5, ctypes.byref(sz)) == 0
    assert sz.value > 1000 * 64 * 16
    assert lib.iso_mst_workspace_size(1, 16, 0, ctypes.byref(sz)) == -1
    assert lib.iso_mst_workspace_size(10, 0, 0, ctypes.byref(sz)) == -1
    assert lib.iso_mst_workspace_size(10, 4, 9, ctypes.byref(sz)) == -1
    assert lib.iso_sub_workspace_size(10, 1, ctypes.byref(sz)) == -1
    assert lib.iso_sub_workspace_size(10, 11, ctypes.byref(sz)) == -1
    assert lib.iso_mst_workspace_size(10, 4, 0, None) == -1


def _p(v):
    return ctypes.c_void_p(v)


def test_mst_argument_validation():
    lib = _lib.load()
    info = _lib.MstInfo()
    dummy = _p(0x1000)
    # NULL points
    assert lib.iso_mst(None, 10, 4, 4, 0, 0, 0, dummy, dummy, ctypes.byref(info), None, 0, None) == -1
    assert b"non-NULL" in lib.iso_last_error()
    # n < 2, d < 1, ld < d, unknown precision / recheck
    assert lib.iso_mst(dummy, 1, 4, 4, 0, 0, 0, dummy, dummy, None, None, 0, None) == -1
    assert lib.iso_mst(dummy, 10, 0, 4, 0, 0, 0, dummy, dummy, None, None, 0, None) == -1
    assert lib.iso_mst(dummy, 10, 4, 3, 0, 0, 0, dummy, dummy, None, None, 0, None) == -1
    assert b"ld" in lib.iso_last_error()
    assert lib.iso_mst(dummy, 10, 4, 4, 7, 0, 0, dummy, dummy, None, None, 0, None) == -1
    assert lib.iso_mst(dummy, 10, 4, 4, 0, 5, 0, dummy, dummy, None, None, 0, None) == -1
    # the old encoding (option bits OR-ed into recheck) is rejected: recheck is
    # only ISO_RECHECK_*, the options have their own argument
    assert lib.iso_mst(dummy, 10, 4, 4, 0, 0x100, 0, dummy, dummy, None, None, 0, None) == -1
    assert b"recheck" in lib.iso_last_error()


def test_mst_flags_validation():
    """iso_mst's flags argument takes exactly the ISO_MST_* bits; unknown
    bits are rejected before any device work."""
    lib = _lib.load()
    dummy = _p(0x1000)
    for bad in (0x20, 0x40, 0x100, 0x80000000):
        assert lib.iso_mst(dummy, 10, 4, 4, 0, 0, bad, dummy, dummy, None, None, 0, None) == -1
        assert b"flag" in lib.iso_last_error()
    assert (_lib.MST_NO_LISTS | _lib.MST_NO_FINAL | _lib.MST_NO_ESCALATE | _lib.MST_PAIR_BOUNDS
            | _lib.MST_NO_PRUNE) == 0x1F


def test_subpartition_argument_validation():
    lib = _lib.load()
    dummy = _p(0x1000)
    ik = ctypes.c_double(0)
    args = dict(parent=dummy, length=dummy, n=10, root=0, k=3, sigma=0.0)

    def call(**kw):
        a = dict(args, **kw)
        return lib.iso_subpartition(a["parent"], a["length"], a["n"], a["root"], a["k"], a["sigma"], None, dummy,
                                    ctypes.byref(ik), None, None, None, None, None, 0, None)

    assert call(parent=None) == -1
    assert call(n=1) == -1
    assert call(k=1) == -1
    assert call(k=11) == -1
    assert call(root=10) == -1
    assert call(root=-1) == -1
    assert call(sigma=-1.0) == -1
    assert call(sigma=float("inf")) == -1
    assert call(sigma=float("nan")) == -1
    bad = _lib.SubOpts(3, 0, 0, 0)
    assert lib.iso_subpartition(dummy, dummy, 10, 0, 3, 0.0, ctypes.byref(bad), dummy, ctypes.byref(ik), None, None,
                                None, None, None, 0, None) == -1


def test_subpartition_noalloc_argument_validation():
    """The allocation-free entry point validates like iso_subpartition and
    rejects n beyond its fixed array's maximum, before any device work."""
    lib = _lib.load()
    dummy = _p(0x1000)
    ik = ctypes.c_double(0)

    def call(n=10, k=3, root=0, sigma=0.0, parent=dummy):
        return lib.iso_subpartition_noalloc(parent, dummy, n, root, k, sigma, None, dummy, ctypes.byref(ik), None,
                                            None, None, None, None)

    assert call(parent=None) == -1
    assert call(n=1) == -1
    assert call(k=11) == -1
    assert call(root=10) == -1
    assert call(sigma=float("nan")) == -1
    assert call(n=32769, k=4) == -1
    assert b"maximum" in lib.iso_last_error()


def test_no_cpu_fallback():
    """The Python API has no CPU path: CPU tensors are rejected."""
    torch = pytest.importorskip("torch")
    import paper_1702_04739_amd as iso
    with pytest.raises(ValueError):
        iso.mst(torch.zeros(4, 2))


def test_header_constants_match_binding():
    """The binding's option and enum values are the header's."""
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                            "isoclust.h")).read()
    defs = {m.group(1): int(m.group(2), 0) for m in re.finditer(r"#define\s+(ISO_\w+)\s+\(?(-?(?:0x)?[0-9A-Fa-f]+)\)?", src)}
    for name, v in _lib.PRECISION.items():
        assert defs["ISO_PREC_" + name.upper()] == v
    for name, v in _lib.RECHECK.items():
        assert defs["ISO_RECHECK_" + name.upper()] == v
    assert defs["ISO_MST_NO_LISTS"] == _lib.MST_NO_LISTS
    assert defs["ISO_MST_NO_FINAL"] == _lib.MST_NO_FINAL
    assert defs["ISO_MST_NO_ESCALATE"] == _lib.MST_NO_ESCALATE
    assert defs["ISO_MST_PAIR_BOUNDS"] == _lib.MST_PAIR_BOUNDS
    assert defs["ISO_OMEGA_FULL"] == _lib.OMEGA["full"]
    for code, name in _lib.ERRORS.items():
        if name in defs:
            assert defs[name] == code
