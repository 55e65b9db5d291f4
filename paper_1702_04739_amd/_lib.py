"""ctypes binding of libisoclust.so (the C ABI declared in include/isoclust.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  There is no fallback: if the library cannot be loaded, or the GPU is
not a gfx950, calls raise.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisoclust.so")

ISO_OK = 0
ERRORS = {
    -1: "ISO_ERR_INVALID_ARG", -2: "ISO_ERR_NONFINITE", -3: "ISO_ERR_NO_DEVICE", -4: "ISO_ERR_HIP",
    -5: "ISO_ERR_OOM", -6: "ISO_ERR_WORKSPACE", -7: "ISO_ERR_INTERNAL",
}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2, "int8": 3}
RECHECK = {"fp32": 0, "fp64": 1}
MST_NO_LISTS = 0x1
MST_NO_FINAL = 0x2
MST_NO_ESCALATE = 0x4
MST_PAIR_BOUNDS = 0x8
MST_NO_PRUNE = 0x10
OMEGA = {"tree": 0, "full": 1}
PHI = {"exp": 0, "gauss_sq": 1}
BRACKET = {"pow2": 0, "paper": 1}

# Every symbol include/isoclust.h declares.
EXPORTS = ["iso_mst_workspace_size", "iso_mst", "iso_sub_workspace_size", "iso_subpartition",
           "iso_subpartition_all_k", "iso_subpartition_noalloc", "iso_backward_workspace_size", "iso_backward", "iso_graph_weights", "iso_sigma_median", "iso_mst_prim_workspace_size", "iso_mst_prim",
           "iso_timing_enable",
           "iso_timing_read", "iso_last_error", "iso_version"]


class IsoError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__("%s returned %s (%d): %s" % (fn, ERRORS.get(code, "?"), code, msg))
        self.code = code


class MstInfo(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("list_rounds", ctypes.c_int32), ("candidates", ctypes.c_int64),
                ("rescanned_rows", ctypes.c_int64), ("mst_weight", ctypes.c_double),
                ("final_components", ctypes.c_int32), ("screen_precision", ctypes.c_int32),
                ("pair_bounds", ctypes.c_int32), ("tile_pairs", ctypes.c_int64),
                ("tile_pairs_full", ctypes.c_int64)]


class SubOpts(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_int32), ("phi", ctypes.c_int32), ("bracket", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("omega0", ctypes.c_void_p), ("p0", ctypes.c_void_p)]


class SubInfo(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("alpha0_raw", ctypes.c_double), ("beta0_raw", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("beta0", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("i_k", ctypes.c_double), ("t_paper", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("passes", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("jstar", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int32), ("screen_launches", ctypes.c_int32), ("screen_ms", ctypes.c_double),
                ("screen_pairs", ctypes.c_double), ("screen_dim", ctypes.c_double), ("mst_calls", ctypes.c_int32),
                ("sub_calls", ctypes.c_int32), ("mst_ms", ctypes.c_double), ("sub_ms", ctypes.c_double),
                ("sub_passes", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


_lib = None


def load(build_if_missing: bool = True):
    """Load libisoclust.so (building it once if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError("libisoclust.so is not built (run __graft_entry__.build())")
        from .csrc import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    lib.iso_mst_workspace_size.argtypes = [I64, I64, I32, ctypes.POINTER(SZ)]
    lib.iso_mst.argtypes = [P, I64, I64, I64, I32, I32, ctypes.c_uint32, P, P, ctypes.POINTER(MstInfo), P, SZ, P]
    lib.iso_sub_workspace_size.argtypes = [I64, I32, ctypes.POINTER(SZ)]
    lib.iso_subpartition.argtypes = [P, P, I64, I32, I32, D, ctypes.POINTER(SubOpts), P, ctypes.POINTER(D), P, P, P,
                                     ctypes.POINTER(SubInfo), P, SZ, P]
    lib.iso_subpartition_noalloc.argtypes = [P, P, I64, I32, I32, D, ctypes.POINTER(SubOpts), P, ctypes.POINTER(D), P,
                                             P, P, ctypes.POINTER(SubInfo), P]
    lib.iso_backward_workspace_size.argtypes = [I64, ctypes.POINTER(SZ)]
    lib.iso_backward.argtypes = [P, I64, I64, I64, P, P, I32, D, I32, D, D, P, I64, ctypes.POINTER(D),
                                 ctypes.POINTER(D), P, SZ, P]
    lib.iso_graph_weights.argtypes = [P, I64, I64, I64, D, I32, D, P, P, P]
    lib.iso_mst_prim_workspace_size.argtypes = [I64, ctypes.POINTER(SZ)]
    lib.iso_mst_prim.argtypes = [P, I64, I64, I64, P, P, P, P, SZ, P]
    lib.iso_subpartition_all_k.argtypes = [P, P, I64, I32, I32, D, ctypes.POINTER(SubOpts), P, P,
                                           ctypes.POINTER(I32), P, SZ, P]
    lib.iso_sigma_median.argtypes = [P, P, I64, ctypes.POINTER(D), P]
    for f in ("iso_mst_workspace_size", "iso_mst", "iso_sub_workspace_size", "iso_subpartition",
              "iso_backward_workspace_size", "iso_backward", "iso_graph_weights", "iso_sigma_median",
              "iso_subpartition_all_k", "iso_subpartition_noalloc", "iso_mst_prim_workspace_size", "iso_mst_prim"):
        getattr(lib, f).restype = ctypes.c_int32
    lib.iso_timing_enable.argtypes = [I32]
    lib.iso_timing_enable.restype = ctypes.c_int32
    lib.iso_timing_read.argtypes = [ctypes.POINTER(Timing)]
    lib.iso_timing_read.restype = ctypes.c_int32
    lib.iso_last_error.restype = ctypes.c_char_p
    lib.iso_last_error.argtypes = []
    lib.iso_version.restype = ctypes.c_char_p
    lib.iso_version.argtypes = []
    _lib = lib
    return lib


def check(rc: int, fn: str):
    if rc != ISO_OK:
        raise IsoError(rc, fn, load().iso_last_error().decode())


def timing_enable(on: bool = True):
    load().iso_timing_enable(1 if on else 0)


def timing_read() -> dict:
    t = Timing()
    check(load().iso_timing_read(ctypes.byref(t)), "iso_timing_read")
    return {f: getattr(t, f) for f, _ in Timing._fields_ if f != "reserved0"}
