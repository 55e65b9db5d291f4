"""FP64 CPU oracle of the clustering method -- TEST INFRASTRUCTURE ONLY.

Thin ctypes binding of ``oracle.c`` (a plain, slow FP64
implementation of the Euclidean MST by dense Prim, Sec. 3.5 / Algorithm 3, and
of the isoperimetric tree search, Sec. 2.2 / Algorithms 1-2, with the labelling
of Algorithm 4).  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the GPU library never
does, and this package imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Every FP64 operation in oracle.c is a separately rounded IEEE operation in the
# order written: no contraction into fused multiply-adds, no fast-math.
# OpenMP is used only by the threaded variant of Prim (its thread count is an
# explicit argument; every other routine runs on one thread).
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (idempotent unless ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _SubInfo(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double),
        ("phi_sum", ctypes.c_double), ("phi_min", ctypes.c_double),
        ("omega_sum", ctypes.c_double), ("omega_min", ctypes.c_double),
        ("p_sum", ctypes.c_double), ("p_min", ctypes.c_double),
        ("alpha0_raw", ctypes.c_double), ("beta0_raw", ctypes.c_double),
        ("alpha0", ctypes.c_double), ("beta0", ctypes.c_double),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("i_k", ctypes.c_double),
        ("t_paper", ctypes.c_int32), ("iters", ctypes.c_int32),
        ("jstar", ctypes.c_int32), ("max_depth", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        D = ctypes.c_double
        lib.orc_sqdist.argtypes = [P, I64, I64, I64, I64]
        lib.orc_sqdist.restype = D
        lib.orc_prim_mst.argtypes = [P, I64, I64, I64, P, P, P, P]
        lib.orc_prim_mst.restype = ctypes.c_int
        lib.orc_prim_mst_threads.argtypes = [P, I64, I64, I64, P, P, P, P, I32]
        lib.orc_prim_mst_threads.restype = ctypes.c_int
        lib.orc_tree_depth.argtypes = [P, I64, I32, P]
        lib.orc_tree_depth.restype = ctypes.c_int
        lib.orc_tree_order.argtypes = [P, I64, P]
        lib.orc_tree_order.restype = ctypes.c_int
        lib.orc_lower_median.argtypes = [P, P, I64]
        lib.orc_lower_median.restype = D
        lib.orc_tree_weights.argtypes = [P, P, I64, I32, D, ctypes.c_int, ctypes.c_int, D, P, I64, I64, P, P, P]
        lib.orc_tree_weights.restype = ctypes.c_int
        lib.orc_decide.argtypes = [P, P, P, P, P, I64, I64, D, P, P, P, P, P, P]
        lib.orc_decide.restype = I64
        lib.orc_subpartition.argtypes = [P, P, I64, I32, I64, D, ctypes.c_int, ctypes.c_int, ctypes.c_int, D, I32,
                                         P, I64, I64, P, P, P, P, ctypes.POINTER(_SubInfo)]
        lib.orc_subpartition.restype = ctypes.c_int
        lib.orc_backward.argtypes = [P, I64, I64, I64, P, I32, P, I32, D, ctypes.c_int, D, D, P, P, P, P, P]
        lib.orc_backward.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _f32(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("points must be a 2-D array")
    return X


def sqdist(X, i: int, j: int) -> float:
    """FP64 squared distance, left-to-right over coordinates."""
    X = _f32(X)
    return _load().orc_sqdist(_ptr(X), X.shape[1], X.shape[1], i, j)


def prim_mst(X, threads: int = 1):
    """Euclidean MST by dense Prim from vertex 0 (Algorithm 3, sequential).

    ``threads`` > 1 splits each step's key update over that many threads (same
    result).  Returns (parent int32[n] with parent[0] = -1, length float64[n]
    with length[0] = 0, depth int32[n], order_added int32[n])."""
    X = _f32(X)
    n, d = X.shape
    parent = np.empty(n, np.int32)
    length = np.empty(n, np.float64)
    depth = np.empty(n, np.int32)
    added = np.empty(n, np.int32)
    rc = _load().orc_prim_mst_threads(_ptr(X), n, d, d, _ptr(parent), _ptr(length), _ptr(depth), _ptr(added),
                                      int(threads))
    if rc != 0:
        raise RuntimeError("orc_prim_mst failed: %d" % rc)
    return parent, length, depth, added


def tree_depth(parent, root: int = 0):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    depth = np.empty(parent.shape[0], np.int32)
    rc = _load().orc_tree_depth(_ptr(parent), parent.shape[0], root, _ptr(depth))
    if rc != 0:
        raise ValueError("not a tree rooted at %d (rc=%d)" % (root, rc))
    return depth


def tree_order(depth):
    depth = np.ascontiguousarray(depth, dtype=np.int32)
    order = np.empty(depth.shape[0], np.int32)
    _load().orc_tree_order(_ptr(depth), depth.shape[0], _ptr(order))
    return order


def lower_median(parent, length) -> float:
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    length = np.ascontiguousarray(length, dtype=np.float64)
    return _load().orc_lower_median(_ptr(parent), _ptr(length), parent.shape[0])


OMEGA = {"tree": 0, "full": 1}
PHI = {"exp": 0, "gauss_sq": 1}
BRACKET = {"pow2": 0, "paper": 1}


def tree_weights(parent, length, sigma, root=0, omega="tree", phi="exp", alpha_pot=0.0, X=None):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    length = np.ascontiguousarray(length, dtype=np.float64)
    n = parent.shape[0]
    Xc = _f32(X) if X is not None else None
    d = Xc.shape[1] if Xc is not None else 0
    ph = np.empty(n, np.float64)
    om = np.empty(n, np.float64)
    p0 = np.empty(n, np.float64)
    rc = _load().orc_tree_weights(_ptr(parent), _ptr(length), n, root, float(sigma), OMEGA[omega], PHI[phi],
                                  float(alpha_pot), _ptr(Xc), d, d, _ptr(ph), _ptr(om), _ptr(p0))
    if rc != 0:
        raise RuntimeError("orc_tree_weights failed: %d" % rc)
    return ph, om, p0


def decide(parent, order, phi, omega0, p0, k: int, N: float, record: bool = False):
    """Algorithm 1 at threshold N.  Returns the number of cuts reached (YES iff
    == k); with ``record`` also (cut vertices, num, den, joined)."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    omega0 = np.ascontiguousarray(omega0, dtype=np.float64)
    p0 = np.ascontiguousarray(p0, dtype=np.float64)
    n = parent.shape[0]
    wb = np.empty(n, np.float64)
    pb = np.empty(n, np.float64)
    if record:
        cut = np.full(k, -1, np.int32)
        num = np.zeros(k, np.float64)
        den = np.zeros(k, np.float64)
        joined = np.zeros(n, np.uint8)
    else:
        cut = num = den = joined = None
    j = _load().orc_decide(_ptr(parent), _ptr(order), _ptr(phi), _ptr(omega0), _ptr(p0), n, k, float(N),
                           _ptr(wb), _ptr(pb), _ptr(cut), _ptr(num), _ptr(den), _ptr(joined))
    if record:
        return j, cut[:j], num[:j], den[:j], joined
    return j


@dataclass
class SubResult:
    labels: np.ndarray
    cl_num: np.ndarray
    cl_den: np.ndarray
    cl_size: np.ndarray
    sigma: float
    i_k: float
    jstar: int
    alpha0_raw: float
    beta0_raw: float
    alpha0: float
    beta0: float
    alpha: float
    beta: float
    t_paper: int
    iters: int
    max_depth: int
    phi_sum: float
    phi_min: float
    omega_sum: float
    omega_min: float
    p_sum: float
    p_min: float


def subpartition(parent, length, k: int, sigma: float = 0.0, root: int = 0, omega="tree", phi="exp",
                 bracket="pow2", alpha_pot=0.0, max_iters=2000, X=None) -> SubResult:
    """Algorithm 2 (to FP64 resolution) + Algorithm 4 labelling on a rooted tree.

    ``sigma`` = 0 selects the lower median of the tree edge lengths."""
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    length = np.ascontiguousarray(length, dtype=np.float64)
    n = parent.shape[0]
    Xc = _f32(X) if X is not None else None
    d = Xc.shape[1] if Xc is not None else 0
    labels = np.empty(n, np.int32)
    num = np.empty(k, np.float64)
    den = np.empty(k, np.float64)
    size = np.empty(k, np.int32)
    info = _SubInfo()
    rc = _load().orc_subpartition(_ptr(parent), _ptr(length), n, root, k, float(sigma), OMEGA[omega], PHI[phi],
                                  BRACKET[bracket], float(alpha_pot), int(max_iters), _ptr(Xc), d, d,
                                  _ptr(labels), _ptr(num), _ptr(den), _ptr(size), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("orc_subpartition failed: %d" % rc)
    return SubResult(labels=labels, cl_num=num, cl_den=den, cl_size=size, sigma=info.sigma, i_k=info.i_k,
                     jstar=info.jstar, alpha0_raw=info.alpha0_raw, beta0_raw=info.beta0_raw, alpha0=info.alpha0,
                     beta0=info.beta0, alpha=info.alpha, beta=info.beta, t_paper=info.t_paper, iters=info.iters,
                     max_depth=info.max_depth, phi_sum=info.phi_sum, phi_min=info.phi_min,
                     omega_sum=info.omega_sum, omega_min=info.omega_min, p_sum=info.p_sum, p_min=info.p_min)


def backward(X, parent, labels, jstar: int, sigma: float, gW: float = 1.0, gI: float = 1.0, root: int = 0,
             phi="exp"):
    """Adjoint of W (total MST length) and I (cost of cluster ``jstar``) with the
    tree and the subpartition fixed.  Returns (gX float64[n,d], gsigma, W, I, n_degenerate)."""
    Xc = _f32(X)
    n, d = Xc.shape
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    gX = np.empty((n, d), np.float64)
    gs = np.zeros(1, np.float64)
    W = np.zeros(1, np.float64)
    I = np.zeros(1, np.float64)
    nd = np.zeros(1, np.int64)
    rc = _load().orc_backward(_ptr(Xc), n, d, d, _ptr(parent), root, _ptr(labels), int(jstar), float(sigma),
                              PHI[phi], float(gW), float(gI), _ptr(gX), _ptr(gs), _ptr(W), _ptr(I), _ptr(nd))
    if rc != 0:
        raise RuntimeError("orc_backward failed: %d" % rc)
    return gX, float(gs[0]), float(W[0]), float(I[0]), int(nd[0])


def run(X, k: int, sigma: float = 0.0, **kw):
    """End-to-end oracle: Prim MST then the tree search."""
    parent, length, _, _ = prim_mst(X)
    res = subpartition(parent, length, k, sigma=sigma, X=X if kw.get("omega", "tree") != "tree" or
                       kw.get("alpha_pot", 0.0) else None, **kw)
    return parent, length, res
